// Device helpers shared by the gfx950 kernel files.
#pragma once
#include "vbd_internal.h"

namespace vbd {

__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float3 a, float s) { return make_float3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float3 operator-(float3 a) { return make_float3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b)
{
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 xyz(float4 a) { return make_float3(a.x, a.y, a.z); }
// X[q] for a slot q >= 0, addressed by a 32-bit byte offset from the array
// base (a topology holds at most 2^28 vertices), so that the load takes its
// base from scalar registers and the address costs one shift.
__device__ __forceinline__ float4 ld_slot(const float4 *X, int q)
{
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(X) + ((unsigned)q << 4));
}
__device__ __forceinline__ float3 ld3(const float *p, int i)
{
    return make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}
__device__ __forceinline__ void st3(float *p, int i, float3 v)
{
    p[3 * i] = v.x; p[3 * i + 1] = v.y; p[3 * i + 2] = v.z;
}

__device__ __forceinline__ float3 normalize3(float3 a)
{
    return a * (1.0f / sqrtf(dot3(a, a)));
}

// Closest point q on triangle (a, b, c) to p, by the Voronoi-region tests of
// Ericson, Real-Time Collision Detection (2005), Sec. 5.1.5.  Returns the
// barycentric weights (w0, w1, w2) of q and its feature:
//   0 face interior, 1/2/3 vertex a/b/c, 4/5/6 edge ab/bc/ca.
struct ClosestPt {
    float3 q;
    float w0, w1, w2;
    int feature;
};

__device__ __forceinline__ ClosestPt closest_on_triangle(float3 p, float3 a, float3 b, float3 c)
{
    ClosestPt r;
    const float3 ab = b - a, ac = c - a, ap = p - a;
    const float d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.f && d2 <= 0.f) { r.q = a; r.w0 = 1.f; r.w1 = 0.f; r.w2 = 0.f; r.feature = 1; return r; }
    const float3 bp = p - b;
    const float d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.f && d4 <= d3) { r.q = b; r.w0 = 0.f; r.w1 = 1.f; r.w2 = 0.f; r.feature = 2; return r; }
    const float vc = d1 * d4 - d3 * d2;
    if (vc <= 0.f && d1 >= 0.f && d3 <= 0.f) {
        const float v = d1 / (d1 - d3);
        r.q = a + ab * v; r.w0 = 1.f - v; r.w1 = v; r.w2 = 0.f; r.feature = 4;
        return r;
    }
    const float3 cp = p - c;
    const float d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0.f && d5 <= d6) { r.q = c; r.w0 = 0.f; r.w1 = 0.f; r.w2 = 1.f; r.feature = 3; return r; }
    const float vb = d5 * d2 - d1 * d6;
    if (vb <= 0.f && d2 >= 0.f && d6 <= 0.f) {
        const float w = d2 / (d2 - d6);
        r.q = a + ac * w; r.w0 = 1.f - w; r.w1 = 0.f; r.w2 = w; r.feature = 6;
        return r;
    }
    const float va = d3 * d6 - d5 * d4;
    if (va <= 0.f && (d4 - d3) >= 0.f && (d5 - d6) >= 0.f) {
        const float w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        r.q = b + (c - b) * w; r.w0 = 0.f; r.w1 = 1.f - w; r.w2 = w; r.feature = 5;
        return r;
    }
    const float den = 1.0f / (va + vb + vc);
    const float v = vb * den, w = vc * den;
    r.q = a + ab * v + ac * w; r.w0 = 1.f - v - w; r.w1 = v; r.w2 = w; r.feature = 0;
    return r;
}


// Closest points of the segments p0 + s (p1 - p0) and q0 + u (q1 - q0), s, u
// in [0, 1], and their squared distance: the clamped solve of Ericson,
// Real-Time Collision Detection (2005), Sec. 5.1.9 (s from the unconstrained
// minimum clamped to [0, 1], u for that s; when u leaves [0, 1] it is clamped
// and s solved again).  Edges have positive length.
struct SegPt {
    float s, u, d2;
};

__device__ __forceinline__ SegPt seg_closest(float3 p0, float3 p1, float3 q0, float3 q1)
{
    const float3 d1 = p1 - p0, d2 = q1 - q0, r = p0 - q0;
    const float a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
    const float c = dot3(d1, r), b = dot3(d1, d2);
    const float den = a * e - b * b;
    float s = den > 0.f ? fminf(fmaxf((b * f - c * e) / den, 0.f), 1.f) : 0.f;
    float u = (b * s + f) / e;
    if (u < 0.f) {
        u = 0.f;
        s = fminf(fmaxf(-c / a, 0.f), 1.f);
    } else if (u > 1.f) {
        u = 1.f;
        s = fminf(fmaxf((b - c) / a, 0.f), 1.f);
    }
    const float3 w = r + d1 * s - d2 * u;
    SegPt out;
    out.s = s;
    out.u = u;
    out.d2 = dot3(w, w);
    return out;
}

}  // namespace vbd
