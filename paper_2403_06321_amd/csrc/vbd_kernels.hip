// gfx950 kernels of the VBD hot path.
//
// Vertex Block Descent (Chen, Liu, Yang, Yuksel, ACM TOG 2024).  A color
// phase updates every free vertex of one color in parallel (Sec. 3.9).  One
// vertex is handled by a group of L lanes of a wave64: the lanes stride over
// the vertex's incident elements (per-color padded records whose addresses
// follow from the vertex's slot), each accumulating the element force and
// 3x3 Hessian block, then the group reduces the 9 values
// with DPP row operations, adds inertia / damping / contact / friction terms
// and solves the 3x3 system analytically (Sec. 3.2).
#include "vbd_device.h"

#include <algorithm>

namespace vbd {

// Lane permutation within a row of 16 lanes.  Every pattern used here reads a
// valid lane of the same row, so the 0 written for an invalid source lane
// (bound_ctrl) never appears; with that 0 (the identity of the add that
// follows) the compiler folds the move into the add as one DPP instruction.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over aligned groups of L lanes (L = 2, 4, 8, 16, 32, 64); every lane of
// the group receives the total.  Must be called with the whole wave active.
template <int L>
__device__ __forceinline__ float group_sum(float v)
{
    v += dpp_mov<0xB1>(v);              // quad_perm [1,0,3,2]  (xor 1)
    if (L >= 4) v += dpp_mov<0x4E>(v);  // quad_perm [2,3,0,1]  (xor 2)
    if (L >= 8) v += dpp_mov<0x141>(v); // row_half_mirror      (lane i <-> 7-i)
    if (L >= 16) v += dpp_mov<0x140>(v);// row_mirror           (lane i <-> 15-i)
    if (L >= 32) v += __shfl_xor(v, 16);
    if (L >= 64) v += __shfl_xor(v, 32);
    return v;
}

// blockIdx -> logical block; the 8 XCDs receive blocks round-robin.
// remap 1: each XCD gets a contiguous range of logical blocks.  remap 2:
// chunks of kXcdChunk consecutive logical blocks are dealt to the XCDs in
// turn (neighbouring vertices share an L2 within a chunk, and the XCDs' work
// stays interleaved over the color); the blocks past the last whole round of
// 8 chunks keep their index.  Both are bijections on [0, nb).
constexpr int kXcdChunk = 16;
__device__ __forceinline__ int xcd_block(int b, int nb, int remap)
{
    // mapping 3 splits colors at mesh boundaries where the launcher has the
    // split (XcdSplit); elsewhere it maps as 1
    if (!remap) return b;
    const int x = b & 7;
    if (remap == 2) {
        const int full = nb / (8 * kXcdChunk) * (8 * kXcdChunk);
        if (b >= full) return b;
        const int k = b >> 3;   // this block's turn on its XCD
        return ((k / kXcdChunk) * 8 + x) * kXcdChunk + k % kXcdChunk;
    }
    const int q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// --------------------------------------------------------- element terms --
struct Acc {
    float fx, fy, fz, hxx, hxy, hxz, hyy, hyz, hzz;
};

__device__ __forceinline__ void acc_zero(Acc &a)
{
    a.fx = a.fy = a.fz = a.hxx = a.hxy = a.hxz = a.hyy = a.hyz = a.hzz = 0.f;
}

// One tet seen from the vertex i it is solved for (stable Neo-Hookean of
// Sec. 5, in the local system of Sec. 3.2): f_i -= V (mu F m + lam (J - alpha) cof(F) m) and
// H_ii += V (mu |m|^2 I + lam (cof(F) m)(cof(F) m)^T), m the vertex's shape
// gradient.  With the pair's rest frame S (F' = D_s' S, D_s' = [e1 e2 e3],
// e_k = x_k - x_i for the other vertices a, b, c):
//   F m = D_s' (S m) = w0 e1 + w1 e2 + w2 e3                (w = S m),
//   cof(F) m = dJ/dx_i = -sigma (x_b - x_a) x (x_c - x_a) = -n (sigma = det S),
//   J = sigma det D_s' = e1 . n,
// so f_i += V lam (J - alpha) n - V mu F m and H_ii += V mu |m|^2 I + V lam n n^T,
// where |m|^2 = -(w0 + w1 + w2) (w_k = s_k . m for the rows s_k of S, which sum
// to -m).  Record: pa.w = V lam, W.xyz = V mu w, hmu = V mu |m|^2.
__device__ __forceinline__ void pair_accumulate(float Vlam, float4 W, float sigma, float hmu,
                                                float4 own, float4 qa, float4 qb, float4 qc,
                                                const StepConsts &K, Acc &a)
{
    const float3 xi = xyz(own), xa = xyz(qa), xb = xyz(qb), xc = xyz(qc);
    const float3 e1 = xa - xi, e2 = xb - xi, e3 = xc - xi;
    const float3 n = cross3(xb - xa, xc - xa) * sigma;
    const float J = dot3(e1, n);
    const float s = Vlam * (J - K.alpha);
    // f += s n - F m, F m = W.x e1 + W.y e2 + W.z e3, as four FMAs per component
    a.fx = fmaf(-W.z, e3.x, fmaf(-W.y, e2.x, fmaf(-W.x, e1.x, fmaf(s, n.x, a.fx))));
    a.fy = fmaf(-W.z, e3.y, fmaf(-W.y, e2.y, fmaf(-W.x, e1.y, fmaf(s, n.y, a.fy))));
    a.fz = fmaf(-W.z, e3.z, fmaf(-W.y, e2.z, fmaf(-W.x, e1.z, fmaf(s, n.z, a.fz))));
    const float3 ln = n * Vlam;
    a.hxx += hmu + ln.x * n.x;
    a.hxy += ln.x * n.y;
    a.hxz += ln.x * n.z;
    a.hyy += hmu + ln.y * n.y;
    a.hyz += ln.y * n.z;
    a.hzz += hmu + ln.z * n.z;
}

// Tet terms of one vertex (permuted slot p) from its D consecutive pair
// records starting at index e0: the lanes of the group take records lane,
// lane + L, ...; each lane issues the loads of KU records together (their
// addresses follow from the slot alone, so they go out with the vertex's own
// state), then the KU x 3 neighbour positions together.  Padding records
// (and slots past D) name p itself as all three neighbours with V lam = 0 and
// V mu w = 0, so they add exactly zero and the accumulation needs no
// per-lane branch.  CR: compact (32-B) records.
template <int L, int KU, bool CR>
__device__ __forceinline__ void tet_terms(const DevTopo &T, const float4 *X, float4 own, int p,
                                          size_t e0, int D, int lane, const StepConsts &K, Acc &a)
{
    for (int base = lane; base < D; base += L * KU) {
        int4 pa[KU];
        float4 pw[KU];
        float pb[KU];
#pragma unroll
        for (int j = 0; j < KU; ++j) {
            const int e = base + j * L;
            if (e < D) {
                pa[j] = T.pa[e0 + e];
                pw[j] = T.pw[e0 + e];
                pb[j] = CR ? 0.f : T.pb[e0 + e];
            } else {
                pa[j] = make_int4(p, p, p, 0);
                pw[j] = make_float4(0.f, 0.f, 0.f, 0.f);
                pb[j] = 0.f;
            }
        }
        // a slot that is padding in every lane of the wave is skipped (the
        // branch is uniform); a real record never names its own vertex
        bool live[KU];
#pragma unroll
        for (int j = 0; j < KU; ++j) live[j] = __builtin_amdgcn_ballot_w64(pa[j].x != p) != 0;
        float4 qa[KU], qb[KU], qc[KU];
#pragma unroll
        for (int j = 0; j < KU; ++j)
            if (live[j]) {
                qa[j] = ld_slot(X, pa[j].x);
                qb[j] = ld_slot(X, pa[j].y);
                qc[j] = ld_slot(X, pa[j].z);
            }
#pragma unroll
        for (int j = 0; j < KU; ++j)
            if (live[j]) {
                const float sigma = CR ? pw[j].w : pb[j];
                const float hmu = CR ? -(pw[j].x + pw[j].y + pw[j].z) : pw[j].w;
                pair_accumulate(__int_as_float(pa[j].w), pw[j], sigma, hmu, own, qa[j], qb[j], qc[j], K, a);
            }
    }
}

// Linear spring E = k/2 (l - L)^2: dE/dx_i = k (l - L) u,
// d2E/dx_i2 = k u u^T + c (I - u u^T) with the transverse stiffness
// c = k (1 - L/l), unprojected (Sec. 3.2) unless the clamp is requested: the
// block's eigenvalues are k along u and c twice across it, so c -> max(c, 0)
// is its PSD projection and leaves the axial k unchanged.
__device__ __forceinline__ void spring_contrib(float3 xi, float3 xj, float L, float k, int psd, Acc &a)
{
    const float3 d = xi - xj;
    const float l2 = dot3(d, d);
    const float inv_l = __builtin_amdgcn_rsqf(l2);   // v_rsq_f32, 1 ulp
    const float l = l2 * inv_l;
    const float3 u = d * inv_l;
    const float g = k * (l - L);
    a.fx -= g * u.x; a.fy -= g * u.y; a.fz -= g * u.z;
    float ci = k * (1.0f - L * inv_l);
    if (psd && ci < 0.f) ci = 0.f;           // transverse stiffness clamped (option)
    const float cu = k - ci;                 // k L / l unclamped, k clamped
    a.hxx += ci + cu * u.x * u.x;
    a.hxy += cu * u.x * u.y;
    a.hxz += cu * u.x * u.z;
    a.hyy += ci + cu * u.y * u.y;
    a.hyz += cu * u.y * u.z;
    a.hzz += ci + cu * u.z * u.z;
}

// Spring terms of one vertex from its D consecutive padded entries at E: each
// lane loads up to 4 entries together, then all their neighbour positions
// before any of the arithmetic (a gather inside each entry's branch would wait
// for the previous entry's terms).
template <int L>
__device__ __forceinline__ void spring_terms(const float4 *X, float3 xi, const int2 *E, int D,
                                             int lane, const StepConsts &K, Acc &a)
{
    constexpr int SU = 4;
    for (int base = lane; base < D; base += L * SU) {
        int2 se[SU];
#pragma unroll
        for (int j = 0; j < SU; ++j) {
            const int e = base + j * L;
            se[j] = (e < D) ? E[e] : make_int2(-1, 0);
        }
        float3 xj[SU];
#pragma unroll
        for (int j = 0; j < SU; ++j)
            if (se[j].x >= 0) xj[j] = xyz(ld_slot(X, se[j].x));
#pragma unroll
        for (int j = 0; j < SU; ++j)
            if (se[j].x >= 0) spring_contrib(xi, xj[j], __int_as_float(se[j].y), K.spring_k, K.spring_psd, a);
    }
}

template <int L>
__device__ __forceinline__ void acc_reduce(Acc &a)
{
    a.fx = group_sum<L>(a.fx); a.fy = group_sum<L>(a.fy); a.fz = group_sum<L>(a.fz);
    a.hxx = group_sum<L>(a.hxx); a.hxy = group_sum<L>(a.hxy); a.hxz = group_sum<L>(a.hxz);
    a.hyy = group_sum<L>(a.hyy); a.hyz = group_sum<L>(a.hyz); a.hzz = group_sum<L>(a.hzz);
    // The sums are consumed only by the group's active vertices; without this
    // use here the compiler moves the last add of each sum below that branch,
    // apart from its cross-lane move, which then cannot fold into a DPP add.
    asm volatile("" ::"v"(a.fx), "v"(a.fy), "v"(a.fz), "v"(a.hxx), "v"(a.hxy), "v"(a.hxz),
                 "v"(a.hyy), "v"(a.hyz), "v"(a.hzz));
}

// Analytic 3x3 solve with the determinant skip of Sec. 3.2:
// skip iff |det H| <= eps_rel * ||H||_F^3.  Returns false when skipped.
__device__ __forceinline__ bool solve_sym3(const Acc &a, float eps_rel, float3 &dx)
{
    const float A00 = a.hyy * a.hzz - a.hyz * a.hyz;
    const float A01 = a.hxz * a.hyz - a.hxy * a.hzz;
    const float A02 = a.hxy * a.hyz - a.hxz * a.hyy;
    const float A11 = a.hxx * a.hzz - a.hxz * a.hxz;
    const float A12 = a.hxy * a.hxz - a.hxx * a.hyz;
    const float A22 = a.hxx * a.hyy - a.hxy * a.hxy;
    const float det = a.hxx * A00 + a.hxy * A01 + a.hxz * A02;
    const float fro = sqrtf(a.hxx * a.hxx + a.hyy * a.hyy + a.hzz * a.hzz +
                            2.f * (a.hxy * a.hxy + a.hxz * a.hxz + a.hyz * a.hyz));
    if (!(fabsf(det) > eps_rel * fro * fro * fro)) return false;
    const float inv = __builtin_amdgcn_rcpf(det);   // v_rcp_f32, 1 ulp
    dx.x = (A00 * a.fx + A01 * a.fy + A02 * a.fz) * inv;
    dx.y = (A01 * a.fx + A11 * a.fy + A12 * a.fz) * inv;
    dx.z = (A02 * a.fx + A12 * a.fy + A22 * a.fz) * inv;
    return true;
}

// Inertia (Eq. VBDForce/VBDHessian), Rayleigh damping on the summed element
// Hessian (Eq. VBDForceWithDamping/VBDHessianWithDamping), penalty contact
// against analytic obstacles with a fixed normal (Eq. collisionEnergy) and
// IPC-style friction with the approximate Hessian (Eq. IPC_friction).
__device__ __forceinline__ bool vertex_terms(const DevTopo &T, const StepConsts &K, int p,
                                             float3 xi, float4 yv, Acc &a)
{
    const float w = yv.w;   // m / h^2
    bool contact = false;
    float3 xt = make_float3(0.f, 0.f, 0.f);
    const bool need_xt = (K.kd_over_h != 0.f) || (K.fric_mu > 0.f);
    if (need_xt) xt = xyz(T.xt[p]);
    if (K.kd_over_h != 0.f) {
        const float3 d = xi - xt;
        const float c = K.kd_over_h;
        a.fx -= c * (a.hxx * d.x + a.hxy * d.y + a.hxz * d.z);
        a.fy -= c * (a.hxy * d.x + a.hyy * d.y + a.hyz * d.z);
        a.fz -= c * (a.hxz * d.x + a.hyz * d.y + a.hzz * d.z);
        a.hxx *= 1.f + c; a.hxy *= 1.f + c; a.hxz *= 1.f + c;
        a.hyy *= 1.f + c; a.hyz *= 1.f + c; a.hzz *= 1.f + c;
    }
    a.fx -= w * (xi.x - yv.x);
    a.fy -= w * (xi.y - yv.y);
    a.fz -= w * (xi.z - yv.z);
    a.hxx += w; a.hyy += w; a.hzz += w;
    const int nobs = K.n_spheres + K.n_planes;
    for (int o = 0; o < nobs; ++o) {
        float3 n;
        float pen;
        if (o < K.n_spheres) {
            const float4 s = K.spheres[o];
            const float3 r = xi - make_float3(s.x, s.y, s.z);
            const float r2 = dot3(r, r);
            const float inv = __builtin_amdgcn_rsqf(r2);   // v_rsq_f32, 1 ulp
            const float dist = r2 * inv;
            n = r * inv;
            pen = s.w + K.delta - dist;
        } else {
            const float4 pl = K.planes[o - K.n_spheres];
            n = make_float3(pl.x, pl.y, pl.z);
            pen = K.delta - (dot3(n, xi) - pl.w);
        }
        if (!(pen > 0.f)) continue;
        contact = true;
        const float kp = K.kc * pen;
        a.fx += kp * n.x; a.fy += kp * n.y; a.fz += kp * n.z;
        a.hxx += K.kc * n.x * n.x; a.hxy += K.kc * n.x * n.y; a.hxz += K.kc * n.x * n.z;
        a.hyy += K.kc * n.y * n.y; a.hyz += K.kc * n.y * n.z; a.hzz += K.kc * n.z * n.z;
        if (K.fric_mu > 0.f) {
            const float3 dx = xi - xt;
            const float dn = dot3(dx, n);
            const float3 u = dx - n * dn;
            const float un = sqrtf(dot3(u, u));
            const float hev = K.fric_hev;
            const float f1u = (un < hev) ? (2.0f / hev - un / (hev * hev)) : (1.0f / un);
            const float s = K.fric_mu * kp * f1u;
            a.fx -= s * u.x; a.fy -= s * u.y; a.fz -= s * u.z;
            a.hxx += s * (1.f - n.x * n.x); a.hxy -= s * n.x * n.y; a.hxz -= s * n.x * n.z;
            a.hyy += s * (1.f - n.y * n.y); a.hyz -= s * n.y * n.z; a.hzz += s * (1.f - n.z * n.z);
        }
    }
    return contact;
}

// Mesh-mesh vertex-triangle contact element (Sec. 3.5) seen from one of its
// vertices: role -1 = the colliding vertex xa, 0..2 = that triangle corner.
// E = k_c/2 d^2, d = delta - (xa - q).n, q the closest point on the triangle
// (recomputed here), n its unit normal; n and q's barycentric weights are held
// fixed in the derivatives: dd/dxa = -n, dd/dc_k = w_k n.  Friction (Sec. 3.6)
// on the relative displacement (xa - xa^t) - sum_k w_k (c_k - c_k^t) with
// lambda = k_c d.  Adds to a and returns true when the element is active.
__device__ __forceinline__ bool vt_term(const StepConsts &K, const float4 *Xt, float3 xa, int ia,
                                        float3 c0, float3 c1, float3 c2, int4 tri, int role,
                                        Acc &a)
{
    const ClosestPt cp = closest_on_triangle(xa, c0, c1, c2);
    const float3 n = normalize3(cross3(c1 - c0, c2 - c0));
    const float d = K.delta - dot3(xa - cp.q, n);
    if (!(d > 0.f)) return false;
    const float g = role < 0 ? -1.f : (role == 0 ? cp.w0 : (role == 1 ? cp.w1 : cp.w2));
    const float kd = K.kc * d * g, kh = K.kc * g * g;
    a.fx -= kd * n.x; a.fy -= kd * n.y; a.fz -= kd * n.z;
    a.hxx += kh * n.x * n.x; a.hxy += kh * n.x * n.y; a.hxz += kh * n.x * n.z;
    a.hyy += kh * n.y * n.y; a.hyz += kh * n.y * n.z; a.hzz += kh * n.z * n.z;
    if (K.fric_mu > 0.f) {
        const float3 dxa = xa - xyz(Xt[ia]);
        const float3 d0 = c0 - xyz(Xt[tri.x]), d1 = c1 - xyz(Xt[tri.y]), d2 = c2 - xyz(Xt[tri.z]);
        const float3 dx = dxa - (d0 * cp.w0 + d1 * cp.w1 + d2 * cp.w2);
        const float3 u = dx - n * dot3(dx, n);
        const float un = sqrtf(dot3(u, u));
        const float hev = K.fric_hev;
        const float f1u = (un < hev) ? (2.0f / hev - un / (hev * hev)) : (1.0f / un);
        const float sf = K.fric_mu * K.kc * d * f1u;
        const float sg = sf * g, sg2 = sf * g * g;
        a.fx += sg * u.x; a.fy += sg * u.y; a.fz += sg * u.z;
        a.hxx += sg2 * (1.f - n.x * n.x); a.hxy -= sg2 * n.x * n.y; a.hxz -= sg2 * n.x * n.z;
        a.hyy += sg2 * (1.f - n.y * n.y); a.hyz -= sg2 * n.y * n.z; a.hzz += sg2 * (1.f - n.z * n.z);
    }
    return true;
}

// Position of a contact partner q during the phase over slots [vb, ve).
// Edge-edge contact element (Sec. 3.5) seen from one of its four vertices:
// role 0, 1 the first edge's ends (x0, x1), 2, 3 the second's (x2, x3).
// E = k_c/2 d^2, d = delta - (x_a - x_b).n with x_a, x_b the closest points
// (recomputed here) and n fixed; with s, u and n held fixed,
// dd/dx0 = -(1 - s) n, dd/dx1 = -s n, dd/dx2 = (1 - u) n, dd/dx3 = u n.
// Friction (Sec. 3.6) on (x_a - x_a^t) - (x_b - x_b^t) with the same weights.
__device__ __forceinline__ bool ee_term(const StepConsts &K, const float4 *Xt, float3 x0, float3 x1,
                                        float3 x2, float3 x3, int4 A, int4 B, float3 n, int role,
                                        Acc &a)
{
    const SegPt sp = seg_closest(x0, x1, x2, x3);
    const float3 xa = x0 + (x1 - x0) * sp.s, xb = x2 + (x3 - x2) * sp.u;
    const float d = K.delta - dot3(xa - xb, n);
    if (!(d > 0.f)) return false;
    const float g = role == 0 ? -(1.f - sp.s) : (role == 1 ? -sp.s : (role == 2 ? 1.f - sp.u : sp.u));
    const float kd = K.kc * d * g, kh = K.kc * g * g;
    a.fx -= kd * n.x; a.fy -= kd * n.y; a.fz -= kd * n.z;
    a.hxx += kh * n.x * n.x; a.hxy += kh * n.x * n.y; a.hxz += kh * n.x * n.z;
    a.hyy += kh * n.y * n.y; a.hyz += kh * n.y * n.z; a.hzz += kh * n.z * n.z;
    if (K.fric_mu > 0.f) {
        const float3 ta0 = xyz(Xt[A.x]), ta1 = xyz(Xt[A.y]), tb0 = xyz(Xt[B.x]), tb1 = xyz(Xt[B.y]);
        const float3 dx = (xa - (ta0 + (ta1 - ta0) * sp.s)) - (xb - (tb0 + (tb1 - tb0) * sp.u));
        const float3 u = dx - n * dot3(dx, n);
        const float un = sqrtf(dot3(u, u));
        const float hev = K.fric_hev;
        const float f1u = (un < hev) ? (2.0f / hev - un / (hev * hev)) : (1.0f / un);
        const float sf = K.fric_mu * K.kc * d * f1u;
        const float sg = sf * g, sg2 = sf * g * g;
        a.fx += sg * u.x; a.fy += sg * u.y; a.fz += sg * u.z;
        a.hxx += sg2 * (1.f - n.x * n.x); a.hxy -= sg2 * n.x * n.y; a.hxz -= sg2 * n.x * n.z;
        a.hyy += sg2 * (1.f - n.y * n.y); a.hyz -= sg2 * n.y * n.z; a.hzz += sg2 * (1.f - n.z * n.z);
    }
    return true;
}

__device__ __forceinline__ float3 phase_pos(const float4 *X, const float4 *Xs, int q, int vb, int ve)
{
    return xyz((q >= vb && q < ve) ? Xs[q] : X[q]);
}

// Contact elements of vertex p: lane 0 takes p's own contact (p is the
// colliding vertex), the lanes stride over the corner entries (p is a corner
// of another vertex's contact triangle).  Partners of p's color (slots in
// [vb, ve)) are read at their positions from before the phase, the others
// at their latest.  Returns the number of active elements this lane added.
// own = S.ctri[p], [e0, e1) = p's corner entries (loaded by the caller with
// the vertex's own state).
template <int L>
__device__ __forceinline__ float contact_terms(const DevTopo &T, const DevSurf &S,
                                               const StepConsts &K, int p, float3 xi, int lane,
                                               int vb, int ve, int own, int e0, int e1, Acc &a)
{
    float nc = 0.f;
    const float4 *X = T.x, *Xs = S.xsnap;
    if (lane == 0) {
        if (own >= 0) {
            const int4 tr = S.tri[own];
            if (vt_term(K, T.xt, xi, p, phase_pos(X, Xs, tr.x, vb, ve), phase_pos(X, Xs, tr.y, vb, ve),
                        phase_pos(X, Xs, tr.z, vb, ve), tr, -1, a))
                nc += 1.f;
        }
    }
    for (int e = e0 + lane; e < e1; e += L) {
        const int va = S.cent[e];
        const int4 tr = S.tri[S.ctri[va]];
        const int role = (tr.x == p) ? 0 : ((tr.y == p) ? 1 : 2);
        const float3 c0 = role == 0 ? xi : phase_pos(X, Xs, tr.x, vb, ve);
        const float3 c1 = role == 1 ? xi : phase_pos(X, Xs, tr.y, vb, ve);
        const float3 c2 = role == 2 ? xi : phase_pos(X, Xs, tr.z, vb, ve);
        if (vt_term(K, T.xt, phase_pos(X, Xs, va, vb, ve), va, c0, c1, c2, tr, role, a)) nc += 1.f;
    }
    if (K.edge_contacts) {
        const int r1 = (int)S.erow[p + 1];
        for (int e = (int)S.erow[p] + lane; e < r1; e += L) {
            const int el = S.eent[e];
            const int4 A = S.edge[el], B = S.edge[S.eb[el]];
            const int role = A.x == p ? 0 : (A.y == p ? 1 : (B.x == p ? 2 : 3));
            const float3 x0 = role == 0 ? xi : phase_pos(X, Xs, A.x, vb, ve);
            const float3 x1 = role == 1 ? xi : phase_pos(X, Xs, A.y, vb, ve);
            const float3 x2 = role == 2 ? xi : phase_pos(X, Xs, B.x, vb, ve);
            const float3 x3 = role == 3 ? xi : phase_pos(X, Xs, B.y, vb, ve);
            if (ee_term(K, T.xt, x0, x1, x2, x3, A, B, xyz(S.en[el]), role, a)) nc += 1.f;
        }
    }
    return nc;
}

// One vertex update by a group of L lanes.  All lanes of the wave must call
// this (inactive groups pass active = false) because of the DPP reduction.
// The phase covers slots [vb, ve) of one color with incidence layout inc.
// MC: mesh-mesh contacts; CR: compact pair records.
template <int L, int KU, bool TETS, bool SPRINGS, bool MC, bool CR>
__device__ __forceinline__ void solve_vertex(const DevTopo &T, const StepConsts &K, int p,
                                             int lane, bool active, int vb, int ve, int4 inc,
                                             const DevSurf *S = nullptr)
{
    Acc a;
    acc_zero(a);
    float4 xi4 = make_float4(0.f, 0.f, 0.f, 0.f), yv = xi4;
    float nc = 0.f;
    int c_own = -1, c_e0 = 0, c_e1 = 0;   // contact lookups, issued with the own state
    if (active) {
        xi4 = T.x[p];
        yv = T.y[p];
        if (MC) {
            c_own = S->ctri[p];
            c_e0 = (int)S->crow[p];
            c_e1 = (int)S->crow[p + 1];
        }
        if (TETS)
            tet_terms<L, KU, CR>(T, T.x, xi4, p, (size_t)inc.x + (size_t)(p - vb) * inc.y, inc.y, lane, K,
                                 a);
        if (SPRINGS)
            spring_terms<L>(T.x, xyz(xi4), T.spr_ell + (size_t)inc.z + (size_t)(p - vb) * inc.w, inc.w,
                            lane, K, a);
    }
    if (MC) {
        // Rayleigh damping applies to the material Hessian only: contact
        // terms are added after it (see below) when damping is on
        if (active && K.kd_over_h == 0.f)
            nc = contact_terms<L>(T, *S, K, p, xyz(xi4), lane, vb, ve, c_own, c_e0, c_e1, a);
    }
    acc_reduce<L>(a);
    if (MC) nc = group_sum<L>(nc);
    if (!active) return;
    const float3 xi = xyz(xi4);
    bool contact = vertex_terms(T, K, p, xi, yv, a);
    if (MC && K.kd_over_h != 0.f) {
        // damping on: the group's lanes are past the reduction, so lane 0
        // alone adds the contact elements to the reduced system
        Acc c;
        acc_zero(c);
        float ncl = 0.f;
        if (lane == 0) {
            ncl = contact_terms<1>(T, *S, K, p, xi, 0, vb, ve, c_own, c_e0, c_e1, c);
            a.fx += c.fx; a.fy += c.fy; a.fz += c.fz;
            a.hxx += c.hxx; a.hxy += c.hxy; a.hxz += c.hxz;
            a.hyy += c.hyy; a.hyz += c.hyz; a.hzz += c.hzz;
        }
        nc += ncl;
    }
    if (MC && nc > 0.f) contact = true;
    float3 dx;
    const bool ok = solve_sym3(a, K.det_eps_rel, dx);
    if (lane == 0) {
        const float4 xo = ok ? make_float4(xi.x + dx.x, xi.y + dx.y, xi.z + dx.z, xi4.w) : xi4;
        if (ok) T.x[p] = xo;
        else atomicAdd(reinterpret_cast<unsigned long long *>(T.flags + kFlagSkips), 1ull);
        if (T.xnext) T.xnext[p] = xo;
        if (contact) T.collided[p] = 1;
    }
}

// ----------------------------------------------------------------- kernels --
// The E-dependent parts of every pair record: V lam into pa.w and V mu w into
// pw, whose last entry is sigma (compact) or V mu |m|^2 = -V mu (w0 + w1 + w2)
// (padding entries have pair_tet = -1).
__global__ void k_material_pairs(int4 *pa, float4 *pw, const float4 *pws, const int *pair_tet,
                                 const float *vol, const int *tet_perm, const float *E, long long n,
                                 float k_mu, float k_lam, int compact)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = pair_tet[i];
    if (t < 0) {
        pw[i] = make_float4(0.f, 0.f, 0.f, 0.f);   // padding: adds zero in the solve
        return;
    }
    const float VE = vol[t] * E[tet_perm[t]];
    const float Vmu = VE * k_mu;
    reinterpret_cast<int *>(pa + i)[3] = __float_as_int(VE * k_lam);
    const float4 w = pws[i];
    pw[i] = make_float4(w.x * Vmu, w.y * Vmu, w.z * Vmu, compact ? w.w : -(w.x + w.y + w.z) * Vmu);
}

// y = x^t + h v^t + h^2 a_ext (Eq. inertia) and the initial guess (Sec. 3.7).
__global__ void k_predict(DevTopo T, const float *x, const float *v, const float *vp,
                          StepConsts K, int reset_flags, int cheb)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (reset_flags) {
        if (p <= kBarGroups) T.flags[kFlagBar + p * kBarStride] = 0u;
        if (p < kBarGroups) T.flags[kFlagCensus + p] = 0u;
        if (p == 0) T.flags[kFlagCensusTotal] = 0u;
    }
    if (p >= T.n_verts) return;
    const int o = T.perm[p];
    const float3 xt = ld3(x, o), vt = ld3(v, o);
    const float h = K.h;
    const float3 g = make_float3(K.gx, K.gy, K.gz);
    const float w = T.mass[p] * K.inv_h * K.inv_h;
    const float3 y = xt + vt * h + g * (h * h);
    T.xt[p] = make_float4(xt.x, xt.y, xt.z, 0.f);
    T.y[p] = make_float4(y.x, y.y, y.z, w);
    float3 x0 = xt;
    if (p < T.n_free) {
        switch (K.init_mode) {
        case 0: break;
        case 1: x0 = xt + vt * h; break;
        case 2: x0 = y; break;
        default: {
            float at = 0.f;
            if (K.gnorm > 0.f) {
                const float3 vpt = ld3(vp, o);
                at = dot3((vt - vpt) * K.inv_h, g) / K.gnorm;
            }
            float atil;
            if (K.gnorm == 0.f) atil = 0.f;
            else if (at > K.gnorm) atil = 1.f;
            else if (at < 0.f) atil = 0.f;
            else atil = at / K.gnorm;
            x0 = xt + vt * h + g * (h * h * atil);
        }
        }
    }
    const float4 x04 = make_float4(x0.x, x0.y, x0.z, 0.f);
    T.x[p] = x04;
    T.collided[p] = 0;
    if (cheb) { T.prev1[p] = x04; T.prev2[p] = x04; }
}

constexpr int kMaxBlock = 512;

// The vertex slot of this thread's group and whether it is in range: with a
// mesh-aligned split (xs, launch mapping 3) block b runs part b mod 8 of the
// color (XCD b mod 8 under round-robin dispatch), else xcd_block's mapping.
template <int L>
__device__ __forceinline__ int phase_slot(int v_begin, int v_end, int remap, const int *xs, bool &act)
{
    if (xs) {
        const int x = blockIdx.x & 7;
        const int lo = xs[x], hi = xs[x + 1];
        const int p = lo + (int)(((blockIdx.x >> 3) * blockDim.x + threadIdx.x) / L);
        act = p < hi;
        return p;
    }
    const int b = xcd_block(blockIdx.x, gridDim.x, remap);
    const int p = v_begin + (int)((b * blockDim.x + threadIdx.x) / L);
    act = p < v_end;
    return p;
}

template <int L, int KU, bool TETS, bool SPRINGS, bool CR>
__global__ __launch_bounds__(kMaxBlock) void k_solve(
    DevTopo T, StepConsts K, int v_begin, int v_end, int4 inc, int remap, const int *xs)
{
    bool act;
    const int p = phase_slot<L>(v_begin, v_end, remap, xs, act);
    solve_vertex<L, KU, TETS, SPRINGS, false, CR>(T, K, p, threadIdx.x & (L - 1), act, v_begin, v_end,
                                                  inc);
}

// Color phase with mesh contacts.  The previously solved color's snapshot is
// refreshed here: during this phase neither its positions change nor its
// snapshot is read.
template <int L, int KU, bool TETS, bool SPRINGS, bool CR>
__global__ __launch_bounds__(kMaxBlock) void k_solve_mc(DevTopo T, DevSurf S, StepConsts K,
                                                        int v_begin, int v_end, int4 inc,
                                                        int prev_begin, int prev_end, int remap,
                                                        const int *xs)
{
    for (int q = prev_begin + blockIdx.x * blockDim.x + threadIdx.x; q < prev_end;
         q += gridDim.x * blockDim.x)
        S.xsnap[q] = T.x[q];
    bool act;
    const int p = phase_slot<L>(v_begin, v_end, remap, xs, act);
    solve_vertex<L, KU, TETS, SPRINGS, true, CR>(T, K, p, threadIdx.x & (L - 1), act, v_begin, v_end,
                                                 inc, &S);
}

__device__ __forceinline__ float cheb_omega(int it, float rho)
{
    // Eq. accelerator: omega_1 = 1, omega_2 = 2/(2 - rho^2),
    // omega_n = 4/(4 - rho^2 omega_{n-1})
    float om = 1.f;
    for (int n = 2; n <= it; ++n) om = (n == 2) ? 2.f / (2.f - rho * rho) : 4.f / (4.f - rho * rho * om);
    return om;
}

__device__ __forceinline__ void cheb_vertex(const DevTopo &T, int p, float om)
{
    const float4 xb = T.x[p], p2 = T.prev2[p];
    float4 xn = xb;
    if (!T.collided[p]) {
        xn.x = om * (xb.x - p2.x) + p2.x;
        xn.y = om * (xb.y - p2.y) + p2.y;
        xn.z = om * (xb.z - p2.z) + p2.z;
    }
    T.prev2[p] = T.prev1[p];
    T.prev1[p] = xn;
    T.x[p] = xn;
}

__global__ void k_cheb(DevTopo T, float rho, int it, float4 *snap)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= T.n_free) return;
    cheb_vertex(T, p, cheb_omega(it, rho));
    if (snap) snap[p] = T.x[p];
}

// v^{t+1} = (x^{t+1} - x^t)/h (Eq. velocity_update); the state's previous
// velocity becomes v^t; results go back in the original vertex order.
__global__ void k_finalize(DevTopo T, float *x, float *v, float *vp, float h)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= T.n_verts) return;
    const int o = T.perm[p];
    const float3 xn = xyz(T.x[p]), xt = xyz(T.xt[p]);
    const float3 vold = ld3(v, o);
    st3(vp, o, vold);
    st3(v, o, (xn - xt) * (1.0f / h));
    st3(x, o, xn);
}

// Device-wide barrier for the persistent kernel.  The XCDs' L2 caches are not
// coherent with each other: a block's writes reach other XCDs only after an
// agent-scope release writes its L2 back, and its reads see other XCDs' writes
// only after an agent-scope acquire.  A write-back covers the whole L2 of the
// XCD, so one per XCD suffices: every block waits until its own stores have
// reached its L2 and arrives at its XCD's counter; the XCD's last arrival
// writes that L2 back once and arrives at the global counter; every block
// waits for the global count and then acquires.  Blocks are grouped by the XCD
// they run on (the hardware XCC_ID register), counted once per launch by
// barrier_census.  Counters only grow (reset to 0 by k_predict before the
// launch): barrier k completes when an XCD's counter reaches k * (its blocks)
// and the global one k * (XCDs in use).  Every wait is bounded: after
// kSpinLimit polls the block raises flags[1] and every block leaves at its next
// barrier, so the kernel always terminates.
constexpr long kSpinLimit = 1L << 20;

struct BarGroup {
    unsigned xcd;        // XCD this block runs on
    unsigned in_grp;     // blocks of the grid on that XCD
    unsigned n_groups;   // XCDs with at least one block
};

// Bounded wait for *ctr >= target; on timeout records what was seen and raises
// the abort flag.  Returns true when the kernel must stop.
__device__ __forceinline__ bool bar_wait(unsigned *flags, unsigned *ctr, unsigned target)
{
    long spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return true;
        if (++spins > kSpinLimit) {
            // record what the waiting block saw, for vbd_check's message
            const unsigned seen = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(&flags[3], seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(&flags[4], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&flags[5], gridDim.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&flags[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return true;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}

// Start of a persistent launch: every block counts itself on its XCD, then
// waits until all blocks are counted.  Returns true when the kernel must stop.
__device__ __forceinline__ bool barrier_census(unsigned *flags, BarGroup &bg)
{
    __shared__ int s_abort;
    __shared__ unsigned s_grp[3];
    if (threadIdx.x == 0) {
        // HW_REG_XCC_ID (register 20), bits 3:0
        const unsigned xcd = __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & (kBarGroups - 1);
        __hip_atomic_fetch_add(&flags[kFlagCensus + xcd], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the XCD count lands before the total that announces it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&flags[kFlagCensusTotal], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int abort = bar_wait(flags, &flags[kFlagCensusTotal], gridDim.x) ? 1 : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        unsigned ng = 0;
        for (int g = 0; g < kBarGroups; ++g)
            ng += __hip_atomic_load(&flags[kFlagCensus + g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        s_grp[0] = xcd;
        s_grp[1] = __hip_atomic_load(&flags[kFlagCensus + xcd], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_grp[2] = ng;
        s_abort = abort;
    }
    __syncthreads();
    bg.xcd = s_grp[0];
    bg.in_grp = s_grp[1];
    bg.n_groups = s_grp[2];
    return s_abort != 0;
}

__device__ __forceinline__ bool grid_barrier(unsigned *flags, unsigned k, const BarGroup &bg)
{
    __shared__ int s_abort;
    // every wave's stores have reached its XCD's L2 (stores count in vmcnt)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned *gc = flags + kFlagBar + bg.xcd * kBarStride;
        unsigned *all = flags + kFlagBar + kBarGroups * kBarStride;
        const unsigned old = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == k * bg.in_grp) {
            // the XCD's last arrival: one write-back of this L2 for all its blocks
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(all, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const int abort = bar_wait(flags, all, k * bg.n_groups) ? 1 : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_abort = abort;
    }
    __syncthreads();
    return s_abort != 0;
}

template <int L, int KU, bool TETS, bool SPRINGS, bool CR>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(kPersistentWavesPerSimd)))
void k_persistent(DevTopo T, StepConsts K, int n_iters, int remap)
{
    const int nb = gridDim.x;
    const int b = xcd_block(blockIdx.x, nb, remap);
    const int G = blockDim.x / L;   // vertex groups per block
    const int g = threadIdx.x / L, lane = threadIdx.x & (L - 1);
    BarGroup bg;
    if (barrier_census(T.flags, bg)) return;
    unsigned nbar = 0;
    for (int it = 1; it <= n_iters; ++it) {
        for (int c = 0; c < T.n_colors; ++c) {
            const int vb = T.color_off[c], ve = T.color_off[c + 1];
            const int2 te = T.ell_info[c], se = T.spr_info[c];
            const int4 inc = make_int4(te.x, te.y, se.x, se.y);
            // contiguous chunk of the color per logical block
            const int n = ve - vb;
            const int chunk = (n + nb - 1) / nb;
            const int cb = vb + b * chunk;
            const int cend = min(cb + chunk, ve);
            for (int base = cb; base < cb + chunk; base += G) {
                const int p = base + g;
                solve_vertex<L, KU, TETS, SPRINGS, false, CR>(T, K, p, lane, p < cend, vb, ve, inc);
            }
            ++nbar;
            if (grid_barrier(T.flags, nbar, bg)) return;
        }
        if (K.cheb_rho > 0.f) {
            const float om = cheb_omega(it, K.cheb_rho);
            for (int p = b * blockDim.x + threadIdx.x; p < T.n_free; p += nb * blockDim.x)
                cheb_vertex(T, p, om);
            ++nbar;
            if (grid_barrier(T.flags, nbar, bg)) return;
        }
    }
}

// Streaming copy: each thread keeps four independent 16-B loads in flight.
// Read-only streaming probe: every thread keeps 8 loads of 16 B in flight
// (grid-stride), sums them, and its block writes one partial sum.
__global__ __launch_bounds__(256) void k_read4(const float4 *src, long long n, float *out)
{
    __shared__ float part[256 / 64];
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.f;
    for (; i + 7 * stride < n; i += 8 * stride) {
        float4 r[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) r[j] = src[i + j * stride];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += (r[j].x + r[j].y) + (r[j].z + r[j].w);
    }
    for (; i < n; i += stride) {
        const float4 r = src[i];
        acc += (r.x + r.y) + (r.z + r.w);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[w];
        out[blockIdx.x] = s;
    }
}

__global__ void k_copy4(float4 *dst, const float4 *src, int n)
{
    const int stride = gridDim.x * blockDim.x;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_zero_u32(unsigned *p, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// Counts the non-finite values among the n floats of a and of b (the step's
// output positions and velocities) into flags[kFlagNonfinite] (cleared by
// vbd_check) and flags[kFlagNonfiniteTotal] (cleared by a counter reset):
// one atomic per wave that found any.
__global__ void k_check_finite(const float *a, const float *b, long long n, unsigned *flags)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    unsigned bad = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        bad += (isfinite(a[i]) ? 0u : 1u) + (isfinite(b[i]) ? 0u : 1u);
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
    if ((threadIdx.x & 63) == 0 && bad != 0) {
        atomicAdd(&flags[kFlagNonfinite], bad);
        atomicAdd(&flags[kFlagNonfiniteTotal], bad);
    }
}

// ---------------------------------------------------------------- adjoint --
__global__ void k_bwd_init(DevTopo T, const float *gx, const float *gv, const float *gvp, float h)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= T.n_verts) return;
    const int o = T.perm[p];
    const float3 a = ld3(gx, o), b = ld3(gv, o), c = ld3(gvp, o);
    const float ih = 1.0f / h;
    T.xbar[p] = make_float4(a.x + b.x * ih, a.y + b.y * ih, a.z + b.z * ih, 0.f);
    T.xtbar[p] = make_float4(-b.x * ih, -b.y * ih, -b.z * ih, 0.f);
    T.vbar[p] = make_float4(c.x, c.y, c.z, 0.f);
    T.ybar[p] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Reverse of one color phase.  The update x_i' = argmin G_i (exact for
// these tets, G_i quadratic in x_i) satisfies grad_i G_i(x_i'; x_nbr, y_i, E)
// = 0, so with w = H_i^{-1} xbar_i:
//   xbar_i <- 0,  ybar_i += (m/h^2) w,  xbar_q -= d(w . grad_i Psi)/dx_q,
//   Ebar_t -= (w . grad_i Psi_t) / E_t,
// all at the state right after the update: vertices of colors <= c from
// iteration n (Sn), the others from iteration n-1 (Sp).  In a tet's pair frame
// (the forward's records: e_k = x_k - x_i for the other vertices a, b, c,
// w_k = (S m)_k, sigma = det S, n = sigma (x_b - x_a) x (x_c - x_a), J = e1 . n):
//   w . grad_i Psi = V mu sum_k w_k (w . e_k) - V lam (J - alpha) (n . w),
// and for the neighbour q (index k of a, b, c)
//   d/dx_q = V mu w_k w - V lam (n . w) c_q - V lam (J - alpha) g_q,
//   c_q = dJ/dx_q = sigma {e2 x e3, e3 x e1, e1 x e2},
//   g_q = d(n . w)/dx_q = sigma {w x (x_c - x_b), (x_c - x_a) x w, w x (x_b - x_a)}.
// H_i = V mu |m|^2 I + V lam n n^T as in the forward solve (|m|^2 = -(w0 + w1 + w2)).
// Neighbour adjoints travel through cells addressed by the receiving
// vertex's pair entry (DevTopo::cin): in a color phase a tet has at most one
// vertex of that color, so each cell has one writer per phase, and between
// two phases of a vertex every other color runs exactly once, so each of its
// three incoming cells per tet holds the latest contribution of its writer
// (all cells start at zero, which covers the colors not yet run in the first
// reverse iteration).  Writes only, no read-modify-write, and the receiver
// reads its cells with its own entries.  Pinned vertices are never updated:
// their contributions accumulate per (tet, slot) in DevTopo::contrib.  At the
// end of the sweep k_bwd_fold adds the cells written after each vertex's
// last update.  Ebar accumulates per pair entry (DevTopo::ebar_pair).
// Position of a neighbour q in the state right after the update of the
// phase's vertex: colors <= c (slots < c_end) from iteration n, the others
// from iteration n - 1.
__device__ __forceinline__ float4 adj_pos(const float4 *Sn, const float4 *Sp, int q, int c_end)
{
    return (q < c_end ? Sn : Sp)[q];
}

// One tet's share of H_i: V mu |m|^2 I + V lam n n^T.
__device__ __forceinline__ void adj_hess(float4 qa, float4 qb, float4 qc, float hmu, float vlam,
                                         float sg, Acc &a)
{
    const float3 xa = xyz(qa);
    const float3 n = cross3(xyz(qb) - xa, xyz(qc) - xa) * sg;
    const float3 ln = n * vlam;
    a.hxx += hmu + ln.x * n.x; a.hxy += ln.x * n.y; a.hxz += ln.x * n.z;
    a.hyy += hmu + ln.y * n.y; a.hyz += ln.y * n.z; a.hzz += hmu + ln.z * n.z;
}

// One tet's reverse terms: -d(w . grad_i Psi)/dx_q added to the cells of the
// other three vertices (c0, c1, c2 in the pair record's order); returns (w . grad_i Psi)/(V E).
__device__ __forceinline__ float adj_pair(float3 xi, float4 qa, float4 qb, float4 qc, float4 ws,
                                          float Vlam, float sg, float3 w, float mu_lam,
                                          const StepConsts &K, float3 &c0, float3 &c1, float3 &c2)
{
    const float3 xa = xyz(qa), xb = xyz(qb), xc = xyz(qc);
    const float3 e1 = xa - xi, e2 = xb - xi, e3 = xc - xi;
    const float3 dab = xb - xa, dac = xc - xa;
    const float3 n = cross3(dab, dac) * sg;
    const float J = dot3(e1, n);
    const float nw = dot3(n, w);
    const float Vmu = Vlam * mu_lam;
    // coefficients of c_q / sigma and g_q / sigma
    const float kc = Vlam * nw * sg, kg = Vlam * (J - K.alpha) * sg;
    const float3 ca = cross3(e2, e3), cb = cross3(e3, e1), cc = cross3(e1, e2);
    const float3 ga = cross3(w, xc - xb), gb = cross3(dac, w), gc = cross3(w, dab);
    const float3 ma = w * (Vmu * ws.x), mb = w * (Vmu * ws.y), mc = w * (Vmu * ws.z);
    c0.x -= ma.x - kc * ca.x - kg * ga.x;
    c0.y -= ma.y - kc * ca.y - kg * ga.y;
    c0.z -= ma.z - kc * ca.z - kg * ga.z;
    c1.x -= mb.x - kc * cb.x - kg * gb.x;
    c1.y -= mb.y - kc * cb.y - kg * gb.y;
    c1.z -= mb.z - kc * cb.z - kg * gb.z;
    c2.x -= mc.x - kc * cc.x - kg * gc.x;
    c2.y -= mc.y - kc * cc.y - kg * gc.y;
    c2.z -= mc.z - kc * cc.z - kg * gc.z;
    // k_mu sum_k w_k (w . e_k) - k_lam (J - alpha) (n . w)
    const float wF = ws.x * dot3(w, e1) + ws.y * dot3(w, e2) + ws.z * dot3(w, e3);
    return K.k_mu * wF - K.k_lam * (J - K.alpha) * nw;
}

// Sends one outgoing contribution (see DevTopo::tgt): into the receiving
// entry's cell, or added to a pinned vertex's (tet, slot) cell.
__device__ __forceinline__ void adj_send(const DevTopo &T, int tg, float3 c)
{
    if (tg >= 0) {
        T.cin[(size_t)(tg & 3) * (size_t)T.n_pairs + (size_t)(tg >> 2)] = c;
    } else {
        float3 *cell = T.contrib + (size_t)(-1 - tg);
        const float3 o = *cell;
        *cell = make_float3(o.x + c.x, o.y + c.y, o.z + c.z);
    }
}

// One entry's loads: pair record (other vertices, V lam), the E-free record
// (w, sigma; sigma = 0 marks padding), targets, incoming cells, Ebar share.
struct AdjEnt {
    int4 pa;
    float4 ws;
    int3 tg;
    float3 g0, g1, g2;
    float eb;
};

__device__ __forceinline__ void adj_load(const DevTopo &T, size_t e, AdjEnt &r)
{
    const size_t np = (size_t)T.n_pairs;
    r.pa = T.pa[e];
    r.ws = T.pws[e];
    r.tg = T.tgt[e];
    r.g0 = T.cin[e];
    r.g1 = T.cin[np + e];
    r.g2 = T.cin[2 * np + e];
    r.eb = T.ebar_pair[e];
}

// The second pass on one entry: outgoing contributions and the Ebar share
// (V = 1 / (6 |sigma|): sigma = det S = 1 / det D_m' with D_m' = Q R, Q proper).
__device__ __forceinline__ void adj_emit(const DevTopo &T, const StepConsts &K, size_t e,
                                         const AdjEnt &r, float3 xi, float4 qa, float4 qb, float4 qc,
                                         float3 w, float mu_lam)
{
    float3 c0 = make_float3(0.f, 0.f, 0.f), c1 = c0, c2 = c0;
    const float vlam = __int_as_float(r.pa.w);
    const float sg = r.ws.w;
    const float rr = adj_pair(xi, qa, qb, qc, r.ws, vlam, sg, w, mu_lam, K, c0, c1, c2);
    adj_send(T, r.tg.x, c0);
    adj_send(T, r.tg.y, c1);
    adj_send(T, r.tg.z, c2);
    T.ebar_pair[e] = r.eb - rr / (6.f * fabsf(sg));
}

// A skipped update sends nothing: its receivers' cells are cleared.
__device__ __forceinline__ void adj_clear(const DevTopo &T, const AdjEnt &r)
{
    const float3 z = make_float3(0.f, 0.f, 0.f);
    if (r.tg.x >= 0) adj_send(T, r.tg.x, z);
    if (r.tg.y >= 0) adj_send(T, r.tg.y, z);
    if (r.tg.z >= 0) adj_send(T, r.tg.z, z);
}

// Reverse of one color phase, every entry of the vertex in registers
// (D <= L * KU): all loads of the phase's vertex are issued before any
// arithmetic (two dependent memory round trips: the entries, then the
// neighbour positions).
template <int L, int KU>
__global__ __launch_bounds__(kMaxBlock) void k_adjoint_one(DevTopo T, StepConsts K,
                                                           const float4 *Sn, const float4 *Sp,
                                                           int v_begin, int v_end, int2 ell,
                                                           int remap)
{
    const int b = xcd_block(blockIdx.x, gridDim.x, remap);
    const int gid = b * blockDim.x + threadIdx.x;
    const int p = v_begin + gid / L;
    const int lane = threadIdx.x & (L - 1);
    const bool active = p < v_end;
    const int c_end = v_end;   // permuted slots < c_end have color <= c
    const int D = active ? ell.y : 0;
    const size_t e0 = (size_t)ell.x + (size_t)(active ? p - v_begin : 0) * ell.y;
    const float mu_lam = K.k_mu / K.k_lam;
    AdjEnt r[KU];
    bool ok[KU];
#pragma unroll
    for (int j = 0; j < KU; ++j) {
        const int e = lane + j * L;
        ok[j] = e < D;
        if (ok[j]) adj_load(T, e0 + e, r[j]);
    }
    float4 own = make_float4(0.f, 0.f, 0.f, 0.f), xb4 = own;
    float wm = 0.f;
    if (active) {
        own = Sn[p];
        xb4 = T.xbar[p];
        wm = T.y[p].w;
    }
    float4 qa[KU], qb[KU], qc[KU];
#pragma unroll
    for (int j = 0; j < KU; ++j) {
        ok[j] = ok[j] && r[j].ws.w != 0.f;
        if (ok[j]) {
            qa[j] = adj_pos(Sn, Sp, r[j].pa.x, c_end);
            qb[j] = adj_pos(Sn, Sp, r[j].pa.y, c_end);
            qc[j] = adj_pos(Sn, Sp, r[j].pa.z, c_end);
        }
    }
    // pass 1: H_i at the post-update state; the incoming cells fold in
    Acc a;
    acc_zero(a);
#pragma unroll
    for (int j = 0; j < KU; ++j)
        if (ok[j]) {
            const float vlam = __int_as_float(r[j].pa.w);
            const float hmu = -(r[j].ws.x + r[j].ws.y + r[j].ws.z) * (vlam * mu_lam);
            adj_hess(qa[j], qb[j], qc[j], hmu, vlam, r[j].ws.w, a);
            a.fx += r[j].g0.x + r[j].g1.x + r[j].g2.x;
            a.fy += r[j].g0.y + r[j].g1.y + r[j].g2.y;
            a.fz += r[j].g0.z + r[j].g1.z + r[j].g2.z;
        }
    acc_reduce<L>(a);
    if (!active) return;
    a.hxx += wm; a.hyy += wm; a.hzz += wm;
    a.fx += xb4.x; a.fy += xb4.y; a.fz += xb4.z;
    float3 w;
    if (!solve_sym3(a, K.det_eps_rel, w)) {
        // skipped update: the adjoint passes through (with the incoming cells)
        if (lane == 0) T.xbar[p] = make_float4(a.fx, a.fy, a.fz, 0.f);
#pragma unroll
        for (int j = 0; j < KU; ++j)
            if (ok[j]) adj_clear(T, r[j]);
        return;
    }
    if (lane == 0) {
        T.xbar[p] = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 yb = T.ybar[p];
        yb.x += wm * w.x; yb.y += wm * w.y; yb.z += wm * w.z;
        T.ybar[p] = yb;
    }
    // pass 2 from the registers
    const float3 xi = xyz(own);
#pragma unroll
    for (int j = 0; j < KU; ++j)
        if (ok[j]) adj_emit(T, K, e0 + lane + j * L, r[j], xi, qa[j], qb[j], qc[j], w, mu_lam);
}

// The general form for any padded degree: the vertex's entries in batches of
// L * KU, loaded again in the second pass.
template <int L, int KU>
__global__ __launch_bounds__(kMaxBlock) void k_adjoint_color(DevTopo T, StepConsts K,
                                                             const float4 *Sn, const float4 *Sp,
                                                             int v_begin, int v_end, int2 ell,
                                                             int remap)
{
    const int b = xcd_block(blockIdx.x, gridDim.x, remap);
    const int gid = b * blockDim.x + threadIdx.x;
    const int p = v_begin + gid / L;
    const int lane = threadIdx.x & (L - 1);
    const bool active = p < v_end;
    const int c_end = v_end;
    const int D = active ? ell.y : 0;
    const size_t e0 = (size_t)ell.x + (size_t)(active ? p - v_begin : 0) * ell.y;
    const float mu_lam = K.k_mu / K.k_lam;
    Acc a;
    acc_zero(a);
    float4 own = make_float4(0.f, 0.f, 0.f, 0.f), xb4 = own;
    float wm = 0.f;
    if (active) {
        own = Sn[p];
        xb4 = T.xbar[p];
        wm = T.y[p].w;
    }
    for (int base = lane; base < D; base += L * KU) {
        AdjEnt r[KU];
        bool ok[KU];
#pragma unroll
        for (int j = 0; j < KU; ++j) {
            const int e = base + j * L;
            ok[j] = e < D;
            if (ok[j]) adj_load(T, e0 + e, r[j]);
        }
#pragma unroll
        for (int j = 0; j < KU; ++j)
            if (ok[j] && r[j].ws.w != 0.f) {
                const float4 qa = adj_pos(Sn, Sp, r[j].pa.x, c_end);
                const float4 qb = adj_pos(Sn, Sp, r[j].pa.y, c_end);
                const float4 qc = adj_pos(Sn, Sp, r[j].pa.z, c_end);
                const float vlam = __int_as_float(r[j].pa.w);
                const float hmu = -(r[j].ws.x + r[j].ws.y + r[j].ws.z) * (vlam * mu_lam);
                adj_hess(qa, qb, qc, hmu, vlam, r[j].ws.w, a);
                a.fx += r[j].g0.x + r[j].g1.x + r[j].g2.x;
                a.fy += r[j].g0.y + r[j].g1.y + r[j].g2.y;
                a.fz += r[j].g0.z + r[j].g1.z + r[j].g2.z;
            }
    }
    acc_reduce<L>(a);
    if (!active) return;
    a.hxx += wm; a.hyy += wm; a.hzz += wm;
    a.fx += xb4.x; a.fy += xb4.y; a.fz += xb4.z;
    float3 w;
    const bool solved = solve_sym3(a, K.det_eps_rel, w);
    if (lane == 0) {
        if (!solved) {
            T.xbar[p] = make_float4(a.fx, a.fy, a.fz, 0.f);
        } else {
            T.xbar[p] = make_float4(0.f, 0.f, 0.f, 0.f);
            float4 yb = T.ybar[p];
            yb.x += wm * w.x; yb.y += wm * w.y; yb.z += wm * w.z;
            T.ybar[p] = yb;
        }
    }
    const float3 xi = xyz(own);
    for (int base = lane; base < D; base += L * KU) {
        AdjEnt r[KU];
        bool ok[KU];
#pragma unroll
        for (int j = 0; j < KU; ++j) {
            const int e = base + j * L;
            ok[j] = e < D;
            if (ok[j]) adj_load(T, e0 + e, r[j]);
        }
#pragma unroll
        for (int j = 0; j < KU; ++j)
            if (ok[j] && r[j].ws.w != 0.f) {
                if (!solved) {
                    adj_clear(T, r[j]);
                    continue;
                }
                const float4 qa = adj_pos(Sn, Sp, r[j].pa.x, c_end);
                const float4 qb = adj_pos(Sn, Sp, r[j].pa.y, c_end);
                const float4 qc = adj_pos(Sn, Sp, r[j].pa.z, c_end);
                adj_emit(T, K, e0 + base + j * L, r[j], xi, qa, qb, qc, w, mu_lam);
            }
    }
}

// End of the reverse sweep: each vertex adds the contributions written after
// its last update: a free vertex the incoming cells from colors below its own
// (its entries' other vertices with smaller slots), a pinned vertex all of
// its (tet, slot) cells.  A group of kFoldLanes lanes per vertex, over its
// entries, then a group sum.  The cells it reads are cleared for the next
// sweep: cells from lower colors are read before they are written in a sweep,
// the other cells of free senders are written first (a skipped update writes
// zeros), and cells of pinned senders are never written.
constexpr int kFoldLanes = 8;
__global__ __launch_bounds__(256) void k_bwd_fold(DevTopo T)
{
    const int L = kFoldLanes;
    const int p = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) / L);
    const int lane = threadIdx.x & (L - 1);
    const bool active = p < T.n_verts;
    float3 g = make_float3(0.f, 0.f, 0.f);
    if (active && p < T.n_free) {
        int c = 0;
        while (c + 1 < T.n_colors && T.color_off[c + 1] <= p) ++c;
        const int lo = T.color_off[c];
        const int2 info = T.ell_info[c];
        const size_t e0 = (size_t)info.x + (size_t)(p - lo) * (size_t)info.y;
        const size_t np = (size_t)T.n_pairs;
        for (int e = lane; e < info.y; e += L) {
            const size_t i = e0 + e;
            if (T.pws[i].w == 0.f) continue;   // padding
            const int4 pa = T.pa[i];
            const int src[3] = {pa.x, pa.y, pa.z};
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (src[j] < lo) {
                    float3 *cell = T.cin + (size_t)j * np + i;
                    const float3 cj = *cell;
                    g.x += cj.x; g.y += cj.y; g.z += cj.z;
                    *cell = make_float3(0.f, 0.f, 0.f);
                }
        }
    } else if (active) {
        for (int e = T.tet_row[p] + lane; e < T.tet_row[p + 1]; e += L) {
            const int ent = T.tet_ent[e].x;
            float3 *cell = T.contrib + 4 * (size_t)(ent >> 2) + (ent & 3);
            const float3 cj = *cell;
            g.x += cj.x; g.y += cj.y; g.z += cj.z;
            *cell = make_float3(0.f, 0.f, 0.f);
        }
    }
    g.x = group_sum<L>(g.x);
    g.y = group_sum<L>(g.y);
    g.z = group_sum<L>(g.z);
    if (!active || lane != 0) return;
    float4 xb = T.xbar[p];
    xb.x += g.x; xb.y += g.y; xb.z += g.z;
    T.xbar[p] = xb;
}

// Start of a recorded step: snapshot 1 = snapshot 0 (the initial guess), and
// the pinned slots of snapshots 2..n_iters from snapshot 0 (pinned vertices
// are never updated; the updates of the free ones are stored into the next
// snapshot by the solve).  blockIdx.y = snapshot - 1.
__global__ void k_seed_snapshots(float4 *snaps, int nv, int n_free)
{
    const int n = (int)blockIdx.y + 1;
    const int lo = n == 1 ? 0 : n_free;
    const int p = lo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= nv) return;
    snaps[(size_t)n * nv + p] = snaps[p];
}

// Adjoint of the initial guess (Sec. 3.7) and of y, written in original order.
__global__ void k_bwd_final(DevTopo T, const float *v_t, const float *v_prev, float *gx_in,
                            float *gv_in, float *gvp_in, float *gE, StepConsts K)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    // Ebar: the shares of the tet's free vertices, added into the caller's
    // order; the shares are cleared for the next sweep
    for (int t = p; t < T.n_tets; t += gridDim.x * blockDim.x) {
        const int4 q = T.tet_pairs[t];
        float eb = 0.f;
        if (q.x >= 0) { eb += T.ebar_pair[q.x]; T.ebar_pair[q.x] = 0.f; }
        if (q.y >= 0) { eb += T.ebar_pair[q.y]; T.ebar_pair[q.y] = 0.f; }
        if (q.z >= 0) { eb += T.ebar_pair[q.z]; T.ebar_pair[q.z] = 0.f; }
        if (q.w >= 0) { eb += T.ebar_pair[q.w]; T.ebar_pair[q.w] = 0.f; }
        gE[T.tet_perm[t]] += eb;
    }
    if (p >= T.n_verts) return;
    const int o = T.perm[p];
    const float3 xb = xyz(T.xbar[p]);
    float3 gx = xyz(T.xtbar[p]) + xb;
    float3 gv = xyz(T.vbar[p]);
    float3 gvp = make_float3(0.f, 0.f, 0.f);
    if (p < T.n_free) {
        const float h = K.h;
        if (K.init_mode != 0) gv = gv + xb * h;
        if (K.init_mode == 3 && K.gnorm > 0.f) {
            const float3 g = make_float3(K.gx, K.gy, K.gz);
            const float at = dot3((ld3(v_t, o) - ld3(v_prev, o)) * K.inv_h, g) / K.gnorm;
            if (at > 0.f && at < K.gnorm) {
                const float s = h * h * dot3(g, xb) / K.gnorm;
                const float3 dd = g * (s / (K.gnorm * h));
                gv = gv + dd;
                gvp = gvp - dd;
            }
        }
        const float3 yb = xyz(T.ybar[p]);
        gx = gx + yb;
        gv = gv + yb * h;
    }
    st3(gx_in, o, gx);
    st3(gv_in, o, gv);
    st3(gvp_in, o, gvp);
}

// -------------------------------------------------------------- launchers --
static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

hipError_t launch_material(const DevTopo &T, const float *tet_E, const StepConsts &K, bool compact,
                           hipStream_t s)
{
    if (T.n_tets == 0) return hipSuccess;
    if (T.n_pairs > 0)
        hipLaunchKernelGGL(k_material_pairs, dim3(cdiv(T.n_pairs, 256)), dim3(256), 0, s, T.pa, T.pw,
                           T.pws, T.pair_tet, T.vol, T.tet_perm, tet_E, T.n_pairs, K.k_mu, K.k_lam,
                           compact ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_predict(const DevTopo &T, const float *x, const float *v, const float *vp,
                          const StepConsts &K, bool reset_flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_predict, dim3(cdiv(T.n_verts > 0 ? T.n_verts : 1, 256)), dim3(256), 0, s,
                       T, x, v, vp, K, reset_flags ? 1 : 0, K.cheb_rho > 0.f ? 1 : 0);
    return hipGetLastError();
}

template <int L, int KU>
static hipError_t solve_dispatch(const DevTopo &T, const StepConsts &K, int vb, int ve, int4 inc,
                                 bool tets, bool springs, const LaunchCfg &cfg, hipStream_t s,
                                 XcdSplit xs)
{
    const int grid = xs.dev ? 8 * cdiv((long)xs.max_size * L, cfg.block) : cdiv((long)(ve - vb) * L, cfg.block);
    const bool cr = cfg.compact != 0;
    if (tets && springs && cr)
        hipLaunchKernelGGL((k_solve<L, KU, true, true, true>), dim3(grid), dim3(cfg.block), 0, s, T, K, vb, ve, inc, cfg.xcd_remap, xs.dev);
    else if (tets && springs)
        hipLaunchKernelGGL((k_solve<L, KU, true, true, false>), dim3(grid), dim3(cfg.block), 0, s, T, K, vb, ve, inc, cfg.xcd_remap, xs.dev);
    else if (tets && cr)
        hipLaunchKernelGGL((k_solve<L, KU, true, false, true>), dim3(grid), dim3(cfg.block), 0, s, T, K, vb, ve, inc, cfg.xcd_remap, xs.dev);
    else if (tets)
        hipLaunchKernelGGL((k_solve<L, KU, true, false, false>), dim3(grid), dim3(cfg.block), 0, s, T, K, vb, ve, inc, cfg.xcd_remap, xs.dev);
    else if (springs)
        hipLaunchKernelGGL((k_solve<L, 1, false, true, false>), dim3(grid), dim3(cfg.block), 0, s, T, K, vb, ve, inc, cfg.xcd_remap, xs.dev);
    else
        hipLaunchKernelGGL((k_solve<L, 1, false, false, false>), dim3(grid), dim3(cfg.block), 0, s, T, K, vb, ve, inc, cfg.xcd_remap, xs.dev);
    return hipGetLastError();
}

template <int L>
static hipError_t solve_unroll(const DevTopo &T, const StepConsts &K, int vb, int ve, int4 inc,
                               bool tets, bool springs, const LaunchCfg &cfg, hipStream_t s, XcdSplit xs)
{
    switch (cfg.unroll) {
    case 1: return solve_dispatch<L, 1>(T, K, vb, ve, inc, tets, springs, cfg, s, xs);
    case 2: return solve_dispatch<L, 2>(T, K, vb, ve, inc, tets, springs, cfg, s, xs);
    case 3: return solve_dispatch<L, 3>(T, K, vb, ve, inc, tets, springs, cfg, s, xs);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve(const DevTopo &T, const StepConsts &K, int vb, int ve, int4 inc, bool tets,
                        bool springs, const LaunchCfg &cfg, hipStream_t s, XcdSplit xs)
{
    if (ve <= vb) return hipSuccess;
    if (cfg.block > kMaxBlock) return hipErrorInvalidValue;
    if (cfg.xcd_remap != 3) xs = XcdSplit{nullptr, 0};
    switch (cfg.lanes) {
    case 2: return solve_unroll<2>(T, K, vb, ve, inc, tets, springs, cfg, s, xs);
    case 4: return solve_unroll<4>(T, K, vb, ve, inc, tets, springs, cfg, s, xs);
    case 8: return solve_unroll<8>(T, K, vb, ve, inc, tets, springs, cfg, s, xs);
    case 16: return solve_unroll<16>(T, K, vb, ve, inc, tets, springs, cfg, s, xs);
    case 32: return solve_unroll<32>(T, K, vb, ve, inc, tets, springs, cfg, s, xs);
    default: return hipErrorInvalidValue;
    }
}

template <int L, int KU>
static hipError_t solve_mc_dispatch(const DevTopo &T, const DevSurf &S, const StepConsts &K, int vb,
                                    int ve, int4 inc, int pb, int pe, bool tets, bool springs,
                                    const LaunchCfg &cfg, hipStream_t s, XcdSplit xs)
{
    const int grid = xs.dev ? 8 * cdiv((long)xs.max_size * L, cfg.block) : cdiv((long)(ve - vb) * L, cfg.block);
    const bool cr = cfg.compact != 0;
    if (tets && springs && cr)
        hipLaunchKernelGGL((k_solve_mc<L, KU, true, true, true>), dim3(grid), dim3(cfg.block), 0, s, T, S, K, vb, ve, inc, pb, pe, cfg.xcd_remap, xs.dev);
    else if (tets && springs)
        hipLaunchKernelGGL((k_solve_mc<L, KU, true, true, false>), dim3(grid), dim3(cfg.block), 0, s, T, S, K, vb, ve, inc, pb, pe, cfg.xcd_remap, xs.dev);
    else if (tets && cr)
        hipLaunchKernelGGL((k_solve_mc<L, KU, true, false, true>), dim3(grid), dim3(cfg.block), 0, s, T, S, K, vb, ve, inc, pb, pe, cfg.xcd_remap, xs.dev);
    else if (tets)
        hipLaunchKernelGGL((k_solve_mc<L, KU, true, false, false>), dim3(grid), dim3(cfg.block), 0, s, T, S, K, vb, ve, inc, pb, pe, cfg.xcd_remap, xs.dev);
    else if (springs)
        hipLaunchKernelGGL((k_solve_mc<L, 1, false, true, false>), dim3(grid), dim3(cfg.block), 0, s, T, S, K, vb, ve, inc, pb, pe, cfg.xcd_remap, xs.dev);
    else
        hipLaunchKernelGGL((k_solve_mc<L, 1, false, false, false>), dim3(grid), dim3(cfg.block), 0, s, T, S, K, vb, ve, inc, pb, pe, cfg.xcd_remap, xs.dev);
    return hipGetLastError();
}

template <int L>
static hipError_t solve_mc_unroll(const DevTopo &T, const DevSurf &S, const StepConsts &K, int vb,
                                  int ve, int4 inc, int pb, int pe, bool tets, bool springs,
                                  const LaunchCfg &cfg, hipStream_t s, XcdSplit xs)
{
    switch (cfg.unroll) {
    case 1: return solve_mc_dispatch<L, 1>(T, S, K, vb, ve, inc, pb, pe, tets, springs, cfg, s, xs);
    case 2: return solve_mc_dispatch<L, 2>(T, S, K, vb, ve, inc, pb, pe, tets, springs, cfg, s, xs);
    case 3: return solve_mc_dispatch<L, 3>(T, S, K, vb, ve, inc, pb, pe, tets, springs, cfg, s, xs);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve_contacts(const DevTopo &T, const DevSurf &S, const StepConsts &K, int vb,
                                 int ve, int4 inc, int pb, int pe, bool tets, bool springs,
                                 const LaunchCfg &cfg, hipStream_t s, XcdSplit xs)
{
    if (ve <= vb) return hipSuccess;
    if (cfg.block > kMaxBlock) return hipErrorInvalidValue;
    if (cfg.xcd_remap != 3) xs = XcdSplit{nullptr, 0};
    switch (cfg.lanes) {
    case 2: return solve_mc_unroll<2>(T, S, K, vb, ve, inc, pb, pe, tets, springs, cfg, s, xs);
    case 4: return solve_mc_unroll<4>(T, S, K, vb, ve, inc, pb, pe, tets, springs, cfg, s, xs);
    case 8: return solve_mc_unroll<8>(T, S, K, vb, ve, inc, pb, pe, tets, springs, cfg, s, xs);
    case 16: return solve_mc_unroll<16>(T, S, K, vb, ve, inc, pb, pe, tets, springs, cfg, s, xs);
    case 32: return solve_mc_unroll<32>(T, S, K, vb, ve, inc, pb, pe, tets, springs, cfg, s, xs);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cheb(const DevTopo &T, const StepConsts &K, int iter, hipStream_t s, float4 *snap)
{
    if (T.n_free == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cheb, dim3(cdiv(T.n_free, 256)), dim3(256), 0, s, T, K.cheb_rho, iter, snap);
    return hipGetLastError();
}

hipError_t launch_finalize(const DevTopo &T, float *x, float *v, float *vp, const StepConsts &K,
                           hipStream_t s)
{
    if (T.n_verts == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(cdiv(T.n_verts, 256)), dim3(256), 0, s, T, x, v, vp, K.h);
    return hipGetLastError();
}

template <int L, int KU, bool TE, bool SP, bool CR>
static hipError_t persistent_go(const DevTopo &T, const StepConsts &K, int n_iters,
                                const LaunchCfg &cfg, int n_cu, bool coop, hipStream_t s,
                                int *grid_out)
{
    auto fn = k_persistent<L, KU, TE, SP, CR>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, cfg.block, 0);
    if (e != hipSuccess) return e;
    if (per_cu <= 0) return hipErrorInvalidConfiguration;
    // The occupancy query does not see every residency limit (on gfx950 a
    // kernel's SGPRs can allow fewer waves than it assumes), so the grid
    // fills kPersistentWavesPerSimd waves per SIMD (4 SIMDs per CU), an
    // occupancy every persistent kernel is compiled for.
    per_cu = std::min(per_cu, std::max(1, kPersistentWavesPerSimd * 4 * 64 / cfg.block));
    if (cfg.blocks_per_cu > 0 && cfg.blocks_per_cu < per_cu) per_cu = cfg.blocks_per_cu;
    const int grid = per_cu * n_cu;
    if (grid_out) *grid_out = grid;
    DevTopo Tc = T;
    StepConsts Kc = K;
    int it = n_iters, rm = cfg.xcd_remap;
    if (coop) {
        void *args[] = {(void *)&Tc, (void *)&Kc, (void *)&it, (void *)&rm};
        return hipLaunchCooperativeKernel((const void *)fn, dim3(grid), dim3(cfg.block), args, 0, s);
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.block), 0, s, Tc, Kc, it, rm);
    return hipGetLastError();
}

template <int L, int KU>
static hipError_t persistent_kinds(const DevTopo &T, const StepConsts &K, int n_iters, bool tets,
                                   bool springs, const LaunchCfg &cfg, int n_cu, bool coop,
                                   hipStream_t s, int *grid_out)
{
    const bool cr = cfg.compact != 0;
    if (tets && springs && cr) return persistent_go<L, KU, true, true, true>(T, K, n_iters, cfg, n_cu, coop, s, grid_out);
    if (tets && springs) return persistent_go<L, KU, true, true, false>(T, K, n_iters, cfg, n_cu, coop, s, grid_out);
    if (tets && cr) return persistent_go<L, KU, true, false, true>(T, K, n_iters, cfg, n_cu, coop, s, grid_out);
    if (tets) return persistent_go<L, KU, true, false, false>(T, K, n_iters, cfg, n_cu, coop, s, grid_out);
    if (springs) return persistent_go<L, 1, false, true, false>(T, K, n_iters, cfg, n_cu, coop, s, grid_out);
    return persistent_go<L, 1, false, false, false>(T, K, n_iters, cfg, n_cu, coop, s, grid_out);
}

template <int L>
static hipError_t persistent_unroll(const DevTopo &T, const StepConsts &K, int n_iters, bool tets,
                                    bool springs, const LaunchCfg &cfg, int n_cu, bool coop,
                                    hipStream_t s, int *grid_out)
{
    switch (cfg.unroll) {
    case 1: return persistent_kinds<L, 1>(T, K, n_iters, tets, springs, cfg, n_cu, coop, s, grid_out);
    case 2: return persistent_kinds<L, 2>(T, K, n_iters, tets, springs, cfg, n_cu, coop, s, grid_out);
    case 3: return persistent_kinds<L, 3>(T, K, n_iters, tets, springs, cfg, n_cu, coop, s, grid_out);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_persistent(const DevTopo &T, const StepConsts &K, int n_iters, bool tets,
                             bool springs, const LaunchCfg &cfg, int n_cu, bool coop,
                             hipStream_t s, int *grid_out)
{
    if (cfg.block > kMaxBlock) return hipErrorInvalidValue;
    switch (cfg.lanes) {
    case 2: return persistent_unroll<2>(T, K, n_iters, tets, springs, cfg, n_cu, coop, s, grid_out);
    case 4: return persistent_unroll<4>(T, K, n_iters, tets, springs, cfg, n_cu, coop, s, grid_out);
    case 8: return persistent_unroll<8>(T, K, n_iters, tets, springs, cfg, n_cu, coop, s, grid_out);
    case 16: return persistent_unroll<16>(T, K, n_iters, tets, springs, cfg, n_cu, coop, s, grid_out);
    case 32: return persistent_unroll<32>(T, K, n_iters, tets, springs, cfg, n_cu, coop, s, grid_out);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_read4(const float4 *src, long long n, float *out, int blocks, hipStream_t s)
{
    if (n <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_read4, dim3(blocks), dim3(256), 0, s, src, n, out);
    return hipGetLastError();
}

hipError_t launch_copy4(float4 *dst, const float4 *src, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int grid = cdiv(n, 256);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_copy4, dim3(grid), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_check_finite(const float *a, const float *b, long long n, unsigned *flags,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)std::min<long long>(blocks, 2048)), dim3(256), 0, s,
                       a, b, n, flags);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned *p, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min<long long>(blocks, 1 << 16)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_bwd_init(const DevTopo &T, const float *gx, const float *gv, const float *gvp,
                           const StepConsts &K, hipStream_t s)
{
    hipLaunchKernelGGL(k_bwd_init, dim3(cdiv(T.n_verts, 256)), dim3(256), 0, s, T, gx, gv, gvp, K.h);
    return hipGetLastError();
}

template <int L>
static void adjoint_go(const DevTopo &T, const StepConsts &K, const float4 *Sn, const float4 *Sp,
                       int vb, int ve, int2 ell, const LaunchCfg &cfg, hipStream_t s)
{
    const int grid = cdiv((long)(ve - vb) * L, cfg.block);
    // a color whose padded degree fits one batch of up to 2 entries per lane
    // takes the single-batch kernel
    if (ell.y <= L)
        hipLaunchKernelGGL((k_adjoint_one<L, 1>), dim3(grid), dim3(cfg.block), 0, s, T, K, Sn, Sp, vb, ve, ell, cfg.xcd_remap);
    else if (ell.y <= 2 * L)
        hipLaunchKernelGGL((k_adjoint_one<L, 2>), dim3(grid), dim3(cfg.block), 0, s, T, K, Sn, Sp, vb, ve, ell, cfg.xcd_remap);
    else if (cfg.unroll >= 2)
        hipLaunchKernelGGL((k_adjoint_color<L, 2>), dim3(grid), dim3(cfg.block), 0, s, T, K, Sn, Sp, vb, ve, ell, cfg.xcd_remap);
    else
        hipLaunchKernelGGL((k_adjoint_color<L, 1>), dim3(grid), dim3(cfg.block), 0, s, T, K, Sn, Sp, vb, ve, ell, cfg.xcd_remap);
}

hipError_t launch_adjoint_color(const DevTopo &T, const StepConsts &K, const float4 *Sn,
                                const float4 *Sp, int vb, int ve, int2 ell, const LaunchCfg &cfg,
                                hipStream_t s)
{
    if (ve <= vb) return hipSuccess;
    // at least 16 lanes per vertex: a phase has few vertices on small meshes
    // and the reverse work per vertex is about three times the forward's; one
    // entry per lane when the padded degree allows (measured faster on the
    // 33^3 cube, degree 24, than 16 lanes with two entries each)
    switch (cfg.lanes) {
    case 2:
    case 4:
    case 8:
    case 16:
        if (ell.y > 16) adjoint_go<32>(T, K, Sn, Sp, vb, ve, ell, cfg, s);
        else adjoint_go<16>(T, K, Sn, Sp, vb, ve, ell, cfg, s);
        break;
    case 32: adjoint_go<32>(T, K, Sn, Sp, vb, ve, ell, cfg, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bwd_fold(const DevTopo &T, hipStream_t s)
{
    if (T.n_verts <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bwd_fold, dim3(cdiv((long)T.n_verts * kFoldLanes, 256)), dim3(256), 0, s, T);
    return hipGetLastError();
}

hipError_t launch_seed_snapshots(const DevTopo &T, int n_iters, hipStream_t s)
{
    if (T.n_verts <= 0 || n_iters < 1) return hipSuccess;
    // snapshot 1 covers every slot; later ones only the pinned range
    hipLaunchKernelGGL(k_seed_snapshots, dim3(cdiv(T.n_verts, 256), n_iters), dim3(256), 0, s, T.snaps,
                       T.n_verts, T.n_free);
    return hipGetLastError();
}

hipError_t launch_bwd_final(const DevTopo &T, const float *v_t, const float *v_prev, float *gx_in,
                            float *gv_in, float *gvp_in, float *gE, const StepConsts &K, hipStream_t s)
{
    hipLaunchKernelGGL(k_bwd_final, dim3(cdiv(T.n_verts, 256)), dim3(256), 0, s, T, v_t, v_prev,
                       gx_in, gv_in, gvp_in, gE, K);
    return hipGetLastError();
}

}  // namespace vbd
