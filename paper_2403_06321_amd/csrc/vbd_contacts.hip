// gfx950 kernels of the mesh-mesh contact detection (Sec. 3.5).
//
// Discrete detection on a set of positions X (x^t at the start of a step,
// the current iterate when it is repeated): every surface vertex takes the
// closest surface triangle of another mesh within the collision radius, and
// the pair becomes a contact element when the vertex lies inside that mesh
// or closer than the contact thickness to its surface.
//
// Broad phase: triangle centroids binned into a hashed uniform grid whose
// cell size s = r + R_max (R_max = largest centroid-to-corner distance of any
// surface triangle at X).  A point within r of a triangle is within
// r + R_max of its centroid, so the 27 cells around the vertex's cell hold
// every candidate.  Buckets are built by counting, an exclusive scan and a
// fill; the query keeps the minimum of (distance, triangle index), which does
// not depend on the order inside a bucket.  Bucket items carry the
// triangle's mesh (same-mesh candidates are skipped without further loads)
// and a bounding sphere rejects triangles that cannot beat the best so far.
//
// Inside test: the sign of (p - q).N with N the angle-weighted pseudonormal of
// the closest feature (face normal, sum of the two face normals of an edge,
// angle-weighted vertex normal), exact for closed, consistently oriented
// surfaces (Baerentzen and Aanaes, IEEE TVCG 11(3), 2005).
//
// The corner incidence (for each vertex, the colliding vertices whose
// contact triangle has it as a corner) is built the same way and each row is
// sorted, so the solve visits the elements in a fixed order.
//
// Self-contact: triangles of the vertex's own mesh are candidates when they
// share no vertex with it and lie farther than the exclusion distance from it
// in the rest shape; such a pair is kept when its element is active.
//
// Edge-edge elements: edge midpoints binned the same way (cell size r +
// 2 L_max, L_max the largest half edge length), every surface edge takes the
// closest eligible edge within r (minimum of (distance, edge index)), and the
// pair is kept when its closest points are interior to both edges, the edges
// are not nearly parallel and the element, with its normal taken from the
// contact points at x^t, is active; a pair found from both edges is kept from
// the lower index.  Each vertex's elements form a sorted incidence row.
#include "vbd_device.h"

namespace vbd {

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------- scan --
// Exclusive scan of n unsigned values into out[0..n], out[n] = total.  Three
// launches: per-block scans of kScanTile values with the block totals in tmp,
// one block scanning tmp, then the block offsets added.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

// In-place exclusive scan of the kScanTile values in lds; returns the total.
__device__ unsigned block_scan_tile(unsigned *lds, unsigned *sums)
{
    const int tid = threadIdx.x;
    unsigned run = 0;
    unsigned v[kScanPer];
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = lds[tid * kScanPer + j];
        run += v[j];
    }
    sums[tid] = run;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread sums
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const unsigned add = tid >= off ? sums[tid - off] : 0u;
        __syncthreads();
        sums[tid] += add;
        __syncthreads();
    }
    const unsigned total = sums[kScanThreads - 1];
    unsigned acc = sums[tid] - run;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        lds[tid * kScanPer + j] = acc;
        acc += v[j];
    }
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const unsigned *in, unsigned *out,
                                                             unsigned *tmp, int n)
{
    __shared__ unsigned lds[kScanTile];
    __shared__ unsigned sums[kScanThreads];
    const long base = (long)blockIdx.x * kScanTile;
    for (int j = threadIdx.x; j < kScanTile; j += kScanThreads)
        lds[j] = (base + j < n) ? in[base + j] : 0u;
    __syncthreads();
    const unsigned total = block_scan_tile(lds, sums);
    for (int j = threadIdx.x; j < kScanTile; j += kScanThreads)
        if (base + j < n) out[base + j] = lds[j];
    if (threadIdx.x == 0) tmp[blockIdx.x] = total;
}

// One block: exclusive scan of the nb block totals (in tiles, with a carry);
// out[n] receives the grand total.
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(unsigned *tmp, int nb, unsigned *out,
                                                              int n)
{
    __shared__ unsigned lds[kScanTile];
    __shared__ unsigned sums[kScanThreads];
    unsigned carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kScanTile) {
        for (int j = threadIdx.x; j < kScanTile; j += kScanThreads)
            lds[j] = (b0 + j < nb) ? tmp[b0 + j] : 0u;
        __syncthreads();
        const unsigned total = block_scan_tile(lds, sums);
        for (int j = threadIdx.x; j < kScanTile; j += kScanThreads)
            if (b0 + j < nb) tmp[b0 + j] = lds[j] + carry;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(unsigned *out, const unsigned *tmp, int n)
{
    const long base = (long)blockIdx.x * kScanTile;
    const unsigned add = tmp[blockIdx.x];
    for (int j = threadIdx.x; j < kScanTile; j += kScanThreads)
        if (base + j < n) out[base + j] += add;
}

static hipError_t scan_exclusive(const unsigned *in, unsigned *out, unsigned *tmp, int n,
                                 hipStream_t s)
{
    const int nb = cdiv(n > 0 ? n : 1, kScanTile);
    hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kScanThreads), 0, s, in, out, tmp, n);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, s, tmp, nb, out, n);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanThreads), 0, s, out, tmp, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------- fill --
__global__ void k_fill_u32(unsigned *p, int n, unsigned v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static hipError_t fill_u32(unsigned *p, int n, unsigned v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(cdiv(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------ grid helpers --
__device__ __forceinline__ int cell_coord(float v, float inv_s)
{
    // clamped so that far-away points still map to valid (if shared) cells
    const float c = floorf(v * inv_s);
    return (int)fminf(fmaxf(c, -1048576.f), 1048576.f);
}

// Spatial hash of a grid cell: the XOR of the cell coordinates times three
// large primes, as proposed by Teschner et al., "Optimized Spatial Hashing for
// Collision Detection of Deformable Objects" (VMV 2003), masked to the
// power-of-two bucket count.
__device__ __forceinline__ unsigned cell_hash(int i, int j, int k, int mask)
{
    const unsigned h = ((unsigned)i * 73856093u) ^ ((unsigned)j * 19349663u) ^ ((unsigned)k * 83492791u);
    return h & (unsigned)mask;
}

__device__ __forceinline__ float grid_cell_size(const DevSurf &S, const StepConsts &K)
{
    const float s = K.col_radius + __uint_as_float(S.gparam[0]);
    return s > 0.f ? s : 1.f;
}

// ---------------------------------------------------------------- kernels --
// Unit normals, bounding spheres, and per block the largest centroid-to-
// corner distance (gmax[block]; k_max_radius reduces them, which avoids
// serialising every block on one atomic).
__global__ __launch_bounds__(256) void k_tri_prep(DevSurf S, const float4 *X)
{
    __shared__ float wmax[4];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    float R = 0.f;
    if (t < S.n_tri) {
        const int4 tr = S.tri[t];
        const float3 a = xyz(X[tr.x]), b = xyz(X[tr.y]), c = xyz(X[tr.z]);
        const float3 n = cross3(b - a, c - a);
        const float l = sqrtf(dot3(n, n));
        const float3 u = l > 0.f ? n * (1.0f / l) : make_float3(0.f, 0.f, 0.f);
        S.tnorm[t] = make_float4(u.x, u.y, u.z, 0.f);
        const float3 g = (a + b + c) * (1.0f / 3.0f);
        const float3 da = a - g, db = b - g, dc = c - g;
        R = sqrtf(fmaxf(dot3(da, da), fmaxf(dot3(db, db), dot3(dc, dc))));
        S.tsph[t] = make_float4(g.x, g.y, g.z, R);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) R = fmaxf(R, __shfl_xor(R, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = R;
    __syncthreads();
    if (threadIdx.x == 0)
        S.gmax[blockIdx.x] = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
}

// One block: *out = float bits of the largest of the nb per-block maxima
// (gparam[0]: triangle radius, gparam[1]: half edge length).
__global__ __launch_bounds__(256) void k_max_radius(const float *gmax, int nb, unsigned *out)
{
    __shared__ float wmax[4];
    float R = 0.f;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) R = fmaxf(R, gmax[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) R = fmaxf(R, __shfl_xor(R, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = R;
    __syncthreads();
    if (threadIdx.x == 0) *out = __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3])));
}

// Angle-weighted pseudonormal of every surface vertex.
__global__ void k_vert_normals(DevSurf S, const float4 *X)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= S.n_sv) return;
    const int slot = S.svert[v].x;
    const float3 xv = xyz(X[slot]);
    float3 acc = make_float3(0.f, 0.f, 0.f);
    for (int e = S.sv_row[v]; e < S.sv_row[v + 1]; ++e) {
        const int t = S.sv_tri[e];
        const int4 tr = S.tri[t];
        int o1, o2;
        if (tr.x == slot) { o1 = tr.y; o2 = tr.z; }
        else if (tr.y == slot) { o1 = tr.z; o2 = tr.x; }
        else { o1 = tr.x; o2 = tr.y; }
        const float3 e1 = xyz(X[o1]) - xv, e2 = xyz(X[o2]) - xv;
        const float3 cr = cross3(e1, e2);
        const float ang = atan2f(sqrtf(dot3(cr, cr)), dot3(e1, e2));
        acc = acc + xyz(S.tnorm[t]) * ang;
    }
    S.vnorm[v] = make_float4(acc.x, acc.y, acc.z, 0.f);
}

__global__ void k_grid_count(DevSurf S, const float4 *X, StepConsts K)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S.n_tri) return;
    const int4 tr = S.tri[t];
    const float3 g = (xyz(X[tr.x]) + xyz(X[tr.y]) + xyz(X[tr.z])) * (1.0f / 3.0f);
    const float inv_s = 1.0f / grid_cell_size(S, K);
    const unsigned h = cell_hash(cell_coord(g.x, inv_s), cell_coord(g.y, inv_s), cell_coord(g.z, inv_s), S.hmask);
    atomicAdd(&S.hcount[h], 1u);
}

__global__ void k_grid_fill(DevSurf S, const float4 *X, StepConsts K)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S.n_tri) return;
    const int4 tr = S.tri[t];
    const float3 g = (xyz(X[tr.x]) + xyz(X[tr.y]) + xyz(X[tr.z])) * (1.0f / 3.0f);
    const float inv_s = 1.0f / grid_cell_size(S, K);
    const unsigned h = cell_hash(cell_coord(g.x, inv_s), cell_coord(g.y, inv_s), cell_coord(g.z, inv_s), S.hmask);
    const unsigned pos = S.hstart[h] + atomicAdd(&S.hcount[h], 1u);
    S.hitems[pos] = make_int2(t, tr.w);
}

// Pseudonormal of the closest feature of triangle t.
__device__ __forceinline__ float3 feature_normal(const DevSurf &S, int t, int feature)
{
    const float3 nt = xyz(S.tnorm[t]);
    if (feature == 0) return nt;
    const int4 tr = S.tri[t];
    if (feature <= 3) {
        const int slot = feature == 1 ? tr.x : (feature == 2 ? tr.y : tr.z);
        const int v = S.svidx[slot];
        return xyz(S.vnorm[v]);
    }
    const int4 adj = S.tadj[t];
    const int o = feature == 4 ? adj.x : (feature == 5 ? adj.y : adj.z);
    return o >= 0 ? nt + xyz(S.tnorm[o]) : nt;
}

// Self-contact eligibility: no shared vertex, farther apart than the
// exclusion distance in the rest shape.
__device__ __forceinline__ bool self_vt_ok(const DevSurf &S, const StepConsts &K, int slot, int4 tr)
{
    if (tr.x == slot || tr.y == slot || tr.z == slot) return false;
    const float3 p = xyz(S.srest[slot]);
    const ClosestPt cp = closest_on_triangle(p, xyz(S.srest[tr.x]), xyz(S.srest[tr.y]), xyz(S.srest[tr.z]));
    const float3 d = p - cp.q;
    return sqrtf(dot3(d, d)) > K.self_excl;
}

__device__ __forceinline__ bool self_ee_ok(const DevSurf &S, const StepConsts &K, int4 A, int4 B)
{
    if (A.x == B.x || A.x == B.y || A.y == B.x || A.y == B.y) return false;
    const SegPt sp = seg_closest(xyz(S.srest[A.x]), xyz(S.srest[A.y]), xyz(S.srest[B.x]), xyz(S.srest[B.y]));
    return sqrtf(sp.d2) > K.self_excl;
}

// One surface vertex per group of kDetLanes lanes: lane l < 27 scans the
// bucket of neighbouring cell l, then the group reduces the (distance^2,
// triangle) minimum with shuffles; the group's first lane decides the contact.
constexpr int kDetLanes = 32;

__global__ __launch_bounds__(256) void k_detect(DevSurf S, const float4 *X, StepConsts K)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = gid / kDetLanes, lane = threadIdx.x & (kDetLanes - 1);
    const bool active = v < S.n_sv;
    int2 sv = make_int2(0, -1);
    float3 p = make_float3(0.f, 0.f, 0.f);
    float best_d2 = K.col_radius * K.col_radius;
    int best = -1;
    if (active) {
        sv = S.svert[v];
        p = xyz(X[sv.x]);
    }
    if (active && lane < 27) {
        const float inv_s = 1.0f / grid_cell_size(S, K);
        const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
        const unsigned h = cell_hash(cell_coord(p.x, inv_s) + dx, cell_coord(p.y, inv_s) + dy,
                                     cell_coord(p.z, inv_s) + dz, S.hmask);
        const unsigned e1 = S.hstart[h + 1];
        for (unsigned e = S.hstart[h]; e < e1; ++e) {
            const int2 item = S.hitems[e];
            const int t = item.x;
            if (item.y == sv.y && !(K.self_contact && self_vt_ok(S, K, sv.x, S.tri[t]))) continue;
            // every point of the triangle lies within R of its centroid; the
            // margin keeps rounding of the bound from deciding a tie
            const float4 sph = S.tsph[t];
            const float3 dc = p - make_float3(sph.x, sph.y, sph.z);
            const float lb = sqrtf(dot3(dc, dc)) - sph.w;
            if (lb > 0.f && lb * lb > 1.001f * best_d2) continue;
            const int4 tr = S.tri[t];
            const ClosestPt cp = closest_on_triangle(p, xyz(X[tr.x]), xyz(X[tr.y]), xyz(X[tr.z]));
            const float3 d = p - cp.q;
            const float d2 = dot3(d, d);
            if (d2 < best_d2 || (d2 == best_d2 && best >= 0 && t < best)) {
                best_d2 = d2;
                best = t;
            }
        }
    }
    // lexicographic minimum of (d2, t) over the group (t = -1: none found)
#pragma unroll
    for (int off = kDetLanes / 2; off > 0; off >>= 1) {
        const float od2 = __shfl_xor(best_d2, off, kDetLanes);
        const int ot = __shfl_xor(best, off, kDetLanes);
        if (ot >= 0 && (best < 0 || od2 < best_d2 || (od2 == best_d2 && ot < best))) {
            best_d2 = od2;
            best = ot;
        }
    }
    if (!active || lane != 0) return;
    int hit = -1;
    if (best >= 0) {
        const int4 tr = S.tri[best];
        const ClosestPt cp = closest_on_triangle(p, xyz(X[tr.x]), xyz(X[tr.y]), xyz(X[tr.z]));
        if (tr.w != sv.y) {
            const bool inside = dot3(p - cp.q, feature_normal(S, best, cp.feature)) < 0.f;
            if (sqrtf(best_d2) < K.delta || inside) hit = best;
        } else if (K.delta - dot3(p - cp.q, xyz(S.tnorm[best])) > 0.f) {
            hit = best;   // own mesh: the element's own activity test
        }
    }
    S.ctri[sv.x] = hit;
    if (hit >= 0) {
        const int4 tr = S.tri[hit];
        atomicAdd(&S.ccount[tr.x], 1u);
        atomicAdd(&S.ccount[tr.y], 1u);
        atomicAdd(&S.ccount[tr.z], 1u);
    }
}

__global__ void k_corner_fill(DevSurf S)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= S.n_sv) return;
    const int slot = S.svert[v].x;
    const int t = S.ctri[slot];
    if (t < 0) return;
    const int4 tr = S.tri[t];
    const int c[3] = {tr.x, tr.y, tr.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const unsigned pos = S.crow[c[k]] + atomicAdd(&S.ccount[c[k]], 1u);
        S.cent[pos] = slot;
    }
}

// Insertion sort of every corner row (rows are short: a handful of entries).
__global__ void k_corner_sort(DevSurf S, int n_verts)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_verts) return;
    const int b = (int)S.crow[p], e = (int)S.crow[p + 1];
    for (int i = b + 1; i < e; ++i) {
        const int key = S.cent[i];
        int j = i - 1;
        while (j >= b && S.cent[j] > key) {
            S.cent[j + 1] = S.cent[j];
            --j;
        }
        S.cent[j + 1] = key;
    }
}

// ---------------------------------------------------------- edge-edge --
// Midpoints and half lengths of the surface edges, and per block the largest
// half length (reduced into gparam[1]).
__global__ __launch_bounds__(256) void k_edge_prep(DevSurf S, const float4 *X)
{
    __shared__ float wmax[4];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    float R = 0.f;
    if (e < S.n_edge) {
        const int4 ed = S.edge[e];
        const float3 a = xyz(X[ed.x]), b = xyz(X[ed.y]);
        const float3 m = (a + b) * 0.5f, h = (b - a) * 0.5f;
        R = sqrtf(dot3(h, h));
        S.emid[e] = make_float4(m.x, m.y, m.z, R);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) R = fmaxf(R, __shfl_xor(R, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = R;
    __syncthreads();
    if (threadIdx.x == 0)
        S.egmax[blockIdx.x] = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
}

__device__ __forceinline__ float edge_cell_size(const DevSurf &S, const StepConsts &K)
{
    const float s = K.col_radius + 2.f * __uint_as_float(S.gparam[1]);
    return s > 0.f ? s : 1.f;
}

__global__ void k_egrid_count(DevSurf S, StepConsts K)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= S.n_edge) return;
    const float4 m = S.emid[e];
    const float inv_s = 1.0f / edge_cell_size(S, K);
    const unsigned h = cell_hash(cell_coord(m.x, inv_s), cell_coord(m.y, inv_s), cell_coord(m.z, inv_s), S.ehmask);
    atomicAdd(&S.ehcount[h], 1u);
}

__global__ void k_egrid_fill(DevSurf S, StepConsts K)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= S.n_edge) return;
    const float4 m = S.emid[e];
    const float inv_s = 1.0f / edge_cell_size(S, K);
    const unsigned h = cell_hash(cell_coord(m.x, inv_s), cell_coord(m.y, inv_s), cell_coord(m.z, inv_s), S.ehmask);
    const unsigned pos = S.ehstart[h] + atomicAdd(&S.ehcount[h], 1u);
    S.ehitems[pos] = make_int2(e, S.edge[e].z);
}

// One surface edge per group of kDetLanes lanes (as k_detect): the closest
// eligible edge within r, then the element tests on the group's first lane.
// A point of an edge lies within its half length of the midpoint, so a pair
// within r has midpoints within r + 2 L_max: the 27 cells hold them all.
__global__ __launch_bounds__(256) void k_detect_ee(DevSurf S, const float4 *X, const float4 *Xt,
                                                   StepConsts K)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int e1 = gid / kDetLanes, lane = threadIdx.x & (kDetLanes - 1);
    const bool active = e1 < S.n_edge;
    int4 A = make_int4(0, 0, -1, 0);
    float3 a0 = make_float3(0.f, 0.f, 0.f), a1 = a0;
    float4 m1 = make_float4(0.f, 0.f, 0.f, 0.f);
    float best_d2 = K.col_radius * K.col_radius;
    int best = -1;
    if (active) {
        A = S.edge[e1];
        a0 = xyz(X[A.x]);
        a1 = xyz(X[A.y]);
        m1 = S.emid[e1];
    }
    if (active && lane < 27) {
        const float inv_s = 1.0f / edge_cell_size(S, K);
        const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
        const unsigned h = cell_hash(cell_coord(m1.x, inv_s) + dx, cell_coord(m1.y, inv_s) + dy,
                                     cell_coord(m1.z, inv_s) + dz, S.ehmask);
        const unsigned c1 = S.ehstart[h + 1];
        for (unsigned c = S.ehstart[h]; c < c1; ++c) {
            const int2 item = S.ehitems[c];
            const int e2 = item.x;
            if (e2 == e1) continue;
            const int4 B = S.edge[e2];
            if (item.y == A.z && !(K.self_contact && self_ee_ok(S, K, A, B))) continue;
            const float4 m2 = S.emid[e2];
            const float3 dm = make_float3(m1.x - m2.x, m1.y - m2.y, m1.z - m2.z);
            const float lb = sqrtf(dot3(dm, dm)) - m1.w - m2.w;
            if (lb > 0.f && lb * lb > 1.001f * best_d2) continue;
            const SegPt sp = seg_closest(a0, a1, xyz(X[B.x]), xyz(X[B.y]));
            if (sp.d2 < best_d2 || (sp.d2 == best_d2 && best >= 0 && e2 < best)) {
                best_d2 = sp.d2;
                best = e2;
            }
        }
    }
#pragma unroll
    for (int off = kDetLanes / 2; off > 0; off >>= 1) {
        const float od2 = __shfl_xor(best_d2, off, kDetLanes);
        const int oe = __shfl_xor(best, off, kDetLanes);
        if (oe >= 0 && (best < 0 || od2 < best_d2 || (od2 == best_d2 && oe < best))) {
            best_d2 = od2;
            best = oe;
        }
    }
    if (!active || lane != 0) return;
    int keep = -1;
    float3 n = make_float3(0.f, 0.f, 0.f);
    if (best >= 0) {
        const int4 B = S.edge[best];
        const float3 b0 = xyz(X[B.x]), b1 = xyz(X[B.y]);
        const SegPt sp = seg_closest(a0, a1, b0, b1);
        const float3 d1 = a1 - a0, d2 = b1 - b0;
        const float3 cr = cross3(d1, d2);
        const bool interior = sp.s > 0.f && sp.s < 1.f && sp.u > 0.f && sp.u < 1.f;
        const bool crossing = sqrtf(dot3(cr, cr)) >= 0.1f * sqrtf(dot3(d1, d1)) * sqrtf(dot3(d2, d2));
        const float3 ta0 = xyz(Xt[A.x]), ta1 = xyz(Xt[A.y]), tb0 = xyz(Xt[B.x]), tb1 = xyz(Xt[B.y]);
        const float3 w = (ta0 + (ta1 - ta0) * sp.s) - (tb0 + (tb1 - tb0) * sp.u);
        const float wl = sqrtf(dot3(w, w));
        if (interior && crossing && wl > 0.f) {
            n = w * (1.0f / wl);
            const float3 xa = a0 + d1 * sp.s, xb = b0 + d2 * sp.u;
            if (K.delta - dot3(xa - xb, n) > 0.f) keep = best;
        }
    }
    S.eb[e1] = keep;
    S.en[e1] = make_float4(n.x, n.y, n.z, 0.f);
}

// A pair found from both of its edges is kept from the lower index.
__device__ __forceinline__ bool ee_kept(const DevSurf &S, int e1)
{
    const int e2 = S.eb[e1];
    return e2 >= 0 && !(S.eb[e2] == e1 && e2 < e1);
}

__global__ void k_ee_count(DevSurf S)
{
    const int e1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (e1 >= S.n_edge || !ee_kept(S, e1)) return;
    const int4 A = S.edge[e1], B = S.edge[S.eb[e1]];
    atomicAdd(&S.ecount[A.x], 1u);
    atomicAdd(&S.ecount[A.y], 1u);
    atomicAdd(&S.ecount[B.x], 1u);
    atomicAdd(&S.ecount[B.y], 1u);
}

__global__ void k_ee_fill(DevSurf S)
{
    const int e1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (e1 >= S.n_edge || !ee_kept(S, e1)) return;
    const int4 A = S.edge[e1], B = S.edge[S.eb[e1]];
    const int v[4] = {A.x, A.y, B.x, B.y};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const unsigned pos = S.erow[v[k]] + atomicAdd(&S.ecount[v[k]], 1u);
        S.eent[pos] = e1;
    }
}

// Insertion sort of every element row (a handful of entries each).
__global__ void k_ee_sort(DevSurf S, int n_verts)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_verts) return;
    const int b = (int)S.erow[p], e = (int)S.erow[p + 1];
    for (int i = b + 1; i < e; ++i) {
        const int key = S.eent[i];
        int j = i - 1;
        while (j >= b && S.eent[j] > key) {
            S.eent[j + 1] = S.eent[j];
            --j;
        }
        S.eent[j + 1] = key;
    }
}

__global__ void k_store_partners(DevSurf S, int *out)
{
    const int e1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (e1 >= S.n_edge) return;
    out[e1] = ee_kept(S, e1) ? S.eb[e1] : -1;
}

__global__ void k_load_x(DevTopo T, const float *x)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= T.n_verts) return;
    const float3 v = ld3(x, T.perm[p]);
    T.x[p] = make_float4(v.x, v.y, v.z, 0.f);
}

__global__ void k_store_ctri(DevTopo T, DevSurf S, int *out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= T.n_verts) return;
    out[T.perm[p]] = S.ctri ? S.ctri[p] : -1;
}

// -------------------------------------------------------------- launchers --
hipError_t launch_detect(const DevTopo &T, const DevSurf &S, const float4 *X, const StepConsts &K,
                         hipStream_t s)
{
    if (S.n_tri == 0 || S.n_sv == 0) return hipSuccess;
    const int H = S.hmask + 1;
    hipError_t e;
    if ((e = fill_u32(S.hcount, H, 0u, s)) != hipSuccess) return e;
    if ((e = fill_u32(S.ccount, T.n_verts, 0u, s)) != hipSuccess) return e;
    const int nb_tri = cdiv(S.n_tri, 256);
    hipLaunchKernelGGL(k_tri_prep, dim3(nb_tri), dim3(256), 0, s, S, X);
    hipLaunchKernelGGL(k_max_radius, dim3(1), dim3(256), 0, s, S.gmax, nb_tri, S.gparam);
    hipLaunchKernelGGL(k_vert_normals, dim3(cdiv(S.n_sv, 256)), dim3(256), 0, s, S, X);
    hipLaunchKernelGGL(k_grid_count, dim3(cdiv(S.n_tri, 256)), dim3(256), 0, s, S, X, K);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(S.hcount, S.hstart, S.scan_tmp, H, s)) != hipSuccess) return e;
    if ((e = fill_u32(S.hcount, H, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_grid_fill, dim3(cdiv(S.n_tri, 256)), dim3(256), 0, s, S, X, K);
    hipLaunchKernelGGL(k_detect, dim3(cdiv((long)S.n_sv * kDetLanes, 256)), dim3(256), 0, s, S, X, K);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(S.ccount, S.crow, S.scan_tmp, T.n_verts, s)) != hipSuccess) return e;
    if ((e = fill_u32(S.ccount, T.n_verts, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_corner_fill, dim3(cdiv(S.n_sv, 256)), dim3(256), 0, s, S);
    hipLaunchKernelGGL(k_corner_sort, dim3(cdiv(T.n_verts, 256)), dim3(256), 0, s, S, T.n_verts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!K.edge_contacts || S.n_edge == 0) return hipSuccess;
    // edge-edge elements, normals from x^t
    const int HE = S.ehmask + 1;
    const int nb_e = cdiv(S.n_edge, 256);
    if ((e = fill_u32(S.ehcount, HE, 0u, s)) != hipSuccess) return e;
    if ((e = fill_u32(S.ecount, T.n_verts, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_prep, dim3(nb_e), dim3(256), 0, s, S, X);
    hipLaunchKernelGGL(k_max_radius, dim3(1), dim3(256), 0, s, S.egmax, nb_e, S.gparam + 1);
    hipLaunchKernelGGL(k_egrid_count, dim3(nb_e), dim3(256), 0, s, S, K);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(S.ehcount, S.ehstart, S.scan_tmp, HE, s)) != hipSuccess) return e;
    if ((e = fill_u32(S.ehcount, HE, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_egrid_fill, dim3(nb_e), dim3(256), 0, s, S, K);
    hipLaunchKernelGGL(k_detect_ee, dim3(cdiv((long)S.n_edge * kDetLanes, 256)), dim3(256), 0, s, S, X,
                       (const float4 *)T.xt, K);
    hipLaunchKernelGGL(k_ee_count, dim3(nb_e), dim3(256), 0, s, S);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(S.ecount, S.erow, S.scan_tmp, T.n_verts, s)) != hipSuccess) return e;
    if ((e = fill_u32(S.ecount, T.n_verts, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ee_fill, dim3(nb_e), dim3(256), 0, s, S);
    hipLaunchKernelGGL(k_ee_sort, dim3(cdiv(T.n_verts, 256)), dim3(256), 0, s, S, T.n_verts);
    return hipGetLastError();
}

hipError_t launch_store_edge_partners(const DevSurf &S, int *partner_out, hipStream_t s)
{
    if (S.n_edge == 0) return hipSuccess;
    hipLaunchKernelGGL(k_store_partners, dim3(cdiv(S.n_edge, 256)), dim3(256), 0, s, S, partner_out);
    return hipGetLastError();
}

hipError_t launch_load_x(const DevTopo &T, const float *x, hipStream_t s)
{
    if (T.n_verts == 0) return hipSuccess;
    hipLaunchKernelGGL(k_load_x, dim3(cdiv(T.n_verts, 256)), dim3(256), 0, s, T, x);
    return hipGetLastError();
}

hipError_t launch_store_ctri(const DevTopo &T, const DevSurf &S, int *out, hipStream_t s)
{
    if (T.n_verts == 0) return hipSuccess;
    hipLaunchKernelGGL(k_store_ctri, dim3(cdiv(T.n_verts, 256)), dim3(256), 0, s, T, S, out);
    return hipGetLastError();
}

}  // namespace vbd
