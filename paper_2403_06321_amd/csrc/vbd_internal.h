// Internal declarations shared by the host orchestration (vbd_host.cpp) and
// the gfx950 kernels (vbd_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace vbd {

static_assert(sizeof(float3) == 12, "float3 cells must be 12 bytes");

// Incidence entry of a (vertex, tet) pair, 16 bytes:
//   x = (stored tet << 2) | slot of the vertex in the tet,
//   y, z, w = permuted ids of the tet's other three vertices in slot order.
// The record and the three neighbour positions depend only on this entry,
// so their loads are issued together.
using PairEnt = int4;

constexpr int kMaxObstacles = 8;

// Entries of the device flag array (DevTopo::flags, kFlagWords x 32 bit):
//   0 barrier arrivals, 1 barrier abort, 3..5 abort diagnostics (arrivals
//   seen, target, grid), kFlagNonfinite / kFlagNonfiniteTotal non-finite
//   output values since the last vbd_check / counter reset, kFlagSkips a
//   64-bit count of determinant-rule skips (8-byte aligned).
constexpr int kFlagNonfinite = 6;
constexpr int kFlagNonfiniteTotal = 7;
constexpr int kFlagSkips = 8;
// The persistent kernel's barrier counters from kFlagBar on, one 128-B line
// each: kBarGroups group counters (one per XCD, by the XCD a block runs on),
// then the global one; then the start-of-launch census: the number of blocks
// on each XCD (one line) and the number counted (one line).
constexpr int kFlagBar = 64;
constexpr int kBarGroups = 8;
constexpr int kBarStride = 32;   // 32 x 4 B = 128 B
constexpr int kFlagCensus = kFlagBar + (kBarGroups + 1) * kBarStride;
constexpr int kFlagCensusTotal = kFlagCensus + kBarStride;
constexpr int kFlagWords = kFlagCensusTotal + kBarStride;
// Waves per SIMD that the persistent grid fills: every persistent kernel is
// compiled for at least this occupancy (amdgpu_waves_per_eu), so the grid is
// resident by construction (a CPU test reads the compiler's occupancy).
constexpr int kPersistentWavesPerSimd = 4;

// Per-step constants passed by value to every kernel.
struct StepConsts {
    float h, inv_h;
    float gx, gy, gz, gnorm;       // external acceleration and its norm
    int init_mode;
    float det_eps_rel;
    float kc, delta;               // penalty stiffness and contact distance
    float kd_over_h;               // Rayleigh damping k_d / h
    float fric_mu, fric_hev;       // friction coefficient and h * eps_v
    float cheb_rho;
    float alpha;                   // 1 + mu/lambda (depends on nu only)
    float k_mu, k_lam;             // mu / E and lambda / E
    float spring_k;
    int spring_psd;
    int n_spheres, n_planes;
    float4 spheres[kMaxObstacles]; // cx, cy, cz, R
    float4 planes[kMaxObstacles];  // unit normal, offset
    float col_radius;              // mesh-mesh detection radius
    int self_contact;              // pairs within one mesh (rest distance > self_excl)
    float self_excl;
    int edge_contacts;             // edge-edge elements
};

// Device-side view of a bound workspace.
struct DevTopo {
    const float *vol;                  // [n_tets] rest volume, in stored order (tet_perm)
    const int *tet_perm;               // stored tet -> caller's tet index
    const int *tet_row;                // CSR over all permuted vertices (adjoint)
    const PairEnt *tet_ent;            // (tet, slot, other vertices) per entry
    // Per-color padded incidence: every free vertex of color c owns
    // ell_info[c].y consecutive entries starting at ell_info[c].x +
    // (slot - color_off[c]) * ell_info[c].y, so entry addresses follow from the
    // slot alone.  Two views of each (vertex, tet) pair:
    //   ell                 (tet, slot, other vertices) entries (adjoint), padding x = -1;
    //   pa / pw / pb        the color solve's pair records, from the rest
    //                       frame S = R^{-1} of the tet's rest edges taken from
    //                       this vertex (D_m' = Q R, Q proper; F' = D_s' S is
    //                       F times a rotation), this vertex's shape gradient
    //                       m = -(rows of S summed), w = S m (so that
    //                       w0 + w1 + w2 = -|m|^2) and sigma = det S:
    //                       pa = {the other three vertices (ascending slot), float
    //                       bits of V lam}, pw = {V mu w, last}, pb = sigma, in
    //                       two layouts: compact (32 B: last = sigma, pb not
    //                       read, V mu |m|^2 summed from w) or full (36 B:
    //                       last = V mu |m|^2); padding entries name the
    //                       vertex itself as all three others, with V lam = 0
    //                       and pw = 0 (written by the material kernel);
    //   pws                 {w, sigma}, the E-free record (material input).
    const PairEnt *ell;
    int4 *pa;
    float4 *pw;
    const float *pb;
    const float4 *pws;
    const int *pair_tet;               // stored tet of each pair entry (-1: padding)
    const int2 *ell_info;              // [n_colors] {first entry, padded degree}
    long long n_pairs;                 // padded entries over all colors
    // springs of every free vertex in the same per-color padded layout:
    // spr_info[c] = {first entry, padded degree}; entries {neighbour slot,
    // float bits of rest length}, padding x = -1
    const int2 *spr_ell;
    const int2 *spr_info;
    const int *perm;                   // permuted slot -> original id
    const float *mass;                 // permuted
    const int *color_off;              // [n_colors + 1]
    float4 *x, *xt, *y;                // current iterate, x^t, inertia target (w = m/h^2)
    float4 *xnext;                     // recording the iterates: each update is also stored
                                       // here (the next iterate's snapshot); else null
    float4 *prev1, *prev2;             // Chebyshev history
    unsigned char *collided;           // sticky contact flag within a step
    unsigned *flags;                   // see kFlag* above
    float4 *snaps;                     // backward: (n_iters + 1) iterates
    float4 *xbar, *ybar, *xtbar, *vbar;
    float3 *contrib;                   // backward: [n_tets][4] pending adjoints of pinned
                                       // vertices (12 B), by (stored tet, slot)
    // backward, per padded pair entry of a receiving vertex: its three incoming
    // contribution cells (cin + j * n_pairs holds the one from the j-th other
    // vertex of the tet in the pair record's order, ascending permuted slot and
    // so ascending color: with a tet's vertices in distinct colors, one color
    // phase writes the cells of one array per receiving color), the targets of
    // its own outgoing contributions ((entry << 2) | j of each other vertex in
    // that order, or -1 - (stored tet * 4 + slot) for a pinned vertex) and its
    // share of Ebar
    float3 *cin;
    const int3 *tgt;
    float *ebar_pair;
    const int4 *tet_pairs;             // [n_tets] stored order: entry of each slot or -1
    int n_verts, n_tets, n_free, n_colors;
};

// Surface of a batched topology and the mesh-mesh contact state (present
// when the topology has more than one mesh).
struct DevSurf {
    const int4 *tri;       // [n_tri] {a, b, c, mesh}, permuted ids, (b-a)x(c-a) outward
    const int4 *tadj;      // [n_tri] triangle across edge (a,b), (b,c), (c,a) or -1
    const int2 *svert;     // [n_sv] {permuted slot, mesh}
    const int *svidx;      // [n_verts] permuted slot -> surface vertex index or -1
    const int *sv_row;     // [n_sv + 1] incident surface triangles of a surface vertex
    const int *sv_tri;
    float4 *tnorm;         // [n_tri] unit normal
    float4 *vnorm;         // [n_sv] angle-weighted pseudonormal
    unsigned *gparam;      // [4] {max centroid radius bits, ...}
    float *gmax;           // [ceil(n_tri / 256)] per-block maximum radius
    unsigned *hcount;      // [H] bucket sizes, then fill cursors
    unsigned *hstart;      // [H + 1]
    unsigned *scan_tmp;    // [n_scan_blocks + 1]
    int2 *hitems;          // [n_tri] {triangle, its mesh} grouped by bucket
    float4 *tsph;          // [n_tri] centroid and centroid-to-corner radius
    int *ctri;             // [n_verts] contact triangle of a permuted slot or -1
    unsigned *ccount;      // [n_verts] corner entries per slot, then fill cursors
    unsigned *crow;        // [n_verts + 1]
    int *cent;             // [3 n_sv] colliding vertex of each corner entry
    float4 *xsnap;         // [n_verts] positions of each color as of the start of its
                           // phase (read for same-color contact partners)
    const float4 *srest;   // [n_verts] rest positions (self-contact exclusion)
    // edge-edge elements
    const int4 *edge;      // [n_edge] {a, b, mesh, 0} permuted ids, ascending original (a, b)
    float4 *emid;          // [n_edge] midpoint and half length
    float *egmax;          // [ceil(n_edge / 256)] per-block maximum half length
    unsigned *ehcount;     // [HE] bucket sizes, then fill cursors
    unsigned *ehstart;     // [HE + 1]
    int2 *ehitems;         // [n_edge] {edge, its mesh} grouped by bucket
    int *eb;               // [n_edge] partner edge of the element found from this edge, or -1
    float4 *en;            // [n_edge] the element's fixed normal
    unsigned *ecount;      // [n_verts] element entries per slot, then fill cursors
    unsigned *erow;        // [n_verts + 1]
    int *eent;             // [4 n_edge] kept elements (their first edge) of each slot, ascending
    int n_tri, n_sv, hmask, n_edge, ehmask;
};

// One color's vertex range split into 8 contiguous parts at mesh boundaries
// (launch mapping 3: part k runs on XCD k): dev = the 9 boundaries (device),
// max_size = the largest part in vertices.  dev == nullptr: no split.
struct XcdSplit {
    const int *dev;
    int max_size;
};

struct LaunchCfg {
    int lanes;        // lanes per vertex
    int block;        // threads per block (<= 512)
    int xcd_remap;    // 0 as launched, 1 contiguous ranges, 2 16-block chunks in turn,
                      // 3 contiguous ranges split at mesh boundaries (XcdSplit)
    int blocks_per_cu;
    int unroll;       // tet entries per lane whose loads are issued together (1..3)
    int compact;      // 1: 32-B pair records (see DevTopo), 0: 36-B
};

// ---- kernel launchers (vbd_kernels.hip) ----
// The E-dependent parts of the pair records (V lam, V mu w).
hipError_t launch_material(const DevTopo &T, const float *tet_E, const StepConsts &K, bool compact,
                           hipStream_t s);
hipError_t launch_predict(const DevTopo &T, const float *x, const float *v, const float *vp,
                          const StepConsts &K, bool reset_flags, hipStream_t s);
// inc: {first tet entry, padded tet degree, first spring entry, padded spring
// degree} of the color (DevTopo::ell_info, DevTopo::spr_info).
hipError_t launch_solve(const DevTopo &T, const StepConsts &K, int v_begin, int v_end, int4 inc,
                        bool tets, bool springs, const LaunchCfg &cfg, hipStream_t s,
                        XcdSplit xs = XcdSplit{nullptr, 0});
// Color solve with mesh-mesh contact elements.  Updates T.x in place; contact
// partners of the same color are read from S.xsnap (their positions before
// the phase).  [prev_begin, prev_end): the previously solved color, whose
// snapshot the kernel refreshes from T.x.
hipError_t launch_solve_contacts(const DevTopo &T, const DevSurf &S, const StepConsts &K,
                                 int v_begin, int v_end, int4 inc, int prev_begin, int prev_end,
                                 bool tets, bool springs, const LaunchCfg &cfg, hipStream_t s,
                                 XcdSplit xs = XcdSplit{nullptr, 0});
// Detection on the permuted positions X (T.xt or T.x) into S.ctri and the
// corner CSR (S.crow, S.cent).
hipError_t launch_detect(const DevTopo &T, const DevSurf &S, const float4 *X,
                         const StepConsts &K, hipStream_t s);
// Edge partners of the kept elements (S.eb filtered) -> partner_out.
hipError_t launch_store_edge_partners(const DevSurf &S, int *partner_out, hipStream_t s);
// x (original order) -> T.x, and S.ctri -> tri_out (original order, or -1).
hipError_t launch_load_x(const DevTopo &T, const float *x, hipStream_t s);
hipError_t launch_store_ctri(const DevTopo &T, const DevSurf &S, int *tri_out, hipStream_t s);
// snap: when not null, also receives the accelerated positions.
hipError_t launch_cheb(const DevTopo &T, const StepConsts &K, int iter, hipStream_t s,
                       float4 *snap = nullptr);
hipError_t launch_finalize(const DevTopo &T, float *x, float *v, float *vp,
                           const StepConsts &K, hipStream_t s);
// Persistent kernel over all iterations and colors.  grid = 0 -> occupancy
// limited.  cooperative: launch through hipLaunchCooperativeKernel.
hipError_t launch_persistent(const DevTopo &T, const StepConsts &K, int n_iters, bool tets,
                             bool springs, const LaunchCfg &cfg, int n_cu, bool cooperative,
                             hipStream_t s, int *grid_out);
hipError_t launch_copy4(float4 *dst, const float4 *src, int n, hipStream_t s);
// Read-only streaming probe: `blocks` blocks of 256 threads sum src[0..n) and
// write one partial sum per block into out[0..blocks).
hipError_t launch_read4(const float4 *src, long long n, float *out, int blocks, hipStream_t s);
hipError_t launch_zero_u32(unsigned *p, long long n, hipStream_t s);
// Non-finite values among a[0..n) and b[0..n) into the flag counters.
hipError_t launch_check_finite(const float *a, const float *b, long long n, unsigned *flags,
                               hipStream_t s);

// backward
hipError_t launch_bwd_init(const DevTopo &T, const float *gx_out, const float *gv_out,
                           const float *gvp_out, const StepConsts &K, hipStream_t s);
hipError_t launch_adjoint_color(const DevTopo &T, const StepConsts &K, const float4 *Sn,
                                const float4 *Sp, int v_begin, int v_end, int2 ell,
                                const LaunchCfg &cfg, hipStream_t s);
hipError_t launch_seed_snapshots(const DevTopo &T, int n_iters, hipStream_t s);
hipError_t launch_bwd_fold(const DevTopo &T, hipStream_t s);
// Also adds the per-pair Ebar shares into g_tet_E (caller's tet order).
hipError_t launch_bwd_final(const DevTopo &T, const float *v_t, const float *v_prev,
                            float *gx_in, float *gv_in, float *gvp_in, float *g_tet_E,
                            const StepConsts &K, hipStream_t s);

}  // namespace vbd
