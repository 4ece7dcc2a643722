// Host side of the VBD library: C ABI, topology preprocessing (FP64 rest
// data, greedy or given coloring, color-sorted incidence, per-color padded
// pair records, mesh surfaces), workspace layout, step orchestration (plain /
// hipGraph / persistent, mesh-contact detection), backward, autotuner and
// profiling.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/vbd.h"
#include "vbd_internal.h"
#include "vbd_static.h"

using namespace vbd;

namespace {

thread_local std::string g_err;

// A named host-side range for tools that trace ROCTx markers (rocprofv3
// --marker-trace): the entry points below open one for their whole call, and
// a step's plain launch sequence one per iteration and per color phase, so a
// trace shows which call, iteration and phase enqueued which kernels.
struct Range {
    explicit Range(const char *name, bool on = true) : on_(on)
    {
        if (on_) roctxRangePushA(name);
    }
    ~Range()
    {
        if (on_) roctxRangePop();
    }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;

private:
    bool on_;
};

vbd_status fail(vbd_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(VBD_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                        __FILE__, __LINE__);                                                   \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t vol, tet_perm, tet_row, tet_ent, ell, pa, pw, pb, pws, pair_tet, ell_info, spr_ell,
        spr_info, perm, mass, color_off, xsplit;
    size_t x, xt, y, prev1, prev2, collided, flags;
    size_t snaps, xbar, ybar, xtbar, vbar, contrib, cin, tgt, ebar_pair, tet_pairs;
    // mesh-mesh contacts (only when the topology has a surface)
    size_t s_tri, s_tadj, s_svert, s_svidx, s_sv_row, s_sv_tri, s_tnorm, s_vnorm, s_gparam, s_gmax;
    size_t s_hcount, s_hstart, s_scan, s_hitems, s_tsph, s_ctri, s_ccount, s_crow, s_cent, s_xsnap;
    size_t s_rest, s_edge, s_emid, s_egmax, s_ehcount, s_ehstart, s_ehitems, s_eb, s_en, s_ecount,
        s_erow, s_eent;
    int hsize, ehsize;
    size_t total;
    int max_bwd_iters;
};

struct GraphKey {
    std::vector<const void *> ptrs;
    void *stream;
    std::vector<uint32_t> params;
    bool operator==(const GraphKey &o) const
    {
        return ptrs == o.ptrs && stream == o.stream && params == o.params;
    }
};

// One captured launch sequence, replayed while its key (device pointers,
// parameters, stream) is unchanged.
struct GraphCache {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GraphKey key{};
    bool have = false;
    void reset()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        have = false;
    }
};

struct ProfileEvent {
    hipEvent_t a, b;
    double bytes;       // algorithmic bytes of the launches inside [a, b]
    int64_t updates;    // vertex updates inside [a, b]
    int64_t launches;   // hot-kernel launches inside [a, b]
};

}  // namespace

struct vbd_topology_s {
    // description
    int nv = 0, nt = 0, ns = 0, n_meshes = 1;
    std::vector<int64_t> vert_off, tet_off;
    std::vector<int32_t> tets, springs;
    std::vector<double> rest, spring_L, mass, Dminv, vol;
    std::vector<uint8_t> pinned;
    double nu = 0.3, spring_k = 0.0;
    // coloring and CSR
    bool colored = false;
    int color_order = -1;               // VBD_COLOR_* of the greedy coloring, -1: given
    int n_colors = 0, n_free = 0;
    std::vector<int32_t> colors, perm, iperm, color_off;
    std::vector<int32_t> tet_row, tet_ent, spr_row, spr_nbr_orig;
    std::vector<int32_t> tet_order, tet_rank;   // stored position <-> caller's tet id
    std::vector<int2> ell_info;                 // per color {first entry, padded degree}
    size_t ell_total = 0;
    std::vector<int2> spr_info;                 // the same for springs
    size_t spr_total = 0;
    std::vector<float> spr_len;
    std::vector<double> phase_bytes;            // for the current launch configuration
    std::vector<double> adj_phase_bytes;        // one reverse color phase (vbd_step_backward)
    std::vector<std::array<int64_t, 3>> phase_cnt;  // per color: pairs, spring entries,
                                                    // distinct neighbours
    std::vector<int64_t> phase_updates;
    // surface (extracted by vbd_color when there is more than one mesh)
    std::vector<int32_t> surf;          // [n_tri][3] original ids, outward
    std::vector<int32_t> surf_adj;      // [n_tri][3] triangle across edge k or -1
    std::vector<int32_t> vert_mesh;     // [nv]
    std::vector<int32_t> sv_slot;       // surface vertices as permuted slots, ascending
    std::vector<int32_t> sv_row, sv_tri;
    std::vector<int32_t> sedge;         // [n_edge][2] surface edges, a < b (original ids), ascending
    std::vector<int32_t> xsplit;        // [n_colors][9] mesh-aligned XCD parts of each color
    std::vector<int32_t> xsplit_max;    // [n_colors] largest part (vertices)
    DevSurf surf_dev{};
    // device
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Layout lay{};
    bool bound = false;
    DevTopo dev{};
    int device = -1;                    // current device at vbd_bind_workspace
    int n_cu = 0;
    std::string arch;
    LaunchCfg cfg{8, 128, 1, 0, 2, 0};
    // graph caches of vbd_step and vbd_step_backward
    hipStream_t cap_stream = nullptr;   // library-owned stream used only for capture
    GraphCache fwd_graph, bwd_graph, rec_graph;
    // profiling
    bool profiling = false;
    // the reverse sweep's accumulators (contribution cells, pinned cells,
    // Ebar shares) are zero: after binding and after every enqueued backward,
    // whose last two kernels clear what they read
    bool bwd_zero = false;
    std::vector<ProfileEvent> events;
    vbd_profile_stats acc{};
    ~vbd_topology_s()
    {
        fwd_graph.reset();
        bwd_graph.reset();
        rec_graph.reset();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (auto &e : events) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    }
};

namespace {

// Algorithmic bytes of one color solve under the current launch
// configuration: per tet pair the 32-B compact or 36-B full record, 8 B per
// spring entry, 48 B own state per vertex (x read, y read, x write), 16 B per
// distinct neighbour position.
void update_phase_bytes(vbd_topology_s &T)
{
    const double rec = T.cfg.compact ? 32.0 : 36.0;
    T.phase_bytes.assign(T.phase_cnt.size(), 0.0);
    T.adj_phase_bytes.assign(T.phase_cnt.size(), 0.0);
    for (size_t c = 0; c < T.phase_cnt.size(); ++c) {
        const auto &n = T.phase_cnt[c];
        T.phase_bytes[c] = rec * (double)n[0] + 8.0 * (double)n[1] + 48.0 * (double)T.phase_updates[c] +
                           16.0 * (double)n[2];
        // reverse phase: per tet pair the 16-B pair record, the 16-B E-free
        // record, the 12-B targets, its three 12-B incoming cells read, three
        // 12-B outgoing cells written and its Ebar share read and written; per
        // vertex its snapshot, xbar and ybar read and written and y read
        // (96 B); 16 B per distinct neighbour position
        T.adj_phase_bytes[c] = (16.0 + 16.0 + 12.0 + 36.0 + 36.0 + 8.0) * (double)n[0] +
                               96.0 * (double)T.phase_updates[c] + 16.0 * (double)n[2];
    }
}

// ----------------------------------------------------------------- layout --
Layout make_layout(const vbd_topology_s &T, int max_bwd_iters)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes ? bytes : 1); return o; };
    const size_t nv = (size_t)T.nv;
    L.vol = take(sizeof(float) * (size_t)T.nt);
    L.tet_perm = take(sizeof(int32_t) * (size_t)T.nt);
    L.tet_row = take(sizeof(int32_t) * (size_t)(T.nv + 1));
    L.tet_ent = take(sizeof(PairEnt) * T.tet_ent.size());
    L.ell = take(sizeof(PairEnt) * T.ell_total);
    L.pa = take(sizeof(int4) * T.ell_total);
    L.pw = take(sizeof(float4) * T.ell_total);
    L.pb = take(sizeof(float) * T.ell_total);
    L.pws = take(sizeof(float4) * T.ell_total);
    L.pair_tet = take(sizeof(int32_t) * T.ell_total);
    L.ell_info = take(sizeof(int2) * (size_t)T.n_colors);
    L.spr_ell = take(sizeof(int2) * T.spr_total);
    L.spr_info = take(sizeof(int2) * (size_t)T.n_colors);
    L.perm = take(sizeof(int32_t) * nv);
    L.mass = take(sizeof(float) * nv);
    L.color_off = take(sizeof(int32_t) * (size_t)(T.n_colors + 1));
    L.xsplit = take(sizeof(int32_t) * 9 * (size_t)T.n_colors);
    L.x = take(sizeof(float4) * nv);
    L.xt = take(sizeof(float4) * nv);
    L.y = take(sizeof(float4) * nv);
    L.prev1 = take(sizeof(float4) * nv);
    L.prev2 = take(sizeof(float4) * nv);
    L.collided = take(nv);
    L.flags = take(sizeof(uint32_t) * kFlagWords);
    L.max_bwd_iters = max_bwd_iters;
    if (max_bwd_iters > 0) {
        L.snaps = take(sizeof(float4) * nv * (size_t)(max_bwd_iters + 1));
        L.xbar = take(sizeof(float4) * nv);
        L.ybar = take(sizeof(float4) * nv);
        L.xtbar = take(sizeof(float4) * nv);
        L.vbar = take(sizeof(float4) * nv);
        L.contrib = take(sizeof(float3) * 4 * (size_t)T.nt);
        L.cin = take(sizeof(float3) * 3 * T.ell_total);
        L.tgt = take(sizeof(int3) * T.ell_total);
        L.ebar_pair = take(sizeof(float) * T.ell_total);
        L.tet_pairs = take(sizeof(int4) * (size_t)T.nt);
    }
    const size_t ntri = T.surf.size() / 3, nsv = T.sv_slot.size();
    if (ntri > 0) {
        int H = 1024;
        while ((size_t)H < 2 * ntri) H <<= 1;
        L.hsize = H;
        L.s_tri = take(sizeof(int4) * ntri);
        L.s_tadj = take(sizeof(int4) * ntri);
        L.s_svert = take(sizeof(int2) * nsv);
        L.s_svidx = take(sizeof(int32_t) * nv);
        L.s_sv_row = take(sizeof(int32_t) * (nsv + 1));
        L.s_sv_tri = take(sizeof(int32_t) * T.sv_tri.size());
        L.s_tnorm = take(sizeof(float4) * ntri);
        L.s_vnorm = take(sizeof(float4) * nsv);
        L.s_gparam = take(sizeof(uint32_t) * 4);
        L.s_gmax = take(sizeof(float) * (ntri / 256 + 1));
        L.s_hcount = take(sizeof(uint32_t) * (size_t)H);
        L.s_hstart = take(sizeof(uint32_t) * ((size_t)H + 1));
        const size_t ne = T.sedge.size() / 2;
        int HE = 1024;
        while ((size_t)HE < 2 * ne) HE <<= 1;
        L.ehsize = HE;
        const size_t big = std::max<size_t>(std::max<size_t>((size_t)H, (size_t)HE), nv + 1);
        L.s_scan = take(sizeof(uint32_t) * (big / 2048 + 2));
        L.s_hitems = take(sizeof(int2) * ntri);
        L.s_tsph = take(sizeof(float4) * ntri);
        L.s_ctri = take(sizeof(int32_t) * nv);
        L.s_ccount = take(sizeof(uint32_t) * nv);
        L.s_crow = take(sizeof(uint32_t) * (nv + 1));
        L.s_cent = take(sizeof(int32_t) * 3 * nsv);
        L.s_xsnap = take(sizeof(float4) * nv);
        L.s_rest = take(sizeof(float4) * nv);
        L.s_edge = take(sizeof(int4) * ne);
        L.s_emid = take(sizeof(float4) * ne);
        L.s_egmax = take(sizeof(float) * (ne / 256 + 1));
        L.s_ehcount = take(sizeof(uint32_t) * (size_t)HE);
        L.s_ehstart = take(sizeof(uint32_t) * ((size_t)HE + 1));
        L.s_ehitems = take(sizeof(int2) * ne);
        L.s_eb = take(sizeof(int32_t) * ne);
        L.s_en = take(sizeof(float4) * ne);
        L.s_ecount = take(sizeof(uint32_t) * nv);
        L.s_erow = take(sizeof(uint32_t) * (nv + 1));
        L.s_eent = take(sizeof(int32_t) * 4 * ne);
    }
    L.total = off;
    return L;
}

void set_dev_pointers(vbd_topology_s &T)
{
    char *b = T.ws;
    const Layout &L = T.lay;
    DevTopo &D = T.dev;
    D.vol = (const float *)(b + L.vol);
    D.tet_perm = (const int *)(b + L.tet_perm);
    D.tet_row = (const int *)(b + L.tet_row);
    D.tet_ent = (const PairEnt *)(b + L.tet_ent);
    D.ell = (const PairEnt *)(b + L.ell);
    D.pa = (int4 *)(b + L.pa);
    D.pw = (float4 *)(b + L.pw);
    D.pb = (const float *)(b + L.pb);
    D.pws = (const float4 *)(b + L.pws);
    D.pair_tet = (const int *)(b + L.pair_tet);
    D.n_pairs = (long long)T.ell_total;
    D.ell_info = (const int2 *)(b + L.ell_info);
    D.spr_ell = (const int2 *)(b + L.spr_ell);
    D.spr_info = (const int2 *)(b + L.spr_info);
    D.perm = (const int *)(b + L.perm);
    D.mass = (const float *)(b + L.mass);
    D.color_off = (const int *)(b + L.color_off);
    D.x = (float4 *)(b + L.x);
    D.xt = (float4 *)(b + L.xt);
    D.y = (float4 *)(b + L.y);
    D.prev1 = (float4 *)(b + L.prev1);
    D.prev2 = (float4 *)(b + L.prev2);
    D.collided = (unsigned char *)(b + L.collided);
    D.flags = (unsigned *)(b + L.flags);
    D.snaps = L.max_bwd_iters > 0 ? (float4 *)(b + L.snaps) : nullptr;
    D.xnext = nullptr;
    D.xbar = L.max_bwd_iters > 0 ? (float4 *)(b + L.xbar) : nullptr;
    D.ybar = L.max_bwd_iters > 0 ? (float4 *)(b + L.ybar) : nullptr;
    D.xtbar = L.max_bwd_iters > 0 ? (float4 *)(b + L.xtbar) : nullptr;
    D.vbar = L.max_bwd_iters > 0 ? (float4 *)(b + L.vbar) : nullptr;
    D.contrib = L.max_bwd_iters > 0 ? (float3 *)(b + L.contrib) : nullptr;
    D.cin = L.max_bwd_iters > 0 ? (float3 *)(b + L.cin) : nullptr;
    D.tgt = L.max_bwd_iters > 0 ? (const int3 *)(b + L.tgt) : nullptr;
    D.ebar_pair = L.max_bwd_iters > 0 ? (float *)(b + L.ebar_pair) : nullptr;
    D.tet_pairs = L.max_bwd_iters > 0 ? (const int4 *)(b + L.tet_pairs) : nullptr;
    D.n_verts = T.nv;
    D.n_tets = T.nt;
    D.n_free = T.n_free;
    D.n_colors = T.n_colors;
    DevSurf &S = T.surf_dev;
    S = DevSurf{};
    S.n_tri = (int)(T.surf.size() / 3);
    S.n_sv = (int)T.sv_slot.size();
    if (S.n_tri > 0) {
        S.tri = (const int4 *)(b + L.s_tri);
        S.tadj = (const int4 *)(b + L.s_tadj);
        S.svert = (const int2 *)(b + L.s_svert);
        S.svidx = (const int *)(b + L.s_svidx);
        S.sv_row = (const int *)(b + L.s_sv_row);
        S.sv_tri = (const int *)(b + L.s_sv_tri);
        S.tnorm = (float4 *)(b + L.s_tnorm);
        S.vnorm = (float4 *)(b + L.s_vnorm);
        S.gparam = (unsigned *)(b + L.s_gparam);
        S.gmax = (float *)(b + L.s_gmax);
        S.hcount = (unsigned *)(b + L.s_hcount);
        S.hstart = (unsigned *)(b + L.s_hstart);
        S.scan_tmp = (unsigned *)(b + L.s_scan);
        S.hitems = (int2 *)(b + L.s_hitems);
        S.tsph = (float4 *)(b + L.s_tsph);
        S.ctri = (int *)(b + L.s_ctri);
        S.ccount = (unsigned *)(b + L.s_ccount);
        S.crow = (unsigned *)(b + L.s_crow);
        S.cent = (int *)(b + L.s_cent);
        S.xsnap = (float4 *)(b + L.s_xsnap);
        S.srest = (const float4 *)(b + L.s_rest);
        S.edge = (const int4 *)(b + L.s_edge);
        S.emid = (float4 *)(b + L.s_emid);
        S.egmax = (float *)(b + L.s_egmax);
        S.ehcount = (unsigned *)(b + L.s_ehcount);
        S.ehstart = (unsigned *)(b + L.s_ehstart);
        S.ehitems = (int2 *)(b + L.s_ehitems);
        S.eb = (int *)(b + L.s_eb);
        S.en = (float4 *)(b + L.s_en);
        S.ecount = (unsigned *)(b + L.s_ecount);
        S.erow = (unsigned *)(b + L.s_erow);
        S.eent = (int *)(b + L.s_eent);
        S.n_edge = (int)(T.sedge.size() / 2);
        S.ehmask = L.ehsize - 1;
        S.hmask = L.hsize - 1;
    }
}

// ------------------------------------------------------------- validation --
vbd_status validate_params(const vbd_topology_s &T, const vbd_step_params *p)
{
    if (!p) return fail(VBD_E_INVALID_ARG, "params is NULL");
    if (!(p->h > 0.f) || !std::isfinite(p->h)) return fail(VBD_E_INVALID_ARG, "h must be > 0");
    if (p->n_iters < 1) return fail(VBD_E_INVALID_ARG, "n_iters must be >= 1");
    if (p->init_mode < 0 || p->init_mode > 3) return fail(VBD_E_INVALID_ARG, "bad init_mode");
    if (p->n_spheres < 0 || p->n_spheres > kMaxObstacles || p->n_planes < 0 ||
        p->n_planes > kMaxObstacles)
        return fail(VBD_E_INVALID_ARG, "at most %d spheres and %d planes", kMaxObstacles, kMaxObstacles);
    if ((p->n_spheres > 0 && !p->spheres) || (p->n_planes > 0 && !p->planes))
        return fail(VBD_E_INVALID_ARG, "obstacle array is NULL");
    if (p->launch_mode < 0 || p->launch_mode > 3) return fail(VBD_E_INVALID_ARG, "bad launch_mode");
    if (p->cheb_rho < 0.f || p->cheb_rho >= 1.f) return fail(VBD_E_INVALID_ARG, "cheb_rho must be in [0,1)");
    if (p->kd < 0.f || p->friction_mu < 0.f || p->contact_k < 0.f)
        return fail(VBD_E_INVALID_ARG, "kd, friction_mu, contact_k must be >= 0");
    if (p->friction_mu > 0.f && !(p->friction_eps_v > 0.f))
        return fail(VBD_E_INVALID_ARG, "friction_eps_v must be > 0");
    if (p->mesh_contacts) {
        if (!(p->collision_radius > 0.f) || !std::isfinite(p->collision_radius))
            return fail(VBD_E_INVALID_ARG, "collision_radius must be > 0 with mesh_contacts");
        if (p->n_col < 0) return fail(VBD_E_INVALID_ARG, "n_col must be >= 0");
        if (p->launch_mode == VBD_LAUNCH_PERSISTENT || p->launch_mode == VBD_LAUNCH_PERSISTENT_GRAPH)
            return fail(VBD_E_UNSUPPORTED, "mesh contacts need launch_mode PLAIN or GRAPH");
        if (p->self_contact && (!(p->self_exclusion >= 0.f) || !std::isfinite(p->self_exclusion)))
            return fail(VBD_E_INVALID_ARG, "self_exclusion must be finite and >= 0");
    } else if (p->self_contact || p->edge_contacts) {
        return fail(VBD_E_INVALID_ARG, "self_contact and edge_contacts need mesh_contacts");
    }
    (void)T;
    return VBD_OK;
}

StepConsts make_consts(const vbd_topology_s &T, const vbd_step_params *p)
{
    StepConsts K{};
    K.h = p->h;
    K.inv_h = 1.0f / p->h;
    K.gx = p->gravity[0]; K.gy = p->gravity[1]; K.gz = p->gravity[2];
    K.gnorm = std::sqrt(K.gx * K.gx + K.gy * K.gy + K.gz * K.gz);
    K.init_mode = p->init_mode;
    K.det_eps_rel = p->det_eps_rel;
    K.kc = p->contact_k;
    K.delta = p->contact_thickness;
    K.kd_over_h = p->kd / p->h;
    K.fric_mu = p->friction_mu;
    K.fric_hev = p->h * p->friction_eps_v;
    K.cheb_rho = p->cheb_rho;
    const double nu = T.nu;
    const double k_mu = 1.0 / (2.0 * (1.0 + nu));
    const double k_lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    K.k_mu = (float)k_mu;
    K.k_lam = (float)k_lam;
    K.alpha = (float)(1.0 + k_mu / k_lam);
    K.spring_k = (float)T.spring_k;
    K.spring_psd = p->spring_psd ? 1 : 0;
    K.n_spheres = p->n_spheres;
    K.n_planes = p->n_planes;
    for (int i = 0; i < p->n_spheres; ++i)
        K.spheres[i] = make_float4(p->spheres[4 * i], p->spheres[4 * i + 1], p->spheres[4 * i + 2],
                                   p->spheres[4 * i + 3]);
    for (int i = 0; i < p->n_planes; ++i) {
        const float *q = p->planes + 4 * i;
        const float n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        const float s = n > 0.f ? 1.0f / n : 0.f;
        K.planes[i] = make_float4(q[0] * s, q[1] * s, q[2] * s, q[3] * s);
    }
    K.col_radius = p->mesh_contacts ? p->collision_radius : 0.f;
    K.self_contact = p->mesh_contacts && p->self_contact ? 1 : 0;
    K.self_excl = p->self_exclusion;
    K.edge_contacts = p->mesh_contacts && p->edge_contacts ? 1 : 0;
    return K;
}

// --------------------------------------------------------------- coloring --
// Vertex adjacency of the tets and springs as CSR, each neighbour once.
// Rows are not sorted: none of the colorings below depends on the order in
// which a vertex's neighbours are visited.
struct Adjacency {
    std::vector<int64_t> row;
    std::vector<int32_t> col;
    int n() const { return (int)row.size() - 1; }
    int32_t degree(int v) const { return (int32_t)(row[v + 1] - row[v]); }
    const int32_t *begin(int v) const { return col.data() + row[v]; }
    const int32_t *end(int v) const { return col.data() + row[v + 1]; }
};

// lower_only: keep only neighbours of smaller id.
Adjacency build_adjacency(const vbd_topology_s &T, bool lower_only)
{
    const int nv = T.nv;
    // vertex -> incident tets and springs, by counting
    std::vector<int64_t> trow((size_t)nv + 1, 0), srow((size_t)nv + 1, 0);
    for (size_t i = 0; i < 4 * (size_t)T.nt; ++i) ++trow[(size_t)T.tets[i] + 1];
    for (size_t i = 0; i < 2 * (size_t)T.ns; ++i) ++srow[(size_t)T.springs[i] + 1];
    for (int v = 0; v < nv; ++v) {
        trow[v + 1] += trow[v];
        srow[v + 1] += srow[v];
    }
    std::vector<int32_t> tinc((size_t)trow[nv]), sinc((size_t)srow[nv]);
    {
        std::vector<int64_t> cur(trow.begin(), trow.end() - 1);
        for (int t = 0; t < T.nt; ++t)
            for (int a = 0; a < 4; ++a) tinc[(size_t)cur[T.tets[4 * (size_t)t + a]]++] = t;
        cur.assign(srow.begin(), srow.end() - 1);
        for (int s = 0; s < T.ns; ++s)
            for (int a = 0; a < 2; ++a) sinc[(size_t)cur[T.springs[2 * (size_t)s + a]]++] = s;
    }
    Adjacency A;
    A.row.assign((size_t)nv + 1, 0);
    A.col.reserve((size_t)trow[nv] * 3 / 2 + (size_t)srow[nv]);
    std::vector<int32_t> stamp(nv, -1);   // last vertex that listed this neighbour
    for (int v = 0; v < nv; ++v) {
        stamp[v] = v;
        auto take = [&](int32_t u) {
            if (stamp[u] == v || (lower_only && u > v)) return;
            stamp[u] = v;
            A.col.push_back(u);
        };
        for (int64_t i = trow[v]; i < trow[v + 1]; ++i) {
            const int32_t *q = &T.tets[4 * (size_t)tinc[(size_t)i]];
            for (int a = 0; a < 4; ++a) take(q[a]);
        }
        for (int64_t i = srow[v]; i < srow[v + 1]; ++i) {
            const int32_t *e = &T.springs[2 * (size_t)sinc[(size_t)i]];
            take(e[0]);
            take(e[1]);
        }
        A.row[(size_t)v + 1] = (int64_t)A.col.size();
    }
    return A;
}

// Vertex order of the greedy coloring.  VBD_COLOR_ID_ORDER: ascending id.
// VBD_COLOR_SMALLEST_LAST: the reverse of the order in which repeatedly
// removing a vertex of smallest remaining degree (ties: smallest id) empties
// the graph (Matula and Beck, J. ACM 30(3), 1983).
std::vector<int32_t> color_order(const Adjacency &nbr, int order)
{
    const int nv = nbr.n();
    std::vector<int32_t> ord(nv);
    if (order == VBD_COLOR_ID_ORDER) {
        for (int v = 0; v < nv; ++v) ord[v] = v;
        return ord;
    }
    // one min-heap of ids per remaining degree, entries invalidated lazily: a
    // vertex enters each bucket at most once (degrees only decrease), so the
    // first live entry of the lowest non-empty bucket is the vertex of
    // smallest remaining degree and, among those, of smallest id
    std::vector<int32_t> deg(nv);
    int maxd = 0;
    for (int v = 0; v < nv; ++v) {
        deg[v] = nbr.degree(v);
        maxd = std::max(maxd, (int)deg[v]);
    }
    std::vector<std::vector<int32_t>> bucket((size_t)maxd + 1);
    for (int v = 0; v < nv; ++v) bucket[deg[v]].push_back(v);   // ascending: already heaps
    const std::greater<int32_t> later;
    std::vector<char> gone(nv, 0);
    int lo = 0;
    for (int i = nv - 1; i >= 0; --i) {
        int v = -1;
        while (v < 0) {
            while (bucket[lo].empty()) ++lo;
            std::vector<int32_t> &b = bucket[lo];
            const int32_t u = b.front();
            std::pop_heap(b.begin(), b.end(), later);
            b.pop_back();
            if (!gone[u] && deg[u] == lo) v = u;
        }
        gone[v] = 1;
        ord[i] = v;
        for (const int32_t *w = nbr.begin(v); w != nbr.end(v); ++w)
            if (!gone[*w]) {
                const int d = --deg[*w];
                bucket[d].push_back(*w);
                std::push_heap(bucket[d].begin(), bucket[d].end(), later);
                if (d < lo) lo = d;
            }
    }
    return ord;
}

// DSATUR (Brelaz, Comm. ACM 22(4), 1979): the next vertex is the uncolored
// one with the most distinct colors among its neighbours (ties: larger
// degree, then smaller id); it takes the smallest color none of them has.
void dsatur_color(const Adjacency &nbr, std::vector<int32_t> &colors, int &nc)
{
    const int nv = nbr.n();
    colors.assign(nv, -1);
    nc = 0;
    std::vector<std::vector<char>> seen(nv);   // neighbour colors seen so far
    std::vector<int32_t> sat(nv, 0);
    // ordered by (saturation desc, degree desc, id asc)
    std::set<std::tuple<int32_t, int32_t, int32_t>> q;
    for (int v = 0; v < nv; ++v) q.insert({0, -nbr.degree(v), v});
    while (!q.empty()) {
        const int v = std::get<2>(*q.begin());
        q.erase(q.begin());
        int c = 0;
        while (c < (int)seen[v].size() && seen[v][c]) ++c;
        colors[v] = c;
        nc = std::max(nc, c + 1);
        for (const int32_t *pw = nbr.begin(v); pw != nbr.end(v); ++pw) {
            const int32_t w = *pw;
            if (colors[w] >= 0) continue;
            if ((int)seen[w].size() <= c) seen[w].resize((size_t)c + 1, 0);
            if (!seen[w][c]) {
                seen[w][c] = 1;
                q.erase({-sat[w], -nbr.degree(w), w});
                ++sat[w];
                q.insert({-sat[w], -nbr.degree(w), w});
            }
        }
    }
}

// First-fit greedy over the union adjacency of tets and springs in the given
// vertex order (DSATUR chooses its order as it colors); neighbour colors are
// tracked in a growable bitset.
void greedy_color(vbd_topology_s &T, int order)
{
    const int nv = T.nv;
    // neighbour lists: in id order only the lower-id neighbours are colored
    // before a vertex; the other orders need them all
    const Adjacency nbr = build_adjacency(T, order == VBD_COLOR_ID_ORDER);
    if (order == VBD_COLOR_DSATUR) {
        int nc = 0;
        dsatur_color(nbr, T.colors, nc);
        T.n_colors = nc;
        return;
    }
    const std::vector<int32_t> ord = color_order(nbr, order);
    T.colors.assign(nv, -1);
    int nc = 0;
    std::vector<uint64_t> used;
    for (int v : ord) {
        used.assign((size_t)(nc / 64 + 1), 0ull);
        for (const int32_t *u = nbr.begin(v); u != nbr.end(v); ++u) {
            const int c = T.colors[*u];
            if (c < 0) continue;
            used[(size_t)c >> 6] |= 1ull << (c & 63);
        }
        int c = 0;
        for (size_t w = 0; w < used.size(); ++w) {
            if (~used[w]) {
                c = (int)(w * 64) + __builtin_ctzll(~used[w]);
                break;
            }
            c = (int)((w + 1) * 64);
        }
        T.colors[v] = c;
        nc = std::max(nc, c + 1);
    }
    T.n_colors = nc;
}

// S = R^{-1} for the rest edge matrix D_m = [X1-X0, X2-X0, X3-X0] = Q R,
// Gram-Schmidt with Q a proper rotation (R's last diagonal entry takes the
// sign of det D_m).  S is upper triangular: {S00, S01, S02, S11, S12, S22}.
void rest_frame_inverse(const std::vector<double> &X, const int32_t *q, double S[6])
{
    double d[3][3];
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) d[c][r] = X[3 * (size_t)q[c + 1] + r] - X[3 * (size_t)q[0] + r];
    auto dotp = [](const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    double q1[3], q2[3], u[3];
    const double r11 = std::sqrt(dotp(d[0], d[0]));
    for (int r = 0; r < 3; ++r) q1[r] = d[0][r] / r11;
    const double r12 = dotp(q1, d[1]);
    for (int r = 0; r < 3; ++r) u[r] = d[1][r] - r12 * q1[r];
    const double r22 = std::sqrt(dotp(u, u));
    for (int r = 0; r < 3; ++r) q2[r] = u[r] / r22;
    const double r13 = dotp(q1, d[2]), r23 = dotp(q2, d[2]);
    for (int r = 0; r < 3; ++r) u[r] = d[2][r] - r13 * q1[r] - r23 * q2[r];
    // third axis q3 = q1 x q2 keeps Q proper; r33 = q3 . d3 carries det's sign
    const double q3[3] = {q1[1] * q2[2] - q1[2] * q2[1], q1[2] * q2[0] - q1[0] * q2[2],
                          q1[0] * q2[1] - q1[1] * q2[0]};
    const double r33 = dotp(q3, d[2]);
    S[0] = 1.0 / r11;
    S[1] = -r12 / (r11 * r22);
    S[2] = (r12 * r23 - r13 * r22) / (r11 * r22 * r33);
    S[3] = 1.0 / r22;
    S[4] = -r23 / (r22 * r33);
    S[5] = 1.0 / r33;
}

void build_csr(vbd_topology_s &T)
{
    const int nv = T.nv;
    // permutation: free vertices by (color, id), then pinned by id
    std::vector<int32_t> count(T.n_colors + 1, 0);
    int n_free = 0;
    for (int v = 0; v < nv; ++v)
        if (!T.pinned[v]) { count[T.colors[v] + 1]++; ++n_free; }
    T.color_off.assign(T.n_colors + 1, 0);
    for (int c = 0; c < T.n_colors; ++c) T.color_off[c + 1] = T.color_off[c] + count[c + 1];
    T.n_free = n_free;
    T.perm.assign(nv, 0);
    T.iperm.assign(nv, 0);
    std::vector<int32_t> fill(T.color_off.begin(), T.color_off.end());
    int pin_slot = n_free;
    for (int v = 0; v < nv; ++v) {
        const int slot = T.pinned[v] ? pin_slot++ : fill[T.colors[v]]++;
        T.perm[slot] = v;
        T.iperm[v] = slot;
    }
    // tet incidence of every vertex slot (free ones first), ascending tet id;
    // the solve kernels only visit the free slots, the adjoint's final fold
    // visits all of them
    std::vector<int32_t> deg(nv + 1, 0);
    for (int t = 0; t < T.nt; ++t)
        for (int k = 0; k < 4; ++k) deg[T.iperm[T.tets[4 * (size_t)t + k]] + 1]++;
    T.tet_row.assign(nv + 1, 0);
    for (int s = 0; s < nv; ++s) T.tet_row[s + 1] = T.tet_row[s] + deg[s + 1];
    T.tet_ent.assign((size_t)T.tet_row[nv], 0);
    std::vector<int32_t> pos(T.tet_row.begin(), T.tet_row.end() - 1);
    for (int t = 0; t < T.nt; ++t)
        for (int k = 0; k < 4; ++k) {
            const int s = T.iperm[T.tets[4 * (size_t)t + k]];
            T.tet_ent[pos[s]++] = (t << 2) | k;
        }
    // spring incidence, ascending spring id
    std::vector<int32_t> sdeg(n_free + 1, 0);
    for (int e = 0; e < T.ns; ++e)
        for (int k = 0; k < 2; ++k) {
            const int s = T.iperm[T.springs[2 * (size_t)e + k]];
            if (s < n_free) sdeg[s + 1]++;
        }
    T.spr_row.assign(n_free + 1, 0);
    for (int s = 0; s < n_free; ++s) T.spr_row[s + 1] = T.spr_row[s] + sdeg[s + 1];
    T.spr_nbr_orig.assign((size_t)T.spr_row[n_free], 0);
    T.spr_len.assign((size_t)T.spr_row[n_free], 0.f);
    std::vector<int32_t> spos(T.spr_row.begin(), T.spr_row.end() - 1);
    for (int e = 0; e < T.ns; ++e)
        for (int k = 0; k < 2; ++k) {
            const int s = T.iperm[T.springs[2 * (size_t)e + k]];
            if (s < n_free) {
                T.spr_nbr_orig[spos[s]] = T.springs[2 * (size_t)e + 1 - k];
                T.spr_len[spos[s]] = (float)T.spring_L[e];
                spos[s]++;
            }
        }
    // color-solve incidence: each color padded to its largest tet count
    T.ell_info.assign(T.n_colors, make_int2(0, 0));
    T.ell_total = 0;
    for (int c = 0; c < T.n_colors; ++c) {
        int dmax = 0;
        for (int s = T.color_off[c]; s < T.color_off[c + 1]; ++s)
            dmax = std::max(dmax, T.tet_row[s + 1] - T.tet_row[s]);
        T.ell_info[c] = make_int2((int)T.ell_total, dmax);
        T.ell_total += (size_t)dmax * (size_t)(T.color_off[c + 1] - T.color_off[c]);
    }
    T.spr_info.assign(T.n_colors, make_int2(0, 0));
    T.spr_total = 0;
    for (int c = 0; c < T.n_colors; ++c) {
        int dmax = 0;
        for (int s = T.color_off[c]; s < T.color_off[c + 1]; ++s)
            dmax = std::max(dmax, T.spr_row[s + 1] - T.spr_row[s]);
        T.spr_info[c] = make_int2((int)T.spr_total, dmax);
        T.spr_total += (size_t)dmax * (size_t)(T.color_off[c + 1] - T.color_off[c]);
    }
    // stored tet order: grouped by the sorted colors of the tet's 4 vertices
    // (then by tet id), so tets sharing a cache line are read in the same
    // color phases
    {
        std::vector<std::pair<uint64_t, int32_t>> key(T.nt);
        for (int t = 0; t < T.nt; ++t) {
            int c[4];
            for (int k = 0; k < 4; ++k) c[k] = T.colors[T.tets[4 * (size_t)t + k]];
            std::sort(c, c + 4);
            uint64_t kk = 0;
            for (int k = 0; k < 4; ++k) kk = (kk << 16) | (uint64_t)(c[k] & 0xffff);
            key[t] = {kk, t};
        }
        std::sort(key.begin(), key.end());
        T.tet_order.assign(T.nt, 0);
        T.tet_rank.assign(T.nt, 0);
        for (int i = 0; i < T.nt; ++i) {
            T.tet_order[i] = key[i].second;
            T.tet_rank[key[i].second] = i;
        }
    }
    // per color: tet pairs, spring entries and distinct neighbours, for the
    // algorithmic bytes of a color solve (update_phase_bytes)
    T.phase_cnt.assign(T.n_colors, {0, 0, 0});
    T.phase_updates.assign(T.n_colors, 0);
    std::vector<int32_t> stamp(nv, -1);
    for (int c = 0; c < T.n_colors; ++c) {
        auto &n = T.phase_cnt[c];
        for (int s = T.color_off[c]; s < T.color_off[c + 1]; ++s) {
            n[0] += T.tet_row[s + 1] - T.tet_row[s];
            n[1] += T.spr_row[s + 1] - T.spr_row[s];
            for (int e = T.tet_row[s]; e < T.tet_row[s + 1]; ++e) {
                const int t = T.tet_ent[e] >> 2;
                for (int k = 0; k < 4; ++k) {
                    const int u = T.iperm[T.tets[4 * (size_t)t + k]];
                    if (u != s && stamp[u] != c) { stamp[u] = c; ++n[2]; }
                }
            }
            for (int e = T.spr_row[s]; e < T.spr_row[s + 1]; ++e) {
                const int u = T.iperm[T.spr_nbr_orig[e]];
                if (stamp[u] != c) { stamp[u] = c; ++n[2]; }
            }
        }
        T.phase_updates[c] = T.color_off[c + 1] - T.color_off[c];
    }
    update_phase_bytes(T);
}

// ----------------------------------------------------------------- surface --
// Faces used by exactly one tet, oriented so (b - a) x (c - a) points away
// from the tet's fourth vertex (out of the mesh), sorted by their ascending
// vertex-id triples; the triangle across each edge; the surface vertices (as
// permuted slots) with their incident triangles.  Only for batched
// topologies (mesh-mesh contacts are between different meshes).
void build_surface(vbd_topology_s &T)
{
    T.surf.clear(); T.surf_adj.clear(); T.sv_slot.clear(); T.sv_row.clear(); T.sv_tri.clear();
    T.vert_mesh.assign(T.nv, 0);
    for (int m = 0; m < T.n_meshes; ++m)
        for (int64_t v = T.vert_off[m]; v < T.vert_off[m + 1]; ++v) T.vert_mesh[v] = m;
    T.sedge.clear();
    if (T.nt == 0) return;
    // faces bucketed by their smallest vertex id (counting sort), then each
    // bucket sorted by the other two ids: the output is in ascending order of
    // the sorted id triples, linear in the number of faces
    struct Face { int32_t mid, hi, t, opp; };
    const int nv = T.nv;
    std::vector<int64_t> off((size_t)nv + 1, 0);
    auto face_ids = [&](int t, int o, int32_t v[3]) {
        int k = 0;
        for (int j = 0; j < 4; ++j)
            if (j != o) v[k++] = T.tets[4 * (size_t)t + j];
    };
    for (int t = 0; t < T.nt; ++t)
        for (int o = 0; o < 4; ++o) {
            int32_t v[3];
            face_ids(t, o, v);
            off[(size_t)std::min(v[0], std::min(v[1], v[2])) + 1]++;
        }
    for (int v = 0; v < nv; ++v) off[v + 1] += off[v];
    std::vector<Face> f((size_t)off[nv]);
    {
        std::vector<int64_t> pos(off.begin(), off.end() - 1);
        for (int t = 0; t < T.nt; ++t)
            for (int o = 0; o < 4; ++o) {
                int32_t v[3];
                face_ids(t, o, v);
                std::sort(v, v + 3);
                f[(size_t)pos[v[0]]++] = Face{v[1], v[2], t, o};
            }
    }
    auto P = [&](int v, int r) { return T.rest[3 * (size_t)v + r]; };
    for (int lo = 0; lo < nv; ++lo) {
        Face *b = f.data() + off[lo], *e = f.data() + off[lo + 1];
        std::sort(b, e, [](const Face &x, const Face &y) {
            return x.mid != y.mid ? x.mid < y.mid : x.hi < y.hi;
        });
        for (Face *i = b; i < e;) {
            Face *j = i + 1;
            while (j < e && j->mid == i->mid && j->hi == i->hi) ++j;
            if (j - i == 1) {
                const int32_t *q = &T.tets[4 * (size_t)i->t];
                int v[3], k = 0;
                for (int a = 0; a < 4; ++a)
                    if (a != i->opp) v[k++] = q[a];
                const int d = q[i->opp];
                double e1[3], e2[3], e3[3];
                for (int r = 0; r < 3; ++r) {
                    e1[r] = P(v[1], r) - P(v[0], r);
                    e2[r] = P(v[2], r) - P(v[0], r);
                    e3[r] = P(d, r) - P(v[0], r);
                }
                const double n0 = e1[1] * e2[2] - e1[2] * e2[1], n1 = e1[2] * e2[0] - e1[0] * e2[2],
                             n2 = e1[0] * e2[1] - e1[1] * e2[0];
                if (n0 * e3[0] + n1 * e3[1] + n2 * e3[2] > 0.0) std::swap(v[1], v[2]);
                T.surf.insert(T.surf.end(), {v[0], v[1], v[2]});
            }
            i = j;
        }
    }
    const int ntri = (int)(T.surf.size() / 3);
    // edge adjacency: (min, max, triangle, edge) sorted by the undirected edge
    std::vector<std::array<int32_t, 4>> ed;
    ed.reserve(3 * (size_t)ntri);
    for (int t = 0; t < ntri; ++t)
        for (int k = 0; k < 3; ++k) {
            const int a = T.surf[3 * (size_t)t + k], b = T.surf[3 * (size_t)t + (k + 1) % 3];
            ed.push_back({std::min(a, b), std::max(a, b), t, k});
        }
    std::sort(ed.begin(), ed.end());
    for (size_t i = 0; i < ed.size(); ++i)
        if (i == 0 || ed[i][0] != ed[i - 1][0] || ed[i][1] != ed[i - 1][1])
            T.sedge.insert(T.sedge.end(), {ed[i][0], ed[i][1]});
    T.surf_adj.assign(3 * (size_t)ntri, -1);
    for (size_t i = 0; i < ed.size();) {
        size_t j = i + 1;
        while (j < ed.size() && ed[j][0] == ed[i][0] && ed[j][1] == ed[i][1]) ++j;
        if (j - i == 2) {
            T.surf_adj[3 * (size_t)ed[i][2] + ed[i][3]] = ed[i + 1][2];
            T.surf_adj[3 * (size_t)ed[i + 1][2] + ed[i + 1][3]] = ed[i][2];
        }
        i = j;
    }
    // surface vertices as ascending permuted slots, with incident triangles
    std::vector<int32_t> idx(T.nv, -1);
    for (int32_t v : T.surf) idx[T.iperm[v]] = 0;
    for (int sl = 0; sl < T.nv; ++sl)
        if (idx[sl] == 0) { idx[sl] = (int32_t)T.sv_slot.size(); T.sv_slot.push_back(sl); }
    const int nsv = (int)T.sv_slot.size();
    T.sv_row.assign(nsv + 1, 0);
    for (int32_t v : T.surf) T.sv_row[idx[T.iperm[v]] + 1]++;
    for (int i = 0; i < nsv; ++i) T.sv_row[i + 1] += T.sv_row[i];
    T.sv_tri.assign((size_t)T.sv_row[nsv], 0);
    std::vector<int32_t> pos(T.sv_row.begin(), T.sv_row.end() - 1);
    for (int t = 0; t < ntri; ++t)
        for (int k = 0; k < 3; ++k) T.sv_tri[pos[idx[T.iperm[T.surf[3 * (size_t)t + k]]]]++] = t;
}

// {first tet entry, padded tet degree, first spring entry, padded spring
// degree} of color c
int4 incidence(const vbd_topology_s &T, int c)
{
    return make_int4(T.ell_info[c].x, T.ell_info[c].y, T.spr_info[c].x, T.spr_info[c].y);
}

// Mesh-aligned XCD parts of every color (launch mapping 3): 8 contiguous
// parts of the color's slot range with about equal work, each cut at the mesh
// boundary nearest its target unless that is more than 1/16 of the color's
// work away (large meshes are cut inside), so that the vertices of one mesh
// and color, which read each other's neighbour positions, mostly run on one
// XCD and share its L2.  Work = vertices: every vertex of a color walks the
// color's padded degree.
void build_xcd_split(vbd_topology_s &T)
{
    T.xsplit.assign(9 * (size_t)T.n_colors, 0);
    T.xsplit_max.assign(T.n_colors, 0);
    for (int c = 0; c < T.n_colors; ++c) {
        const int b = T.color_off[c], e = T.color_off[c + 1], n = e - b;
        std::vector<double> cum((size_t)n + 1, 0.0);
        for (int i = 0; i < n; ++i) {
            const int sl = b + i;
            (void)sl;
            cum[i + 1] = cum[i] + 1.0;
        }
        std::vector<int> bounds{0};
        for (int i = 1; i < n; ++i)
            if (T.vert_mesh[T.perm[b + i]] != T.vert_mesh[T.perm[b + i - 1]]) bounds.push_back(i);
        bounds.push_back(n);
        int32_t *xs = &T.xsplit[9 * (size_t)c];
        xs[0] = b;
        xs[8] = e;
        int prev = 0;
        for (int k = 1; k < 8; ++k) {
            const double target = cum[n] * k / 8.0;
            // nearest mesh boundary to the target
            auto it = std::lower_bound(bounds.begin(), bounds.end(), 0, [&](int pos, int) {
                return cum[pos] < target;
            });
            int best = it == bounds.end() ? n : *it;
            if (it != bounds.begin() && it != bounds.end()) {
                const int lo = *(it - 1);
                if (target - cum[lo] < cum[best] - target) best = lo;
            }
            if (std::fabs(cum[best] - target) > cum[n] / 16.0) {
                // cut inside the mesh at the target
                best = (int)(std::lower_bound(cum.begin(), cum.end(), target) - cum.begin());
            }
            best = std::max(best, prev);
            xs[k] = b + best;
            prev = best;
        }
        for (int k = 0; k < 8; ++k) T.xsplit_max[c] = std::max(T.xsplit_max[c], xs[k + 1] - xs[k]);
    }
}

XcdSplit xcd_split(const vbd_topology_s &T, int c)
{
    return XcdSplit{(const int *)(T.ws + T.lay.xsplit) + 9 * (size_t)c, T.xsplit_max[c]};
}

// --------------------------------------------------------------- profiling --
vbd_status prof_begin(vbd_topology_s &T, hipStream_t s, ProfileEvent &ev)
{
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    HIP_TRY(hipEventRecord(ev.a, s));
    (void)T;
    return VBD_OK;
}

// ------------------------------------------------------------ enqueue step --
// D: the device view the kernels use (D, or T.dev with the per-step state
// buffers moved to the static scratch); profile: allow the event brackets.
vbd_status enqueue_step(vbd_topology_s &T, const DevTopo &D, const vbd_step_params *p,
                        const StepConsts &K, float *x, float *v, float *vp, const float *E,
                        hipStream_t s, bool persistent, bool in_capture, bool profile = true)
{
    const bool tets = T.nt > 0, springs = T.ns > 0;
    HIP_TRY(launch_material(D, E, K, T.cfg.compact != 0, s));
    HIP_TRY(launch_predict(D, x, v, vp, K, persistent, s));
    const bool prof = profile && T.profiling && !in_capture;
    if (persistent) {
        ProfileEvent ev{};
        if (prof) {
            vbd_status st = prof_begin(T, s, ev);
            if (st) return st;
        }
        int grid = 0;
        HIP_TRY(launch_persistent(D, K, p->n_iters, tets, springs, T.cfg, T.n_cu,
                                  /*cooperative=*/!in_capture, s, &grid));
        if (prof) {
            HIP_TRY(hipEventRecord(ev.b, s));
            double bytes = 0;
            int64_t upd = 0;
            for (int c = 0; c < T.n_colors; ++c) { bytes += T.phase_bytes[c]; upd += T.phase_updates[c]; }
            ev.bytes = bytes * p->n_iters;
            ev.updates = upd * p->n_iters;
            ev.launches = 1;
            T.events.push_back(ev);
        }
    } else {
        // profiling brackets the whole sequence of color-solve launches of the
        // step with one event pair (no per-launch event overhead)
        ProfileEvent ev{};
        if (prof) {
            vbd_status st = prof_begin(T, s, ev);
            if (st) return st;
        }
        int64_t launches = 0;
        const bool mc = p->mesh_contacts && T.surf_dev.n_tri > 0;
        // mesh contacts: the snapshot starts equal to the initial guess; each
        // phase refreshes the snapshot of the color solved before it
        int pend_b = 0, pend_e = 0;
        if (mc) {
            HIP_TRY(launch_copy4(T.surf_dev.xsnap, D.x, T.nv, s));
            HIP_TRY(launch_detect(D, T.surf_dev, D.xt, K, s));
        }
        for (int it = 1; it <= p->n_iters; ++it) {
            Range iteration("vbd iteration", profile);
            // Alg. 1: detection on the current iterate before iterations
            // 1, 1 + n_col, ... (n mod n_col = 1; the first on the initial guess)
            if (mc && p->n_col > 0 && (it - 1) % p->n_col == 0)
                HIP_TRY(launch_detect(D, T.surf_dev, D.x, K, s));
            for (int c = 0; c < T.n_colors; ++c) {
                Range phase("vbd color phase", profile);
                if (mc) {
                    if (T.color_off[c + 1] > T.color_off[c]) {
                        HIP_TRY(launch_solve_contacts(D, T.surf_dev, K, T.color_off[c], T.color_off[c + 1],
                                                      incidence(T, c), pend_b, pend_e, tets, springs, T.cfg, s,
                                                      xcd_split(T, c)));
                        pend_b = T.color_off[c];
                        pend_e = T.color_off[c + 1];
                    }
                } else
                    HIP_TRY(launch_solve(D, K, T.color_off[c], T.color_off[c + 1], incidence(T, c), tets, springs,
                                         T.cfg, s, xcd_split(T, c)));
                if (T.color_off[c + 1] > T.color_off[c]) {
                    ++launches;
                    ev.bytes += T.phase_bytes[c];
                    ev.updates += T.phase_updates[c];
                }
            }
            if (p->cheb_rho > 0.f) {
                HIP_TRY(launch_cheb(D, K, it, s, mc ? T.surf_dev.xsnap : nullptr));
                pend_b = pend_e = 0;
            }
        }
        if (prof) {
            HIP_TRY(hipEventRecord(ev.b, s));
            ev.launches = launches;
            T.events.push_back(ev);
        }
    }
    HIP_TRY(launch_finalize(D, x, v, vp, K, s));
    if (p->check_finite) HIP_TRY(launch_check_finite(x, v, 3 * (long long)T.nv, D.flags, s));
    return VBD_OK;
}

GraphKey make_key(const vbd_step_params *p, std::vector<const void *> ptrs, void *stream)
{
    GraphKey k;
    k.ptrs = std::move(ptrs);
    k.stream = stream;
    auto push = [&](const void *src, size_t n) {
        const uint32_t *w = (const uint32_t *)src;
        for (size_t i = 0; i < n / 4; ++i) k.params.push_back(w[i]);
    };
    push(&p->h, 4); push(&p->n_iters, 4); push(p->gravity, 12); push(&p->init_mode, 4);
    push(&p->det_eps_rel, 4); push(&p->contact_k, 4); push(&p->contact_thickness, 4);
    push(&p->n_spheres, 4); if (p->n_spheres) push(p->spheres, 16 * (size_t)p->n_spheres);
    push(&p->n_planes, 4); if (p->n_planes) push(p->planes, 16 * (size_t)p->n_planes);
    push(&p->kd, 4); push(&p->cheb_rho, 4); push(&p->friction_mu, 4); push(&p->friction_eps_v, 4);
    push(&p->spring_psd, 4);
    push(&p->launch_mode, 4);
    push(&p->mesh_contacts, 4); push(&p->collision_radius, 4); push(&p->n_col, 4);
    push(&p->backward_recorded, 4);
    push(&p->check_finite, 4);
    push(&p->self_contact, 4); push(&p->self_exclusion, 4); push(&p->edge_contacts, 4);
    return k;
}

// Replays C's graph when its key matches, else captures `enqueue` on the
// library-owned capture stream (the caller's may be the null stream, which
// cannot be captured) and replays that; the graph is launched on `s`.
template <class F>
vbd_status run_graph(vbd_topology_s &T, GraphCache &C, GraphKey key, hipStream_t s, F enqueue)
{
    if (!C.have || !(key == C.key)) {
        C.reset();
        if (!T.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&T.cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(T.cap_stream, hipStreamCaptureModeThreadLocal));
        vbd_status cs = enqueue(T.cap_stream);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(T.cap_stream, &g);
        if (cs != VBD_OK) {
            if (g) (void)hipGraphDestroy(g);
            return cs;
        }
        if (ce != hipSuccess) return fail(VBD_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
        HIP_TRY(hipGraphInstantiate(&C.exec, g, nullptr, nullptr, 0));
        C.graph = g;
        C.key = std::move(key);
        C.have = true;
    }
    HIP_TRY(hipGraphLaunch(C.exec, s));
    return VBD_OK;
}

// Backward of one step: forward recompute with an iterate snapshot per
// iteration, then the reverse color sweeps, the fold of the pending cells and
// the adjoints of the initial guess and of y.
// The step's iterates into the workspace snapshots: snapshot n = the iterate
// after iteration n (snapshot 0 = the initial guess).
vbd_status enqueue_record(vbd_topology_s &T, const vbd_step_params *p, const StepConsts &K,
                          const float *x_t, const float *v_t, const float *v_prev, const float *E,
                          hipStream_t s)
{
    const size_t nv = (size_t)T.nv;
    DevTopo D = T.dev;
    D.x = D.snaps;
    HIP_TRY(launch_material(D, E, K, T.cfg.compact != 0, s));
    HIP_TRY(launch_predict(D, x_t, v_t, v_prev, K, false, s));
    // snapshot 1 starts as the initial guess and every snapshot holds the
    // pinned positions; the updates of iteration n are stored into snapshot
    // n and, as the start of iteration n + 1, into snapshot n + 1
    HIP_TRY(launch_seed_snapshots(D, p->n_iters, s));
    for (int it = 1; it <= p->n_iters; ++it) {
        Range iteration("vbd iteration");
        float4 *Sn = T.dev.snaps + nv * it;
        D.x = Sn;
        D.xnext = it < p->n_iters ? Sn + nv : nullptr;
        for (int c = 0; c < T.n_colors; ++c) {
            Range phase("vbd color phase");
            HIP_TRY(launch_solve(D, K, T.color_off[c], T.color_off[c + 1], incidence(T, c), true, false, T.cfg, s,
                                 xcd_split(T, c)));
        }
    }
    return VBD_OK;
}

// Clears the reverse sweep's accumulators: the contribution cells, the pinned
// vertices' (tet, slot) cells and the Ebar shares.
hipError_t zero_bwd_accumulators(vbd_topology_s &T, hipStream_t s)
{
    if (T.lay.max_bwd_iters <= 0 || T.nt == 0) return hipSuccess;
    const DevTopo &D = T.dev;
    hipError_t e = launch_zero_u32((unsigned *)D.contrib, 12 * (long long)T.nt, s);
    if (e == hipSuccess) e = launch_zero_u32((unsigned *)D.cin, 9 * (long long)T.ell_total, s);
    if (e == hipSuccess) e = launch_zero_u32((unsigned *)D.ebar_pair, (long long)T.ell_total, s);
    return e;
}

vbd_status enqueue_backward(vbd_topology_s &T, const vbd_step_params *p, const StepConsts &K,
                            const float *x_t, const float *v_t, const float *v_prev, const float *E,
                            const float *gx_out, const float *gv_out, const float *gvp_out,
                            float *gx_in, float *gv_in, float *gvp_in, float *g_E, hipStream_t s,
                            bool in_capture)
{
    const size_t nv = (size_t)T.nv;
    DevTopo D = T.dev;
    if (p->backward_recorded) {
        // the snapshots hold this step's iterates already: only the material
        // records and the inertia target (into the library's own x, so that
        // snapshot 0 stays as recorded) are rebuilt
        HIP_TRY(launch_material(D, E, K, T.cfg.compact != 0, s));
        HIP_TRY(launch_predict(D, x_t, v_t, v_prev, K, false, s));
    } else {
        vbd_status st = enqueue_record(T, p, K, x_t, v_t, v_prev, E, s);
        if (st) return st;
    }
    D.x = T.dev.snaps;
    // reverse sweep
    HIP_TRY(launch_bwd_init(D, gx_out, gv_out, gvp_out, K, s));
    // profiling: one event pair around the reverse sweep's adjoint launches
    ProfileEvent ev{};
    const bool prof = T.profiling && !in_capture;
    if (prof) {
        vbd_status st = prof_begin(T, s, ev);
        if (st) return st;
    }
    // the reverse phases map each XCD to a contiguous range of vertices
    // whatever the forward's mapping: a phase's senders and the cells they
    // write then stay in one L2 (measured fastest on the 33^3 cube: 8.4 us
    // against 8.9-9.8 us with the other mappings, at any block size)
    LaunchCfg acfg = T.cfg;
    acfg.xcd_remap = 1;
    for (int it = p->n_iters; it >= 1; --it) {
        Range iteration("vbd reverse iteration");
        const float4 *Sn = T.dev.snaps + nv * it, *Sp = Sn - nv;
        for (int c = T.n_colors - 1; c >= 0; --c) {
            Range phase("vbd reverse color phase");
            HIP_TRY(launch_adjoint_color(D, K, Sn, Sp, T.color_off[c], T.color_off[c + 1], T.ell_info[c],
                                         acfg, s));
            if (T.color_off[c + 1] > T.color_off[c]) {
                ++ev.launches;
                ev.bytes += T.adj_phase_bytes[c];
                ev.updates += T.phase_updates[c];
            }
        }
    }
    if (prof) {
        HIP_TRY(hipEventRecord(ev.b, s));
        T.events.push_back(ev);
    }
    HIP_TRY(launch_bwd_fold(D, s));
    HIP_TRY(launch_bwd_final(D, v_t, v_prev, gx_in, gv_in, gvp_in, g_E, K, s));
    return VBD_OK;
}

// autotune cache: (arch, log2 size buckets, kinds, persistent) -> config
std::mutex g_tune_mu;
std::map<std::tuple<std::string, int, int, int, int, int>, LaunchCfg> g_tune_cache;

int log2_bucket(int64_t n)
{
    int b = 0;
    while (n > 1) { n >>= 1; ++b; }
    return b;
}

}  // namespace

// ===================================================================== ABI ==
extern "C" {

const char *vbd_last_error(void) { return g_err.c_str(); }

vbd_status vbd_build_topology(const vbd_mesh_desc *d, vbd_topology *out)
{
    Range range("vbd_build_topology");
    if (!d || !out) return fail(VBD_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (d->n_verts < 0 || d->n_tets < 0 || d->n_springs < 0 || d->n_meshes < 1)
        return fail(VBD_E_INVALID_ARG, "negative counts or n_meshes < 1");
    if (d->n_verts > 0 && !d->rest_pos) return fail(VBD_E_INVALID_ARG, "rest_pos is NULL");
    if (d->n_tets > 0 && !d->tets) return fail(VBD_E_INVALID_ARG, "tets is NULL");
    if (d->n_springs > 0 && !d->springs) return fail(VBD_E_INVALID_ARG, "springs is NULL");
    if (d->n_tets > (1 << 29)) return fail(VBD_E_INVALID_ARG, "too many tets (max 2^29)");
    if (d->n_verts > (1 << 28)) return fail(VBD_E_INVALID_ARG, "too many vertices (max 2^28)");
    // The stable Neo-Hookean energy as read here, mu/2 (tr F^T F - 3) +
    // lam/2 (J - alpha)^2 with alpha = 1 + mu/lam, needs lam > 0, i.e. nu > 0.
    if (!(d->poisson_nu > 0.0 && d->poisson_nu < 0.5) && d->n_tets > 0)
        return fail(VBD_E_INVALID_ARG, "poisson_nu must be in (0, 0.5)");
    if (d->n_meshes > 1 && (!d->vert_offsets || !d->tet_offsets))
        return fail(VBD_E_INVALID_ARG, "batched description needs vert_offsets and tet_offsets");
    auto *T = new vbd_topology_s();
    T->nv = d->n_verts; T->nt = d->n_tets; T->ns = d->n_springs; T->n_meshes = d->n_meshes;
    T->nu = d->poisson_nu;
    T->spring_k = d->spring_k;
    T->rest.assign(d->rest_pos, d->rest_pos + 3 * (size_t)d->n_verts);
    if (d->n_tets) T->tets.assign(d->tets, d->tets + 4 * (size_t)d->n_tets);
    if (d->n_springs) T->springs.assign(d->springs, d->springs + 2 * (size_t)d->n_springs);
    T->pinned.assign(d->n_verts, 0);
    if (d->pinned)
        for (int i = 0; i < d->n_verts; ++i) T->pinned[i] = d->pinned[i] ? 1 : 0;
    if (d->n_meshes > 1) {
        T->vert_off.assign(d->vert_offsets, d->vert_offsets + d->n_meshes + 1);
        T->tet_off.assign(d->tet_offsets, d->tet_offsets + d->n_meshes + 1);
    } else {
        T->vert_off = {0, d->n_verts};
        T->tet_off = {0, d->n_tets};
    }
    auto reject = [&](vbd_status s, const char *fmt, auto... a) {
        delete T;
        return fail(s, fmt, a...);
    };
    if (T->vert_off.front() != 0 || T->vert_off.back() != d->n_verts || T->tet_off.front() != 0 ||
        T->tet_off.back() != d->n_tets)
        return reject(VBD_E_INVALID_ARG, "offsets must start at 0 and end at the counts");
    for (int m = 0; m < T->n_meshes; ++m)
        if (T->vert_off[m + 1] < T->vert_off[m] || T->tet_off[m + 1] < T->tet_off[m])
            return reject(VBD_E_INVALID_ARG, "offsets must be non-decreasing");
    // tets: ids in range, distinct, inside their mesh; FP64 rest data
    T->Dminv.assign(9 * (size_t)T->nt, 0.0);
    T->vol.assign(T->nt, 0.0);
    for (int m = 0; m < T->n_meshes; ++m) {
        for (int64_t t = T->tet_off[m]; t < T->tet_off[m + 1]; ++t) {
            const int32_t *q = &T->tets[4 * (size_t)t];
            for (int a = 0; a < 4; ++a) {
                if (q[a] < T->vert_off[m] || q[a] >= T->vert_off[m + 1])
                    return reject(VBD_E_TOPOLOGY, "tet %lld vertex %d out of range of mesh %d",
                                  (long long)t, q[a], m);
                for (int b = 0; b < a; ++b)
                    if (q[a] == q[b]) return reject(VBD_E_TOPOLOGY, "tet %lld repeats vertex %d", (long long)t, q[a]);
            }
            double D[3][3];
            double lmax = 0.0;
            for (int c = 0; c < 3; ++c)
                for (int r = 0; r < 3; ++r) {
                    D[r][c] = T->rest[3 * (size_t)q[c + 1] + r] - T->rest[3 * (size_t)q[0] + r];
                    lmax = std::max(lmax, std::fabs(D[r][c]));
                }
            // adjugate inverse
            const double A00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
            const double A01 = D[0][2] * D[2][1] - D[0][1] * D[2][2];
            const double A02 = D[0][1] * D[1][2] - D[0][2] * D[1][1];
            const double A10 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
            const double A11 = D[0][0] * D[2][2] - D[0][2] * D[2][0];
            const double A12 = D[0][2] * D[1][0] - D[0][0] * D[1][2];
            const double A20 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
            const double A21 = D[0][1] * D[2][0] - D[0][0] * D[2][1];
            const double A22 = D[0][0] * D[1][1] - D[0][1] * D[1][0];
            const double det = D[0][0] * A00 + D[0][1] * A10 + D[0][2] * A20;
            if (!(std::fabs(det) > 1e-12 * lmax * lmax * lmax))
                return reject(VBD_E_TOPOLOGY, "tet %lld is degenerate in the rest shape", (long long)t);
            const double inv = 1.0 / det;
            const double Ai[9] = {A00, A01, A02, A10, A11, A12, A20, A21, A22};
            for (int k = 0; k < 9; ++k) T->Dminv[9 * (size_t)t + k] = Ai[k] * inv;
            T->vol[t] = std::fabs(det) / 6.0;
        }
    }
    // springs
    T->spring_L.assign(T->ns, 0.0);
    for (int s = 0; s < T->ns; ++s) {
        const int a = T->springs[2 * (size_t)s], b = T->springs[2 * (size_t)s + 1];
        if (a < 0 || a >= T->nv || b < 0 || b >= T->nv)
            return reject(VBD_E_TOPOLOGY, "spring %d endpoint out of range", s);
        if (a == b) return reject(VBD_E_TOPOLOGY, "spring %d connects a vertex to itself", s);
        double L;
        if (d->spring_rest) {
            L = d->spring_rest[s];
        } else {
            double d2 = 0;
            for (int r = 0; r < 3; ++r) {
                const double dd = T->rest[3 * (size_t)a + r] - T->rest[3 * (size_t)b + r];
                d2 += dd * dd;
            }
            L = std::sqrt(d2);
        }
        if (!(L > 0.0)) return reject(VBD_E_TOPOLOGY, "spring %d has zero rest length", s);
        T->spring_L[s] = L;
    }
    // masses
    if (d->mass) {
        T->mass.assign(d->mass, d->mass + d->n_verts);
    } else {
        T->mass.assign(T->nv, 0.0);
        for (int t = 0; t < T->nt; ++t)
            for (int a = 0; a < 4; ++a) T->mass[T->tets[4 * (size_t)t + a]] += d->density * T->vol[t] / 4.0;
    }
    // a free vertex may be massless: its local Hessian then comes from its
    // elements alone and the determinant rule skips it while that is singular
    for (int i = 0; i < T->nv; ++i)
        if (!(T->mass[i] >= 0.0) || !std::isfinite(T->mass[i]))
            return reject(VBD_E_INVALID_ARG, "vertex %d has mass %g (must be finite and >= 0)", i,
                          T->mass[i]);
    *out = T;
    return VBD_OK;
}

vbd_status vbd_color(vbd_topology T, int32_t *n_colors_out, int32_t *colors_out)
{
    return vbd_color_greedy(T, VBD_COLOR_ID_ORDER, n_colors_out, colors_out);
}

vbd_status vbd_color_greedy(vbd_topology T, int32_t order, int32_t *n_colors_out, int32_t *colors_out)
{
    Range range("vbd_color_greedy");
    if (!T) return fail(VBD_E_INVALID_ARG, "NULL topology");
    if (order != VBD_COLOR_ID_ORDER && order != VBD_COLOR_SMALLEST_LAST && order != VBD_COLOR_DSATUR)
        return fail(VBD_E_INVALID_ARG, "unknown coloring order %d", order);
    if (T->colored && T->color_order != order) {
        if (T->bound) return fail(VBD_E_INVALID_ARG, "the topology is bound: color before vbd_bind_workspace");
        T->colored = false;
    }
    if (!T->colored) {
        greedy_color(*T, order);
        T->color_order = order;
        build_csr(*T);
        build_surface(*T);
        build_xcd_split(*T);
        T->colored = true;
    }
    if (n_colors_out) *n_colors_out = T->n_colors;
    if (colors_out) std::copy(T->colors.begin(), T->colors.end(), colors_out);
    return VBD_OK;
}

vbd_status vbd_color_given(vbd_topology T, const int32_t *colors)
{
    Range range("vbd_color_given");
    if (!T || (!colors && T->nv > 0)) return fail(VBD_E_INVALID_ARG, "NULL argument");
    if (T->bound) return fail(VBD_E_INVALID_ARG, "the topology is bound: color before vbd_bind_workspace");
    int nc = 0;
    for (int v = 0; v < T->nv; ++v) {
        if (colors[v] < 0 || colors[v] >= 65536)
            return fail(VBD_E_INVALID_ARG, "color of vertex %d out of range [0, 65536)", v);
        nc = std::max(nc, colors[v] + 1);
    }
    for (int t = 0; t < T->nt; ++t) {
        const int32_t *q = &T->tets[4 * (size_t)t];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < a; ++b)
                if (colors[q[a]] == colors[q[b]])
                    return fail(VBD_E_INVALID_ARG, "tet %d has two vertices of color %d", t, colors[q[a]]);
    }
    for (int e = 0; e < T->ns; ++e)
        if (colors[T->springs[2 * (size_t)e]] == colors[T->springs[2 * (size_t)e + 1]])
            return fail(VBD_E_INVALID_ARG, "spring %d joins two vertices of one color", e);
    T->colors.assign(colors, colors + T->nv);
    T->n_colors = nc;
    T->color_order = -1;
    build_csr(*T);
    build_surface(*T);
    build_xcd_split(*T);
    T->colored = true;
    return VBD_OK;
}

vbd_status vbd_workspace_size(vbd_topology T, int32_t max_backward_iters, size_t *bytes)
{
    if (!T || !bytes) return fail(VBD_E_INVALID_ARG, "NULL argument");
    if (!T->colored) return fail(VBD_E_NOT_COLORED, "call vbd_color first");
    if (max_backward_iters < 0) return fail(VBD_E_INVALID_ARG, "max_backward_iters < 0");
    *bytes = make_layout(*T, max_backward_iters).total;
    return VBD_OK;
}

vbd_status vbd_bind_workspace(vbd_topology T, void *dev_ptr, size_t bytes, void *stream)
{
    Range range("vbd_bind_workspace");
    if (!T || !dev_ptr) return fail(VBD_E_INVALID_ARG, "NULL argument");
    if (!T->colored) return fail(VBD_E_NOT_COLORED, "call vbd_color first");
    if ((uintptr_t)dev_ptr % kAlign) return fail(VBD_E_INVALID_ARG, "workspace must be 256-byte aligned");
    if (T->ell_total > (size_t)INT32_MAX || T->spr_total > (size_t)INT32_MAX)
        return fail(VBD_E_INVALID_ARG, "topology too large: %zu / %zu padded incidence entries",
                    T->ell_total, T->spr_total);
    // the largest backward iteration count that fits
    Layout L0 = make_layout(*T, 0);
    if (bytes < L0.total) return fail(VBD_E_NO_WORKSPACE, "workspace too small: %zu < %zu", bytes, L0.total);
    int nb = 0;
    {
        // largest backward iteration count whose layout fits: estimate from
        // the snapshot size (an upper bound), then step down until it fits
        Layout L1 = make_layout(*T, 1);
        const size_t snap = sizeof(float4) * (size_t)T->nv;
        if (bytes >= L1.total) nb = 2 + (int)std::min<size_t>((bytes - L1.total) / (snap ? snap : 1), 1 << 20);
        while (nb > 0 && make_layout(*T, nb).total > bytes) --nb;
        // the reverse sweep addresses cells by (entry << 2) | index
        if (T->ell_total >= ((size_t)1 << 29)) nb = 0;
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    T->device = dev;
    T->n_cu = prop.multiProcessorCount;
    T->arch = prop.gcnArchName;
    T->ws = (char *)dev_ptr;
    T->ws_bytes = bytes;
    T->lay = make_layout(*T, nb);
    set_dev_pointers(*T);
    // host staging of every static array
    std::vector<float> volf(T->nt);
    for (int i = 0; i < T->nt; ++i) volf[i] = (float)T->vol[T->tet_order[i]];
    std::vector<PairEnt> tet_ent_dev(T->tet_ent.size());
    for (size_t e = 0; e < tet_ent_dev.size(); ++e) {
        const int32_t v = T->tet_ent[e];
        const int t = v >> 2, k = v & 3;
        const int32_t *q = &T->tets[4 * (size_t)t];
        int o[3], n = 0;
        for (int j = 0; j < 4; ++j)
            if (j != k) o[n++] = T->iperm[q[j]];
        tet_ent_dev[e] = make_int4((T->tet_rank[t] << 2) | k, o[0], o[1], o[2]);
    }
    std::vector<int2> spr(T->spr_total, make_int2(-1, 0));
    for (int c = 0; c < T->n_colors; ++c) {
        const int2 info = T->spr_info[c];
        for (int sl = T->color_off[c]; sl < T->color_off[c + 1]; ++sl) {
            const size_t base = (size_t)info.x + (size_t)(sl - T->color_off[c]) * (size_t)info.y;
            for (int e = T->spr_row[sl]; e < T->spr_row[sl + 1]; ++e) {
                float L = T->spr_len[e];
                int bits;
                std::memcpy(&bits, &L, 4);
                spr[base + (size_t)(e - T->spr_row[sl])] = make_int2(T->iperm[T->spr_nbr_orig[e]], bits);
            }
        }
    }
    std::vector<float> massp(T->nv);
    for (int sl = 0; sl < T->nv; ++sl) massp[sl] = (float)T->mass[T->perm[sl]];
    auto up = [&](size_t off, const void *src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(T->ws + off, src, n, hipMemcpyHostToDevice, s);
    };
    HIP_TRY(up(T->lay.vol, volf.data(), 4 * volf.size()));
    HIP_TRY(up(T->lay.tet_perm, T->tet_order.data(), 4 * T->tet_order.size()));
    HIP_TRY(up(T->lay.tet_row, T->tet_row.data(), 4 * T->tet_row.size()));
    HIP_TRY(up(T->lay.tet_ent, tet_ent_dev.data(), sizeof(PairEnt) * tet_ent_dev.size()));
    {
        std::vector<PairEnt> ell(T->ell_total, make_int4(-1, 0, 0, 0));
        for (int c = 0; c < T->n_colors; ++c) {
            const int2 info = T->ell_info[c];
            for (int sl = T->color_off[c]; sl < T->color_off[c + 1]; ++sl) {
                const size_t base = (size_t)info.x + (size_t)(sl - T->color_off[c]) * (size_t)info.y;
                for (int e = T->tet_row[sl]; e < T->tet_row[sl + 1]; ++e)
                    ell[base + (size_t)(e - T->tet_row[sl])] = tet_ent_dev[e];
            }
        }
        HIP_TRY(up(T->lay.ell, ell.data(), sizeof(PairEnt) * ell.size()));
        // pair records: from the rest frame S of each (vertex, tet) pair with
        // the vertex as origin and the other three vertices in ascending
        // permuted slot, i.e. ascending color (the reverse sweep's cells are
        // numbered in the same order, so that one color phase writes one
        // cell array per receiving color), in double: m = -(rows of S
        // summed), w = S m, sigma = det S
        std::vector<int4> pa(T->ell_total, make_int4(-1, 0, 0, 0));
        std::vector<float4> pws(T->ell_total, make_float4(0.f, 0.f, 0.f, 0.f));
        std::vector<float> pb(T->ell_total, 0.f);
        std::vector<int32_t> ptet(T->ell_total, -1);
        for (int c = 0; c < T->n_colors; ++c) {
            const int2 info = T->ell_info[c];
            for (int sl = T->color_off[c]; sl < T->color_off[c + 1]; ++sl) {
                const size_t base = (size_t)info.x + (size_t)(sl - T->color_off[c]) * (size_t)info.y;
                for (int e = T->tet_row[sl]; e < T->tet_row[sl + 1]; ++e) {
                    const int t = T->tet_ent[e] >> 2, k = T->tet_ent[e] & 3;
                    const int32_t *q = &T->tets[4 * (size_t)t];
                    int32_t ord[4] = {q[k], 0, 0, 0};
                    int n = 1;
                    for (int j = 0; j < 4; ++j)
                        if (j != k) ord[n++] = q[j];
                    std::sort(ord + 1, ord + 4, [&](int32_t a, int32_t b) { return T->iperm[a] < T->iperm[b]; });
                    double S[6];   // S00, S01, S02, S11, S12, S22
                    rest_frame_inverse(T->rest, ord, S);
                    const double m0 = -S[0], m1 = -(S[1] + S[3]), m2 = -(S[2] + S[4] + S[5]);
                    const double w0 = S[0] * m0 + S[1] * m1 + S[2] * m2;
                    const double w1 = S[3] * m1 + S[4] * m2;
                    const double w2 = S[5] * m2;
                    const size_t i = base + (size_t)(e - T->tet_row[sl]);
                    pa[i] = make_int4(T->iperm[ord[1]], T->iperm[ord[2]], T->iperm[ord[3]], 0);
                    pws[i] = make_float4((float)w0, (float)w1, (float)w2, (float)(S[0] * S[3] * S[5]));
                    pb[i] = pws[i].w;
                    ptet[i] = T->tet_rank[t];
                }
                // padding: the vertex itself as all three neighbours, V lam = 0
                for (size_t i = base + (size_t)(T->tet_row[sl + 1] - T->tet_row[sl]); i < base + (size_t)info.y; ++i)
                    pa[i] = make_int4(sl, sl, sl, 0);
            }
        }
        HIP_TRY(up(T->lay.pa, pa.data(), sizeof(int4) * pa.size()));
        HIP_TRY(up(T->lay.pws, pws.data(), sizeof(float4) * pws.size()));
        HIP_TRY(up(T->lay.pb, pb.data(), sizeof(float) * pb.size()));
        HIP_TRY(up(T->lay.pair_tet, ptet.data(), 4 * ptet.size()));
        HIP_TRY(up(T->lay.ell_info, T->ell_info.data(), sizeof(int2) * T->ell_info.size()));
        if (T->lay.max_bwd_iters > 0) {
            // the reverse sweep's contribution cells, addressed by the pair of
            // the receiving vertex: pos_of[t*4 + k] = padded entry of (slot k's
            // vertex, t) or -1 for a pinned vertex
            std::vector<int32_t> pos_of(4 * (size_t)T->nt, -1);
            for (int c = 0; c < T->n_colors; ++c) {
                const int2 info = T->ell_info[c];
                for (int sl = T->color_off[c]; sl < T->color_off[c + 1]; ++sl) {
                    const size_t base = (size_t)info.x + (size_t)(sl - T->color_off[c]) * (size_t)info.y;
                    for (int e = T->tet_row[sl]; e < T->tet_row[sl + 1]; ++e)
                        pos_of[T->tet_ent[e]] = (int32_t)(base + (size_t)(e - T->tet_row[sl]));
                }
            }
            // per pair (slot k of tet t) and each other slot q in the pair
            // record's order (ascending permuted slot): (entry of (q, t) << 2)
            // | index of k among q's other vertices in that order, or
            // -1 - (stored tet * 4 + q) when q's vertex is pinned
            std::vector<int3> tgt(T->ell_total, make_int3(0, 0, 0));
            for (int t = 0; t < T->nt; ++t) {
                const int32_t *qv = &T->tets[4 * (size_t)t];
                for (int k = 0; k < 4; ++k) {
                    const int32_t e = pos_of[4 * (size_t)t + k];
                    if (e < 0) continue;
                    int32_t os[3], n = 0;
                    for (int q = 0; q < 4; ++q)
                        if (q != k) os[n++] = q;
                    std::sort(os, os + 3, [&](int a, int b) { return T->iperm[qv[a]] < T->iperm[qv[b]]; });
                    int32_t o[3];
                    for (int j = 0; j < 3; ++j) {
                        const int q = os[j];
                        const int32_t eq = pos_of[4 * (size_t)t + q];
                        int rank = 0;   // k among q's others: those of smaller permuted slot
                        for (int r = 0; r < 4; ++r)
                            if (r != q && T->iperm[qv[r]] < T->iperm[qv[k]]) ++rank;
                        o[j] = eq >= 0 ? (eq << 2) | rank : -1 - (T->tet_rank[t] * 4 + q);
                    }
                    tgt[e] = make_int3(o[0], o[1], o[2]);
                }
            }
            std::vector<int4> tpairs(T->nt);
            for (int t = 0; t < T->nt; ++t) {
                const int32_t *q = &pos_of[4 * (size_t)t];
                tpairs[T->tet_rank[t]] = make_int4(q[0], q[1], q[2], q[3]);
            }
            HIP_TRY(up(T->lay.tgt, tgt.data(), sizeof(int3) * tgt.size()));
            HIP_TRY(up(T->lay.tet_pairs, tpairs.data(), sizeof(int4) * tpairs.size()));
        }
    }
    HIP_TRY(up(T->lay.spr_ell, spr.data(), sizeof(int2) * spr.size()));
    HIP_TRY(up(T->lay.spr_info, T->spr_info.data(), sizeof(int2) * T->spr_info.size()));
    HIP_TRY(up(T->lay.perm, T->perm.data(), 4 * T->perm.size()));
    HIP_TRY(up(T->lay.mass, massp.data(), 4 * massp.size()));
    HIP_TRY(up(T->lay.color_off, T->color_off.data(), 4 * T->color_off.size()));
    HIP_TRY(up(T->lay.xsplit, T->xsplit.data(), 4 * T->xsplit.size()));
    const int ntri = (int)(T->surf.size() / 3), nsv = (int)T->sv_slot.size();
    std::vector<int4> stri(ntri), sadj(ntri);
    std::vector<int2> svert(nsv);
    std::vector<int32_t> svidx(T->nv, -1), ctri(T->nv, -1);
    if (ntri > 0) {
        for (int t = 0; t < ntri; ++t) {
            const int32_t *q = &T->surf[3 * (size_t)t];
            stri[t] = make_int4(T->iperm[q[0]], T->iperm[q[1]], T->iperm[q[2]], T->vert_mesh[q[0]]);
            const int32_t *a = &T->surf_adj[3 * (size_t)t];
            sadj[t] = make_int4(a[0], a[1], a[2], -1);
        }
        for (int i = 0; i < nsv; ++i) {
            svert[i] = make_int2(T->sv_slot[i], T->vert_mesh[T->perm[T->sv_slot[i]]]);
            svidx[T->sv_slot[i]] = i;
        }
        HIP_TRY(up(T->lay.s_tri, stri.data(), sizeof(int4) * stri.size()));
        HIP_TRY(up(T->lay.s_tadj, sadj.data(), sizeof(int4) * sadj.size()));
        HIP_TRY(up(T->lay.s_svert, svert.data(), sizeof(int2) * svert.size()));
        HIP_TRY(up(T->lay.s_svidx, svidx.data(), 4 * svidx.size()));
        HIP_TRY(up(T->lay.s_sv_row, T->sv_row.data(), 4 * T->sv_row.size()));
        HIP_TRY(up(T->lay.s_sv_tri, T->sv_tri.data(), 4 * T->sv_tri.size()));
        HIP_TRY(up(T->lay.s_ctri, ctri.data(), 4 * ctri.size()));
        HIP_TRY(launch_zero_u32((unsigned *)(T->ws + T->lay.s_crow), T->nv + 1, s));
        // rest positions (self-contact exclusion) and surface edges as
        // {permuted a, permuted b, mesh, 0} in ascending original-id order
        std::vector<float4> srest(T->nv);
        for (int sl = 0; sl < T->nv; ++sl) {
            const double *r = &T->rest[3 * (size_t)T->perm[sl]];
            srest[sl] = make_float4((float)r[0], (float)r[1], (float)r[2], 0.f);
        }
        const size_t ne = T->sedge.size() / 2;
        std::vector<int4> sedge(ne);
        for (size_t e = 0; e < ne; ++e) {
            const int32_t a = T->sedge[2 * e], b = T->sedge[2 * e + 1];
            sedge[e] = make_int4(T->iperm[a], T->iperm[b], T->vert_mesh[a], 0);
        }
        HIP_TRY(up(T->lay.s_rest, srest.data(), sizeof(float4) * srest.size()));
        HIP_TRY(up(T->lay.s_edge, sedge.data(), sizeof(int4) * sedge.size()));
        HIP_TRY(launch_zero_u32((unsigned *)(T->ws + T->lay.s_erow), T->nv + 1, s));
        std::vector<int32_t> no_partner(ne, -1);
        HIP_TRY(up(T->lay.s_eb, no_partner.data(), 4 * no_partner.size()));
    }
    HIP_TRY(launch_zero_u32(T->dev.flags, kFlagWords, s));
    HIP_TRY(hipStreamSynchronize(s));
    T->bound = true;
    T->bwd_zero = false;
    T->fwd_graph.reset();
    T->bwd_graph.reset();
    T->rec_graph.reset();
    return VBD_OK;
}

vbd_status vbd_topology_query(vbd_topology T, int32_t what, void *out, size_t bytes)
{
    if (!T || !out) return fail(VBD_E_INVALID_ARG, "NULL argument");
    auto give = [&](const void *src, size_t n) -> vbd_status {
        if (bytes < n) return fail(VBD_E_INVALID_ARG, "output buffer too small (%zu < %zu)", bytes, n);
        if (n) std::memcpy(out, src, n);
        return VBD_OK;
    };
    if (what == VBD_Q_COUNTS) {
        int64_t c[8] = {T->nv, T->nt, T->ns, T->n_colors, T->n_free, (int64_t)T->tet_ent.size(),
                        (int64_t)T->spr_nbr_orig.size(), T->n_meshes};
        return give(c, sizeof(c));
    }
    if (what == VBD_Q_MASS) return give(T->mass.data(), 8 * T->mass.size());
    if (what == VBD_Q_DMINV) return give(T->Dminv.data(), 8 * T->Dminv.size());
    if (what == VBD_Q_VOLUME) return give(T->vol.data(), 8 * T->vol.size());
    if (!T->colored) return fail(VBD_E_NOT_COLORED, "call vbd_color first");
    switch (what) {
    case VBD_Q_COLORS: return give(T->colors.data(), 4 * T->colors.size());
    case VBD_Q_PERM: return give(T->perm.data(), 4 * T->perm.size());
    case VBD_Q_COLOR_OFFSETS: return give(T->color_off.data(), 4 * T->color_off.size());
    case VBD_Q_TET_ROWS: return give(T->tet_row.data(), 4 * T->tet_row.size());
    case VBD_Q_TET_ENTRIES: return give(T->tet_ent.data(), 4 * T->tet_ent.size());
    case VBD_Q_SPRING_ROWS: return give(T->spr_row.data(), 4 * T->spr_row.size());
    case VBD_Q_SPRING_NBRS: return give(T->spr_nbr_orig.data(), 4 * T->spr_nbr_orig.size());
    case VBD_Q_PHASE_BYTES: return give(T->phase_bytes.data(), 8 * T->phase_bytes.size());
    case VBD_Q_ADJ_PHASE_BYTES: return give(T->adj_phase_bytes.data(), 8 * T->adj_phase_bytes.size());
    case VBD_Q_PHASE_COUNTS: {
        std::vector<int64_t> q(4 * (size_t)T->n_colors);
        for (int c = 0; c < T->n_colors; ++c) {
            q[4 * c] = T->phase_cnt[c][0];
            q[4 * c + 1] = T->phase_cnt[c][1];
            q[4 * c + 2] = T->phase_cnt[c][2];
            q[4 * c + 3] = T->phase_updates[c];
        }
        return give(q.data(), 8 * q.size());
    }
    case VBD_Q_TET_ORDER: return give(T->tet_order.data(), 4 * T->tet_order.size());
    case VBD_Q_SURFACE: return give(T->surf.data(), 4 * T->surf.size());
    case VBD_Q_SURFACE_EDGES: return give(T->sedge.data(), 4 * T->sedge.size());
    case VBD_Q_XCD_SPLIT: return give(T->xsplit.data(), 4 * T->xsplit.size());
    case VBD_Q_SURFACE_COUNTS: {
        int64_t c[3] = {(int64_t)(T->surf.size() / 3), (int64_t)T->sv_slot.size(),
                        (int64_t)(T->sedge.size() / 2)};
        return give(c, sizeof(c));
    }
    case VBD_Q_SNAPSHOT_REGION: {
        if (!T->bound) return fail(VBD_E_NO_WORKSPACE, "no workspace bound");
        int64_t c[3] = {(int64_t)T->lay.snaps, (int64_t)(sizeof(float4) * (size_t)T->nv),
                        (int64_t)T->lay.max_bwd_iters};
        if (T->lay.max_bwd_iters <= 0) c[0] = -1;
        return give(c, sizeof(c));
    }
    case VBD_Q_REST_FRAME: {
        std::vector<double> S(6 * (size_t)T->nt);
        for (int t = 0; t < T->nt; ++t) rest_frame_inverse(T->rest, &T->tets[4 * (size_t)t], &S[6 * (size_t)t]);
        return give(S.data(), 8 * S.size());
    }
    default: return fail(VBD_E_INVALID_ARG, "unknown query %d", what);
    }
}

vbd_status vbd_topology_destroy(vbd_topology T)
{
    delete T;
    return VBD_OK;
}

static vbd_status check_ready(vbd_topology T)
{
    if (!T) return fail(VBD_E_INVALID_ARG, "NULL topology");
    if (!T->colored) return fail(VBD_E_NOT_COLORED, "call vbd_color before stepping");
    if (!T->bound) return fail(VBD_E_NO_WORKSPACE, "call vbd_bind_workspace before stepping");
    return VBD_OK;
}

vbd_status vbd_step(vbd_topology T, const vbd_step_params *p, float *x, float *v, float *vp,
                    const float *E, void *stream)
{
    Range range("vbd_step");
    vbd_status st = check_ready(T);
    if (st) return st;
    if ((st = validate_params(*T, p))) return st;
    if (T->nv > 0 && (!x || !v || !vp)) return fail(VBD_E_INVALID_ARG, "state pointer is NULL");
    if (T->nt > 0 && !E) return fail(VBD_E_INVALID_ARG, "tet_E is NULL");
    const StepConsts K = make_consts(*T, p);
    hipStream_t s = (hipStream_t)stream;
    const int mode = p->launch_mode;
    const bool persistent = mode == VBD_LAUNCH_PERSISTENT || mode == VBD_LAUNCH_PERSISTENT_GRAPH;
    if (T->nv == 0) return VBD_OK;
    if (mode == VBD_LAUNCH_PLAIN || mode == VBD_LAUNCH_PERSISTENT || T->profiling)
        return enqueue_step(*T, T->dev, p, K, x, v, vp, E, s, persistent, false);
    // graph modes: capture once per (pointers, parameters, stream), replay after
    return run_graph(*T, T->fwd_graph, make_key(p, {x, v, vp, E}, stream), s, [&](hipStream_t cs) {
        return enqueue_step(*T, T->dev, p, K, x, v, vp, E, cs, persistent, true);
    });
}

vbd_status vbd_step_static(vbd_topology T, const vbd_step_params *p, float *x, float *v, float *vp,
                           const float *E, void *stream)
{
    vbd_status st = check_ready(T);
    if (st) return st;
    if ((st = validate_params(*T, p))) return st;
    if (T->nv > 0 && (!x || !v || !vp)) return fail(VBD_E_INVALID_ARG, "state pointer is NULL");
    if (T->nt > 0 && !E) return fail(VBD_E_INVALID_ARG, "tet_E is NULL");
    const int mode = p->launch_mode;
    if (mode != VBD_LAUNCH_PLAIN && mode != VBD_LAUNCH_PERSISTENT)
        return fail(VBD_E_UNSUPPORTED, "vbd_step_static: launch_mode must be PLAIN or PERSISTENT "
                                       "(graph instantiation allocates)");
    if (p->mesh_contacts)
        return fail(VBD_E_UNSUPPORTED, "vbd_step_static: mesh contacts are not supported");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != T->device)
        return fail(VBD_E_INVALID_ARG, "vbd_step_static: the workspace is bound on device %d, "
                                       "the current device is %d", T->device, dev);
    // the per-step state sections, each 256-B aligned
    const size_t nv = (size_t)T->nv;
    const bool cheb = p->cheb_rho > 0.f;
    const size_t s4 = align_up(sizeof(float4) * nv), need = (cheb ? 5 : 3) * s4 + align_up(nv);
    if (need > kStaticScratchBytes)
        return fail(VBD_E_INVALID_ARG, "vbd_step_static: %d vertices need %zu bytes of state, the "
                                       "static scratch holds %zu (at most %zu vertices%s)", T->nv,
                    need, kStaticScratchBytes,
                    (size_t)((kStaticScratchBytes - 256) / (16 * (cheb ? 5 : 3) + 1)),
                    cheb ? " with acceleration" : "");
    if (T->nv == 0) return VBD_OK;
    void *base = nullptr;
    HIP_TRY(static_scratch(dev, &base));
    char *b = (char *)base;
    DevTopo D = T->dev;
    D.x = (float4 *)b;
    D.xt = (float4 *)(b + s4);
    D.y = (float4 *)(b + 2 * s4);
    D.prev1 = cheb ? (float4 *)(b + 3 * s4) : nullptr;
    D.prev2 = cheb ? (float4 *)(b + 4 * s4) : nullptr;
    D.collided = (unsigned char *)(b + (cheb ? 5 : 3) * s4);
    const StepConsts K = make_consts(*T, p);
    return enqueue_step(*T, D, p, K, x, v, vp, E, (hipStream_t)stream,
                        mode == VBD_LAUNCH_PERSISTENT, false, /*profile=*/false);
}

namespace {
// What the differentiable step supports, and the workspace it needs.
vbd_status check_differentiable(vbd_topology T, const vbd_step_params *p)
{
    vbd_status st = check_ready(T);
    if (st) return st;
    if ((st = validate_params(*T, p))) return st;
    if (T->ns > 0 || p->n_spheres > 0 || p->n_planes > 0 || p->kd != 0.f || p->cheb_rho > 0.f ||
        p->friction_mu > 0.f || p->mesh_contacts)
        return fail(VBD_E_UNSUPPORTED, "backward supports tets, inertia and pins only");
    if (p->n_iters > T->lay.max_bwd_iters)
        return fail(VBD_E_NO_WORKSPACE, "workspace holds %d backward iterations, need %d",
                    T->lay.max_bwd_iters, p->n_iters);
    return VBD_OK;
}
}  // namespace

vbd_status vbd_step_record(vbd_topology T, const vbd_step_params *p, float *x, float *v, float *vp,
                           const float *E, void *stream)
{
    Range range("vbd_step_record");
    vbd_status st = check_differentiable(T, p);
    if (st) return st;
    if (T->nv == 0) return VBD_OK;
    if (!x || !v || !vp || (T->nt > 0 && !E)) return fail(VBD_E_INVALID_ARG, "NULL array");
    const StepConsts K = make_consts(*T, p);
    hipStream_t s = (hipStream_t)stream;
    auto enqueue = [&](hipStream_t q) -> vbd_status {
        vbd_status r = enqueue_record(*T, p, K, x, v, vp, E, q);
        if (r) return r;
        DevTopo D = T->dev;
        D.x = T->dev.snaps + (size_t)T->nv * p->n_iters;
        HIP_TRY(launch_finalize(D, x, v, vp, K, q));
        if (p->check_finite) HIP_TRY(launch_check_finite(x, v, 3 * (long long)T->nv, T->dev.flags, q));
        return VBD_OK;
    };
    if (p->launch_mode == VBD_LAUNCH_PLAIN || p->launch_mode == VBD_LAUNCH_PERSISTENT || T->profiling)
        return enqueue(s);
    return run_graph(*T, T->rec_graph, make_key(p, {x, v, vp, E}, stream), s, enqueue);
}

vbd_status vbd_step_backward(vbd_topology T, const vbd_step_params *p, const float *x_t,
                             const float *v_t, const float *v_prev, const float *E,
                             const float *gx_out, const float *gv_out, const float *gvp_out,
                             float *gx_in, float *gv_in, float *gvp_in, float *g_E, void *stream)
{
    Range range("vbd_step_backward");
    vbd_status st = check_differentiable(T, p);
    if (st) return st;
    if (T->nv == 0) return VBD_OK;
    if (!x_t || !v_t || !v_prev || !gx_out || !gv_out || !gvp_out || !gx_in || !gv_in || !gvp_in ||
        (T->nt > 0 && (!E || !g_E)))
        return fail(VBD_E_INVALID_ARG, "NULL array");
    const StepConsts K = make_consts(*T, p);
    hipStream_t s = (hipStream_t)stream;
    // the sweep starts from zero accumulators; they are left zero by the last
    // backward unless its enqueue stopped part way
    if (!T->bwd_zero) {
        HIP_TRY(zero_bwd_accumulators(*T, s));
        T->bwd_zero = true;
    }
    auto enqueue = [&](hipStream_t q, bool in_capture) {
        return enqueue_backward(*T, p, K, x_t, v_t, v_prev, E, gx_out, gv_out, gvp_out, gx_in, gv_in,
                                gvp_in, g_E, q, in_capture);
    };
    T->bwd_zero = false;
    if (p->launch_mode == VBD_LAUNCH_PLAIN || p->launch_mode == VBD_LAUNCH_PERSISTENT || T->profiling)
        st = enqueue(s, false);
    else
        st = run_graph(*T, T->bwd_graph,
                       make_key(p, {x_t, v_t, v_prev, E, gx_out, gv_out, gvp_out, gx_in, gv_in, gvp_in, g_E},
                                stream),
                       s, [&](hipStream_t q) { return enqueue(q, true); });
    if (st == VBD_OK) T->bwd_zero = true;
    return st;
}

vbd_status vbd_detect_edges(vbd_topology T, const vbd_step_params *p, const float *x,
                            const float *x_t, int32_t *partner_out, void *stream)
{
    Range range("vbd_detect_edges");
    vbd_status st = check_ready(T);
    if (st) return st;
    if ((st = validate_params(*T, p))) return st;
    if (!p->mesh_contacts || !p->edge_contacts)
        return fail(VBD_E_INVALID_ARG, "params->mesh_contacts and edge_contacts must be 1");
    if (T->nv > 0 && (!x || !x_t || (!partner_out && !T->sedge.empty())))
        return fail(VBD_E_INVALID_ARG, "NULL device pointer");
    if (T->nv == 0 || T->sedge.empty()) return VBD_OK;
    const StepConsts K = make_consts(*T, p);
    hipStream_t s = (hipStream_t)stream;
    DevTopo Dt = T->dev;
    Dt.x = T->dev.xt;
    HIP_TRY(launch_load_x(Dt, x_t, s));
    HIP_TRY(launch_load_x(T->dev, x, s));
    HIP_TRY(launch_detect(T->dev, T->surf_dev, T->dev.x, K, s));
    HIP_TRY(launch_store_edge_partners(T->surf_dev, partner_out, s));
    return VBD_OK;
}

vbd_status vbd_detect_contacts(vbd_topology T, const vbd_step_params *p, const float *x,
                               int32_t *tri_out, void *stream)
{
    Range range("vbd_detect_contacts");
    vbd_status st = check_ready(T);
    if (st) return st;
    if ((st = validate_params(*T, p))) return st;
    if (!p->mesh_contacts) return fail(VBD_E_INVALID_ARG, "params->mesh_contacts must be 1");
    if (T->nv > 0 && (!x || !tri_out)) return fail(VBD_E_INVALID_ARG, "NULL device pointer");
    if (T->nv == 0) return VBD_OK;
    const StepConsts K = make_consts(*T, p);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_load_x(T->dev, x, s));
    HIP_TRY(launch_detect(T->dev, T->surf_dev, T->dev.x, K, s));
    HIP_TRY(launch_store_ctri(T->dev, T->surf_dev, tri_out, s));
    return VBD_OK;
}

vbd_status vbd_get_launch_config(vbd_topology T, vbd_launch_config *c)
{
    if (!T || !c) return fail(VBD_E_INVALID_ARG, "NULL argument");
    c->lanes_per_vertex = T->cfg.lanes;
    c->block_size = T->cfg.block;
    c->xcd_remap = T->cfg.xcd_remap;
    c->blocks_per_cu = T->cfg.blocks_per_cu;
    c->tet_unroll = T->cfg.unroll;
    c->compact_records = T->cfg.compact;
    return VBD_OK;
}

vbd_status vbd_set_launch_config(vbd_topology T, const vbd_launch_config *c)
{
    if (!T || !c) return fail(VBD_E_INVALID_ARG, "NULL argument");
    const int L = c->lanes_per_vertex;
    if (L != 2 && L != 4 && L != 8 && L != 16 && L != 32)
        return fail(VBD_E_INVALID_ARG, "lanes_per_vertex must be 2, 4, 8, 16 or 32");
    if (c->block_size < 64 || c->block_size > 512 || c->block_size % 64)
        return fail(VBD_E_INVALID_ARG, "block_size must be a multiple of 64 in [64, 512]");
    if (c->blocks_per_cu < 0) return fail(VBD_E_INVALID_ARG, "blocks_per_cu < 0");
    if (c->tet_unroll < 1 || c->tet_unroll > 3) return fail(VBD_E_INVALID_ARG, "tet_unroll must be 1, 2 or 3");
    if (c->compact_records != 0 && c->compact_records != 1)
        return fail(VBD_E_INVALID_ARG, "compact_records must be 0 or 1");
    if (c->xcd_remap < 0 || c->xcd_remap > 3) return fail(VBD_E_INVALID_ARG, "xcd_remap must be 0, 1, 2 or 3");
    T->cfg = LaunchCfg{L, c->block_size, c->xcd_remap, c->blocks_per_cu, c->tet_unroll,
                       c->compact_records};
    update_phase_bytes(*T);
    T->fwd_graph.reset();
    T->bwd_graph.reset();
    T->rec_graph.reset();
    return VBD_OK;
}

vbd_status vbd_autotune(vbd_topology T, const vbd_step_params *p, const float *x, const float *v,
                        const float *vp, const float *E, void *stream)
{
    Range range("vbd_autotune");
    vbd_status st = check_ready(T);
    if (st) return st;
    if ((st = validate_params(*T, p))) return st;
    const bool persistent = p->launch_mode >= VBD_LAUNCH_PERSISTENT;
    const auto key = std::make_tuple(T->arch, log2_bucket(T->nv), log2_bucket(T->nt),
                                     log2_bucket(T->ns), persistent ? 1 : 0, T->n_colors);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            T->cfg = it->second;
            update_phase_bytes(*T);
            return VBD_OK;
        }
    }
    const StepConsts K = make_consts(*T, p);
    hipStream_t s = (hipStream_t)stream;
    const bool tets = T->nt > 0, springs = T->ns > 0;
    std::vector<LaunchCfg> cands;
    for (int cr : {0, 1}) {
        if (!tets && cr) continue;
        for (int L : {2, 4, 8, 16}) {
            if (tets && L == 2) continue;   // tets: 24 pairs per vertex want more lanes
            for (int U : {1, 2, 3}) {
                if (!tets && U > 1) continue;
                for (int B : {64, 128, 256, 512})
                    for (int rm : {0, 1, 2, 3}) {
                        if (rm == 3 && (T->n_meshes < 2 || persistent)) continue;
                        if (persistent)
                            for (int bpc : {0, 2, 1}) cands.push_back(LaunchCfg{L, B, rm, bpc, U, cr});
                        else
                            cands.push_back(LaunchCfg{L, B, rm, 0, U, cr});
                    }
            }
        }
    }
    // the timed sweeps must not show in the caller's skip counter
    uint32_t saved_skips[2] = {0, 0};
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(saved_skips, T->dev.flags + kFlagSkips, sizeof(saved_skips), hipMemcpyDeviceToHost));
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    const int sweeps = std::max(1, std::min(p->n_iters, 8));
    // one untimed run, then every candidate timed in each of three rounds; a
    // candidate's time is its best round (single timings of launches of a few
    // microseconds spread by several percent)
    constexpr int kRounds = 3;
    std::vector<float> t_best(cands.size(), 1e30f);
    for (int round = -1; round < kRounds; ++round) {
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            if (round < 0 && ci > 0) break;
            if (t_best[ci] < 0.f) continue;   // discarded
            const LaunchCfg &cf = cands[ci];
            HIP_TRY(launch_material(T->dev, E, K, cf.compact != 0, s));
            HIP_TRY(launch_predict(T->dev, x, v, vp, K, true, s));
            HIP_TRY(hipEventRecord(a, s));
            if (persistent) {
                hipError_t e = launch_persistent(T->dev, K, sweeps, tets, springs, cf, T->n_cu, true, s, nullptr);
                if (e != hipSuccess) { (void)hipGetLastError(); t_best[ci] = -1.f; continue; }
            } else {
                for (int it = 0; it < sweeps; ++it)
                    for (int c = 0; c < T->n_colors; ++c)
                        HIP_TRY(launch_solve(T->dev, K, T->color_off[c], T->color_off[c + 1], incidence(*T, c), tets,
                                             springs, cf, s, xcd_split(*T, c)));
            }
            HIP_TRY(hipEventRecord(b, s));
            HIP_TRY(hipEventSynchronize(b));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, a, b));
            if (persistent) {
                // a configuration whose blocks were not all resident trips the
                // barrier guard: discard it and clear the flag
                uint32_t f[2] = {0, 0};
                HIP_TRY(hipMemcpy(f, T->dev.flags, sizeof(f), hipMemcpyDeviceToHost));
                if (f[1] != 0) {
                    HIP_TRY(launch_zero_u32(T->dev.flags + 1, 5, s));
                    HIP_TRY(hipStreamSynchronize(s));
                    t_best[ci] = -1.f;
                    continue;
                }
            }
            if (round >= 0) t_best[ci] = std::min(t_best[ci], ms);
        }
    }
    float best = 1e30f;
    LaunchCfg best_cfg = T->cfg;
    for (size_t ci = 0; ci < cands.size(); ++ci)
        if (t_best[ci] >= 0.f && t_best[ci] < best) {
            best = t_best[ci];
            best_cfg = cands[ci];
        }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(T->dev.flags + kFlagSkips, saved_skips, sizeof(saved_skips), hipMemcpyHostToDevice));
    T->cfg = best_cfg;
    update_phase_bytes(*T);
    T->fwd_graph.reset();
    T->bwd_graph.reset();
    T->rec_graph.reset();
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = best_cfg;
    return VBD_OK;
}

vbd_status vbd_profile_enable(vbd_topology T, int32_t enable)
{
    if (!T) return fail(VBD_E_INVALID_ARG, "NULL topology");
    T->profiling = enable != 0;
    return VBD_OK;
}

vbd_status vbd_profile_read(vbd_topology T, vbd_profile_stats *out, int32_t reset)
{
    if (!T || !out) return fail(VBD_E_INVALID_ARG, "NULL argument");
    for (auto &e : T->events) {
        HIP_TRY(hipEventSynchronize(e.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
        T->acc.n_launches += e.launches;
        T->acc.total_ms += ms;
        T->acc.total_bytes += e.bytes;
        T->acc.n_vertex_updates += e.updates;
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    T->events.clear();
    *out = T->acc;
    if (reset) T->acc = vbd_profile_stats{};
    return VBD_OK;
}

vbd_status vbd_check(vbd_topology T, void *stream)
{
    vbd_status st = check_ready(T);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    uint32_t f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(f, T->dev.flags, sizeof(f), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (f[1] != 0) {
        HIP_TRY(launch_zero_u32(T->dev.flags + 1, 1, s));
        HIP_TRY(launch_zero_u32(T->dev.flags + 3, 3, s));
        HIP_TRY(hipStreamSynchronize(s));
        return fail(VBD_E_DEVICE,
                    "persistent kernel barrier timed out: arrivals seen %u of target %u, grid %u blocks "
                    "(%d CUs)", f[3], f[4], f[5], T->n_cu);
    }
    if (f[kFlagNonfinite] != 0) {
        HIP_TRY(launch_zero_u32(T->dev.flags + kFlagNonfinite, 1, s));
        HIP_TRY(hipStreamSynchronize(s));
        return fail(VBD_E_NONFINITE, "%u non-finite position or velocity values after a step run with "
                    "check_finite", f[kFlagNonfinite]);
    }
    return VBD_OK;
}

vbd_status vbd_read_counters(vbd_topology T, vbd_counters *out, int32_t reset, void *stream)
{
    vbd_status st = check_ready(T);
    if (st) return st;
    if (!out) return fail(VBD_E_INVALID_ARG, "out is NULL");
    hipStream_t s = (hipStream_t)stream;
    uint32_t f[4] = {0, 0, 0, 0};   // flags kFlagNonfinite .. kFlagSkips + 1
    static_assert(kFlagNonfiniteTotal + 1 == kFlagSkips, "counter layout");
    HIP_TRY(hipMemcpyAsync(f, T->dev.flags + kFlagNonfinite, sizeof(f), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->n_skips = (int64_t)((uint64_t)f[2] | ((uint64_t)f[3] << 32));
    out->n_nonfinite = (int64_t)f[1];
    if (reset) {
        HIP_TRY(launch_zero_u32(T->dev.flags + kFlagNonfiniteTotal, 3, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return VBD_OK;
}

vbd_status vbd_probe_copy(void *dst, const void *src, size_t n_bytes, void *stream)
{
    if (!dst || !src || n_bytes % 16) return fail(VBD_E_INVALID_ARG, "bad copy arguments");
    if (n_bytes / 16 > (size_t)INT32_MAX) return fail(VBD_E_INVALID_ARG, "copy too large");
    HIP_TRY(launch_copy4((float4 *)dst, (const float4 *)src, (int)(n_bytes / 16), (hipStream_t)stream));
    return VBD_OK;
}

vbd_status vbd_probe_read(const void *src, size_t n_bytes, float *partials, int32_t n_blocks,
                          void *stream)
{
    if (!src || !partials || n_bytes % 16 || n_blocks < 1 || n_blocks > 65535)
        return fail(VBD_E_INVALID_ARG, "bad read-probe arguments");
    HIP_TRY(launch_read4((const float4 *)src, (long long)(n_bytes / 16), partials, n_blocks,
                         (hipStream_t)stream));
    return VBD_OK;
}

}  // extern "C"
