// Drives the host side of the C ABI (no device needed) for an
// AddressSanitizer / UndefinedBehaviorSanitizer build of the library:
// topology building for tets, springs and batched meshes, the three greedy
// coloring orders and a given coloring, every host query, workspace sizing
// and the argument errors.  Exit status 0 when every call behaved.
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/vbd.h"

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "failed: %s (line %d): %s\n", #c, __LINE__,       \
                         vbd_last_error());                                        \
            return 1;                                                              \
        }                                                                          \
    } while (0)

static void lattice(int n, double x0, std::vector<double> &rest, std::vector<int32_t> &tets)
{
    const int base = (int)rest.size() / 3;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                rest.push_back(x0 + 0.1 * i);
                rest.push_back(0.1 * j);
                rest.push_back(0.1 * k);
            }
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int k = 0; k + 1 < n; ++k)
        for (int j = 0; j + 1 < n; ++j)
            for (int i = 0; i + 1 < n; ++i)
                for (auto &p : perm) {
                    int c[3] = {i, j, k}, id[4];
                    id[0] = c[0] + n * (c[1] + n * c[2]);
                    for (int r = 0; r < 3; ++r) {
                        c[p[r]] += 1;
                        id[r + 1] = c[0] + n * (c[1] + n * c[2]);
                    }
                    const double *a = &rest[3 * (base + id[0])], *b = &rest[3 * (base + id[1])],
                                 *cc = &rest[3 * (base + id[2])], *d = &rest[3 * (base + id[3])];
                    double e1[3], e2[3], e3[3];
                    for (int r = 0; r < 3; ++r) { e1[r] = b[r] - a[r]; e2[r] = cc[r] - a[r]; e3[r] = d[r] - a[r]; }
                    const double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) -
                                       e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                                       e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
                    if (det < 0) std::swap(id[2], id[3]);
                    for (int r = 0; r < 4; ++r) tets.push_back(base + id[r]);
                }
}

static int queries(vbd_topology t)
{
    int64_t counts[8];
    CHECK(vbd_topology_query(t, VBD_Q_COUNTS, counts, sizeof(counts)) == VBD_OK);
    const int64_t nv = counts[0], nt = counts[1], nc = counts[3], nfree = counts[4];
    int64_t sc[3];
    CHECK(vbd_topology_query(t, VBD_Q_SURFACE_COUNTS, sc, sizeof(sc)) == VBD_OK);
    struct Q { int what; size_t bytes; } qs[] = {
        {VBD_Q_COLORS, 4 * (size_t)nv}, {VBD_Q_PERM, 4 * (size_t)nv},
        {VBD_Q_COLOR_OFFSETS, 4 * (size_t)(nc + 1)}, {VBD_Q_TET_ROWS, 4 * (size_t)(nv + 1)},
        {VBD_Q_TET_ENTRIES, 4 * (size_t)counts[5]}, {VBD_Q_SPRING_ROWS, 4 * (size_t)(nfree + 1)},
        {VBD_Q_SPRING_NBRS, 4 * (size_t)counts[6]}, {VBD_Q_MASS, 8 * (size_t)nv},
        {VBD_Q_DMINV, 72 * (size_t)nt}, {VBD_Q_VOLUME, 8 * (size_t)nt},
        {VBD_Q_PHASE_BYTES, 8 * (size_t)nc}, {VBD_Q_TET_ORDER, 4 * (size_t)nt},
        {VBD_Q_REST_FRAME, 48 * (size_t)nt}, {VBD_Q_SURFACE, 12 * (size_t)sc[0]},
        {VBD_Q_ADJ_PHASE_BYTES, 8 * (size_t)nc}, {VBD_Q_PHASE_COUNTS, 32 * (size_t)nc},
        {VBD_Q_SURFACE_EDGES, 8 * (size_t)sc[2]}, {VBD_Q_XCD_SPLIT, 36 * (size_t)nc}};
    for (auto &q : qs) {
        std::vector<unsigned char> buf(q.bytes + 1);
        CHECK(vbd_topology_query(t, q.what, buf.data(), q.bytes) == VBD_OK);
        if (q.bytes > 0) CHECK(vbd_topology_query(t, q.what, buf.data(), q.bytes - 1) == VBD_E_INVALID_ARG);
    }
    size_t ws = 0;
    CHECK(vbd_workspace_size(t, 0, &ws) == VBD_OK && ws > 0);
    CHECK(vbd_workspace_size(t, 20, &ws) == VBD_OK && ws > 0);
    return 0;
}

int main()
{
    // two meshes (batched), lumped masses, the bottom layer pinned
    std::vector<double> rest;
    std::vector<int32_t> tets;
    lattice(4, 0.0, rest, tets);
    const int nv1 = (int)rest.size() / 3, nt1 = (int)tets.size() / 4;
    lattice(3, 1.0, rest, tets);
    const int nv = (int)rest.size() / 3, nt = (int)tets.size() / 4;
    std::vector<uint8_t> pinned(nv, 0);
    for (int v = 0; v < nv; ++v) pinned[v] = rest[3 * v + 2] < 1e-12;
    const int64_t vo[3] = {0, nv1, nv}, to[3] = {0, nt1, nt};
    vbd_mesh_desc d{};
    d.n_verts = nv; d.n_tets = nt; d.n_meshes = 2; d.vert_offsets = vo; d.tet_offsets = to;
    d.tets = tets.data(); d.rest_pos = rest.data(); d.density = 1000.0; d.poisson_nu = 0.3;
    d.pinned = pinned.data();
    for (int order : {VBD_COLOR_ID_ORDER, VBD_COLOR_SMALLEST_LAST, VBD_COLOR_DSATUR}) {
        vbd_topology t = nullptr;
        CHECK(vbd_build_topology(&d, &t) == VBD_OK);
        int32_t nc = 0;
        std::vector<int32_t> colors(nv);
        CHECK(vbd_color_greedy(t, order, &nc, colors.data()) == VBD_OK && nc > 0);
        if (queries(t)) return 1;
        vbd_launch_config c{};
        CHECK(vbd_get_launch_config(t, &c) == VBD_OK);
        c.xcd_remap = 3;
        CHECK(vbd_set_launch_config(t, &c) == VBD_OK);
        c.lanes_per_vertex = 3;
        CHECK(vbd_set_launch_config(t, &c) == VBD_E_INVALID_ARG);
        // a given coloring: valid, then one with a tet of two equal colors
        vbd_topology g = nullptr;
        CHECK(vbd_build_topology(&d, &g) == VBD_OK);
        CHECK(vbd_color_given(g, colors.data()) == VBD_OK);
        if (queries(g)) return 1;
        vbd_topology h = nullptr;
        CHECK(vbd_build_topology(&d, &h) == VBD_OK);
        std::vector<int32_t> bad = colors;
        bad[tets[1]] = bad[tets[0]];
        CHECK(vbd_color_given(h, bad.data()) == VBD_E_INVALID_ARG);
        // stepping without a workspace is refused before any device work
        vbd_step_params p{};
        p.h = 1.f / 60.f; p.n_iters = 1;
        CHECK(vbd_step(g, &p, nullptr, nullptr, nullptr, nullptr, nullptr) == VBD_E_NO_WORKSPACE);
        CHECK(vbd_topology_destroy(t) == VBD_OK);
        CHECK(vbd_topology_destroy(g) == VBD_OK);
        CHECK(vbd_topology_destroy(h) == VBD_OK);
    }
    // springs with given masses and rest lengths, one massless free vertex
    {
        std::vector<double> r = {0, 0, 0, 0.1, 0, 0, 0.2, 0, 0, 0.3, 0, 0};
        std::vector<int32_t> sp = {0, 1, 1, 2, 2, 3};
        std::vector<double> L = {0.1, 0.1, 0.12}, m = {1, 1, 0, 1};
        std::vector<uint8_t> pin = {1, 0, 0, 0};
        vbd_mesh_desc s{};
        s.n_verts = 4; s.n_springs = 3; s.n_meshes = 1; s.springs = sp.data(); s.rest_pos = r.data();
        s.spring_rest = L.data(); s.spring_k = 100.0; s.mass = m.data(); s.density = 1000.0;
        s.poisson_nu = 0.3; s.pinned = pin.data();
        vbd_topology t = nullptr;
        CHECK(vbd_build_topology(&s, &t) == VBD_OK);
        int32_t nc = 0;
        CHECK(vbd_color(t, &nc, nullptr) == VBD_OK && nc == 2);
        if (queries(t)) return 1;
        CHECK(vbd_topology_destroy(t) == VBD_OK);
        m[2] = -1.0;
        CHECK(vbd_build_topology(&s, &t) == VBD_E_INVALID_ARG);
    }
    // argument errors
    {
        vbd_topology t = nullptr;
        vbd_mesh_desc e = d;
        e.poisson_nu = 0.0;
        CHECK(vbd_build_topology(&e, &t) == VBD_E_INVALID_ARG);
        e = d;
        std::vector<int32_t> bt = tets;
        bt[5] = nv + 7;
        e.tets = bt.data();
        CHECK(vbd_build_topology(&e, &t) == VBD_E_TOPOLOGY);
        CHECK(vbd_build_topology(nullptr, &t) == VBD_E_INVALID_ARG);
    }
    std::printf("host driver: %d vertices, %d tets, all calls behaved\n", nv, nt);
    return 0;
}
