/* Drives the FP64 oracle (test infrastructure) through every entry point on
 * small inputs, for an AddressSanitizer / UndefinedBehaviorSanitizer build:
 * two stacked lattice cubes with mesh contacts (vertex-triangle, edge-edge,
 * self-contact), friction, damping, Chebyshev, springs, the coloring orders,
 * the surface, the adjoint and the complex-step build.  Exit status 0 when
 * every call returned success. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/vbd_oracle.h"

static int lattice(int n, double z0, double shift, int base, double *rest, int32_t *tets)
{
    /* n^3 vertices, 6 tets per cell (Kuhn split), vertex id = base + i + n (j + n k) */
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double *p = rest + 3 * (size_t)(i + n * (j + n * k));
                p[0] = 0.1 * i + shift; p[1] = 0.1 * j + 0.5 * shift; p[2] = z0 + 0.1 * k;
            }
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int nt = 0;
    for (int k = 0; k + 1 < n; ++k)
        for (int j = 0; j + 1 < n; ++j)
            for (int i = 0; i + 1 < n; ++i)
                for (int q = 0; q < 6; ++q) {
                    int c[3] = {i, j, k}, id[4];
                    id[0] = c[0] + n * (c[1] + n * c[2]);
                    for (int r = 0; r < 3; ++r) {
                        c[perm[q][r]] += 1;
                        id[r + 1] = c[0] + n * (c[1] + n * c[2]);
                    }
                    /* positive orientation */
                    const double *a = rest + 3 * id[0], *b = rest + 3 * id[1], *cc = rest + 3 * id[2],
                                 *d = rest + 3 * id[3];
                    double e1[3], e2[3], e3[3];
                    for (int r = 0; r < 3; ++r) { e1[r] = b[r] - a[r]; e2[r] = cc[r] - a[r]; e3[r] = d[r] - a[r]; }
                    double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                                 e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
                    if (det < 0) { int t = id[2]; id[2] = id[3]; id[3] = t; }
                    for (int r = 0; r < 4; ++r) tets[4 * nt + r] = base + id[r];
                    ++nt;
                }
    return nt;
}

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

int main(void)
{
    const int n = 4, nv1 = n * n * n, nv = 2 * nv1, nt1 = 6 * (n - 1) * (n - 1) * (n - 1), nt = 2 * nt1;
    double *rest = calloc(3 * (size_t)nv, sizeof(double));
    int32_t *tets = calloc(4 * (size_t)nt, sizeof(int32_t));
    lattice(n, 0.0, 0.0, 0, rest, tets);
    lattice(n, 0.299, 0.033, nv1, rest + 3 * nv1, tets + 4 * nt1);
    double *Dminv = calloc(9 * (size_t)nt, sizeof(double)), *vol = calloc(nt, sizeof(double));
    double *mass = calloc(nv, sizeof(double));
    CHECK(oracle_tet_rest(nt, tets, rest, Dminv, vol) == 0);
    oracle_lumped_mass(nv, nt, tets, vol, 1000.0, mass);
    int32_t *colors = calloc(nv, sizeof(int32_t));
    CHECK(oracle_color_smallest_last(nv, nt, tets, 0, NULL, colors) > 0);
    CHECK(oracle_color_dsatur(nv, nt, tets, 0, NULL, colors) > 0);
    const int nc = oracle_color_greedy(nv, nt, tets, 0, NULL, colors);
    CHECK(nc > 0);
    int32_t *tris = calloc(3 * 4 * (size_t)nt, sizeof(int32_t));
    const int ntri = oracle_surface(nt, tets, rest, tris);
    CHECK(ntri == 2 * 2 * 6 * (n - 1) * (n - 1));
    uint8_t *pinned = calloc(nv, 1);
    for (int v = 0; v < nv1; ++v) pinned[v] = rest[3 * v + 2] < 1e-12;
    int32_t *vmesh = calloc(nv, sizeof(int32_t));
    for (int v = nv1; v < nv; ++v) vmesh[v] = 1;
    oracle_model M = {nv, nt, 0, nc, tets, NULL, Dminv, vol, NULL, mass, pinned, colors, 0.3, 0.0,
                      ntri, tris, vmesh, rest};
    oracle_params P;
    memset(&P, 0, sizeof(P));
    P.h = 1.0 / 60.0; P.n_iters = 6; P.gravity[2] = -9.8; P.init_mode = OR_INIT_ADAPTIVE;
    P.det_eps_rel = 1e-6; P.contact_k = 1e4; P.contact_thickness = 5e-3;
    double plane[4] = {0.0, 0.0, 1.0, -0.01}, sphere[4] = {0.15, 0.15, 0.8, 0.1};
    P.n_planes = 1; P.planes = plane; P.n_spheres = 1; P.spheres = sphere;
    P.kd = 1e-5; P.cheb_rho = 0.5; P.friction_mu = 0.3; P.friction_eps_v = 1e-2;
    P.mesh_contacts = 1; P.collision_radius = 0.02; P.n_col = 2;
    P.self_contact = 1; P.self_exclusion = 0.05; P.edge_contacts = 1;
    double *x = calloc(3 * (size_t)nv, sizeof(double)), *v = calloc(3 * (size_t)nv, sizeof(double));
    double *vp = calloc(3 * (size_t)nv, sizeof(double)), *E = calloc(nt, sizeof(double));
    for (int t = 0; t < nt; ++t) E[t] = 1e5;
    memcpy(x, rest, sizeof(double) * 3 * nv);
    oracle_stats st;
    memset(&st, 0, sizeof(st));
    double *G = calloc((size_t)P.n_iters * nc, sizeof(double));
    CHECK(oracle_step(&M, &P, x, v, vp, E, NULL, G, 1, &st) == 0);
    int32_t *tri_v = calloc(nv, sizeof(int32_t));
    oracle_detect_contacts(&M, &P, x, tri_v);
    int32_t ev[4 * 64];
    double en[3 * 64];
    CHECK(oracle_detect_edges(&M, &P, x, rest, 64, ev, en) >= 0);
    double s, u, g12[12], x12[12] = {0, 0, 0, 1, 0, 0, 0.5, -0.5, 0.001, 0.5, 0.5, 0.001}, nn[3] = {0, 0, -1};
    CHECK(oracle_segment_closest(x12, x12 + 3, x12 + 6, x12 + 9, &s, &u) >= 0.0);
    oracle_edge_element(x12, nn, 1e4, 5e-3, g12);
    double xe12[12];
    for (int i = 0; i < 12; ++i) xe12[i] = x12[i] - 1e-4 * (i % 3 == 0);
    oracle_edge_element_friction(x12, xe12, nn, 1e4, 5e-3, 0.3, 1e-2, 1.0 / 60.0, g12);
    double p0[3] = {0.1, 0.1, 0.5};
    (void)oracle_winding_number(&M, 1, p0, x);
    /* energies, derivatives, predict */
    double *y = calloc(3 * (size_t)nv, sizeof(double)), *grad = calloc(3 * (size_t)nv, sizeof(double));
    oracle_predict(&M, &P, x, v, y);
    (void)oracle_energy_G(&M, &P, x, y, E, grad, NULL);
    double hess[144], gt[12], mu, lam;
    oracle_lame(1e5, 0.3, &mu, &lam);
    double xt12[12];
    for (int k = 0; k < 4; ++k)
        for (int a = 0; a < 3; ++a) xt12[3 * k + a] = rest[3 * tets[k] + a];
    (void)oracle_tet_energy(xt12, Dminv, vol[0], mu, lam);
    oracle_tet_derivs(xt12, Dminv, vol[0], mu, lam, gt, hess);
    /* adjoint (tets, inertia, pins) */
    oracle_params Pa;
    memset(&Pa, 0, sizeof(Pa));
    Pa.h = 1.0 / 60.0; Pa.n_iters = 4; Pa.gravity[2] = -9.8; Pa.init_mode = OR_INIT_ADAPTIVE;
    Pa.det_eps_rel = 1e-6;
    double *gx = calloc(3 * (size_t)nv, sizeof(double)), *gv = calloc(3 * (size_t)nv, sizeof(double));
    double *gvp = calloc(3 * (size_t)nv, sizeof(double)), *gE = calloc(nt, sizeof(double));
    double *ox = calloc(3 * (size_t)nv, sizeof(double)), *ov = calloc(3 * (size_t)nv, sizeof(double));
    double *ovp = calloc(3 * (size_t)nv, sizeof(double));
    for (int i = 0; i < 3 * nv; ++i) gx[i] = 1e-3 * (i % 7);
    CHECK(oracle_step_backward(&M, &Pa, rest, v, vp, E, gx, gv, gvp, ox, ov, ovp, gE) == 0);
    /* complex-step build */
    double _Complex *xc = calloc(3 * (size_t)nv, sizeof(double _Complex));
    double _Complex *vc = calloc(3 * (size_t)nv, sizeof(double _Complex));
    double _Complex *vpc = calloc(3 * (size_t)nv, sizeof(double _Complex));
    double _Complex *Ec = calloc(nt, sizeof(double _Complex));
    for (int i = 0; i < 3 * nv; ++i) xc[i] = rest[i];
    for (int t = 0; t < nt; ++t) Ec[t] = 1e5 + 1e-20 * I;
    CHECK(oracle_step_cs(&M, &Pa, xc, vc, vpc, Ec, NULL, NULL, 0, &st) == 0);
    /* springs */
    int32_t spr[6] = {0, 1, 1, 2, 2, 3};
    double L[3];
    oracle_spring_rest(3, spr, rest, L);
    double gs[6], hs[36];
    (void)oracle_spring_energy(rest, rest + 3, L[0], 100.0);
    oracle_spring_derivs(rest, rest + 3, L[0] * 1.1, 100.0, gs, hs);
    printf("oracle driver: %d colors, %d surface triangles, %lld contacts\n", nc, ntri,
           (long long)st.n_contacts);
    free(rest); free(tets); free(Dminv); free(vol); free(mass); free(colors); free(tris); free(pinned);
    free(vmesh); free(x); free(v); free(vp); free(E); free(G); free(tri_v); free(y); free(grad);
    free(gx); free(gv); free(gvp); free(gE); free(ox); free(ov); free(ovp); free(xc); free(vc); free(vpc);
    free(Ec);
    return 0;
}
