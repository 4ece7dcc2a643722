/* FP64 oracle: element derivatives and the VBD time step (test infrastructure).
 *
 * Compiled twice: with OR_COMPLEX=0 (real, public names) and OR_COMPLEX=1
 * (double complex, names with suffix _cs) for complex-step derivatives.
 * Branches (pivoting, clamps, contact activity, skip test) are decided on real
 * parts so the complex build stays analytic in its inputs.
 *
 * Element derivatives take the textbook route: Psi(F) -> P = dPsi/dF ->
 * d2Psi/dF2 (9x9), contracted with dF/dx_k = m_k (x) I.  No closed-form
 * shortcut is used here.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "vbd_oracle.h"

#if OR_COMPLEX
typedef double _Complex R;
#define RE(a) creal(a)
#define RSQRT(a) csqrt(a)
#define FN(n) n##_cs
#else
typedef double R;
#define RE(a) (a)
#define RSQRT(a) sqrt(a)
#define FN(n) n
#endif

#ifdef _OPENMP
#include <omp.h>
#endif

static const int LC[3][3][3] = {  /* Levi-Civita symbol */
    {{0, 0, 0}, {0, 0, 1}, {0, -1, 0}},
    {{0, 0, -1}, {0, 0, 0}, {1, 0, 0}},
    {{0, 1, 0}, {-1, 0, 0}, {0, 0, 0}},
};

/* ---------------------------------------------------------------------------
 * Stable Neo-Hookean tet without the logarithmic term (Sec. 5, citing Smith
 * et al. 2018):  Psi = mu/2 (tr F^T F - 3) + lam/2 (J - alpha)^2,
 * alpha = 1 + mu/lam, J = det F, F = D_s Dm^{-1}.  Element energy V * Psi.
 * Lame parameters from (E, nu) by the textbook conversion.
 * ------------------------------------------------------------------------- */
static void lame_R(R E, double nu, R *mu, R *lam)
{
    *mu = E / (2.0 * (1.0 + nu));
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

/* m_l = gradient of the barycentric shape function of vertex l:
 * m_1..m_3 = rows of Dm^{-1}, m_0 = -(m_1 + m_2 + m_3), so F = sum_l x_l m_l^T. */
static void shape_grads(const double B[9], double m[4][3])
{
    for (int b = 0; b < 3; ++b) {
        m[1][b] = B[0 * 3 + b];
        m[2][b] = B[1 * 3 + b];
        m[3][b] = B[2 * 3 + b];
        m[0][b] = -(m[1][b] + m[2][b] + m[3][b]);
    }
}

static void tet_F(const R x[4][3], const double B[9], R F[3][3])
{
    /* F = D_s B with D_s = [x1-x0, x2-x0, x3-x0] (columns) */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            R s = 0;
            for (int c = 0; c < 3; ++c) s += (x[c + 1][a] - x[0][a]) * B[c * 3 + b];
            F[a][b] = s;
        }
}

static R det3(const R F[3][3])
{
    R s = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                if (LC[i][j][k]) s += LC[i][j][k] * F[0][i] * F[1][j] * F[2][k];
    return s;
}

/* cofactor matrix: cof_ab = 1/2 eps_acd eps_bef F_ce F_df  (= dJ/dF_ab) */
static void cof3(const R F[3][3], R C[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            R s = 0;
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d) {
                    if (!LC[a][c][d]) continue;
                    for (int e = 0; e < 3; ++e)
                        for (int f = 0; f < 3; ++f)
                            if (LC[b][e][f]) s += 0.5 * LC[a][c][d] * LC[b][e][f] * F[c][e] * F[d][f];
                }
            C[a][b] = s;
        }
}

static R psi_R(const R F[3][3], R mu, R lam)
{
    R alpha = 1.0 + mu / lam;
    R Ic = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Ic += F[a][b] * F[a][b];
    R J = det3(F);
    return 0.5 * mu * (Ic - 3.0) + 0.5 * lam * (J - alpha) * (J - alpha);
}

/* P = dPsi/dF = mu F + lam (J - alpha) cof(F) */
static void P_of_F(const R F[3][3], R mu, R lam, R P[3][3])
{
    R alpha = 1.0 + mu / lam;
    R C[3][3];
    cof3(F, C);
    R J = det3(F);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) P[a][b] = mu * F[a][b] + lam * (J - alpha) * C[a][b];
}

/* D[ab][ce] = d2Psi/dF_ab dF_ce
 *           = mu d_ac d_be + lam cof_ab cof_ce + lam (J-alpha) dcof_ab/dF_ce,
 * dcof_ab/dF_ce = sum_df eps_acd eps_bef F_df. */
static void dPdF(const R F[3][3], R mu, R lam, R D[9][9])
{
    R alpha = 1.0 + mu / lam;
    R C[3][3];
    cof3(F, C);
    R J = det3(F);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c)
                for (int e = 0; e < 3; ++e) {
                    R dc = 0;
                    for (int d = 0; d < 3; ++d)
                        for (int f = 0; f < 3; ++f)
                            if (LC[a][c][d] && LC[b][e][f]) dc += LC[a][c][d] * LC[b][e][f] * F[d][f];
                    R v = lam * C[a][b] * C[c][e] + lam * (J - alpha) * dc;
                    if (a == c && b == e) v += mu;
                    D[a * 3 + b][c * 3 + e] = v;
                }
}

/* gradient dE/dx_k and Hessian block d2E/dx_k dx_l of one tet */
static void tet_grad_k(const R F[3][3], const double m[4][3], double vol, R mu, R lam,
                       int k, R g[3])
{
    R P[3][3];
    P_of_F(F, mu, lam, P);
    for (int c = 0; c < 3; ++c) {
        R s = 0;
        for (int b = 0; b < 3; ++b) s += P[c][b] * m[k][b];
        g[c] = vol * s;
    }
}

static void tet_hess_kl(const R D[9][9], const double m[4][3], double vol, int k, int l,
                        R Hb[3][3])
{
    for (int c = 0; c < 3; ++c)
        for (int e = 0; e < 3; ++e) {
            R s = 0;
            for (int b = 0; b < 3; ++b)
                for (int f = 0; f < 3; ++f) s += D[c * 3 + b][e * 3 + f] * m[k][b] * m[l][f];
            Hb[c][e] = vol * s;
        }
}

/* ---------------------------------------------------------------------------
 * Linear spring E = k/2 (l - L)^2, l = |x_a - x_b| (Sec. 5, Sec. 6.1).
 * dl/dx_a = d/l, d2l/dx_a2 = (I - d d^T / l^2) / l.
 * ------------------------------------------------------------------------- */
static void spring_block(const R xa[3], const R xb[3], double L, double k, int psd, R g[3],
                         R Hb[3][3])
{
    R d[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
    R l = RSQRT(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    R u[3] = {d[0] / l, d[1] / l, d[2] / l};
    for (int a = 0; a < 3; ++a) g[a] = k * (l - L) * u[a];
    /* psd: the block has eigenvalues k (along u) and k (l - L)/l (twice,
     * across u); clamping the latter at 0 is its exact PSD projection */
    R tr = (l - L);
    if (psd && RE(tr) < 0.0) tr = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            R d2l = ((a == b ? 1.0 : 0.0) - u[a] * u[b]) / l;
            Hb[a][b] = k * (u[a] * u[b] + tr * d2l);
        }
}

/* ---------------------------------------------------------------------------
 * Gaussian elimination with partial pivoting on a 3x3 system.  Returns det(A)
 * (product of pivots with the permutation sign); x is valid when det != 0.
 * ------------------------------------------------------------------------- */
static R solve3(const R Ain[3][3], const R bin[3], R x[3])
{
    R A[3][4];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) A[r][c] = Ain[r][c];
        A[r][3] = bin[r];
    }
    R det = 1.0;
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(RE(A[r][col])) > fabs(RE(A[piv][col]))) piv = r;
        if (piv != col) {
            for (int c = 0; c < 4; ++c) { R t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
            det = -det;
        }
        det *= A[col][col];
        if (RE(A[col][col]) == 0.0) { x[0] = x[1] = x[2] = 0; return 0.0; }
        for (int r = col + 1; r < 3; ++r) {
            R fct = A[r][col] / A[col][col];
            for (int c = col; c < 4; ++c) A[r][c] -= fct * A[col][c];
        }
    }
    for (int r = 2; r >= 0; --r) {
        R s = A[r][3];
        for (int c = r + 1; c < 3; ++c) s -= A[r][c] * x[c];
        x[r] = s / A[r][r];
    }
    return det;
}

/* skip rule of Sec. 3.2: |det H| <= eps, with eps = det_eps_rel * ||H||_F^3 */
static int skip_solve(const R H[3][3], R det, double eps_rel)
{
    double fn = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) fn += RE(H[a][b]) * RE(H[a][b]);
    fn = sqrt(fn);
    return fabs(RE(det)) <= eps_rel * fn * fn * fn;
}

/* ---------------------------------------------------------------------------
 * Incidence lists: for each vertex the incident tets (tet, slot) and springs
 * (spring, other end), each in ascending element id.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t *tet_row, *tet_ent;   /* ent = tet*4 + slot */
    int32_t *spr_row, *spr_ent;   /* ent = spring*2 + end */
} Inc;

static void inc_build(const oracle_model *M, Inc *ic)
{
    int nv = M->n_verts;
    ic->tet_row = (int32_t *)calloc((size_t)nv + 1, sizeof(int32_t));
    ic->spr_row = (int32_t *)calloc((size_t)nv + 1, sizeof(int32_t));
    for (int t = 0; t < M->n_tets; ++t)
        for (int s = 0; s < 4; ++s) ic->tet_row[M->tets[t * 4 + s] + 1]++;
    for (int e = 0; e < M->n_springs; ++e)
        for (int s = 0; s < 2; ++s) ic->spr_row[M->springs[e * 2 + s] + 1]++;
    for (int i = 0; i < nv; ++i) {
        ic->tet_row[i + 1] += ic->tet_row[i];
        ic->spr_row[i + 1] += ic->spr_row[i];
    }
    ic->tet_ent = (int32_t *)malloc(sizeof(int32_t) * ((size_t)ic->tet_row[nv] + 1));
    ic->spr_ent = (int32_t *)malloc(sizeof(int32_t) * ((size_t)ic->spr_row[nv] + 1));
    int32_t *fill = (int32_t *)calloc((size_t)nv, sizeof(int32_t));
    for (int t = 0; t < M->n_tets; ++t)
        for (int s = 0; s < 4; ++s) {
            int v = M->tets[t * 4 + s];
            ic->tet_ent[ic->tet_row[v] + fill[v]++] = t * 4 + s;
        }
    memset(fill, 0, sizeof(int32_t) * (size_t)nv);
    for (int e = 0; e < M->n_springs; ++e)
        for (int s = 0; s < 2; ++s) {
            int v = M->springs[e * 2 + s];
            ic->spr_ent[ic->spr_row[v] + fill[v]++] = e * 2 + s;
        }
    free(fill);
}

static void inc_free(Inc *ic)
{
    free(ic->tet_row); free(ic->tet_ent); free(ic->spr_row); free(ic->spr_ent);
}

/* ---------------------------------------------------------------------------
 * Mesh-mesh vertex-triangle contacts (Sec. 3.5).  Closest point on a triangle:
 * the projection onto its plane if that lies inside, otherwise the nearest
 * of the three edge projections (each clamped to its segment).  Region
 * decisions use real parts.
 * ------------------------------------------------------------------------- */
static void closest_point_R(const R p[3], const R a[3], const R b[3], const R c[3], R q[3],
                            R bary[3])
{
    R ab[3], ac[3], n[3];
    for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; }
    n[0] = ab[1] * ac[2] - ab[2] * ac[1];
    n[1] = ab[2] * ac[0] - ab[0] * ac[2];
    n[2] = ab[0] * ac[1] - ab[1] * ac[0];
    R nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    R t = ((p[0] - a[0]) * n[0] + (p[1] - a[1]) * n[1] + (p[2] - a[2]) * n[2]) / nn;
    R q0[3] = {p[0] - t * n[0], p[1] - t * n[1], p[2] - t * n[2]};
    /* barycentric weights by signed sub-triangle areas */
    const R *V[3] = {a, b, c};
    R w[3];
    for (int k = 0; k < 3; ++k) {
        const R *u = V[(k + 1) % 3], *v = V[(k + 2) % 3];
        R e1[3] = {u[0] - q0[0], u[1] - q0[1], u[2] - q0[2]};
        R e2[3] = {v[0] - q0[0], v[1] - q0[1], v[2] - q0[2]};
        R cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        w[k] = (cr[0] * n[0] + cr[1] * n[1] + cr[2] * n[2]) / nn;
    }
    if (RE(w[0]) >= 0.0 && RE(w[1]) >= 0.0 && RE(w[2]) >= 0.0) {
        for (int k = 0; k < 3; ++k) { q[k] = q0[k]; bary[k] = w[k]; }
        return;
    }
    double best = -1.0;
    for (int e = 0; e < 3; ++e) {
        const int i0 = e, i1 = (e + 1) % 3;
        const R *u = V[i0], *v = V[i1];
        R d[3] = {v[0] - u[0], v[1] - u[1], v[2] - u[2]};
        R sn = ((p[0] - u[0]) * d[0] + (p[1] - u[1]) * d[1] + (p[2] - u[2]) * d[2]) /
               (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (RE(sn) < 0.0) sn = 0.0;
        if (RE(sn) > 1.0) sn = 1.0;
        R c0[3] = {u[0] + sn * d[0], u[1] + sn * d[1], u[2] + sn * d[2]};
        double dd = 0.0;
        for (int k = 0; k < 3; ++k) dd += RE(p[k] - c0[k]) * RE(p[k] - c0[k]);
        if (best < 0.0 || dd < best) {
            best = dd;
            for (int k = 0; k < 3; ++k) { q[k] = c0[k]; bary[k] = 0.0; }
            bary[i0] = 1.0 - sn;
            bary[i1] = sn;
        }
    }
}

static void tri_normal_R(const R a[3], const R b[3], const R c[3], R n[3])
{
    R ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, ac[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    n[0] = ab[1] * ac[2] - ab[2] * ac[1];
    n[1] = ab[2] * ac[0] - ab[0] * ac[2];
    n[2] = ab[0] * ac[1] - ab[1] * ac[0];
    R l = RSQRT(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int k = 0; k < 3; ++k) n[k] /= l;
}

/* Closest points of the segments p0 + s (p1 - p0) and q0 + u (q1 - q0),
 * s, u in [0, 1]: the minimum of |p0 - q0 + s d1 - u d2|^2 over the unit
 * square is its stationary point when that lies inside and the segments are
 * not parallel, else it lies on one of the square's four sides, where the
 * minimisation is one-dimensional (solve, then clamp to [0, 1]).  Every
 * candidate is evaluated and the smallest distance wins (ties: the first in
 * the order interior, s = 0, s = 1, u = 0, u = 1).  Decisions on real parts. */
static double segment_closest_R(const R p0[3], const R p1[3], const R q0[3], const R q1[3], R *s_out,
                                R *u_out)
{
    R d1[3], d2[3], r[3];
    for (int k = 0; k < 3; ++k) { d1[k] = p1[k] - p0[k]; d2[k] = q1[k] - q0[k]; r[k] = p0[k] - q0[k]; }
    R a = 0, b = 0, c = 0, d = 0, e = 0;
    for (int k = 0; k < 3; ++k) {
        a += d1[k] * d1[k]; b += d1[k] * d2[k]; c += d2[k] * d2[k];
        d += d1[k] * r[k]; e += d2[k] * r[k];
    }
    R cs[5], cu[5];
    int nc = 0;
    const R den = a * c - b * b;
    if (RE(den) > 1e-14 * RE(a) * RE(c)) {
        const R s = (b * e - c * d) / den, u = (a * e - b * d) / den;
        if (RE(s) >= 0.0 && RE(s) <= 1.0 && RE(u) >= 0.0 && RE(u) <= 1.0) { cs[nc] = s; cu[nc] = u; ++nc; }
    }
    for (int side = 0; side < 2; ++side) {       /* s fixed at 0 or 1 */
        R u = (b * (double)side + e) / c;
        if (RE(u) < 0.0) u = 0.0;
        if (RE(u) > 1.0) u = 1.0;
        cs[nc] = (double)side; cu[nc] = u; ++nc;
    }
    for (int side = 0; side < 2; ++side) {       /* u fixed at 0 or 1 */
        R s = (b * (double)side - d) / a;
        if (RE(s) < 0.0) s = 0.0;
        if (RE(s) > 1.0) s = 1.0;
        cs[nc] = s; cu[nc] = (double)side; ++nc;
    }
    double best = -1.0;
    for (int k = 0; k < nc; ++k) {
        double dd = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double w = RE(r[j]) + RE(cs[k]) * RE(d1[j]) - RE(cu[k]) * RE(d2[j]);
            dd += w * w;
        }
        if (best < 0.0 || dd < best) { best = dd; *s_out = cs[k]; *u_out = cu[k]; }
    }
    return sqrt(best);
}

/* Edge-edge pairs (Sec. 3.5, Fig. CollisionPotential) are kept only when the
 * closest points are interior to both segments (at an end point the pair is
 * a vertex-triangle contact of that end point) and the edges are not nearly
 * parallel (sine of their angle at least EE_MIN_SIN: for parallel edges the
 * closest points are not unique). */
#define EE_MIN_SIN 0.1

typedef struct {
    int32_t *tri;          /* [n_verts] contact triangle of a surface vertex or -1 */
    int32_t *crow, *cent;  /* corner incidence: vertices whose contact triangle uses v */
    int32_t n_ee;          /* edge-edge elements */
    int32_t *ee;           /* [n_ee*4]: first edge a, b, second edge a, b */
    double *ee_n;          /* [n_ee*3]: fixed normal, from the second edge to the first */
    int32_t *erow, *eent;  /* per vertex: the elements it belongs to (ascending) */
} Contacts;

static int cmp_i64(const void *a, const void *b)
{
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Surface edges: the distinct vertex pairs (a < b) of the surface triangles,
 * in ascending (a, b) order.  Returns the count; *out holds 2 ids per edge. */
static int surface_edges(const oracle_model *M, int32_t **out)
{
    const int nt = M->n_surf_tris;
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (3 * (size_t)nt + 1));
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            int64_t a = M->surf_tris[3 * t + k], b = M->surf_tris[3 * t + (k + 1) % 3];
            if (a > b) { int64_t w = a; a = b; b = w; }
            key[3 * t + k] = (a << 32) | b;
        }
    qsort(key, 3 * (size_t)nt, sizeof(int64_t), cmp_i64);
    int n = 0;
    for (int i = 0; i < 3 * nt; ++i)
        if (i == 0 || key[i] != key[i - 1]) key[n++] = key[i];
    *out = (int32_t *)malloc(sizeof(int32_t) * (2 * (size_t)n + 1));
    for (int i = 0; i < n; ++i) {
        (*out)[2 * i] = (int32_t)(key[i] >> 32);
        (*out)[2 * i + 1] = (int32_t)(key[i] & 0xffffffff);
    }
    free(key);
    return n;
}

static int mesh_of(const oracle_model *M, int v) { return M->vert_mesh ? M->vert_mesh[v] : 0; }

/* Self-contact eligibility (Sec. 3.5 self-collisions): two primitives of one
 * mesh may collide when they share no vertex and lie farther apart than
 * self_exclusion in the rest shape (closer ones are neighbours of the
 * material, not contacts). */
static int self_pair_vt(const oracle_model *M, const oracle_params *P, int v, const int32_t *T)
{
    if (!P->self_contact || !M->rest_pos) return 0;
    if (T[0] == v || T[1] == v || T[2] == v) return 0;
    R pv[3], a[3], b[3], c[3], q[3], bary[3];
    for (int k = 0; k < 3; ++k) {
        pv[k] = M->rest_pos[3 * v + k];
        a[k] = M->rest_pos[3 * T[0] + k];
        b[k] = M->rest_pos[3 * T[1] + k];
        c[k] = M->rest_pos[3 * T[2] + k];
    }
    closest_point_R(pv, a, b, c, q, bary);
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) d2 += RE(pv[k] - q[k]) * RE(pv[k] - q[k]);
    return sqrt(d2) > P->self_exclusion;
}

static int self_pair_ee(const oracle_model *M, const oracle_params *P, const int32_t *e1,
                        const int32_t *e2)
{
    if (!P->self_contact || !M->rest_pos) return 0;
    if (e1[0] == e2[0] || e1[0] == e2[1] || e1[1] == e2[0] || e1[1] == e2[1]) return 0;
    R a0[3], a1[3], b0[3], b1[3], s, u;
    for (int k = 0; k < 3; ++k) {
        a0[k] = M->rest_pos[3 * e1[0] + k];
        a1[k] = M->rest_pos[3 * e1[1] + k];
        b0[k] = M->rest_pos[3 * e2[0] + k];
        b1[k] = M->rest_pos[3 * e2[1] + k];
    }
    return segment_closest_R(a0, a1, b0, b1, &s, &u) > P->self_exclusion;
}


/* detection: for each surface vertex, the closest surface triangle of another
 * mesh within collision_radius whose outward side is closer than delta */
/* generalized winding number of the closed surface of mesh `mesh` at p:
 * sum of the signed solid angles of its triangles over 4 pi (Van Oosterom and
 * Strackee's formula for the solid angle of a triangle); 1 inside, 0 outside
 * for outward-oriented triangles. */
static double winding_number(const oracle_model *M, int mesh, const double p[3], const R *x)
{
    double w = 0.0;
    for (int t = 0; t < M->n_surf_tris; ++t) {
        const int32_t *T = M->surf_tris + 3 * t;
        if ((M->vert_mesh ? M->vert_mesh[T[0]] : 0) != mesh) continue;
        double a[3], b[3], c[3];
        for (int k = 0; k < 3; ++k) {
            a[k] = RE(x[3 * T[0] + k]) - p[k];
            b[k] = RE(x[3 * T[1] + k]) - p[k];
            c[k] = RE(x[3 * T[2] + k]) - p[k];
        }
        const double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        const double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        const double lc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        const double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                           a[2] * (b[0] * c[1] - b[1] * c[0]);
        const double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
        const double ac = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
        const double bc = b[0] * c[0] + b[1] * c[1] + b[2] * c[2];
        w += 2.0 * atan2(det, la * lb * lc + ab * lc + ac * lb + bc * la);
    }
    return w / (4.0 * 3.14159265358979323846);
}

/* discrete detection (Sec. 3.5): for each surface vertex, the closest surface
 * triangle of any other mesh (and, with self-contact, of its own mesh when
 * eligible) within collision_radius (ties: lower index); the pair is a
 * contact when the vertex has penetrated that other mesh (winding number
 * above 1/2) or lies closer than the contact thickness to its surface; for a
 * triangle of its own mesh, when the element is active (d > 0). */
static void detect_R(const oracle_model *M, const oracle_params *P, const R *x, int32_t *tri_out)
{
    const int nv = M->n_verts;
    uint8_t *on_surf = (uint8_t *)calloc((size_t)nv + 1, 1);
    for (int t = 0; t < M->n_surf_tris; ++t)
        for (int k = 0; k < 3; ++k) on_surf[M->surf_tris[3 * t + k]] = 1;
    for (int v = 0; v < nv; ++v) {
        tri_out[v] = -1;
        if (!on_surf[v]) continue;
        const int mv = M->vert_mesh ? M->vert_mesh[v] : 0;
        double best = 0.0;
        int bt = -1;
        for (int t = 0; t < M->n_surf_tris; ++t) {
            const int32_t *T = M->surf_tris + 3 * t;
            if (mesh_of(M, T[0]) == mv && !self_pair_vt(M, P, v, T)) continue;
            R q[3], bary[3];
            closest_point_R(x + 3 * v, x + 3 * T[0], x + 3 * T[1], x + 3 * T[2], q, bary);
            double dist = 0.0;
            for (int k = 0; k < 3; ++k) dist += RE(x[3 * v + k] - q[k]) * RE(x[3 * v + k] - q[k]);
            dist = sqrt(dist);
            if (!(dist < P->collision_radius)) continue;
            if (bt < 0 || dist < best) { best = dist; bt = t; }
        }
        if (bt < 0) continue;
        const double p[3] = {RE(x[3 * v]), RE(x[3 * v + 1]), RE(x[3 * v + 2])};
        const int32_t *B = M->surf_tris + 3 * bt;
        const int mb = mesh_of(M, B[0]);
        if (mb != mv) {
            if (best < P->contact_thickness || winding_number(M, mb, p, x) > 0.5) tri_out[v] = bt;
        } else {
            /* own mesh: the element's own activity test, d = delta - (p - q).n > 0
             * (closer than delta in front of the triangle, or behind it) */
            R q[3], bary[3], n[3];
            closest_point_R(x + 3 * v, x + 3 * B[0], x + 3 * B[1], x + 3 * B[2], q, bary);
            tri_normal_R(x + 3 * B[0], x + 3 * B[1], x + 3 * B[2], n);
            double dn = 0.0;
            for (int k = 0; k < 3; ++k) dn += (p[k] - RE(q[k])) * RE(n[k]);
            if (P->contact_thickness - dn > 0.0) tri_out[v] = bt;
        }
    }
    free(on_surf);
}

static void contacts_index(const oracle_model *M, Contacts *C)
{
    const int nv = M->n_verts;
    free(C->crow); free(C->cent);
    C->crow = (int32_t *)calloc((size_t)nv + 1, sizeof(int32_t));
    for (int v = 0; v < nv; ++v)
        if (C->tri[v] >= 0)
            for (int k = 0; k < 3; ++k) C->crow[M->surf_tris[3 * C->tri[v] + k] + 1]++;
    for (int v = 0; v < nv; ++v) C->crow[v + 1] += C->crow[v];
    C->cent = (int32_t *)malloc(sizeof(int32_t) * ((size_t)C->crow[nv] + 1));
    int32_t *fill = (int32_t *)calloc((size_t)nv + 1, sizeof(int32_t));
    for (int v = 0; v < nv; ++v)
        if (C->tri[v] >= 0)
            for (int k = 0; k < 3; ++k) {
                const int c = M->surf_tris[3 * C->tri[v] + k];
                C->cent[C->crow[c] + fill[c]++] = v;
            }
    free(fill);
}

/* Edge-edge detection (Sec. 3.5): for each surface edge e1, the closest
 * eligible surface edge e2 (another mesh, or its own mesh under the
 * self-contact rule) within collision_radius (ties: lower index).  The pair
 * becomes an element when its closest points are interior to both edges, the
 * edges are not nearly parallel (EE_MIN_SIN) and the element is active,
 * d = delta - (x_a - x_b).n > 0, with n the unit direction from x_b to x_a at
 * x^t (closest-point parameters of x, positions of x^t: the side each edge
 * was on before the step's motion; the paper's edge-edge normal is the
 * direction between the two contact points).  A pair found from both of its
 * edges is kept once, from the edge with the lower index. */
static void detect_ee(const oracle_model *M, const oracle_params *P, const R *x, const R *xt,
                      Contacts *C)
{
    free(C->ee); free(C->ee_n);
    C->ee = NULL; C->ee_n = NULL; C->n_ee = 0;
    int32_t *E = NULL;
    const int ne = surface_edges(M, &E);
    int32_t *best = (int32_t *)malloc(sizeof(int32_t) * ((size_t)ne + 1));
    double *bn = (double *)malloc(sizeof(double) * (3 * (size_t)ne + 1));
    for (int e1 = 0; e1 < ne; ++e1) {
        best[e1] = -1;
        const int32_t *A = E + 2 * e1;
        const int ma = mesh_of(M, A[0]);
        double bd = 0.0;
        int b = -1;
        for (int e2 = 0; e2 < ne; ++e2) {
            if (e2 == e1) continue;
            const int32_t *B = E + 2 * e2;
            if (mesh_of(M, B[0]) == ma && !self_pair_ee(M, P, A, B)) continue;
            R s, u;
            const double dist = segment_closest_R(x + 3 * A[0], x + 3 * A[1], x + 3 * B[0], x + 3 * B[1], &s, &u);
            if (!(dist < P->collision_radius)) continue;
            if (b < 0 || dist < bd) { bd = dist; b = e2; }
        }
        if (b < 0) continue;
        const int32_t *B = E + 2 * b;
        R s, u;
        segment_closest_R(x + 3 * A[0], x + 3 * A[1], x + 3 * B[0], x + 3 * B[1], &s, &u);
        if (!(RE(s) > 0.0 && RE(s) < 1.0 && RE(u) > 0.0 && RE(u) < 1.0)) continue;
        double d1[3], d2[3];
        for (int k = 0; k < 3; ++k) {
            d1[k] = RE(x[3 * A[1] + k] - x[3 * A[0] + k]);
            d2[k] = RE(x[3 * B[1] + k] - x[3 * B[0] + k]);
        }
        const double cr[3] = {d1[1] * d2[2] - d1[2] * d2[1], d1[2] * d2[0] - d1[0] * d2[2],
                              d1[0] * d2[1] - d1[1] * d2[0]};
        const double l1 = sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);
        const double l2 = sqrt(d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2]);
        if (!(sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]) >= EE_MIN_SIN * l1 * l2)) continue;
        double w[3], wl = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double xa = RE(xt[3 * A[0] + k]) + RE(s) * RE(xt[3 * A[1] + k] - xt[3 * A[0] + k]);
            const double xb = RE(xt[3 * B[0] + k]) + RE(u) * RE(xt[3 * B[1] + k] - xt[3 * B[0] + k]);
            w[k] = xa - xb;
            wl += w[k] * w[k];
        }
        wl = sqrt(wl);
        if (!(wl > 0.0)) continue;
        double gap = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double xa = RE(x[3 * A[0] + k] + s * (x[3 * A[1] + k] - x[3 * A[0] + k]));
            const double xb = RE(x[3 * B[0] + k] + u * (x[3 * B[1] + k] - x[3 * B[0] + k]));
            gap += (xa - xb) * w[k] / wl;
        }
        if (!(P->contact_thickness - gap > 0.0)) continue;
        best[e1] = b;
        for (int k = 0; k < 3; ++k) bn[3 * e1 + k] = w[k] / wl;
    }
    int n = 0;
    for (int e1 = 0; e1 < ne; ++e1)
        if (best[e1] >= 0 && !(best[best[e1]] == e1 && best[e1] < e1)) ++n;
    C->ee = (int32_t *)malloc(sizeof(int32_t) * (4 * (size_t)n + 1));
    C->ee_n = (double *)malloc(sizeof(double) * (3 * (size_t)n + 1));
    n = 0;
    for (int e1 = 0; e1 < ne; ++e1) {
        const int e2 = best[e1];
        if (e2 < 0 || (best[e2] == e1 && e2 < e1)) continue;
        C->ee[4 * n] = E[2 * e1];
        C->ee[4 * n + 1] = E[2 * e1 + 1];
        C->ee[4 * n + 2] = E[2 * e2];
        C->ee[4 * n + 3] = E[2 * e2 + 1];
        for (int k = 0; k < 3; ++k) C->ee_n[3 * n + k] = bn[3 * e1 + k];
        ++n;
    }
    C->n_ee = n;
    free(best); free(bn); free(E);
}

/* per vertex, the edge-edge elements it belongs to, ascending */
static void ee_index(const oracle_model *M, Contacts *C)
{
    const int nv = M->n_verts;
    free(C->erow); free(C->eent);
    C->erow = (int32_t *)calloc((size_t)nv + 1, sizeof(int32_t));
    for (int e = 0; e < C->n_ee; ++e)
        for (int k = 0; k < 4; ++k) C->erow[C->ee[4 * e + k] + 1]++;
    for (int v = 0; v < nv; ++v) C->erow[v + 1] += C->erow[v];
    C->eent = (int32_t *)malloc(sizeof(int32_t) * ((size_t)C->erow[nv] + 1));
    int32_t *fill = (int32_t *)calloc((size_t)nv + 1, sizeof(int32_t));
    for (int e = 0; e < C->n_ee; ++e)
        for (int k = 0; k < 4; ++k) {
            const int v = C->ee[4 * e + k];
            C->eent[C->erow[v] + fill[v]++] = e;
        }
    free(fill);
}

/* one edge-edge element seen from its vertex `role` (0, 1: the first edge's
 * ends, 2, 3: the second's).  E = 1/2 k_c d^2 with d = delta - (x_a - x_b).n,
 * x_a = x0 + s (x1 - x0), x_b = x2 + u (x3 - x2) at the closest points of the
 * current positions, n fixed (Sec. 3.5); s, u and n held fixed in the
 * derivatives: dd/dx0 = -(1 - s) n, dd/dx1 = -s n, dd/dx2 = (1 - u) n,
 * dd/dx3 = u n.  IPC-style friction on (x_a - x_a^t) - (x_b - x_b^t) with the
 * same weights (Sec. 3.6). */
static int ee_contact(const oracle_params *P, const R *xv[4], const R *xvt[4], const double n[3],
                      int role, R f[3], R H[3][3])
{
    R s, u;
    segment_closest_R(xv[0], xv[1], xv[2], xv[3], &s, &u);
    R xa[3], xb[3];
    for (int k = 0; k < 3; ++k) {
        xa[k] = xv[0][k] + s * (xv[1][k] - xv[0][k]);
        xb[k] = xv[2][k] + u * (xv[3][k] - xv[2][k]);
    }
    R d = P->contact_thickness;
    for (int k = 0; k < 3; ++k) d -= (xa[k] - xb[k]) * n[k];
    if (!(RE(d) > 0.0)) return 0;
    const R g = role == 0 ? -(1.0 - s) : (role == 1 ? -s : (role == 2 ? 1.0 - u : u));
    for (int a = 0; a < 3; ++a) {
        f[a] -= P->contact_k * d * g * n[a];
        for (int b = 0; b < 3; ++b) H[a][b] += P->contact_k * g * g * n[a] * n[b];
    }
    if (P->friction_mu > 0.0) {
        R dx[3];
        for (int a = 0; a < 3; ++a) {
            const R xat = xvt[0][a] + s * (xvt[1][a] - xvt[0][a]);
            const R xbt = xvt[2][a] + u * (xvt[3][a] - xvt[2][a]);
            dx[a] = (xa[a] - xat) - (xb[a] - xbt);
        }
        R dn = dx[0] * n[0] + dx[1] * n[1] + dx[2] * n[2];
        R uu[3] = {dx[0] - dn * n[0], dx[1] - dn * n[1], dx[2] - dn * n[2]};
        R un = RSQRT(uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]);
        double hev = P->h * P->friction_eps_v;
        R f1u = (RE(un) < hev) ? (2.0 / hev - un / (hev * hev)) : (1.0 / un);
        R sf = P->friction_mu * P->contact_k * d * f1u;
        for (int a = 0; a < 3; ++a) {
            f[a] += sf * g * uu[a];
            for (int b = 0; b < 3; ++b) H[a][b] += sf * g * g * ((a == b ? 1.0 : 0.0) - n[a] * n[b]);
        }
    }
    return 1;
}

/* one vertex-triangle element seen from vertex `role` (-1: the colliding
 * vertex a, 0..2: that corner of the triangle).  E = 1/2 k_c d^2 with
 * d = delta - (x_a - x_b).n, x_b = closest point, n and the barycentric
 * weights held fixed (Sec. 3.5); IPC-style friction with the relative
 * displacement (x_a - x_a^t) - sum_k beta_k (x_k - x_k^t) (Sec. 3.6). */
static int vt_contact(const oracle_params *P, const R xa[3], const R *xc[3], const R xat[3],
                      const R *xct[3], int role, R f[3], R H[3][3])
{
    R q[3], bary[3], n[3];
    closest_point_R(xa, xc[0], xc[1], xc[2], q, bary);
    tri_normal_R(xc[0], xc[1], xc[2], n);
    R d = P->contact_thickness - ((xa[0] - q[0]) * n[0] + (xa[1] - q[1]) * n[1] + (xa[2] - q[2]) * n[2]);
    if (!(RE(d) > 0.0)) return 0;
    /* dd/dx_a = -n, dd/dx_j = beta_j n */
    R g = (role < 0) ? -1.0 : bary[role];
    for (int a = 0; a < 3; ++a) {
        f[a] -= P->contact_k * d * g * n[a];
        for (int b = 0; b < 3; ++b) H[a][b] += P->contact_k * g * g * n[a] * n[b];
    }
    if (P->friction_mu > 0.0) {
        R dx[3];
        for (int a = 0; a < 3; ++a)
            dx[a] = (xa[a] - xat[a]) - (bary[0] * (xc[0][a] - xct[0][a]) + bary[1] * (xc[1][a] - xct[1][a]) +
                                        bary[2] * (xc[2][a] - xct[2][a]));
        R dn = dx[0] * n[0] + dx[1] * n[1] + dx[2] * n[2];
        R u[3] = {dx[0] - dn * n[0], dx[1] - dn * n[1], dx[2] - dn * n[2]};
        R un = RSQRT(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double hev = P->h * P->friction_eps_v;
        R f1u = (RE(un) < hev) ? (2.0 / hev - un / (hev * hev)) : (1.0 / un);
        R s = P->friction_mu * P->contact_k * d * f1u;
        /* d(dx)/dx_role = -g I  (a: +I) */
        for (int a = 0; a < 3; ++a) {
            f[a] += s * g * u[a];
            for (int b = 0; b < 3; ++b) H[a][b] += s * g * g * ((a == b ? 1.0 : 0.0) - n[a] * n[b]);
        }
    }
    return 1;
}

/* ---------------------------------------------------------------------------
 * Local system of vertex i (Eq. VBDForce / VBDHessian, damping Eq.
 * VBDForceWithDamping / VBDHessianWithDamping on material elements,
 * penalty contact Eq. collisionEnergy with the normal held fixed, IPC-style
 * friction Eq. IPC_friction with the approximate Hessian).
 * xi_over: optional replacement of x_i (used to evaluate after an update).
 * ------------------------------------------------------------------------- */
static void local_system(const oracle_model *M, const oracle_params *P, const Inc *ic,
                         const Contacts *CT, int i, const R *x, const R *xi_over, const R *y,
                         const R *xt, const R *E, R f[3], R H[3][3], int *in_contact)
{
    const double h = P->h;
    const double mh2 = M->mass[i] / (h * h);
    R xi[3];
    for (int a = 0; a < 3; ++a) xi[a] = xi_over ? xi_over[a] : x[3 * i + a];
    for (int a = 0; a < 3; ++a) {
        f[a] = -mh2 * (xi[a] - y[3 * i + a]);
        for (int b = 0; b < 3; ++b) H[a][b] = (a == b) ? mh2 : 0.0;
    }
    const double kdh = P->kd / h;
    for (int e = ic->tet_row[i]; e < ic->tet_row[i + 1]; ++e) {
        int t = ic->tet_ent[e] >> 2, k = ic->tet_ent[e] & 3;
        R xl[4][3];
        for (int l = 0; l < 4; ++l) {
            int vl = M->tets[t * 4 + l];
            for (int a = 0; a < 3; ++a) xl[l][a] = (vl == i) ? xi[a] : x[3 * vl + a];
        }
        double m[4][3];
        shape_grads(M->Dminv + 9 * t, m);
        R F[3][3], D[9][9], g[3], Hb[3][3], mu, lam;
        lame_R(E[t], M->nu, &mu, &lam);
        tet_F((const R(*)[3])xl, M->Dminv + 9 * t, F);
        tet_grad_k((const R(*)[3])F, (const double(*)[3])m, M->vol[t], mu, lam, k, g);
        dPdF((const R(*)[3])F, mu, lam, D);
        tet_hess_kl((const R(*)[9])D, (const double(*)[3])m, M->vol[t], k, k, Hb);
        for (int a = 0; a < 3; ++a) {
            f[a] -= g[a];
            for (int b = 0; b < 3; ++b) H[a][b] += Hb[a][b];
        }
        if (P->kd != 0.0) {
            for (int a = 0; a < 3; ++a) {
                R s = 0;
                for (int b = 0; b < 3; ++b) s += Hb[a][b] * (xi[b] - xt[3 * i + b]);
                f[a] -= kdh * s;
            }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) H[a][b] += kdh * Hb[a][b];
        }
    }
    for (int e = ic->spr_row[i]; e < ic->spr_row[i + 1]; ++e) {
        int s = ic->spr_ent[e] >> 1, end = ic->spr_ent[e] & 1;
        int o = M->springs[2 * s + (1 - end)];
        R xo[3] = {x[3 * o], x[3 * o + 1], x[3 * o + 2]};
        R g[3], Hb[3][3];
        spring_block(xi, xo, M->spring_rest[s], M->spring_k, P->spring_psd, g, Hb);
        for (int a = 0; a < 3; ++a) {
            f[a] -= g[a];
            for (int b = 0; b < 3; ++b) H[a][b] += Hb[a][b];
        }
        if (P->kd != 0.0) {
            for (int a = 0; a < 3; ++a) {
                R sm = 0;
                for (int b = 0; b < 3; ++b) sm += Hb[a][b] * (xi[b] - xt[3 * i + b]);
                f[a] -= kdh * sm;
            }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) H[a][b] += kdh * Hb[a][b];
        }
    }
    /* mesh-mesh vertex-triangle contacts, at the current iterate */
    if (CT) {
        if (CT->tri[i] >= 0) {
            const int32_t *T = M->surf_tris + 3 * CT->tri[i];
            const R *xc[3] = {x + 3 * T[0], x + 3 * T[1], x + 3 * T[2]};
            const R *xct[3] = {xt + 3 * T[0], xt + 3 * T[1], xt + 3 * T[2]};
            if (vt_contact(P, xi, xc, xt + 3 * i, xct, -1, f, H)) *in_contact = 1;
        }
        for (int e = CT->crow[i]; e < CT->crow[i + 1]; ++e) {
            const int a = CT->cent[e];
            const int32_t *T = M->surf_tris + 3 * CT->tri[a];
            int role = 0;
            while (T[role] != i) ++role;
            const R *xc[3], *xct[3];
            for (int k = 0; k < 3; ++k) {
                xc[k] = (k == role) ? xi : x + 3 * T[k];
                xct[k] = xt + 3 * T[k];
            }
            if (vt_contact(P, x + 3 * a, xc, xt + 3 * a, xct, role, f, H)) *in_contact = 1;
        }
        for (int e = CT->erow ? CT->erow[i] : 0; CT->erow && e < CT->erow[i + 1]; ++e) {
            const int el = CT->eent[e];
            const int32_t *V4 = CT->ee + 4 * el;
            const R *xv[4], *xvt[4];
            int role = 0;
            for (int k = 0; k < 4; ++k) {
                if (V4[k] == i) role = k;
                xv[k] = (V4[k] == i) ? xi : x + 3 * V4[k];
                xvt[k] = xt + 3 * V4[k];
            }
            if (ee_contact(P, xv, xvt, CT->ee_n + 3 * el, role, f, H)) *in_contact = 1;
        }
    }
    /* contacts against analytic spheres and planes, at the current iterate */
    int nobs = P->n_spheres + P->n_planes;
    for (int o = 0; o < nobs; ++o) {
        R n[3], pen;
        if (o < P->n_spheres) {
            const double *s = P->spheres + 4 * o;
            R r[3] = {xi[0] - s[0], xi[1] - s[1], xi[2] - s[2]};
            R dist = RSQRT(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            for (int a = 0; a < 3; ++a) n[a] = r[a] / dist;
            pen = s[3] + P->contact_thickness - dist;
        } else {
            const double *pl = P->planes + 4 * (o - P->n_spheres);
            for (int a = 0; a < 3; ++a) n[a] = pl[a];
            pen = P->contact_thickness - (pl[0] * xi[0] + pl[1] * xi[1] + pl[2] * xi[2] - pl[3]);
        }
        if (!(RE(pen) > 0.0)) continue;
        *in_contact = 1;
        /* E_c = 1/2 k_c pen^2 with pen = (x_b - x_i).n and n fixed:
         * dE/dx_i = -k_c pen n, d2E/dx_i2 = k_c n n^T */
        for (int a = 0; a < 3; ++a) {
            f[a] += P->contact_k * pen * n[a];
            for (int b = 0; b < 3; ++b) H[a][b] += P->contact_k * n[a] * n[b];
        }
        if (P->friction_mu > 0.0) {
            /* relative tangential displacement u = (I - n n^T)(x_i - x_i^t)
             * (the obstacle is static); lambda = contact force magnitude */
            R dx[3] = {xi[0] - xt[3 * i], xi[1] - xt[3 * i + 1], xi[2] - xt[3 * i + 2]};
            R dn = dx[0] * n[0] + dx[1] * n[1] + dx[2] * n[2];
            R u[3] = {dx[0] - dn * n[0], dx[1] - dn * n[1], dx[2] - dn * n[2]};
            R un = RSQRT(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            double hev = h * P->friction_eps_v;
            R f1_over_u; /* f1(u)/u, f1 as in Eq. IPC_friction */
            if (RE(un) < hev) f1_over_u = 2.0 / hev - un / (hev * hev);
            else f1_over_u = 1.0 / un;
            R lamc = P->contact_k * pen;
            R s = P->friction_mu * lamc * f1_over_u;
            for (int a = 0; a < 3; ++a) {
                f[a] -= s * u[a];
                for (int b = 0; b < 3; ++b) H[a][b] += s * ((a == b ? 1.0 : 0.0) - n[a] * n[b]);
            }
        }
    }
}

/* variational energy G (Eq. VariantionalFormOfImplicitEuler); grad/hess optional */
static double energy_G_impl(const oracle_model *M, const oracle_params *P, const R *x,
                            const R *y, const R *E, double *grad, double *hess)
{
    const int nv = M->n_verts, n3 = 3 * nv;
    const double h2 = P->h * P->h;
    double G = 0;
    if (grad) memset(grad, 0, sizeof(double) * (size_t)n3);
    if (hess) memset(hess, 0, sizeof(double) * (size_t)n3 * (size_t)n3);
    for (int i = 0; i < nv; ++i) {
        if (M->pinned[i]) continue;
        double mh2 = M->mass[i] / h2;
        for (int a = 0; a < 3; ++a) {
            double d = RE(x[3 * i + a]) - RE(y[3 * i + a]);
            G += 0.5 * mh2 * d * d;
            if (grad) grad[3 * i + a] += mh2 * d;
            if (hess) hess[(size_t)(3 * i + a) * n3 + 3 * i + a] += mh2;
        }
    }
    for (int t = 0; t < M->n_tets; ++t) {
        R xl[4][3];
        for (int l = 0; l < 4; ++l)
            for (int a = 0; a < 3; ++a) xl[l][a] = RE(x[3 * M->tets[4 * t + l] + a]);
        R F[3][3], mu, lam;
        lame_R(RE(E[t]), M->nu, &mu, &lam);
        tet_F((const R(*)[3])xl, M->Dminv + 9 * t, F);
        G += M->vol[t] * RE(psi_R((const R(*)[3])F, mu, lam));
        if (grad || hess) {
            double m[4][3];
            shape_grads(M->Dminv + 9 * t, m);
            R D[9][9];
            dPdF((const R(*)[3])F, mu, lam, D);
            for (int k = 0; k < 4; ++k) {
                int vk = M->tets[4 * t + k];
                if (grad) {
                    R g[3];
                    tet_grad_k((const R(*)[3])F, (const double(*)[3])m, M->vol[t], mu, lam, k, g);
                    for (int a = 0; a < 3; ++a) grad[3 * vk + a] += RE(g[a]);
                }
                if (hess)
                    for (int l = 0; l < 4; ++l) {
                        int vl = M->tets[4 * t + l];
                        R Hb[3][3];
                        tet_hess_kl((const R(*)[9])D, (const double(*)[3])m, M->vol[t], k, l, Hb);
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b)
                                hess[(size_t)(3 * vk + a) * n3 + 3 * vl + b] += RE(Hb[a][b]);
                    }
            }
        }
    }
    for (int s = 0; s < M->n_springs; ++s) {
        int va = M->springs[2 * s], vb = M->springs[2 * s + 1];
        R xa[3], xb[3];
        for (int a = 0; a < 3; ++a) { xa[a] = RE(x[3 * va + a]); xb[a] = RE(x[3 * vb + a]); }
        R d[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
        double l = sqrt(RE(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
        G += 0.5 * M->spring_k * (l - M->spring_rest[s]) * (l - M->spring_rest[s]);
        if (grad || hess) {
            R g[3], Hb[3][3];
            spring_block(xa, xb, M->spring_rest[s], M->spring_k, P->spring_psd, g, Hb);
            for (int a = 0; a < 3; ++a) {
                if (grad) { grad[3 * va + a] += RE(g[a]); grad[3 * vb + a] -= RE(g[a]); }
                if (hess)
                    for (int b = 0; b < 3; ++b) {
                        double v = RE(Hb[a][b]);
                        hess[(size_t)(3 * va + a) * n3 + 3 * va + b] += v;
                        hess[(size_t)(3 * vb + a) * n3 + 3 * vb + b] += v;
                        hess[(size_t)(3 * va + a) * n3 + 3 * vb + b] -= v;
                        hess[(size_t)(3 * vb + a) * n3 + 3 * va + b] -= v;
                    }
            }
        }
    }
    int nobs = P->n_spheres + P->n_planes;
    for (int i = 0; i < nv && nobs > 0; ++i) {
        if (M->pinned[i]) continue;
        double xi[3] = {RE(x[3 * i]), RE(x[3 * i + 1]), RE(x[3 * i + 2])};
        for (int o = 0; o < nobs; ++o) {
            double n[3], pen;
            if (o < P->n_spheres) {
                const double *s = P->spheres + 4 * o;
                double r[3] = {xi[0] - s[0], xi[1] - s[1], xi[2] - s[2]};
                double dist = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                for (int a = 0; a < 3; ++a) n[a] = r[a] / dist;
                pen = s[3] + P->contact_thickness - dist;
            } else {
                const double *pl = P->planes + 4 * (o - P->n_spheres);
                for (int a = 0; a < 3; ++a) n[a] = pl[a];
                pen = P->contact_thickness - (pl[0] * xi[0] + pl[1] * xi[1] + pl[2] * xi[2] - pl[3]);
            }
            if (!(pen > 0.0)) continue;
            G += 0.5 * P->contact_k * pen * pen;
            for (int a = 0; a < 3; ++a) {
                if (grad) grad[3 * i + a] -= P->contact_k * pen * n[a];
                if (hess)
                    for (int b = 0; b < 3; ++b)
                        hess[(size_t)(3 * i + a) * n3 + 3 * i + b] += P->contact_k * n[a] * n[b];
            }
        }
    }
    return G;
}

/* y = x^t + h v^t + h^2 a_ext (Eq. inertia) */
static void predict_R(const oracle_model *M, const oracle_params *P, const R *x, const R *v, R *y)
{
    const double h = P->h;
    for (int i = 0; i < M->n_verts; ++i)
        for (int a = 0; a < 3; ++a)
            y[3 * i + a] = x[3 * i + a] + h * v[3 * i + a] + h * h * P->gravity[a];
}

/* Initial guess (Sec. 3.7): options (a) previous position, (b) inertia,
 * (c) inertia and acceleration (= y), (d) adaptive.  Pinned vertices: x^t.
 * For (d), a_t = (v^t - v^{t-1})/h, a_ext^t = a_t . a_hat, and the factor
 * a~ = 1 if a_ext^t > |a_ext|, 0 if a_ext^t < 0, a_ext^t/|a_ext| otherwise. */
static void init_R(const oracle_model *M, const oracle_params *P, const R *xt, const R *v,
                   const R *vp, const R *y, R *x)
{
    const double h = P->h;
    const double *g = P->gravity;
    const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    for (int i = 0; i < M->n_verts; ++i) {
        for (int a = 0; a < 3; ++a) x[3 * i + a] = xt[3 * i + a];
        if (M->pinned[i]) continue;
        switch (P->init_mode) {
        case OR_INIT_PREV:
            break;
        case OR_INIT_INERTIA:
            for (int a = 0; a < 3; ++a) x[3 * i + a] = xt[3 * i + a] + h * v[3 * i + a];
            break;
        case OR_INIT_Y:
            for (int a = 0; a < 3; ++a) x[3 * i + a] = y[3 * i + a];
            break;
        default: {
            R at = 0;
            if (gn > 0.0)
                for (int a = 0; a < 3; ++a) at += (v[3 * i + a] - vp[3 * i + a]) / h * (g[a] / gn);
            R atil;
            if (gn == 0.0) atil = 0.0;
            else if (RE(at) > gn) atil = 1.0;
            else if (RE(at) < 0.0) atil = 0.0;
            else atil = at / gn;
            for (int a = 0; a < 3; ++a)
                x[3 * i + a] = xt[3 * i + a] + h * v[3 * i + a] + h * h * atil * g[a];
        }
        }
    }
}

static int check_args(const oracle_model *M, const oracle_params *P)
{
    if (!M || !P || P->h <= 0.0 || P->n_iters < 0 || M->n_verts < 0) return -1;
    if (M->n_tets > 0 && (!M->tets || !M->Dminv || !M->vol)) return -1;
    if (M->n_springs > 0 && (!M->springs || !M->spring_rest)) return -1;
    if (!M->mass || !M->pinned || !M->colors) return -1;
    return 0;
}

/* Chebyshev weights (Eq. accelerator): omega_1 = 1, omega_2 = 2/(2-rho^2),
 * omega_n = 4/(4 - rho^2 omega_{n-1}). */
static double cheb_omega(int n, double rho, double prev)
{
    if (n <= 1) return 1.0;
    if (n == 2) return 2.0 / (2.0 - rho * rho);
    return 4.0 / (4.0 - rho * rho * prev);
}

/* One VBD time step, following Alg. 1 in order. */
int32_t FN(oracle_step)(const oracle_model *M, const oracle_params *P, R *x, R *v, R *vprev,
                        const R *E, const int32_t *order, double *G_trace,
                        int32_t track_local_grad, oracle_stats *st)
{
    if (check_args(M, P)) return -1;
    const int nv = M->n_verts, C = M->n_colors;
    const size_t n3 = 3 * (size_t)nv;
    Inc inc;
    inc_build(M, &inc);
    R *xt = (R *)malloc(sizeof(R) * n3 + 1), *y = (R *)malloc(sizeof(R) * n3 + 1);
    R *xnew = (R *)malloc(sizeof(R) * n3 + 1);
    R *pr1 = NULL, *pr2 = NULL;
    uint8_t *collided = (uint8_t *)calloc((size_t)nv + 1, 1);
    memcpy(xt, x, sizeof(R) * n3);

    /* vertices of each color in processing order */
    int32_t *crow = (int32_t *)calloc((size_t)C + 2, sizeof(int32_t));
    int32_t *clist = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nv + 1));
    for (int i = 0; i < nv; ++i) crow[M->colors[i] + 1]++;
    for (int c = 0; c < C; ++c) crow[c + 1] += crow[c];
    {
        int32_t *fill = (int32_t *)calloc((size_t)C + 1, sizeof(int32_t));
        for (int q = 0; q < nv; ++q) {
            int i = order ? order[q] : q;
            int c = M->colors[i];
            clist[crow[c] + fill[c]++] = i;
        }
        free(fill);
    }

    predict_R(M, P, xt, v, y);                       /* Alg. 1: y */
    init_R(M, P, xt, v, vprev, y, x);                /* Alg. 1: initial guess */
    memcpy(xnew, x, sizeof(R) * n3);
    if (P->cheb_rho > 0.0) {
        pr1 = (R *)malloc(sizeof(R) * n3 + 1);
        pr2 = (R *)malloc(sizeof(R) * n3 + 1);
        memcpy(pr1, x, sizeof(R) * n3);
        memcpy(pr2, x, sizeof(R) * n3);
    }
    int64_t n_upd = 0, n_skip = 0, n_con = 0;
    double max_lg = 0.0, omega = 1.0;
    Contacts CTs = {NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL};
    const Contacts *CT = NULL;
    if (P->mesh_contacts && M->n_surf_tris > 0) {
        /* discrete detection at x^t (Sec. 3.5, Alg. 1) */
        CTs.tri = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nv + 1));
        detect_R(M, P, xt, CTs.tri);
        contacts_index(M, &CTs);
        if (P->edge_contacts) {
            detect_ee(M, P, xt, xt, &CTs);
            ee_index(M, &CTs);
        }
        CT = &CTs;
    }

    for (int it = 1; it <= P->n_iters; ++it) {
        /* Alg. 1: the collision pass on the current iterate runs when
         * n mod n_col = 1, i.e. before iterations 1, 1 + n_col, ... (the
         * first one on the initial guess); n_col = 1 means every iteration */
        if (CT && P->n_col > 0 && (it - 1) % P->n_col == 0) {
            detect_R(M, P, x, CTs.tri);
            contacts_index(M, &CTs);
            if (P->edge_contacts) {
                detect_ee(M, P, x, xt, &CTs);
                ee_index(M, &CTs);
            }
        }
        for (int c = 0; c < C; ++c) {
            const int cb = crow[c], ce = crow[c + 1];
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_upd, n_skip, n_con) reduction(max : max_lg)
#endif
            for (int q = cb; q < ce; ++q) {
                int i = clist[q];
                if (M->pinned[i]) continue;
                R f[3], H[3][3], dx[3];
                int con = 0;
                local_system(M, P, &inc, CT, i, x, NULL, y, xt, E, f, H, &con);
                if (con) { collided[i] = 1; n_con++; }
                R det = solve3((const R(*)[3])H, f, dx);
                n_upd++;
                if (skip_solve((const R(*)[3])H, det, P->det_eps_rel)) {
                    n_skip++;
                    for (int a = 0; a < 3; ++a) xnew[3 * i + a] = x[3 * i + a];
                    continue;
                }
                for (int a = 0; a < 3; ++a) xnew[3 * i + a] = x[3 * i + a] + dx[a];
                if (track_local_grad) {
                    R f2[3], H2[3][3];
                    int con2 = 0;
                    local_system(M, P, &inc, CT, i, x, xnew + 3 * i, y, xt, E, f2, H2, &con2);
                    double gmax = 0;
                    for (int a = 0; a < 3; ++a) gmax = fmax(gmax, fabs(RE(f2[a])));
                    if (gmax > max_lg) max_lg = gmax;
                }
            }
            /* copy updated positions of this color back (x_new buffer, Sec. 3.9) */
            for (int q = cb; q < ce; ++q) {
                int i = clist[q];
                for (int a = 0; a < 3; ++a) x[3 * i + a] = xnew[3 * i + a];
            }
            if (G_trace && !OR_COMPLEX)
                G_trace[(size_t)(it - 1) * C + c] = energy_G_impl(M, P, x, y, E, NULL, NULL);
        }
        if (P->cheb_rho > 0.0) {
            /* accelerated iteration, skipping vertices that collided in this step */
            omega = cheb_omega(it, P->cheb_rho, omega);
            for (int i = 0; i < nv; ++i) {
                if (M->pinned[i] || collided[i]) continue;
                for (int a = 0; a < 3; ++a)
                    x[3 * i + a] = omega * (x[3 * i + a] - pr2[3 * i + a]) + pr2[3 * i + a];
            }
            memcpy(pr2, pr1, sizeof(R) * n3);
            memcpy(pr1, x, sizeof(R) * n3);
            memcpy(xnew, x, sizeof(R) * n3);
        }
    }
    /* Eq. velocity_update; the state's previous velocity becomes v^t */
    for (size_t q = 0; q < n3; ++q) {
        R vn = (x[q] - xt[q]) / P->h;
        vprev[q] = v[q];
        v[q] = vn;
    }
    if (st) {
        st->n_updates += n_upd;
        st->n_skips += n_skip;
        st->n_contacts += n_con;
        if (max_lg > st->max_local_grad) st->max_local_grad = max_lg;
    }
    free(xt); free(y); free(xnew); free(pr1); free(pr2); free(collided);
    free(crow); free(clist);
    free(CTs.tri); free(CTs.crow); free(CTs.cent);
    free(CTs.ee); free(CTs.ee_n); free(CTs.erow); free(CTs.eent);
    inc_free(&inc);
    return 0;
}

#if !OR_COMPLEX
/* ------------------------------- real-only API ---------------------------- */
void oracle_lame(double E, double nu, double *mu, double *lam) { lame_R(E, nu, mu, lam); }

double oracle_tet_energy(const double x[12], const double Dminv[9], double vol, double mu,
                         double lam)
{
    double xl[4][3], F[3][3];
    memcpy(xl, x, sizeof(xl));
    tet_F((const double(*)[3])xl, Dminv, F);
    return vol * psi_R((const double(*)[3])F, mu, lam);
}

void oracle_tet_derivs(const double x[12], const double Dminv[9], double vol, double mu,
                       double lam, double grad[12], double hess[144])
{
    double xl[4][3], F[3][3], D[9][9], m[4][3];
    memcpy(xl, x, sizeof(xl));
    shape_grads(Dminv, m);
    tet_F((const double(*)[3])xl, Dminv, F);
    dPdF((const double(*)[3])F, mu, lam, D);
    for (int k = 0; k < 4; ++k) {
        tet_grad_k((const double(*)[3])F, (const double(*)[3])m, vol, mu, lam, k, grad + 3 * k);
        for (int l = 0; l < 4; ++l) {
            double Hb[3][3];
            tet_hess_kl((const double(*)[9])D, (const double(*)[3])m, vol, k, l, Hb);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) hess[(3 * k + a) * 12 + 3 * l + b] = Hb[a][b];
        }
    }
}

double oracle_spring_energy(const double xa[3], const double xb[3], double L, double k)
{
    double d[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
    double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    return 0.5 * k * (l - L) * (l - L);
}

void oracle_spring_derivs(const double xa[3], const double xb[3], double L, double k,
                          double grad[6], double hess[36])
{
    double g[3], Hb[3][3];
    spring_block(xa, xb, L, k, 0, g, Hb);
    for (int a = 0; a < 3; ++a) {
        grad[a] = g[a];
        grad[3 + a] = -g[a];
        for (int b = 0; b < 3; ++b) {
            hess[a * 6 + b] = Hb[a][b];
            hess[(3 + a) * 6 + 3 + b] = Hb[a][b];
            hess[a * 6 + 3 + b] = -Hb[a][b];
            hess[(3 + a) * 6 + b] = -Hb[a][b];
        }
    }
}

void oracle_predict(const oracle_model *M, const oracle_params *P, const double *x,
                    const double *v, double *y)
{
    predict_R(M, P, x, v, y);
}

double oracle_energy_G(const oracle_model *M, const oracle_params *P, const double *x,
                       const double *y, const double *tet_E, double *grad, double *hess)
{
    return energy_G_impl(M, P, x, y, tet_E, grad, hess);
}

void oracle_closest_point_triangle(const double p[3], const double a[3], const double b[3],
                                   const double c[3], double q[3], double bary[3])
{
    closest_point_R(p, a, b, c, q, bary);
}

void oracle_detect_contacts(const oracle_model *M, const oracle_params *P, const double *x,
                            int32_t *tri_of_vertex)
{
    detect_R(M, P, x, tri_of_vertex);
}

double oracle_segment_closest(const double p0[3], const double p1[3], const double q0[3],
                              const double q1[3], double *s, double *u)
{
    return segment_closest_R(p0, p1, q0, q1, s, u);
}

int32_t oracle_detect_edges(const oracle_model *M, const oracle_params *P, const double *x,
                            const double *xt, int32_t max_out, int32_t *out_v, double *out_n)
{
    Contacts C = {NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL};
    detect_ee(M, P, x, xt, &C);
    const int n = C.n_ee;
    for (int e = 0; e < n && e < max_out; ++e) {
        for (int k = 0; k < 4; ++k) out_v[4 * e + k] = C.ee[4 * e + k];
        for (int k = 0; k < 3; ++k) out_n[3 * e + k] = C.ee_n[3 * e + k];
    }
    free(C.ee); free(C.ee_n);
    return n;
}

double oracle_edge_element(const double x[12], const double n[3], double k, double delta,
                           double grad[12])
{
    oracle_params P;
    memset(&P, 0, sizeof(P));
    P.contact_k = k;
    P.contact_thickness = delta;
    const double *xv[4] = {x, x + 3, x + 6, x + 9};
    double s, u, d = delta;
    segment_closest_R(xv[0], xv[1], xv[2], xv[3], &s, &u);
    for (int a = 0; a < 3; ++a)
        d -= (xv[0][a] + s * (xv[1][a] - xv[0][a]) - xv[2][a] - u * (xv[3][a] - xv[2][a])) * n[a];
    for (int role = 0; role < 4; ++role) {
        double f[3] = {0, 0, 0}, H[3][3] = {{0}};
        ee_contact(&P, xv, xv, n, role, f, H);
        for (int a = 0; a < 3; ++a) grad[3 * role + a] = -f[a];
    }
    return d;
}

double oracle_edge_element_friction(const double x[12], const double xt[12], const double n[3], double k,
                                    double delta, double mu, double eps_v, double h, double grad[12])
{
    oracle_params P;
    memset(&P, 0, sizeof(P));
    P.contact_k = k;
    P.contact_thickness = delta;
    P.friction_mu = mu;
    P.friction_eps_v = eps_v;
    P.h = h;
    const double *xv[4] = {x, x + 3, x + 6, x + 9};
    const double *xvt[4] = {xt, xt + 3, xt + 6, xt + 9};
    double s, u, d = delta;
    segment_closest_R(xv[0], xv[1], xv[2], xv[3], &s, &u);
    for (int a = 0; a < 3; ++a)
        d -= (xv[0][a] + s * (xv[1][a] - xv[0][a]) - xv[2][a] - u * (xv[3][a] - xv[2][a])) * n[a];
    for (int role = 0; role < 4; ++role) {
        double f[3] = {0, 0, 0}, H[3][3] = {{0}};
        ee_contact(&P, xv, xvt, n, role, f, H);
        for (int a = 0; a < 3; ++a) grad[3 * role + a] = -f[a];
    }
    return d;
}

double oracle_winding_number(const oracle_model *M, int32_t mesh, const double p[3], const double *x)
{
    return winding_number(M, mesh, p, x);
}

/* d2J/dx_k dx_l: (M_kl)_ac = sum_b,e (m_k)_b (m_l)_e dcof_ab/dF_ce,
 * with dcof_ab/dF_ce = sum_df eps_acd eps_bef F_df. */
static void d2J_kl(const double F[3][3], const double m[4][3], int k, int l, double Mk[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int b = 0; b < 3; ++b)
                for (int e = 0; e < 3; ++e) {
                    double dc = 0;
                    for (int d = 0; d < 3; ++d)
                        for (int f = 0; f < 3; ++f)
                            if (LC[a][c][d] && LC[b][e][f]) dc += LC[a][c][d] * LC[b][e][f] * F[d][f];
                    s += m[k][b] * m[l][e] * dc;
                }
            Mk[a][c] = s;
        }
}

/* Reverse mode of one step, explicit form.  Each local update is
 *   x_i' = x_i + D,  D = H_i^{-1} f_i,
 * with f_i, H_i evaluated at the state before the color pass.  For an input z,
 *   dD = H^{-1} (df/dz - dH/dz D) dz,
 * so with w = H^{-1} xbar_i:  zbar += (df/dz)^T w - (dH/dz : w D^T).
 * For a tet with vertex i in slot k:
 *   df/dx_i = -H_i, dH_i/dx_i = 0 (J is affine in x_k, so c_k = cof(F) m_k
 *   does not depend on x_k),
 *   df/dx_j = -K_kj,  dH/dx_j : w D^T = V lam [(c.D) M^T w + (c.w) M^T D]
 *   with c = c_k, M = d2J/dx_k dx_j  (H_kk = V(mu |m_k|^2 I + lam c c^T)),
 *   df/dy_i = m/h^2 I,  df/dE_t = -grad_k U_t / E_t,  dH/dE_t = H_t,kk / E_t.
 * Then the adjoints of the initial guess and of y are applied. */
int32_t oracle_step_backward(const oracle_model *M, const oracle_params *P, const double *x_t,
                             const double *v_t, const double *v_prev, const double *E,
                             const double *gx_out, const double *gv_out, const double *gvp_out,
                             double *gx_in, double *gv_in, double *gvp_in, double *g_E)
{
    if (check_args(M, P)) return -1;
    if (M->n_springs > 0 || P->n_spheres > 0 || P->n_planes > 0 || P->kd != 0.0 ||
        P->cheb_rho > 0.0 || P->mesh_contacts)
        return -2;
    const int nv = M->n_verts, C = M->n_colors, N = P->n_iters;
    const size_t n3 = 3 * (size_t)nv;
    const double h = P->h;
    Inc inc;
    inc_build(M, &inc);
    double *S = (double *)malloc(sizeof(double) * n3 * (size_t)(N + 1) + 8);
    double *y = (double *)malloc(sizeof(double) * n3 + 8);
    double *x = (double *)malloc(sizeof(double) * n3 + 8);
    double *xnew = (double *)malloc(sizeof(double) * n3 + 8);
    double *cur = (double *)malloc(sizeof(double) * n3 + 8);
    double *xb = (double *)calloc(n3 + 1, sizeof(double));
    double *yb = (double *)calloc(n3 + 1, sizeof(double));
    double *xtb = (double *)calloc(n3 + 1, sizeof(double));
    double *vb = (double *)calloc(n3 + 1, sizeof(double));
    double *vpb = (double *)calloc(n3 + 1, sizeof(double));

    /* forward recompute with a snapshot after every iteration */
    predict_R(M, P, x_t, v_t, y);
    init_R(M, P, x_t, v_t, v_prev, y, x);
    memcpy(S, x, sizeof(double) * n3);
    memcpy(xnew, x, sizeof(double) * n3);
    for (int it = 1; it <= N; ++it) {
        for (int c = 0; c < C; ++c) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
            for (int i = 0; i < nv; ++i) {
                if (M->colors[i] != c || M->pinned[i]) continue;
                double f[3], H[3][3], dx[3];
                int con = 0;
                local_system(M, P, &inc, NULL, i, x, NULL, y, x_t, E, f, H, &con);
                double det = solve3((const double(*)[3])H, f, dx);
                for (int a = 0; a < 3; ++a)
                    xnew[3 * i + a] = skip_solve((const double(*)[3])H, det, P->det_eps_rel)
                                          ? x[3 * i + a] : x[3 * i + a] + dx[a];
            }
            for (int i = 0; i < nv; ++i)
                if (M->colors[i] == c)
                    for (int a = 0; a < 3; ++a) x[3 * i + a] = xnew[3 * i + a];
        }
        memcpy(S + n3 * (size_t)it, x, sizeof(double) * n3);
    }

    /* outputs: x^{t+1} = x^(N), v^{t+1} = (x^(N) - x^t)/h, v_out_prev = v^t */
    for (size_t q = 0; q < n3; ++q) {
        xb[q] = gx_out[q] + gv_out[q] / h;
        xtb[q] = -gv_out[q] / h;
        vb[q] = gvp_out[q];
    }
    for (int it = N; it >= 1; --it) {
        const double *Sn = S + n3 * (size_t)it, *Sp = S + n3 * (size_t)(it - 1);
        for (int c = C - 1; c >= 0; --c) {
            /* state before color pass c of iteration it */
            for (int l = 0; l < nv; ++l)
                for (int a = 0; a < 3; ++a)
                    cur[3 * l + a] = (M->colors[l] < c) ? Sn[3 * l + a] : Sp[3 * l + a];
            /* vertices of one color are independent; their scatters into
             * neighbours (other colors) are summed with atomic adds */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
            for (int i = 0; i < nv; ++i) {
                if (M->colors[i] != c || M->pinned[i]) continue;
                double f[3], H[3][3], D[3], w[3];
                int con = 0;
                local_system(M, P, &inc, NULL, i, cur, NULL, y, x_t, E, f, H, &con);
                double det = solve3((const double(*)[3])H, f, D);
                if (skip_solve((const double(*)[3])H, det, P->det_eps_rel)) continue;
                double g[3] = {xb[3 * i], xb[3 * i + 1], xb[3 * i + 2]};
                solve3((const double(*)[3])H, g, w);
                for (int a = 0; a < 3; ++a) {
                    double Hw = H[a][0] * w[0] + H[a][1] * w[1] + H[a][2] * w[2];
                    xb[3 * i + a] = g[a] - Hw;
                    yb[3 * i + a] += M->mass[i] / (h * h) * w[a];
                }
                for (int e = inc.tet_row[i]; e < inc.tet_row[i + 1]; ++e) {
                    int t = inc.tet_ent[e] >> 2, k = inc.tet_ent[e] & 3;
                    double xl[4][3], F[3][3], Dm[9][9], Cf[3][3], m[4][3], mu, lam;
                    for (int l = 0; l < 4; ++l)
                        for (int a = 0; a < 3; ++a) xl[l][a] = cur[3 * M->tets[4 * t + l] + a];
                    shape_grads(M->Dminv + 9 * t, m);
                    lame_R(E[t], M->nu, &mu, &lam);
                    tet_F((const double(*)[3])xl, M->Dminv + 9 * t, F);
                    dPdF((const double(*)[3])F, mu, lam, Dm);
                    cof3((const double(*)[3])F, Cf);
                    double ck[3];
                    for (int a = 0; a < 3; ++a)
                        ck[a] = Cf[a][0] * m[k][0] + Cf[a][1] * m[k][1] + Cf[a][2] * m[k][2];
                    double cD = ck[0] * D[0] + ck[1] * D[1] + ck[2] * D[2];
                    double cw = ck[0] * w[0] + ck[1] * w[1] + ck[2] * w[2];
                    double V = M->vol[t];
                    for (int j = 0; j < 4; ++j) {
                        if (j == k) continue;
                        int vj = M->tets[4 * t + j];
                        double K[3][3], Mkj[3][3];
                        tet_hess_kl((const double(*)[9])Dm, (const double(*)[3])m, V, k, j, K);
                        d2J_kl((const double(*)[3])F, (const double(*)[3])m, k, j, Mkj);
                        for (int e2 = 0; e2 < 3; ++e2) {
                            double Ktw = 0, Mtw = 0, MtD = 0;
                            for (int a = 0; a < 3; ++a) {
                                Ktw += K[a][e2] * w[a];
                                Mtw += Mkj[a][e2] * w[a];
                                MtD += Mkj[a][e2] * D[a];
                            }
                            const double add = -Ktw - V * lam * (cD * Mtw + cw * MtD);
#ifdef _OPENMP
#pragma omp atomic
#endif
                            xb[3 * vj + e2] += add;
                        }
                    }
                    double gk[3], Hkk[3][3];
                    tet_grad_k((const double(*)[3])F, (const double(*)[3])m, V, mu, lam, k, gk);
                    tet_hess_kl((const double(*)[9])Dm, (const double(*)[3])m, V, k, k, Hkk);
                    double s = 0;
                    for (int a = 0; a < 3; ++a) {
                        double HD = Hkk[a][0] * D[0] + Hkk[a][1] * D[1] + Hkk[a][2] * D[2];
                        s += w[a] * (gk[a] + HD);
                    }
                    g_E[t] += -s / E[t];
                }
            }
        }
    }
    /* adjoint of the initial guess (Sec. 3.7) */
    const double *gr = P->gravity;
    const double gn = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
    for (int i = 0; i < nv; ++i) {
        double *b = xb + 3 * i;
        for (int a = 0; a < 3; ++a) xtb[3 * i + a] += b[a];
        if (M->pinned[i]) continue;
        if (P->init_mode == OR_INIT_PREV) continue;
        for (int a = 0; a < 3; ++a) vb[3 * i + a] += h * b[a];
        if (P->init_mode == OR_INIT_ADAPTIVE && gn > 0.0) {
            double at = 0;
            for (int a = 0; a < 3; ++a) at += (v_t[3 * i + a] - v_prev[3 * i + a]) / h * (gr[a] / gn);
            if (at > 0.0 && at < gn) {
                /* x = ... + h^2 (at/gn) g, d(at)/dv = ghat/h, d(at)/dvp = -ghat/h */
                double s = h * h * (gr[0] * b[0] + gr[1] * b[1] + gr[2] * b[2]) / gn;
                for (int a = 0; a < 3; ++a) {
                    vb[3 * i + a] += s * gr[a] / gn / h;
                    vpb[3 * i + a] -= s * gr[a] / gn / h;
                }
            }
        }
    }
    /* adjoint of y = x^t + h v^t + h^2 a_ext */
    for (int i = 0; i < nv; ++i) {
        if (M->pinned[i]) continue;
        for (int a = 0; a < 3; ++a) {
            xtb[3 * i + a] += yb[3 * i + a];
            vb[3 * i + a] += h * yb[3 * i + a];
        }
    }
    memcpy(gx_in, xtb, sizeof(double) * n3);
    memcpy(gv_in, vb, sizeof(double) * n3);
    memcpy(gvp_in, vpb, sizeof(double) * n3);
    free(S); free(y); free(x); free(xnew); free(cur);
    free(xb); free(yb); free(xtb); free(vb); free(vpb);
    inc_free(&inc);
    return 0;
}
#endif
