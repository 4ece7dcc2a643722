/* FP64 reference ("oracle") for the Vertex Block Descent time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential CPU
 * implementation of what the GPU library computes.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never does.  It shares no code, headers or tables with the HIP library.
 *
 * Paper: A. H. Chen, Z. Liu, Y. Yang, C. Yuksel, "Vertex Block Descent",
 * ACM TOG 43(4), 2024.  Each function names the passage it follows.
 *
 * All floating point is IEEE double.  The forward step is also compiled in
 * double complex (suffix _cs) so that tests can take complex-step directional
 * derivatives (Squire & Trapp 1998) of a whole rollout.
 */
#ifndef VBD_ORACLE_H
#define VBD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_INIT_PREV = 0, OR_INIT_INERTIA = 1, OR_INIT_Y = 2, OR_INIT_ADAPTIVE = 3 };

typedef struct {
    int32_t n_verts, n_tets, n_springs, n_colors;
    const int32_t *tets;        /* [n_tets*4] */
    const int32_t *springs;     /* [n_springs*2] or NULL */
    const double  *Dminv;       /* [n_tets*9] row-major inverse of the rest edge matrix */
    const double  *vol;         /* [n_tets] rest volume */
    const double  *spring_rest; /* [n_springs] rest length */
    const double  *mass;        /* [n_verts] */
    const uint8_t *pinned;      /* [n_verts] 0/1 */
    const int32_t *colors;      /* [n_verts] */
    double nu;                  /* Poisson ratio (tets) */
    double spring_k;            /* spring stiffness */
    int32_t n_surf_tris;        /* surface triangles for mesh-mesh contacts (0 = none) */
    const int32_t *surf_tris;   /* [n_surf_tris*3], outward oriented */
    const int32_t *vert_mesh;   /* [n_verts] mesh id of each vertex, or NULL (one mesh) */
    const double  *rest_pos;    /* [n_verts*3] rest positions (self-contact exclusion), or NULL */
} oracle_model;

typedef struct {
    double h;
    int32_t n_iters;
    double gravity[3];
    int32_t init_mode;
    double det_eps_rel;
    double contact_k, contact_thickness;
    int32_t n_spheres; const double *spheres;  /* [n*4] cx cy cz R */
    int32_t n_planes;  const double *planes;   /* [n*4] nx ny nz offset, unit normal */
    double kd;                 /* Rayleigh damping (Sec. 3.3) */
    double cheb_rho;           /* Chebyshev spectral radius (Sec. 3.8), 0 = off */
    double friction_mu, friction_eps_v;        /* Sec. 3.6 */
    int32_t spring_psd;        /* 1: clamp the transverse spring stiffness at 0 */
    int32_t mesh_contacts;     /* 1: vertex-triangle contacts between different meshes */
    double collision_radius;   /* detection radius for mesh-mesh contacts */
    int32_t n_col;             /* re-detect every n_col iterations (0 = only at x^t) */
    int32_t self_contact;      /* 1: contacts within one mesh too (Sec. 3.5, self-collisions) */
    double self_exclusion;     /* same-mesh primitives closer than this at rest never collide */
    int32_t edge_contacts;     /* 1: edge-edge elements (Sec. 3.5, Fig. CollisionPotential) */
} oracle_params;

typedef struct {
    int64_t n_updates;       /* local solves attempted on free vertices */
    int64_t n_skips;         /* solves skipped by the determinant test */
    double  max_local_grad;  /* max |grad_i G_i| right after an update (if tracked) */
    int64_t n_contacts;      /* local solves with at least one active contact */
} oracle_stats;

/* ---- preprocessing (real only) ------------------------------------------ */
/* Greedy first-fit vertex coloring in ascending vertex id over the adjacency
 * of all material elements (Sec. 3.9).  Returns the number of colors. */
int32_t oracle_color_greedy(int32_t n_verts, int32_t n_tets, const int32_t *tets,
                            int32_t n_springs, const int32_t *springs, int32_t *colors);
/* Greedy first fit over the smallest-last order (min remaining degree, ties
 * by smallest id; colored in reverse removal order).  Returns n_colors. */
int32_t oracle_color_smallest_last(int32_t n_verts, int32_t n_tets, const int32_t *tets,
                                   int32_t n_springs, const int32_t *springs, int32_t *colors);
/* DSATUR: most distinct neighbour colors first (ties: larger degree, then
 * smaller id), smallest free color.  Returns n_colors. */
int32_t oracle_color_dsatur(int32_t n_verts, int32_t n_tets, const int32_t *tets,
                            int32_t n_springs, const int32_t *springs, int32_t *colors);
/* Rest edge matrix inverse and volume per tet; returns 0, or -1-t for the first
 * degenerate tet t. */
int32_t oracle_tet_rest(int32_t n_tets, const int32_t *tets, const double *rest,
                        double *Dminv, double *vol);
/* Lumped mass: each tet adds density*V/4 to each of its vertices. */
void oracle_lumped_mass(int32_t n_verts, int32_t n_tets, const int32_t *tets,
                        const double *vol, double density, double *mass);
void oracle_spring_rest(int32_t n_springs, const int32_t *springs, const double *rest,
                        double *L);

/* Surface triangles of a tet mesh (faces used by exactly one tet), oriented
 * so the normal points away from the tet's fourth vertex.  tris_out needs
 * room for 4*n_tets triangles; returns the number written. */
int32_t oracle_surface(int32_t n_tets, const int32_t *tets, const double *rest, int32_t *tris_out);
/* Closest point q on triangle (a, b, c) to p and its barycentric weights. */
void oracle_closest_point_triangle(const double p[3], const double a[3], const double b[3],
                                   const double c[3], double q[3], double bary[3]);
/* Mesh-mesh contact detection used by the step: for each surface vertex the
 * closest surface triangle of another mesh within collision_radius, kept when
 * the vertex is inside that mesh or closer than the contact thickness to its
 * surface (-1 if none). */
void oracle_detect_contacts(const oracle_model *M, const oracle_params *P, const double *x,
                            int32_t *tri_of_vertex);
/* Closest points of segments [p0, p1] and [q0, q1]: parameters s, u in
 * [0, 1] of p0 + s (p1 - p0) and q0 + u (q1 - q0); returns the distance. */
double oracle_segment_closest(const double p0[3], const double p1[3], const double q0[3],
                              const double q1[3], double *s, double *u);
/* Edge-edge contact elements the step would detect on positions x (with x^t
 * = xt for the normals): up to max_out elements, each {e1 a, e1 b, e2 a,
 * e2 b} vertex ids into out_v and its fixed normal into out_n.  Returns the
 * number of elements. */
int32_t oracle_detect_edges(const oracle_model *M, const oracle_params *P, const double *x,
                            const double *xt, int32_t max_out, int32_t *out_v, double *out_n);
/* One edge-edge element (Sec. 3.5): E = k/2 d^2, d = delta - (x_a - x_b).n,
 * x_a on [x0, x1], x_b on [x2, x3] at their closest points (held fixed with
 * n in the derivatives).  grad[12] = dE/dx of the four vertices; returns d
 * (the element is active when d > 0; grad is zero otherwise). */
double oracle_edge_element(const double x[12], const double n[3], double k, double delta,
                           double grad[12]);
/* The same element with its friction (Sec. 3.6): the relative displacement
 * (x_a - x_a^t) - (x_b - x_b^t) from positions xt at the start of the step,
 * friction coefficient mu, eps_v and time step h; grad[12] = the negated
 * forces of penalty and friction (lambda = k d, s, u and n held fixed). */
double oracle_edge_element_friction(const double x[12], const double xt[12], const double n[3], double k,
                                    double delta, double mu, double eps_v, double h, double grad[12]);
/* Generalized winding number of mesh `mesh`'s surface at p (positions x). */
double oracle_winding_number(const oracle_model *M, int32_t mesh, const double p[3], const double *x);

/* ---- element energies and derivatives (real) ------------------------------ */
void   oracle_lame(double E, double nu, double *mu, double *lam);
double oracle_tet_energy(const double x[12], const double Dminv[9], double vol,
                         double mu, double lam);
/* full 12-gradient and 12x12 Hessian of one tet (row-major) */
void   oracle_tet_derivs(const double x[12], const double Dminv[9], double vol,
                         double mu, double lam, double grad[12], double hess[144]);
double oracle_spring_energy(const double xa[3], const double xb[3], double L, double k);
void   oracle_spring_derivs(const double xa[3], const double xb[3], double L, double k,
                            double grad[6], double hess[36]);

/* ---- one time step (Alg. 1) --------------------------------------------- */
/* In place: (x, v, vprev) = (x^t, v^t, v^{t-1}) -> (x^{t+1}, v^{t+1}, v^t).
 * order: optional processing order of vertices inside each color (NULL =
 * ascending id).  G_trace: optional [n_iters*n_colors] variational energy
 * after each color pass.  track_local_grad: record max |grad_i G_i| after each
 * update.  Returns 0, or <0 on bad arguments. */
int32_t oracle_step(const oracle_model *M, const oracle_params *P,
                    double *x, double *v, double *vprev, const double *tet_E,
                    const int32_t *order, double *G_trace, int32_t track_local_grad,
                    oracle_stats *st);
int32_t oracle_step_cs(const oracle_model *M, const oracle_params *P,
                       double _Complex *x, double _Complex *v, double _Complex *vprev,
                       const double _Complex *tet_E, const int32_t *order,
                       double *G_trace, int32_t track_local_grad, oracle_stats *st);

/* Inertia target y = x^t + h v^t + h^2 a_ext (Eq. inertia). */
void oracle_predict(const oracle_model *M, const oracle_params *P,
                    const double *x, const double *v, double *y);
/* Variational energy G (Eq. VariantionalFormOfImplicitEuler), its gradient
 * [3n] and (if hess != NULL) dense Hessian [3n x 3n].  Inertia over free
 * vertices; contacts with the normal held fixed (Sec. 3.5). */
double oracle_energy_G(const oracle_model *M, const oracle_params *P,
                       const double *x, const double *y, const double *tet_E,
                       double *grad, double *hess);

/* ---- reverse mode of one step ---------------------------------------------- */
/* Adjoint of oracle_step for tets + inertia + pins (no springs, contacts,
 * damping or acceleration: returns -2 then).  Recomputes the step's iterates
 * from (x_t, v_t, v_prev).  Inputs: adjoints of (x^{t+1}, v^{t+1}, v^t_out).
 * Outputs: adjoints of (x^t, v^t, v^{t-1}); g_E is accumulated (+=). */
int32_t oracle_step_backward(const oracle_model *M, const oracle_params *P,
                             const double *x_t, const double *v_t, const double *v_prev,
                             const double *tet_E,
                             const double *gx_out, const double *gv_out, const double *gvp_out,
                             double *gx_in, double *gv_in, double *gvp_in, double *g_E);

void oracle_set_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
