/* vbd.h - C ABI of the MI355X (gfx950) Vertex Block Descent library.
 *
 * Method: A. H. Chen, Z. Liu, Y. Yang, C. Yuksel, "Vertex Block Descent",
 * ACM TOG 43(4), 2024.  One call of vbd_step advances every mesh of a
 * topology by one implicit-Euler time step (Sec. 3.1, Eq.
 * VariantionalFormOfImplicitEuler) using the per-color Gauss-Seidel vertex
 * updates of Alg. 1.
 *
 * Conventions
 *   - Every call returns a vbd_status: VBD_OK (0) or a negative error code.
 *     vbd_last_error() returns a thread-local, library-owned, NUL-terminated
 *     message for the last failing call on this thread (valid until the next
 *     call on the thread).
 *   - Host pointers are read during the call only; the caller keeps ownership.
 *   - Device memory is always caller-owned (for example torch tensors).  The
 *     library never allocates device memory: it works inside one workspace
 *     bound by vbd_bind_workspace.
 *   - Device state buffers are float32, row-major [n_verts][3] in the
 *     ORIGINAL vertex order.  The library keeps its own color-sorted copies in
 *     the workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Compute calls are asynchronous with respect to the host.
 *   - A topology may be used by one host thread at a time.
 */
#ifndef VBD_H
#define VBD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vbd_topology_s *vbd_topology;

typedef enum {
    VBD_OK = 0,
    VBD_E_INVALID_ARG = -1,   /* NULL pointer, bad size, bad parameter value */
    VBD_E_TOPOLOGY = -2,      /* id out of range, repeated vertex in an element,
                                 degenerate rest tet, zero-length spring,
                                 element crossing meshes */
    VBD_E_NOT_COLORED = -3,   /* vbd_workspace_size/bind/step before vbd_color */
    VBD_E_NO_WORKSPACE = -4,  /* step before bind, or workspace too small */
    VBD_E_HIP = -5,           /* HIP runtime failure (message has hipGetErrorString) */
    VBD_E_UNSUPPORTED = -6,   /* a feature combination this entry point does not do */
    VBD_E_NONFINITE = -7,     /* a step run with check_finite left a non-finite value (vbd_check) */
    VBD_E_DEVICE = -8         /* a device-side guard fired (see vbd_check) */
} vbd_status;

/* Initial guess options of Sec. 3.7: (a) previous position, (b) inertia,
 * (c) inertia and acceleration (= y), (d) adaptive (default). */
enum { VBD_INIT_PREV = 0, VBD_INIT_INERTIA = 1, VBD_INIT_Y = 2, VBD_INIT_ADAPTIVE = 3 };

/* Launch modes of vbd_step.
 *   PLAIN            host loop of kernel launches: per color one solve kernel
 *   GRAPH            the same launch sequence captured once into a hipGraph and
 *                    replayed (re-captured when pointers or parameters change)
 *   PERSISTENT       one persistent kernel runs all iterations and colors with
 *                    a device-wide barrier between color phases
 *   PERSISTENT_GRAPH the persistent launch plus its pre/post kernels in a hipGraph */
enum { VBD_LAUNCH_PLAIN = 0, VBD_LAUNCH_GRAPH = 1, VBD_LAUNCH_PERSISTENT = 2,
       VBD_LAUNCH_PERSISTENT_GRAPH = 3 };

/* Mesh description (host memory).  A batch is a concatenation of meshes that
 * share no vertices; element ids are global vertex ids. */
typedef struct {
    int32_t n_verts, n_tets, n_springs;
    int32_t n_meshes;              /* >= 1 */
    const int64_t *vert_offsets;   /* [n_meshes+1] or NULL when n_meshes == 1 */
    const int64_t *tet_offsets;    /* [n_meshes+1] or NULL when n_meshes == 1 */
    const int32_t *tets;           /* [n_tets][4] or NULL when n_tets == 0 */
    const int32_t *springs;        /* [n_springs][2] or NULL when n_springs == 0 */
    const double *rest_pos;        /* [n_verts][3] FP64 rest shape */
    const double *spring_rest;     /* [n_springs] or NULL -> rest distance */
    double spring_k;               /* spring stiffness (N/m), global */
    const double *mass;            /* [n_verts] finite, >= 0, or NULL -> lumped:
                                      each tet adds density*V/4 to each of its
                                      vertices.  A massless free vertex is
                                      allowed: while its local Hessian is
                                      singular the determinant rule skips it */
    double density;                /* kg/m^3, used for lumped masses */
    double poisson_nu;             /* Poisson ratio of all tets, 0 < nu < 0.5 (the
                                      energy's rest offset alpha = 1 + mu/lambda
                                      needs lambda > 0) */
    const uint8_t *pinned;         /* [n_verts] 0/1 or NULL (none pinned) */
} vbd_mesh_desc;

/* Validates the description and precomputes, in FP64, each tet's inverse
 * rest edge matrix and rest volume and the lumped vertex masses.
 * Sec. 5: tets carry the stable Neo-Hookean energy V Psi(F) (Smith et al.
 * 2018, without the logarithmic term) of the deformation gradient
 * F = D_s D_m^{-1} (D_s, D_m: current and rest edge matrices, V = |det D_m|/6);
 * Sec. 3.1, Eq. VariantionalFormOfImplicitEuler / VBDEnergy: the vertex masses
 * m_i of the inertia term, lumped as density*V/4 per incident tet unless
 * given.  Host only, synchronous.  Errors:
 * VBD_E_INVALID_ARG (also for more than 2^28 vertices or 2^29 tets, and for
 * a negative or non-finite mass),
 * VBD_E_TOPOLOGY (|det D_m| <= 1e-12 * (max edge)^3 counts as degenerate).
 * *out receives a library-owned handle. */
vbd_status vbd_build_topology(const vbd_mesh_desc *desc, vbd_topology *out);

/* Greedy vertex coloring (Sec. 3.9): no force element (tet, spring) may use
 * two vertices of one color; first-fit in ascending vertex id.  Then builds
 * the color-sorted vertex permutation (free vertices by (color, id), pinned
 * vertices last by id), the tet incidence CSR of every vertex slot and the
 * spring incidence CSR of every free slot (from which vbd_bind_workspace lays
 * out the per-color padded records the kernels read).  Host, synchronous.
 * colors_out: host [n_verts] or NULL. */
vbd_status vbd_color(vbd_topology topo, int32_t *n_colors_out, int32_t *colors_out);

/* Vertex orders of the greedy first-fit coloring (vbd_color_greedy). */
enum { VBD_COLOR_ID_ORDER = 0,      /* ascending vertex id (what vbd_color uses) */
       VBD_COLOR_SMALLEST_LAST = 1, /* smallest-last order: repeatedly remove a vertex of
                                       smallest remaining degree (ties: smallest id),
                                       color in reverse removal order (Matula and Beck
                                       1983); 4 colors on a Kuhn-split lattice */
       VBD_COLOR_DSATUR = 2         /* DSATUR (Brelaz 1979): next the uncolored vertex with
                                       the most distinct neighbour colors (ties: larger
                                       degree, then smaller id), smallest free color; 5
                                       colors on the spring cloth */
};
/* vbd_color with a choice of vertex order: each vertex, in that order, takes
 * the smallest color not used by an already colored neighbour (for DSATUR
 * the order is chosen as the coloring proceeds).  Recoloring
 * with another order is allowed before vbd_bind_workspace. */
vbd_status vbd_color_greedy(vbd_topology topo, int32_t order, int32_t *n_colors_out,
                            int32_t *colors_out);

/* Alternative to vbd_color: the caller supplies the coloring (host
 * colors[n_verts], values in [0, 65536)), for example a lattice coloring with
 * fewer colors than first-fit greedy finds.  Validated as Sec. 3.9 requires:
 * no tet or spring may have two vertices of one color (VBD_E_INVALID_ARG
 * otherwise, naming the element).  Colors are processed in ascending order;
 * unused color values give empty phases.  Then builds the same permutation
 * and incidence as vbd_color.  Must precede vbd_bind_workspace. */
vbd_status vbd_color_given(vbd_topology topo, const int32_t *colors);

/* Device bytes the workspace needs.  max_backward_iters: largest n_iters that
 * vbd_step_backward will be called with (0 = forward only). */
vbd_status vbd_workspace_size(vbd_topology topo, int32_t max_backward_iters, size_t *bytes);

/* Binds caller-owned device memory (>= vbd_workspace_size bytes, 256-byte
 * aligned) and uploads the topology into it on `stream`.  The memory must
 * stay valid until the topology is destroyed or rebound.  The upload goes
 * through host staging and finishes before the call returns. */
vbd_status vbd_bind_workspace(vbd_topology topo, void *dev_ptr, size_t bytes, void *stream);

/* Read-only queries of host-side topology arrays (tests of bit-exactness). */
enum {
    VBD_Q_COUNTS = 0,       /* int64[8]: n_verts, n_tets, n_springs, n_colors, n_free,
                               tet CSR entries, spring CSR entries, n_meshes */
    VBD_Q_COLORS = 1,       /* int32[n_verts] */
    VBD_Q_PERM = 2,         /* int32[n_verts]: permuted slot -> original id */
    VBD_Q_COLOR_OFFSETS = 3,/* int32[n_colors+1] over the free permuted slots */
    VBD_Q_TET_ROWS = 4,     /* int32[n_verts+1] over permuted slots (free slots first) */
    VBD_Q_TET_ENTRIES = 5,  /* int32[entries]: (tet << 2) | slot, ascending tet */
    VBD_Q_SPRING_ROWS = 6,  /* int32[n_free+1] */
    VBD_Q_SPRING_NBRS = 7,  /* int32[entries]: original id of the other end */
    VBD_Q_MASS = 8,         /* double[n_verts] lumped or given masses (original order) */
    VBD_Q_DMINV = 9,        /* double[n_tets][9] */
    VBD_Q_VOLUME = 10,      /* double[n_tets] */
    VBD_Q_PHASE_BYTES = 11, /* double[n_colors]: algorithmic HBM bytes of one color solve */
    VBD_Q_TET_ORDER = 12,   /* int32[n_tets]: stored tet position -> caller's tet id
                               (tets grouped by the colors of their vertices) */
    VBD_Q_REST_FRAME = 13,  /* double[n_tets][6]: upper triangle of R^{-1}, D_m = Q R with
                               Q a proper rotation (caller's tet order) */
    VBD_Q_SURFACE = 14,     /* int32[n_surf_tris][3]: surface triangles (faces of exactly
                               one tet), original vertex ids, ordered so (b - a) x (c - a)
                               points out of the mesh; sorted by their ascending vertex-id
                               triples */
    VBD_Q_SURFACE_COUNTS = 15, /* int64[3]: n_surf_tris, n_surf_verts, n_surf_edges */
    VBD_Q_SNAPSHOT_REGION = 16,/* int64[3]: byte offset of the iterate snapshots in the bound
                                  workspace (-1 when max_backward_iters is 0), bytes per
                                  snapshot (n_verts float4 in slot order), snapshot count - 1
                                  (max_backward_iters); a step of n_iters iterations uses the
                                  first (n_iters + 1) snapshots */
    VBD_Q_ADJ_PHASE_BYTES = 17,/* double[n_colors]: algorithmic HBM bytes of one reverse color
                                  phase of vbd_step_backward */
    VBD_Q_PHASE_COUNTS = 18,   /* int64[n_colors][4]: tet pairs, spring entries, distinct
                                  neighbour vertices and free vertices of each color */
    VBD_Q_SURFACE_EDGES = 19,  /* int32[n_surf_edges][2]: the distinct edges of the surface
                                  triangles, original ids a < b, ascending (a, b) */
    VBD_Q_XCD_SPLIT = 20       /* int32[n_colors][9]: slot boundaries of the 8 parts of each
                                  color that launch mapping 3 runs on XCDs 0..7 */
};
vbd_status vbd_topology_query(vbd_topology topo, int32_t what, void *host_out, size_t bytes);
vbd_status vbd_topology_destroy(vbd_topology topo);

/* Parameters of one time step (FP32, the kernels' precision). */
typedef struct {
    float h;                       /* time step (s), > 0 */
    int32_t n_iters;               /* VBD iterations n_max, >= 1 */
    float gravity[3];              /* external acceleration a_ext */
    int32_t init_mode;             /* VBD_INIT_* */
    float det_eps_rel;             /* skip a vertex iff |det H| <= det_eps_rel*||H||_F^3 */
    float contact_k;               /* penalty stiffness k_c (Sec. 3.5) */
    float contact_thickness;       /* contact distance delta */
    int32_t n_spheres;             /* <= 8 */
    const float *spheres;          /* host [n_spheres][4]: cx, cy, cz, R */
    int32_t n_planes;              /* <= 8 */
    const float *planes;           /* host [n_planes][4]: nx, ny, nz, offset (n.x = offset);
                                      the normal is normalised by the library */
    float kd;                      /* Rayleigh damping coefficient (Sec. 3.3) */
    float cheb_rho;                /* Chebyshev spectral radius (Sec. 3.8), 0 = off */
    float friction_mu;             /* friction coefficient mu_c (Sec. 3.6), 0 = off */
    float friction_eps_v;          /* friction velocity threshold eps_v */
    int32_t spring_psd;            /* 0: spring Hessian as is (Sec. 3.2, no projection);
                                      1: transverse stiffness k(1 - L/l) clamped at 0,
                                      the exact PSD projection of a spring block */
    int32_t launch_mode;           /* VBD_LAUNCH_* */
    /* Mesh-mesh vertex-triangle contacts (Sec. 3.5, 3.9), between different
     * meshes of a batched topology (and within one mesh with self_contact,
     * below).  Detection at x^t: each
     * surface vertex takes the closest surface triangle of another mesh within
     * collision_radius; the pair is a contact element when the vertex is inside
     * that mesh or closer than contact_thickness to its surface.  Detection is
     * repeated on the current iterate before iterations 1 + k n_col, k >= 0
     * (Alg. 1's n mod n_col = 1, the first on the initial guess; n_col = 0:
     * only at x^t).  Elements use the penalty energy with the closest point
     * recomputed at every evaluation and the triangle normal held fixed; same-
     * color updates read the positions from before the color (x_new buffer).
     * Needs launch_mode PLAIN or GRAPH (else VBD_E_UNSUPPORTED). */
    int32_t mesh_contacts;         /* 1 = on */
    float collision_radius;        /* > 0 when mesh_contacts is on */
    int32_t n_col;                 /* >= 0 */
    /* vbd_step_backward only: 1 = the workspace snapshot region already holds
     * this step's iterates (left there by vbd_step_record with the same
     * inputs, or copied back by the caller, see VBD_Q_SNAPSHOT_REGION), so the
     * forward recompute is skipped; 0 = recompute them. */
    int32_t backward_recorded;
    /* 1 = after the step, count the non-finite values of the output x and v
     * on the device (one extra pass over them); vbd_check then returns
     * VBD_E_NONFINITE when any was found.  0 = no check. */
    int32_t check_finite;
    /* Self-contact (Sec. 3.5 self-collisions), with mesh_contacts only: the
     * detection also pairs primitives of one mesh that share no vertex and
     * lie farther apart than self_exclusion in the rest shape; such a
     * vertex-triangle pair is a contact element when the element is active
     * (d > 0, closer than the contact thickness in front of the triangle or
     * behind it).  Else VBD_E_INVALID_ARG. */
    int32_t self_contact;          /* 1 = on */
    float self_exclusion;          /* >= 0, rest-shape distance */
    /* Edge-edge elements (Sec. 3.5, Fig. CollisionPotential), with
     * mesh_contacts only: at every detection each surface edge takes the
     * closest eligible surface edge (another mesh, or its own under the
     * self-contact rule) within collision_radius; the pair is an element when
     * its closest points are interior to both edges, the edges are not nearly
     * parallel (sine of their angle >= 0.1; parallel pairs are left to the
     * vertex-triangle elements of their end points) and the element is
     * active.  Energy k_c/2 d^2, d = delta - (x_a - x_b).n, x_a, x_b the
     * closest points (recomputed at every evaluation), n the unit direction
     * from x_b to x_a at x^t (held fixed); a pair found from both edges is
     * kept once (the lower edge index's).  Friction as for vertex-triangle
     * elements.  Up to two same-color vertex pairs per element read the
     * positions from before their color (x_new buffer, Sec. 3.9). */
    int32_t edge_contacts;         /* 1 = on */
} vbd_step_params;

/* One implicit-Euler time step of every mesh (Alg. 1):
 *   S^t = (x^t, v^t, v^{t-1}) -> S^{t+1} = (x^{t+1}, v^{t+1}, v^t), in place.
 * y = x^t + h v^t + h^2 a_ext (Eq. inertia); initial guess (Sec. 3.7);
 * n_iters sweeps over the colors in ascending order, each free vertex of a
 * color solving H_i dx = f_i (Eq. VBDLocalSystem, VBDForce, VBDHessian) over
 * its tets, springs and active contacts; optional Chebyshev acceleration
 * after each sweep; v^{t+1} = (x^{t+1} - x^t)/h (Eq. velocity_update).
 * x, v, v_prev: device float [n_verts][3]; tet_E: device float [n_tets]
 * Young's modulus per tet (may be NULL when n_tets == 0).  Pinned vertices
 * keep x^t and get v = 0.  Errors: VBD_E_NOT_COLORED, VBD_E_NO_WORKSPACE,
 * VBD_E_INVALID_ARG, VBD_E_HIP. */
vbd_status vbd_step(vbd_topology topo, const vbd_step_params *params, float *x, float *v,
                    float *v_prev, const float *tet_E, void *stream);

/* vbd_step for callers that cannot allocate device memory during the call
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same step, arguments, results and errors, with the per-step
 * state buffers (iterate, x^t, y, Chebyshev history, contact flags) taken
 * from a fixed device array of 96 MiB that the library holds on every device
 * it runs on until the process ends, instead of from the bound workspace.
 * Nothing is allocated: no hipMalloc, no graph, no profiling events.  Limits:
 * 3 x 16 + 1 bytes of state per vertex (5 x 16 + 1 with Chebyshev
 * acceleration), each section 256-B aligned, within 96 MiB (about 2.0M
 * vertices, 1.2M with acceleration; more: VBD_E_INVALID_ARG); launch_mode
 * PLAIN or PERSISTENT (graph modes: VBD_E_UNSUPPORTED); no mesh contacts
 * (VBD_E_UNSUPPORTED); the current device must be the one the workspace was
 * bound on (VBD_E_INVALID_ARG).  Every call on a device shares that device's
 * array: calls that overlap on one device (other streams, other topologies,
 * other threads) race and must be ordered by the caller.  Each step writes
 * every state entry it reads before reading it, so nothing carries over
 * between calls.  The skip and non-finite counters stay in the workspace. */
vbd_status vbd_step_static(vbd_topology topo, const vbd_step_params *params, float *x, float *v,
                           float *v_prev, const float *tet_E, void *stream);

/* Reverse mode of one vbd_step (tets + inertia + pins; springs, contacts,
 * damping and acceleration give VBD_E_UNSUPPORTED).  Recomputes the step's
 * iterates from the checkpoint S^t = (x_t, v_t, v_prev) and runs the adjoint
 * of the color sweeps in reverse order (n = N..1, colors descending), then the
 * adjoints of the initial guess and of y.  Each local update is the exact
 * minimiser of the vertex energy G_i (Eq. VBDEnergy; G_i is quadratic in x_i
 * for these tets), so its derivative is taken by the implicit function
 * theorem at the updated position.
 * Inputs gx_out, gv_out, gvp_out: adjoints of (x^{t+1}, v^{t+1}, v^t) as
 * device float [n_verts][3].  Outputs gx_in, gv_in, gvp_in: adjoints of
 * (x^t, v^t, v^{t-1}) (overwritten); g_tet_E: device float [n_tets],
 * ACCUMULATED (+=).  The workspace must have been sized with
 * max_backward_iters >= params->n_iters.  launch_mode GRAPH or
 * PERSISTENT_GRAPH: the launch sequence is captured into a hipGraph and
 * replayed while the pointers, parameters and stream stay the same (callers
 * that keep their buffers fixed pay the launch cost once); PLAIN or
 * PERSISTENT: plain launches. */
vbd_status vbd_step_backward(vbd_topology topo, const vbd_step_params *params,
                             const float *x_t, const float *v_t, const float *v_prev,
                             const float *tet_E, const float *gx_out, const float *gv_out,
                             const float *gvp_out, float *gx_in, float *gv_in, float *gvp_in,
                             float *g_tet_E, void *stream);

/* vbd_step for the differentiable path (tets, inertia and pins only, as
 * vbd_step_backward), in the form vbd_step_backward recomputes: the same
 * update, with snapshot n of the workspace left holding the iterate after
 * iteration n (0: the initial guess).  The caller may copy the snapshot
 * region (VBD_Q_SNAPSHOT_REGION) away and back, then call vbd_step_backward
 * with backward_recorded = 1 and the same x^t, v^t, v^{t-1}, tet_E to skip the
 * recompute.  x, v, v_prev: device float [n_verts][3], updated in place as by
 * vbd_step; tet_E as for vbd_step.  The workspace must have been sized with
 * max_backward_iters >= params->n_iters.  Launch modes as for
 * vbd_step_backward (GRAPH: captured and replayed while pointers, parameters
 * and stream stay the same).  Errors: as vbd_step_backward. */
vbd_status vbd_step_record(vbd_topology topo, const vbd_step_params *params, float *x, float *v,
                           float *v_prev, const float *tet_E, void *stream);

/* Runs the edge-edge detection that vbd_step does (params: mesh_contacts and
 * edge_contacts must be 1) with closest points on x and normals from x_t
 * (device float [n_verts][3] each, original order; x = x_t is the detection
 * at the start of a step) and writes, for every surface edge in
 * VBD_Q_SURFACE_EDGES order, the second edge of the element kept from it
 * (the elements are the pairs (e, partner_out[e]) with partner_out[e] >= 0),
 * or -1 (partner_out: device int32 [n_surf_edges]).  Uses the library's
 * internal state buffers.  Errors as vbd_detect_contacts. */
vbd_status vbd_detect_edges(vbd_topology topo, const vbd_step_params *params, const float *x,
                            const float *x_t, int32_t *partner_out, void *stream);

/* Runs the mesh-mesh contact detection that vbd_step does at x^t (params:
 * mesh_contacts must be 1; collision_radius and contact_thickness are used) on
 * the positions x (device float [n_verts][3], original order) and writes, for
 * every vertex, the index of its contact triangle in VBD_Q_SURFACE order or -1
 * (tri_out: device int32 [n_verts], original order).  Uses the library's
 * internal state buffers (a following vbd_step is unaffected).  Errors:
 * VBD_E_NOT_COLORED, VBD_E_NO_WORKSPACE, VBD_E_INVALID_ARG, VBD_E_HIP. */
vbd_status vbd_detect_contacts(vbd_topology topo, const vbd_step_params *params, const float *x,
                               int32_t *tri_out, void *stream);

/* Kernel launch configuration of the color solve. */
typedef struct {
    int32_t lanes_per_vertex;   /* 2, 4, 8, 16 or 32 lanes of a wave64 per vertex */
    int32_t block_size;         /* 64..512, multiple of 64 */
    int32_t xcd_remap;          /* 0: blocks as launched (round-robin over the 8
                                   XCDs), 1: each XCD a contiguous range of blocks,
                                   2: chunks of 16 consecutive blocks dealt to the
                                   XCDs in turn, 3: each XCD a contiguous part of the
                                   color cut at mesh boundaries with about equal work
                                   (VBD_Q_XCD_SPLIT; the color solve only, elsewhere
                                   as 1); other values: VBD_E_INVALID_ARG.  The
                                   backward's reverse phases always map as 1. */
    int32_t blocks_per_cu;      /* persistent kernel: resident blocks per CU (0 = max) */
    int32_t tet_unroll;         /* 1..3 tet entries per lane loaded together */
    int32_t compact_records;    /* 1: 32-B pair records (|m|^2 summed from w in the
                                   solve; fewer bytes), 0: 36-B records (|m|^2
                                   stored; fewer registers) */
} vbd_launch_config;
vbd_status vbd_get_launch_config(vbd_topology topo, vbd_launch_config *cfg);
vbd_status vbd_set_launch_config(vbd_topology topo, const vbd_launch_config *cfg);

/* Autotuner: times the color-solve sweep for each candidate configuration on
 * this topology (predict from the given state, then sweeps on the library's
 * internal copy; the caller's x, v, v_prev are not modified) and keeps the
 * fastest.  Results are cached in-process per (device arch, size bucket,
 * element kinds, launch mode); a cached entry is reused without timing.
 * Synchronizes `stream`. */
vbd_status vbd_autotune(vbd_topology topo, const vbd_step_params *params, const float *x,
                        const float *v, const float *v_prev, const float *tet_E, void *stream);

/* Marker ranges: vbd_build_topology, vbd_color_greedy (and so vbd_color),
 * vbd_color_given, vbd_bind_workspace, vbd_step, vbd_step_record,
 * vbd_step_backward, vbd_detect_edges, vbd_detect_contacts and vbd_autotune
 * each open a ROCTx range named after the call for its whole duration (host
 * time: the enqueue, plus the synchronizations the call itself makes), seen
 * by tools that trace markers (rocprofv3 --marker-trace); inside them, the
 * plain launch sequence of a step opens "vbd iteration" and "vbd color phase"
 * ranges (the backward's "vbd reverse iteration" and "vbd reverse color
 * phase"), around the enqueue of each (a graph replays them without host
 * work, a persistent launch has no host-side phases); vbd_step_static opens
 * none.  Without such a tool the ranges cost a function call each.
 *
 * Timing of the hot kernel (hipEvents on the launch stream).  When enabled,
 * vbd_step runs its plain launch sequence and records one event pair around
 * the step's back-to-back color-solve launches (or around the persistent
 * kernel), and vbd_step_backward (plain launches) one around its reverse
 * sweep's adjoint color phases, with VBD_Q_ADJ_PHASE_BYTES as their bytes;
 * total_ms / n_launches is the average launch duration.
 * vbd_profile_read synchronizes and reports totals since the last reset. */
typedef struct {
    int64_t n_launches;        /* timed hot-kernel launches */
    double total_ms;           /* summed event time of those launches */
    double total_bytes;        /* summed algorithmic HBM bytes of those launches */
    int64_t n_vertex_updates;  /* local solves of free vertices inside them */
} vbd_profile_stats;
vbd_status vbd_profile_enable(vbd_topology topo, int32_t enable);
vbd_status vbd_profile_read(vbd_topology topo, vbd_profile_stats *out, int32_t reset);

/* Reads the device-side guard flags on `stream` (synchronizes).
 * VBD_E_DEVICE if the persistent kernel's barrier guard fired since the last
 * check; VBD_E_NONFINITE if a step run with check_finite produced a
 * non-finite position or velocity since the last check.  The flag that is
 * reported is then cleared. */
vbd_status vbd_check(vbd_topology topo, void *stream);

/* Event counters of a topology, accumulated on the device over every step
 * (vbd_step, vbd_step_record and the backward's recompute; the autotuner's
 * timed sweeps are not counted) since the last reset. */
typedef struct {
    int64_t n_skips;       /* local solves skipped by the determinant rule of
                              Sec. 3.2 (|det H_i| <= det_eps_rel ||H_i||_F^3:
                              the vertex keeps its position) */
    int64_t n_nonfinite;   /* non-finite output values found by check_finite */
} vbd_counters;
/* Copies the counters to *out on `stream` (synchronizes); reset != 0 then
 * clears them.  Errors: VBD_E_INVALID_ARG, VBD_E_NOT_COLORED,
 * VBD_E_NO_WORKSPACE, VBD_E_HIP. */
vbd_status vbd_read_counters(vbd_topology topo, vbd_counters *out, int32_t reset, void *stream);

/* Device copy probe: copies n_bytes (multiple of 16) from src to dst with
 * the library's own streaming kernel; used to measure achievable HBM
 * bandwidth and to calibrate traffic counters. */
vbd_status vbd_probe_copy(void *dst, const void *src, size_t n_bytes, void *stream);

/* Device read probe: n_blocks (1..65535) blocks of 256 threads read n_bytes
 * (multiple of 16) from src, 8 loads of 16 B in flight per thread, and write
 * one partial sum per block into partials (device float[n_blocks]); the
 * achievable read-dominant HBM bandwidth that the solve kernels, whose traffic
 * is almost all reads, are quoted against. */
vbd_status vbd_probe_read(const void *src, size_t n_bytes, float *partials, int32_t n_blocks,
                          void *stream);

const char *vbd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
