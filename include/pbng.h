/*
 * pbng.h -- C ABI of libpbng: Position-Based Nonlinear Gauss-Seidel (PBNG)
 * for quasistatic hyperelasticity on linear-tetrahedral meshes, on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Chen, Han, Chen & Teran, "Position-Based Nonlinear Gauss-Seidel
 * for Quasistatic Hyperelasticity" (arXiv 2306.09021).  The problem solved
 * is the Dirichlet-constrained minimisation of the discrete potential
 * energy minus external work (Sec. "Discretization", Eq. fem_qs / fem_d and
 * the argmin over W that follows them), with the hyperelastic energies of
 * Sec. "Constitutive Models" (Eq. cor, Eq. nh) and the weak constraints of
 * Sec. "Weak Constraints".  The iteration is the position-based nonlinear
 * Gauss-Seidel of Sec. "Position-Based Nonlinear Gauss-Seidel" (Eq.
 * pbgn_update, pbgn_dx) with the modified Hessian of Eq. mod_hess_dens /
 * mod_hess, run over the node colouring of Sec. "Coloring and Parallelism",
 * with the Chebyshev / SOR blends of Sec. "Acceleration Techniques".
 *
 * Conventions
 *  - Every function returns an int32_t status: 0 = PBNG_OK, positive =
 *    warning (results valid), negative = error (outputs unspecified).  The
 *    thread-local text of the last error is returned by pbng_last_error().
 *    No C++ exception crosses this interface.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *    device allocations on the current device (e.g. torch cuda tensors).
 *  - The caller owns every buffer it passes.  The library keeps no caller
 *    pointer after a call returns; a workspace copies what it needs.
 *  - Positions are row-major [n][3] arrays of the workspace's position type
 *    (float for PBNG_F32, double for PBNG_F64 and PBNG_MIXED), in the
 *    caller's vertex order; batched problems are concatenated instance
 *    after instance.
 *  - hip_stream may be NULL (the null stream).  Calls that return host
 *    results (stats, norms) synchronise that stream before returning.
 */
#ifndef PBNG_H
#define PBNG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PBNG_ABI_VERSION 1

/* ---- status codes ---------------------------------------------------- */
#define PBNG_OK 0
#define PBNG_NOT_CONVERGED 1      /* iteration cap reached; outputs valid */
#define PBNG_EINVAL (-1)          /* null pointer, bad size or option      */
#define PBNG_EMESH (-2)           /* index out of range, repeated vertex,  */
                                  /* rest volume <= 0                      */
#define PBNG_EMATERIAL (-3)       /* mu <= 0 or lambda <= 0 (the modified  */
                                  /* Hessian is SPD only for lambda > 0)   */
#define PBNG_ECOLOR (-4)          /* colouring invalid or > 64 colours     */
#define PBNG_ENAN (-5)            /* non-finite input or iterate           */
#define PBNG_EHIP (-6)            /* HIP runtime failure                   */
#define PBNG_ENOMEM (-7)          /* allocation failure                    */
#define PBNG_EUNSUPPORTED (-8)    /* e.g. a workspace too large for 32-bit offsets */

/* ---- enumerations ---------------------------------------------------- */
#define PBNG_NEOHOOKEAN 0   /* Eq. nh: 1/2 mu |F|^2 + lhat/2 (J - 1 - mu/lhat)^2, lhat = mu + lambda */
#define PBNG_COROTATED 1    /* Eq. cor: mu |F - R(F)|^2 + lambda/2 (J - 1)^2 */
/* Eq. snh with the Lame lambda on its volume term (the printed equation
 * lacks it; with it the rest state is stress free):
 * 1/2 mu (|F|^2 - 3) + 1/2 lambda (J - 1 - 3 mu / (4 lambda))^2 - 1/2 mu log(1 + |F|^2).
 * Needs lambda > 0. */
#define PBNG_STABLE_NEOHOOKEAN 2

#define PBNG_F32 0    /* positions and sweep arithmetic in float             */
#define PBNG_F64 1    /* positions and sweep arithmetic in double            */
#define PBNG_MIXED 2  /* positions in double (an FP64 master copy of the    */
                      /* iterate), sweep arithmetic in float on edge vectors */
                      /* x_j - x_i formed in double                          */

#define PBNG_ACCEL_NONE 0
#define PBNG_ACCEL_CHEBYSHEV 1  /* x^{l+1} = w_{l+1}(gamma (x_P - x^l) + x^l - x^{l-1}) + x^{l-1} */
#define PBNG_ACCEL_SOR 2        /* x^{l+1} = omega (x_P - x^{l-1}) + x^{l-1} */

#define PBNG_SAFEGUARD_NONE 0       /* the paper's plain single step       */
#define PBNG_SAFEGUARD_BACKTRACK 1  /* halve the step until the local      */
                                    /* energy does not increase            */

/* ---- problem statement (host memory, one struct per instance) --------- */
/*
 * One quasistatic problem (Sec. "Discretization"): rest mesh, material,
 * Dirichlet targets, external force and weak constraints.
 *
 *  n_verts, n_tets      mesh size (n_tets may be 0 for spring-only systems)
 *  rest_pos  [n_verts][3]  rest positions X_i (double)
 *  tets      [n_tets][4]   vertex indices; every tet must have positive rest
 *                          volume det[X1-X0, X2-X0, X3-X0] / 6 > 0
 *  model                PBNG_NEOHOOKEAN, PBNG_COROTATED or PBNG_STABLE_NEOHOOKEAN
 *                       (one model per workspace)
 *  mu, lambda           uniform Lame parameters (Eq. lame), used when
 *                       mu_tet / lambda_tet are NULL
 *  mu_tet, lambda_tet   optional [n_tets] per-tet Lame parameters
 *  density, gravity[3]  body force density R0 g; lumped as R0 g V0_e / 4
 *                       onto each vertex of tet e
 *  nodal_force [n_verts][3]  optional extra lumped load (e.g. tractions);
 *                       may be NULL
 *  n_dirichlet, dirichlet_idx [n_dirichlet], dirichlet_x [n_dirichlet][3]
 *                       prescribed vertices and their targets x_D
 *  n_wc, wc_ptr [n_wc+1], wc_vert [nnz], wc_w [nnz], wc_K [n_wc][6]
 *                       weak constraints (Sec. "Weak Constraints"):
 *                       C_c = sum_j wc_w[j] y_{wc_vert[j]} over
 *                       j in [wc_ptr[c], wc_ptr[c+1]) with wc_w = w0 - w1,
 *                       energy 1/2 C_c^T K_c C_c, K_c symmetric stored as
 *                       (xx, xy, xz, yy, yz, zz).  NULL when n_wc == 0.
 *  n_planes, planes [n_planes][5]
 *                       contact half-spaces (n_x, n_y, n_z, d, k): every
 *                       vertex with phi = n . y - d < 0 carries the
 *                       penalty 1/2 k phi^2 (a zero-rest-length spring to
 *                       its projection with stiffness k n n^T).
 */
typedef struct pbng_problem {
    int32_t n_verts;
    int32_t n_tets;
    const double* rest_pos;
    const int32_t* tets;
    int32_t model;
    double mu;
    double lambda;
    const double* mu_tet;
    const double* lambda_tet;
    double density;
    double gravity[3];
    const double* nodal_force;
    int32_t n_dirichlet;
    const int32_t* dirichlet_idx;
    const double* dirichlet_x;
    int32_t n_wc;
    const int32_t* wc_ptr;
    const int32_t* wc_vert;
    const double* wc_w;
    const double* wc_K;
    int32_t n_planes;
    const double* planes;
} pbng_problem;

/* ---- solver options --------------------------------------------------- */
/*
 *  max_sweeps      Gauss-Seidel sweeps (iterations l) at most
 *  rel_tol         stop an instance when ||r(x^l)|| / ||r(x^0)|| <= rel_tol,
 *                  r = f + fhat over free vertices in FP64 (0 disables)
 *  check_every     sweeps between FP64 residual checks (>= 1)
 *  accel           PBNG_ACCEL_*; rho / gamma for Chebyshev, omega for SOR
 *  safeguard       PBNG_SAFEGUARD_*; max_halvings step halvings at most
 *                  (a vertex whose step never passes keeps its position)
 *  lanes           lanes of a 64-wide wavefront per vertex (1, 2, 4, 8,
 *                  16, 32, 64); 0 = per colour, the power of two covering
 *                  half the colour's mean number of incident tets
 *  sweeps_per_graph  >0: once the blend weight is at its fixed point,
 *                  capture that many sweeps (rounded up to even with a
 *                  blend) in one HIP graph and replay it between residual
 *                  checks; 0 = plain launches.  Needs a non-null stream.
 *  resume          1: continue the acceleration state (x^{l-1}, l,
 *                  omega_l) left in the workspace by the previous solve
 *                  instead of starting a new iteration at l = 0
 */
typedef struct pbng_solve_opts {
    int32_t max_sweeps;
    double rel_tol;
    int32_t check_every;
    int32_t accel;
    double rho;
    double gamma;
    double omega;
    int32_t safeguard;
    int32_t max_halvings;
    int32_t lanes;
    int32_t sweeps_per_graph;
    int32_t resume;
} pbng_solve_opts;

/* Per-instance results. */
typedef struct pbng_stats {
    int32_t sweeps;          /* sweeps applied to this instance            */
    int32_t converged;       /* 1 if rel_residual <= rel_tol was reached   */
    int32_t n_colors;        /* colours of this instance                   */
    int32_t rejected;        /* safeguard: vertex updates left unapplied   */
    double residual0;        /* ||r(x^0)||_2, FP64                         */
    double residual;         /* ||r|| at the last check, FP64              */
    double rel_residual;     /* residual / residual0                       */
    double energy;           /* total energy at the last check, FP64       */
    double time_ms;          /* wall time of the whole (batched) call      */
    double time_to_tol_ms;   /* time at which rel_tol was first met, or -1 */
    double vertex_updates;   /* free-vertex local updates performed        */
} pbng_stats;

/* Adjoint options (block Gauss-Seidel on the true Hessian). */
typedef struct pbng_adjoint_opts {
    int32_t max_sweeps;
    double rel_tol;          /* on ||b - H lam|| / ||b||, FP64             */
    int32_t check_every;
    int32_t accel;           /* PBNG_ACCEL_NONE or PBNG_ACCEL_CHEBYSHEV    */
    double rho;
    double gamma;
    int32_t lanes;
} pbng_adjoint_opts;

typedef struct pbng_workspace pbng_workspace;

/* ---- functions -------------------------------------------------------- */

/* ABI version (PBNG_ABI_VERSION). */
int32_t pbng_version(void);

/* Thread-local text of the last error (never NULL). */
const char* pbng_last_error(void);

/* Eq. lame, element-wise over n host values: mu = E / (2 (1 + nu)),
 * lambda = E nu / ((1 + nu)(1 - 2 nu)).  E, nu: host [n] inputs; mu_out,
 * lambda_out: host [n] outputs.  Returns PBNG_EINVAL for a nu outside
 * (-1, 0.5), an E <= 0 or a null pointer (outputs then unspecified). */
int32_t pbng_lame(int64_t n, const double* E, const double* nu, double* mu_out, double* lambda_out);

/* Fill *o with defaults: 1000 sweeps, rel_tol 1e-5, check_every 10, no
 * acceleration (rho 0.95, gamma 1.7, omega 1.7 when enabled), backtracking
 * safeguard with 8 halvings, automatic lanes, plain launches. */
int32_t pbng_default_solve_opts(pbng_solve_opts* o);
int32_t pbng_default_adjoint_opts(pbng_adjoint_opts* o);

/*
 * Node colouring, Sec. "Coloring and Parallelism".  Host memory only.
 * Free vertices are visited in ascending index; each takes the least
 * colour absent from the used-colour sets S_c of its incident tets and
 * weak constraints, then registers it in each of them.  Dirichlet vertices
 * get -1.  colors_out [p->n_verts]; *n_colors_out = number of colours.
 * Reads n_verts, n_tets, tets, the Dirichlet list and the weak-constraint
 * CSR (wc_ptr, wc_vert), which are checked first as in
 * pbng_workspace_create.  Errors: PBNG_EINVAL (bad sizes, n_tets >= 2^29,
 * a null array, a repeated or out-of-range Dirichlet index, a malformed
 * wc_ptr), PBNG_EMESH (tet or constraint vertex out of range, a repeated
 * vertex), PBNG_ECOLOR (more than 64 colours would be needed).
 */
int32_t pbng_color(const pbng_problem* p, int32_t* colors_out, int32_t* n_colors_out);

/*
 * Validate and pack n_problems instances (host array p[n_problems]) for
 * the device: rest-state gradients and volumes, lumped loads, colour-major
 * vertex order and per-visit records.  colors (host, concatenated
 * [sum n_verts], -1 on Dirichlet vertices) may be NULL to colour with
 * pbng_color; a supplied colouring is checked (no two same-coloured
 * vertices may share a tet or weak constraint).  real = PBNG_F32, PBNG_F64
 * or PBNG_MIXED selects the sweep arithmetic and the position type.
 * Allocates device memory on the current device; *ws_out receives the
 * handle.  Errors: PBNG_EINVAL, PBNG_EMESH, PBNG_EMATERIAL, PBNG_ECOLOR,
 * PBNG_ENAN, PBNG_EHIP, PBNG_ENOMEM.
 */
int32_t pbng_workspace_create(const pbng_problem* p, int32_t n_problems, const int32_t* colors,
                              int32_t real, pbng_workspace** ws_out);

/* Release a workspace (NULL is accepted). */
int32_t pbng_workspace_destroy(pbng_workspace* ws);

/* Sizes of a workspace: total vertices, tets, free vertices, colours
 * (maximum over instances), visits (free vertex, incident tet) per sweep,
 * instances.  Any output may be NULL. */
int32_t pbng_workspace_info(const pbng_workspace* ws, int64_t* n_verts, int64_t* n_tets,
                            int64_t* n_free, int32_t* n_colors, int64_t* n_visits,
                            int32_t* n_instances);

/* Replace the Lame parameters (device double arrays [sum n_tets]) or the
 * Dirichlet targets (device double array [sum n_dirichlet][3], in the order
 * given at creation) of a workspace.  Errors: PBNG_EINVAL, PBNG_EHIP. */
int32_t pbng_workspace_set_materials(pbng_workspace* ws, const double* mu_dev,
                                     const double* lambda_dev, void* hip_stream);
int32_t pbng_workspace_set_dirichlet(pbng_workspace* ws, const double* xd_dev, void* hip_stream);

/* Backward-Euler inertia (Eq. fem_be, minimised as the incremental
 * potential): with dt > 0 every later solve, residual and adjoint of the
 * workspace adds sum over free vertices i of 1/2 m_ii / dt^2 |y_i - xhat_i|^2
 * to the energy, with xhat = 2 x^n - x^{n-1} and the lumped mass
 * m_ii = R0 sum_{e incident to i} V0_e / 4 (R0 = each problem's `density`).
 * Then A_i gains m_ii / dt^2 I and g_i gains m_ii / dt^2 (y_i - xhat_i).
 * x_n_dev, x_prev_dev: device double arrays [n_verts][3] over all instances
 * in the caller's order (Dirichlet rows are ignored), read on hip_stream
 * before the call returns to the stream; the workspace keeps its own copy of
 * xhat.  dt <= 0 switches inertia off (the pointers may then be NULL).
 * Errors: PBNG_EINVAL (null arrays with dt > 0, non-finite dt), PBNG_EHIP. */
int32_t pbng_workspace_set_inertia(pbng_workspace* ws, double dt, const double* x_n_dev,
                                   const double* x_prev_dev, void* hip_stream);

/* Dynamic weak constraints (Sec. "Weak Constraints" with Sec. "Collisions"
 * and "Collision Coloring"): replaces the workspace's contact set by n
 * vertex-vertex contacts, each the weak constraint C = y_a - y_b with the
 * anisotropic stiffness K = k_n n n^T (n normalised here; the tangential
 * stiffness is 0), next to the problems' static weak constraints.
 * pairs_dev: device int32 [n][2] of caller vertex indices over the whole
 * workspace (both vertices of one instance, distinct); normals_dev: device
 * double [n][3].  Then recolours as the paper prescribes: every free vertex
 * incident to a contact, in ascending caller index, keeps its colour unless
 * a vertex sharing a tet or a weak constraint with it has it, and otherwise
 * takes the least colour none of them has.  Vertices keep their storage;
 * a recoloured vertex runs in its new colour's phase.  Synchronises
 * hip_stream.  n = 0 removes the contacts (colours stay valid).
 * Errors: PBNG_EINVAL (bad pairs, normals or stiffness), PBNG_EHIP. */
int32_t pbng_workspace_set_contacts(pbng_workspace* ws, int32_t n, const int32_t* pairs_dev,
                                    const double* normals_dev, double k_n, void* hip_stream);

/* Vertex-vertex proximity detection for pbng_workspace_set_contacts: all
 * pairs (a, b), a < b in caller order, of surface vertices (vertices of a
 * face that belongs to one tet) of different connected parts of one
 * instance whose distance is at most radius and positive, not both
 * Dirichlet, at the positions x_dev (device [n_verts][3] of the position
 * type: float for PBNG_F32, double otherwise, caller order).  Outputs
 * (device): pairs_dev int32 [max_pairs][2] sorted by (a, b), normals_dev
 * double [max_pairs][3] = (x_b - x_a) / |x_b - x_a|; *n_found (host) the
 * number of pairs.  Uses a uniform grid of cell size radius (sorted cell
 * keys, 27-cell search); allocates its scratch on first use or growth.
 * Synchronises hip_stream.  Errors: PBNG_EINVAL (bad radius or arrays, or
 * more than max_pairs pairs: *n_found then holds the count), PBNG_EHIP. */
int32_t pbng_detect_contacts(pbng_workspace* ws, const void* x_dev, double radius, int32_t max_pairs,
                             int32_t* pairs_dev, double* normals_dev, int32_t* n_found,
                             void* hip_stream);

/* The current colouring: colors_out host int32 [n_verts] in the caller's
 * order, -1 on Dirichlet vertices. */
int32_t pbng_workspace_colors(const pbng_workspace* ws, int32_t* colors_out);

/*
 * Solve (Eq. pbgn_update / pbgn_dx over the colours, with the optional
 * Chebyshev / SOR blend of Sec. "Acceleration Techniques").  x_inout
 * (device, [sum n_verts][3] of the workspace's real type) holds the initial
 * iterate on entry and the result on exit; Dirichlet rows are overwritten
 * with their targets.  stats (host, [n_instances]) may be NULL.  Returns
 * PBNG_OK when every instance met rel_tol, PBNG_NOT_CONVERGED when some did
 * not within max_sweeps (outputs valid), PBNG_ENAN when an iterate became
 * non-finite, or another error.
 */
int32_t pbng_solve(pbng_workspace* ws, void* x_inout, const pbng_solve_opts* o,
                   pbng_stats* stats, void* hip_stream);

/*
 * FP64 residual and energy (Eq. fem_qs, pe_hat): for every instance,
 * res_norm[q] = ||f(x) + fhat||_2 over free vertices and energy[q] =
 * PE(x) - x . fhat (+ plane penalties).  x: device, [sum n_verts][3] of the
 * workspace's real type.  res_norm, energy: host [n_instances], either may
 * be NULL.  r_out: optional device double [sum n_verts][3] receiving r
 * (zero on Dirichlet rows).
 */
int32_t pbng_residual(pbng_workspace* ws, const void* x, double* res_norm, double* energy,
                      double* r_out, void* hip_stream);

/*
 * Adjoint of the equilibrium.  At an equilibrium x_eq
 * (device, workspace real type), solve H lam = dL/dx restricted to free
 * vertices, H the true energy Hessian (Eq. hess with the exact density), by
 * block Gauss-Seidel over the same colouring (diagonal blocks: the true
 * H_ii for Neo-Hookean, the modified A_ii >= H_ii for the corotated and
 * stable Neo-Hookean models, whose H_ii need not be positive away from a
 * stable equilibrium; the corotated rotation derivative is singular where
 * two signed singular values sum to zero, so inverted elements are not
 * supported there), then assemble
 *   dL/dmu_e     = -V0_e < dP/dmu (F_e) , Lam_e >
 *   dL/dlambda_e = -V0_e < (J_e - 1) cof F_e , Lam_e >
 * with dP/dmu = F + (J - 2) cof F (Neo-Hookean), 2 (F - R) (corotated),
 * (1 - 1/(1 + |F|^2)) F - 3/4 cof F (stable Neo-Hookean), and
 *   dL/dx_k      = (dL/dx)_k - (H lam)_k  for Dirichlet vertices k
 * (the first term because x*_k = x_D,k), Lam_e = sum_j lam_j dN_j^T.
 * dL_dx: device [sum n_verts][3] (workspace real type).  Outputs (device, double, any may be
 * NULL): dL_dxD [sum n_dirichlet][3] in creation order, dL_dmu and
 * dL_dlambda [sum n_tets], lam_out [sum n_verts][3] (zero on Dirichlet
 * rows).  stats [n_instances] (host, may be NULL): sweeps, residuals of
 * the adjoint system.
 */
int32_t pbng_adjoint(pbng_workspace* ws, const void* x_eq, const void* dL_dx, double* dL_dxD,
                     double* dL_dmu, double* dL_dlambda, double* lam_out,
                     const pbng_adjoint_opts* o, pbng_stats* stats, void* hip_stream);

/*
 * Autotuner: on the iterate x (device, position type), times, colour by
 * colour, each lanes-per-vertex candidate (1 .. 64 around the colour's mean
 * visit count) inside whole sweeps (best of 3 x 16 sweeps, the other colours
 * at their current choice) and keeps a candidate only when it beats the
 * automatic heuristic by more than 2%; the result becomes the workspace's
 * automatic choice (o->lanes = 0).  It then times 64 sweeps as plain
 * launches and as replays of graphs of 2, 8 and 32 sweeps.  *tuned receives *o with lanes = 0 and the chosen
 * sweeps_per_graph; lanes_out [n_colors] (host, nullable) the lanes per
 * colour.  hip_stream must not be NULL.  The workspace's internal iterate is
 * left undefined (the next pbng_solve reloads it).
 */
int32_t pbng_autotune(pbng_workspace* ws, const void* x, const pbng_solve_opts* o,
                      pbng_solve_opts* tuned, int32_t* lanes_out, void* hip_stream);

/*
 * Launch-level access for measurement: run n_sweeps sweeps (with the
 * blend of o->accel, no residual) on the workspace's internal iterate, or a
 * single colour phase (the same kernel the solve launches for o; with
 * acceleration it blends with omega = gamma = 1 and does not advance the
 * iteration), on hip_stream without synchronising.  The internal iterate
 * is loaded from x (device) by pbng_load, and written back by pbng_store.
 * Algorithmic bytes of one colour phase are reported by
 * pbng_phase_bytes (sum over its visits of the 56-byte visit record and
 * 4-byte visit index, 24 bytes per updated vertex, 12 bytes per distinct
 * neighbour read).
 */
int32_t pbng_load(pbng_workspace* ws, const void* x, void* hip_stream);
int32_t pbng_store(pbng_workspace* ws, void* x, void* hip_stream);
int32_t pbng_sweeps(pbng_workspace* ws, int32_t n_sweeps, const pbng_solve_opts* o,
                    void* hip_stream);
int32_t pbng_phase(pbng_workspace* ws, int32_t color, const pbng_solve_opts* o, void* hip_stream);
int32_t pbng_phase_bytes(const pbng_workspace* ws, int32_t color, int64_t* bytes,
                         int64_t* vertices, int64_t* visits);

#ifdef __cplusplus
}
#endif

#endif /* PBNG_H */
