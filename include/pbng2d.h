/*
 * pbng2d.h -- C ABI of libpbng for planar problems: Position-Based
 * Nonlinear Gauss-Seidel on triangle meshes (d = 2) on AMD Instinct MI355X
 * (gfx950).
 *
 * The method is the one of pbng.h with d = 2 (Sec. "Discretization":
 * piecewise-linear interpolation over a triangle mesh; positions in R^2).
 * The deformation gradient of a triangle is 2x2; the constitutive models
 * are Eq. (cor) and Eq. (nh) with 2x2 F, det F and the 2x2 cofactor
 * matrix; the modified Hessian density of Eq. (mod_hess_dens) and the nodal
 * matrix of Eq. (mod_hess) are 2x2; each vertex update of Eq. (pbgn_update)
 * / (pbgn_dx) solves a 2x2 SPD system.  The planar experiment of Sec.
 * "PBNG vs. PBD and Limited Newton" is of this kind.
 *
 * Weak constraints (Sec. "Weak Constraints"), contact half-planes and the
 * backward-Euler inertia of Eq. (fem_be) enter as in pbng.h with d = 2.
 *
 * Conventions are those of pbng.h (status codes, pbng_last_error(), host
 * and device pointers, ownership, streams), with positions as row-major
 * [n][2] arrays in the caller's vertex order.  One problem per workspace.
 * Not supported in the planar family: the stable Neo-Hookean model (its
 * printed rest-state constant 3 mu / (4 lambda) makes F = I stress free
 * only for d = 3), and contact detection with recolouring.
 */
#ifndef PBNG2D_H
#define PBNG2D_H

#include <stdint.h>

#include "pbng.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * One planar quasistatic problem (host memory):
 *  n_verts, n_tris      mesh size (n_tris >= 1)
 *  rest_pos [n_verts][2] rest positions X_i
 *  tris     [n_tris][3]  vertex indices, counter-clockwise: every triangle
 *                        needs positive rest area det[X1-X0, X2-X0] / 2 > 0
 *  model                PBNG_NEOHOOKEAN or PBNG_COROTATED
 *  mu, lambda           uniform Lame parameters, used when mu_tri /
 *                        lambda_tri are NULL (both must be > 0)
 *  mu_tri, lambda_tri   optional [n_tris] per-triangle Lame parameters
 *  density, gravity[2]  body force R0 g, lumped as R0 g A0_e / 3 onto each
 *                        vertex of triangle e (unit thickness)
 *  nodal_force [n_verts][2]  optional extra lumped load (may be NULL)
 *  n_dirichlet, dirichlet_idx [n_dirichlet], dirichlet_x [n_dirichlet][2]
 *                        prescribed vertices (distinct) and their targets
 *  n_wc, wc_ptr [n_wc+1], wc_vert [nnz], wc_w [nnz], wc_K [n_wc][3]
 *                        weak constraints: C_c = sum_j wc_w[j] y_{wc_vert[j]}
 *                        over j in [wc_ptr[c], wc_ptr[c+1]) (wc_ptr[0] = 0,
 *                        non-decreasing, distinct vertices per constraint),
 *                        energy 1/2 C_c^T K_c C_c with K_c symmetric stored
 *                        as (xx, xy, yy); arrays may be NULL when n_wc == 0
 *  n_planes, planes [n_planes][4]
 *                        contact half-planes (n_x, n_y, d, k), k >= 0: every
 *                        vertex with phi = n . y - d < 0 carries the penalty
 *                        1/2 k phi^2
 * Fields after dirichlet_x were added with the constraints; zero them
 * (n_wc = n_planes = 0) for a purely elastic problem.
 */
typedef struct pbng2d_problem {
    int32_t n_verts;
    int32_t n_tris;
    const double* rest_pos;
    const int32_t* tris;
    int32_t model;
    double mu;
    double lambda;
    const double* mu_tri;
    const double* lambda_tri;
    double density;
    double gravity[2];
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
} pbng2d_problem;

typedef struct pbng2d_workspace pbng2d_workspace;

/*
 * Node colouring (Sec. "Coloring and Parallelism"), host only: free
 * vertices in ascending index each take the least colour used by no
 * already coloured vertex of an incident triangle or weak constraint;
 * Dirichlet vertices get -1.  colors_out [n_verts]; *n_colors_out the number of colours.
 * Errors: PBNG_EINVAL, PBNG_EMESH, PBNG_ECOLOR (more than 64 colours),
 * PBNG_EUNSUPPORTED (n_tris above INT32_MAX / 3, checked before tris is
 * read).
 */
int32_t pbng2d_color(const pbng2d_problem* p, int32_t* colors_out, int32_t* n_colors_out);

/*
 * Validate and pack a problem for the device (current device).  colors
 * (host [n_verts], -1 on Dirichlet vertices) may be NULL to colour with
 * pbng2d_color; a supplied colouring is checked.  real = PBNG_F32 or
 * PBNG_F64 (positions and sweep arithmetic; PBNG_MIXED is not offered).
 * Errors: PBNG_EINVAL, PBNG_EMESH, PBNG_EMATERIAL, PBNG_ECOLOR, PBNG_ENAN,
 * PBNG_EUNSUPPORTED (a model other than the two above, or a mesh too large
 * for the 32-bit indices and stream offsets), PBNG_EHIP, PBNG_ENOMEM.
 */
int32_t pbng2d_workspace_create(const pbng2d_problem* p, const int32_t* colors, int32_t real,
                                pbng2d_workspace** ws_out);
int32_t pbng2d_workspace_destroy(pbng2d_workspace* ws);

/* Sizes: vertices, triangles, free vertices, colours, visits (free vertex,
 * incident triangle) per sweep.  Any output may be NULL. */
int32_t pbng2d_workspace_info(const pbng2d_workspace* ws, int64_t* n_verts, int64_t* n_tris,
                              int64_t* n_free, int32_t* n_colors, int64_t* n_visits);

/* The colouring in use: colors_out host int32 [n_verts], caller order. */
int32_t pbng2d_workspace_colors(const pbng2d_workspace* ws, int32_t* colors_out);

/*
 * Solve: x_inout (device [n_verts][2] of the workspace's real type) holds
 * the initial iterate and receives the result; Dirichlet rows are set to
 * their targets.  Uses max_sweeps, rel_tol, check_every, accel (rho,
 * gamma / omega), safeguard, max_halvings and lanes (0 = 4 lanes per
 * vertex) of o; sweeps_per_graph and resume are ignored.  The backtracking
 * safeguard is exact for the Neo-Hookean model (its local energy is a
 * quadratic along the step, |F|^2 being quadratic and det F affine in
 * x_i, and so are the weak constraints and the inertia; half-plane
 * penalties are evaluated exactly); for the corotated model the full step
 * never increases the local energy (mu |F' - R(F')|^2 <= mu |F' - R(F)|^2
 * majorises it by the quadratic whose Hessian is the modified matrix A_i)
 * unless it enters a half-plane, so halvings are only ever tested, on the
 * exact energy, when that bound fails.  stats (host, one entry) may be NULL.  Returns PBNG_OK,
 * PBNG_NOT_CONVERGED (outputs valid), PBNG_ENAN or another error.
 */
int32_t pbng2d_solve(pbng2d_workspace* ws, void* x_inout, const pbng_solve_opts* o,
                     pbng_stats* stats, void* hip_stream);

/*
 * FP64 residual and energy (Eq. fem_qs): *res_norm = ||f(x) + fhat||_2
 * over free vertices, *energy = sum A0 Psi(F) - x . fhat plus the weak
 * constraint, half-plane and inertia terms (either may be NULL); r_out: optional device double [n_verts][2] (zero on Dirichlet
 * rows).  x: device [n_verts][2] of the workspace's real type.
 */
int32_t pbng2d_residual(pbng2d_workspace* ws, const void* x, double* res_norm, double* energy,
                        double* r_out, void* hip_stream);

/*
 * Adjoint of a planar equilibrium (the planar form of pbng_adjoint): at
 * x_eq (device [n_verts][2], workspace real type) solve H lam = dL/dx on
 * the free vertices, H the true Hessian of the energy (triangles, weak
 * constraints, active half-planes, inertia), by block Gauss-Seidel over the
 * colours (diagonal blocks: the true H_ii for Neo-Hookean, which in 2-D is
 * sum A0 (mu |dN_i|^2 I + lhat c c^T); the modified A_ii for corotated),
 * then assemble
 *   dL/dmu_e     = -A0_e < dP/dmu (F_e), Lam_e >,
 *   dL/dlambda_e = -A0_e (J_e - 1) < cof F_e, Lam_e >,
 *   dL/dx_k      = (dL/dx)_k - (H lam)_k for Dirichlet vertices k,
 * Lam_e = sum_j lam_j dN_j^T, dP/dmu = F + (J - 2) cof F (Neo-Hookean) or
 * 2 (F - R) (corotated).  dL_dx: device [n_verts][2], workspace real type.
 * Outputs (device, double, any may be NULL): dL_dxD [n_dirichlet][2] in the
 * order of dirichlet_idx, dL_dmu and dL_dlambda [n_tris], lam_out
 * [n_verts][2] (zero on Dirichlet rows).  o: max_sweeps, rel_tol on
 * ||b - H lam|| / ||b|| (FP64, free rows), check_every, accel
 * (PBNG_ACCEL_NONE or PBNG_ACCEL_CHEBYSHEV with rho, gamma), lanes.  stats
 * (host, one entry, may be NULL): sweeps and the adjoint residuals.
 * Returns PBNG_OK, PBNG_NOT_CONVERGED (outputs valid), PBNG_ENAN or
 * another error.
 */
int32_t pbng2d_adjoint(pbng2d_workspace* ws, const void* x_eq, const void* dL_dx, double* dL_dxD,
                       double* dL_dmu, double* dL_dlambda, double* lam_out, const pbng_adjoint_opts* o,
                       pbng_stats* stats, void* hip_stream);

/*
 * Backward-Euler inertia (Eq. fem_be, minimised as the incremental
 * potential) with d = 2: with dt > 0 every later solve and residual adds
 * sum over free vertices i of 1/2 m_ii / dt^2 |y_i - xhat_i|^2 to the
 * energy, xhat = 2 x^n - x^{n-1}, lumped mass m_ii = R0 sum_{e incident to
 * i} A0_e / 3 (R0 = the problem's density, unit thickness).  x_n_dev,
 * x_prev_dev: device double arrays [n_verts][2] in the caller's order
 * (Dirichlet rows ignored), read on hip_stream before the call returns;
 * the workspace keeps its own xhat.  dt <= 0 switches inertia off (the
 * pointers may then be NULL).  Errors: PBNG_EINVAL (null arrays with
 * dt > 0, non-finite dt), PBNG_EHIP.
 */
int32_t pbng2d_workspace_set_inertia(pbng2d_workspace* ws, double dt, const double* x_n_dev,
                                     const double* x_prev_dev, void* hip_stream);

/*
 * Launch-level access for measurement, as in pbng.h: load the internal
 * iterate from x (device), run n_sweeps sweeps (with o's blend, no
 * residual) on hip_stream without synchronising, store it back.
 * pbng2d_phase_bytes: algorithmic bytes of colour `color`'s phase in the
 * FP32 form -- 32 bytes per visit record (two int32 vertex indices, four
 * float shape-function gradients, V0 mu and V0 lambda), per updated vertex
 * 28 bytes (position read and written, external force, CSR offset), 8
 * bytes per distinct neighbour position read; doubled floats in FP64.  A
 * workspace whose triangles share one (mu, lambda) streams 24 of the 32
 * record bytes (the rest area follows from the gradients); the figure
 * stays defined on the full record.
 */
int32_t pbng2d_load(pbng2d_workspace* ws, const void* x, void* hip_stream);
int32_t pbng2d_store(pbng2d_workspace* ws, void* x, void* hip_stream);
int32_t pbng2d_sweeps(pbng2d_workspace* ws, int32_t n_sweeps, const pbng_solve_opts* o,
                      void* hip_stream);
int32_t pbng2d_phase_bytes(const pbng2d_workspace* ws, int32_t color, int64_t* bytes,
                           int64_t* vertices, int64_t* visits);

#ifdef __cplusplus
}
#endif

#endif /* PBNG2D_H */
