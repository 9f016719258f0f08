/*
 * pbng_oracle2d.c -- plain, serial FP64 reference for PBNG on triangle
 * meshes (d = 2), the planar case of the same method (Chen, Han, Chen &
 * Teran, arXiv 2306.09021): piecewise-linear interpolation over triangles
 * (Sec. "Discretization"), 2x2 deformation gradients, the constitutive
 * models of Eq. (cor) and Eq. (nh) with d = 2, the modified Hessian of
 * Eq. (mod_hess_dens) / (mod_hess) with the 2x2 cofactor matrix, and 2x2
 * local systems in the update of Eq. (pbgn_update) / (pbgn_dx), with the
 * weak constraints of Sec. "Weak Constraints", contact half-planes and the
 * backward-Euler inertia of Eq. (fem_be) in their d = 2 form.
 *
 * TEST INFRASTRUCTURE ONLY.  Built into oracle/liboracle.so next to the
 * 3-D oracle and loaded by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py -- nothing else.  It shares no code with the
 * HIP library and none with the 3-D oracle file either.  Every quantity is
 * computed from its definition; colours run in sequence, vertices of one
 * colour in ascending index.
 *
 * Only the Neo-Hookean and corotated models are defined here: the stable
 * Neo-Hookean density as printed (Eq. snh) carries the 3-D rest-state
 * constant 3 mu / (4 lambda) and is not stress free at F = I when d = 2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR2_NEOHOOKEAN 0
#define OR2_COROTATED 1

#define OR2_ACCEL_NONE 0
#define OR2_ACCEL_CHEBYSHEV 1
#define OR2_ACCEL_SOR 2

#define OR2_SAFEGUARD_BACKTRACK 1

/* A planar problem; arrays owned by the caller.  Matrices are row-major
 * 2x2, M[2 * r + c].  The energy is the sum of A0 Psi(F) over triangles,
 * -y . fhat, the weak constraints of Sec. "Weak Constraints" with d = 2
 * (1/2 C_c^T K_c C_c, C_c = sum_j w_j y_{v_j}, K_c symmetric 2x2 stored as
 * (xx, xy, yy)), for every vertex and contact half-plane (n_x, n_y, d, k)
 * the penalty 1/2 k min(0, n . y - d)^2, and, with minert non-null, the
 * backward-Euler inertia of Eq. (fem_be) written as the incremental
 * potential: sum_i 1/2 minert_i |y_i - xhat_i|^2, minert_i = m_ii / dt^2
 * (zero on Dirichlet vertices), xhat = 2 x^n - x^{n-1}. */
typedef struct {
    int32_t nv, nt, model;
    const double* X;        /* [nv][2] rest positions                    */
    const int32_t* tris;    /* [nt][3], counter-clockwise (area > 0)     */
    const double* mu;       /* [nt]                                      */
    const double* lam;      /* [nt] Lame lambda                          */
    const double* fext;     /* [nv][2] lumped external force             */
    const uint8_t* is_dir;  /* [nv] 1 = Dirichlet                        */
    int32_t n_wc;
    const int32_t* wc_ptr;  /* [n_wc + 1]                                */
    const int32_t* wc_vert; /* [nnz]                                     */
    const double* wc_w;     /* [nnz] w0 - w1                             */
    const double* wc_K;     /* [n_wc][3] (xx, xy, yy)                    */
    int32_t n_planes;
    const double* planes;   /* [n_planes][4] (n_x, n_y, d, k)            */
    const double* minert;   /* [nv] or NULL                              */
    const double* xhat;     /* [nv][2]                                   */
} or2_problem;

/* Same field layout as the 3-D oracle's options and statistics. */
typedef struct {
    int32_t max_sweeps;
    int32_t check_every;
    double rel_tol;
    int32_t accel;
    double rho, gamma, omega;
    int32_t safeguard;
    int32_t max_halvings;
    double skip_tol;        /* unused in 2-D                             */
    int32_t emulate_f32;    /* round every stored position to float      */
    int32_t n_threads;      /* unused in 2-D                             */
} or2_opts;

typedef struct {
    int32_t sweeps;
    int32_t converged;
    int64_t rejected;
    int64_t halvings;
    double res0, res, rel, energy;
} or2_stats;

/* ------------------------------------------------------------------ */
/* 2x2 algebra                                                          */
/* ------------------------------------------------------------------ */
static double det2(const double* A) { return A[0] * A[3] - A[1] * A[2]; }

/* cof(A) = det(A) A^{-T}, defined for every A: [[a11, -a10], [-a01, a00]]. */
static void cofactor2(const double* A, double* C)
{
    C[0] = A[3];
    C[1] = -A[2];
    C[2] = -A[1];
    C[3] = A[0];
}

/* Closest rotation to F (maximiser of tr(R^T F) over proper rotations),
 * i.e. the rotation of the polar decomposition F = R S for det F > 0 and
 * of the signed one otherwise.  With R = [[c, -s], [s, c]],
 * tr(R^T F) = c (F00 + F11) + s (F10 - F01), maximised by (c, s) parallel
 * to (F00 + F11, F10 - F01); when both vanish every rotation is optimal and
 * R = I is taken. */
void or2_rotation(const double* F, double* R)
{
    double a = F[0] + F[3], b = F[2] - F[1];
    double r = sqrt(a * a + b * b);
    double c = 1.0, s = 0.0;
    if (r > 0.0) {
        c = a / r;
        s = b / r;
    }
    R[0] = c;
    R[1] = -s;
    R[2] = s;
    R[3] = c;
}

/* ------------------------------------------------------------------ */
/* Constitutive models with d = 2                                        */
/* ------------------------------------------------------------------ */
/* Corotated, Eq. (cor): mu |F - R(F)|^2 + lambda/2 (det F - 1)^2.
 * Neo-Hookean, Eq. (nh): 1/2 mu |F|^2 + lhat/2 (det F - 1 - mu/lhat)^2,
 * lhat = mu + lambda. */
double or2_psi(int model, double mu, double lam, const double* F)
{
    double J = det2(F);
    if (model == OR2_NEOHOOKEAN) {
        double lh = mu + lam, f2 = 0.0;
        for (int k = 0; k < 4; ++k) f2 += F[k] * F[k];
        double q = J - 1.0 - mu / lh;
        return 0.5 * mu * f2 + 0.5 * lh * q * q;
    }
    double R[4], d2 = 0.0;
    or2_rotation(F, R);
    for (int k = 0; k < 4; ++k) d2 += (F[k] - R[k]) * (F[k] - R[k]);
    return mu * d2 + 0.5 * lam * (J - 1.0) * (J - 1.0);
}

/* P = dPsi/dF; d det F / dF = cof F and d/dF |F - R(F)|^2 = 2 (F - R). */
void or2_pk1(int model, double mu, double lam, const double* F, double* P)
{
    double C[4], J = det2(F);
    cofactor2(F, C);
    if (model == OR2_NEOHOOKEAN) {
        double lh = mu + lam, q = J - 1.0 - mu / lh;
        for (int k = 0; k < 4; ++k) P[k] = mu * F[k] + lh * q * C[k];
    } else {
        double R[4];
        or2_rotation(F, R);
        for (int k = 0; k < 4; ++k) P[k] = 2.0 * mu * (F[k] - R[k]) + lam * (J - 1.0) * C[k];
    }
}

/* Modified Hessian density, Eq. (mod_hess_dens) with d = 2, as the tensor
 * Ct[alpha][gamma][beta][delta] (index ((a*2+g)*2+b)*2+d):
 * 2 mu delta_ab delta_gd + lambda cof(F)_ag cof(F)_bd. */
void or2_mod_hess_density(double mu, double lam, const double* F, double* Ct)
{
    double C[4];
    cofactor2(F, C);
    for (int a = 0; a < 2; ++a)
        for (int g = 0; g < 2; ++g)
            for (int b = 0; b < 2; ++b)
                for (int d = 0; d < 2; ++d)
                    Ct[((a * 2 + g) * 2 + b) * 2 + d] =
                        2.0 * mu * (a == b) * (g == d) + lam * C[2 * a + g] * C[2 * b + d];
}

/* ------------------------------------------------------------------ */
/* Discretisation                                                       */
/* ------------------------------------------------------------------ */
/* Per triangle: dN[e][j][:] = dN_j/dX, A0[e] = rest area.  With
 * Dm = [X1 - X0, X2 - X0] (columns), dN_j (j = 1, 2) is row j-1 of Dm^{-1}
 * and dN_0 = -(dN_1 + dN_2).  Returns -1 for a triangle of area <= 0, -2
 * for an index out of range. */
int or2_prep(int32_t nv, int32_t nt, const double* X, const int32_t* tris, double* dN /* [nt][3][2] */,
             double* A0 /* [nt] */)
{
    for (int e = 0; e < nt; ++e) {
        const int32_t* t = tris + 3 * e;
        for (int j = 0; j < 3; ++j)
            if (t[j] < 0 || t[j] >= nv) return -2;
        double Dm[4];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) Dm[2 * r + c] = X[2 * t[c + 1] + r] - X[2 * t[0] + r];
        double det = det2(Dm);
        if (!(det > 0.0)) return -1;
        A0[e] = 0.5 * det;
        double* g = dN + 6 * e;
        /* Dm^{-1} = cof(Dm)^T / det */
        g[2] = Dm[3] / det;
        g[3] = -Dm[1] / det;
        g[4] = -Dm[2] / det;
        g[5] = Dm[0] / det;
        g[0] = -(g[2] + g[4]);
        g[1] = -(g[3] + g[5]);
    }
    return 0;
}

/* Lumped mass of Eq. (fem_be) with d = 2: m_ii = int R0 N_i dX, i.e.
 * R0 A0_e / 3 from every incident triangle (unit thickness).  Accumulates
 * into m[nv]. */
void or2_lumped_mass(int32_t nv, int32_t nt, const int32_t* tris, const double* A0, double density,
                     double* m)
{
    (void)nv;
    for (int e = 0; e < nt; ++e)
        for (int j = 0; j < 3; ++j) m[tris[3 * e + j]] += density * A0[e] / 3.0;
}

/* Lumped body force: a linear basis function integrates to A0 / 3 over a
 * triangle, so fhat_i += R0 g A0_e / 3 from every incident triangle. */
void or2_body_force(int32_t nv, int32_t nt, const int32_t* tris, const double* A0, double density,
                    const double* grav, double* fext /* [nv][2], accumulated */)
{
    (void)nv;
    for (int e = 0; e < nt; ++e)
        for (int j = 0; j < 3; ++j)
            for (int c = 0; c < 2; ++c) fext[2 * tris[3 * e + j] + c] += density * grav[c] * A0[e] / 3.0;
}

static void deformation_gradient(const double* y, const int32_t* t, const double* g, double* F)
{
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += y[2 * t[j] + a] * g[2 * j + b];
            F[2 * a + b] = s;
        }
}

/* vertex -> incident triangles (with local slot); vertex -> incident weak
 * constraints (with the position of the vertex in the constraint) */
typedef struct {
    int32_t *tptr, *tlist, *tslot;
    int32_t *cptr, *clist, *cpos;
    double *dN, *A0;
} or2_adj;

static void adj_free(or2_adj* A)
{
    free(A->tptr); free(A->tlist); free(A->tslot); free(A->dN); free(A->A0);
    free(A->cptr); free(A->clist); free(A->cpos);
    memset(A, 0, sizeof *A);
}

static int adj_build(const or2_problem* p, or2_adj* A)
{
    memset(A, 0, sizeof *A);
    int nv = p->nv, nt = p->nt;
    A->dN = (double*)malloc(sizeof(double) * 6 * (size_t)(nt > 0 ? nt : 1));
    A->A0 = (double*)malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
    int rc = or2_prep(nv, nt, p->X, p->tris, A->dN, A->A0);
    if (rc) { adj_free(A); return rc; }
    A->tptr = (int32_t*)calloc((size_t)nv + 1, sizeof(int32_t));
    for (int e = 0; e < nt; ++e)
        for (int j = 0; j < 3; ++j) A->tptr[p->tris[3 * e + j] + 1]++;
    for (int i = 0; i < nv; ++i) A->tptr[i + 1] += A->tptr[i];
    A->tlist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(3 * nt + 1));
    A->tslot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(3 * nt + 1));
    int32_t* fill = (int32_t*)calloc((size_t)nv + 1, sizeof(int32_t));
    for (int e = 0; e < nt; ++e)
        for (int j = 0; j < 3; ++j) {
            int v = p->tris[3 * e + j];
            int k = A->tptr[v] + fill[v]++;
            A->tlist[k] = e;
            A->tslot[k] = j;
        }
    int nnz = p->n_wc > 0 ? p->wc_ptr[p->n_wc] : 0;
    A->cptr = (int32_t*)calloc((size_t)nv + 1, sizeof(int32_t));
    for (int k = 0; k < nnz; ++k) {
        int v = p->wc_vert[k];
        if (v < 0 || v >= nv) { free(fill); adj_free(A); return -2; }
        A->cptr[v + 1]++;
    }
    for (int i = 0; i < nv; ++i) A->cptr[i + 1] += A->cptr[i];
    A->clist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    A->cpos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    memset(fill, 0, sizeof(int32_t) * ((size_t)nv + 1));
    for (int c = 0; c < p->n_wc; ++c)
        for (int k = p->wc_ptr[c]; k < p->wc_ptr[c + 1]; ++k) {
            int v = p->wc_vert[k];
            int q = A->cptr[v] + fill[v]++;
            A->clist[q] = c;
            A->cpos[q] = k;
        }
    free(fill);
    return 0;
}

/* K_c entry (a, b) from the stored (xx, xy, yy). */
static double symK(const double* K, int a, int b) { return (a == b) ? K[2 * a] : K[1]; }

/* C_c = sum_j w_j y_{v_j}, with y_i replaced by yi when yi is non-null. */
static void constraint_value(const or2_problem* p, int c, const double* y, int i, const double* yi, double* C)
{
    C[0] = C[1] = 0.0;
    for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s) {
        int v = p->wc_vert[s];
        const double* yv = (yi && v == i) ? yi : y + 2 * v;
        C[0] += p->wc_w[s] * yv[0];
        C[1] += p->wc_w[s] * yv[1];
    }
}

/* phi = n . y - d of half-plane q at position y. */
static double plane_phi(const double* pl, const double* y) { return pl[0] * y[0] + pl[1] * y[1] - pl[2]; }

/* ------------------------------------------------------------------ */
/* Node colouring, Sec. "Coloring and Parallelism"                       */
/* ------------------------------------------------------------------ */
/* Free vertices in ascending index each take the least colour used by no
 * already coloured vertex of an incident triangle or weak constraint (the
 * union of the sets S_c of those elements).  Dirichlet vertices get -1.
 * Returns the number of colours or < 0 on error. */
int32_t or2_color(const or2_problem* p, int32_t* colors)
{
    or2_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    int ncol = 0;
    char used[256];
    for (int i = 0; i < p->nv; ++i) colors[i] = -1;
    for (int i = 0; i < p->nv; ++i) {
        if (p->is_dir[i]) continue;
        memset(used, 0, sizeof used);
        for (int k = A.tptr[i]; k < A.tptr[i + 1]; ++k) {
            const int32_t* t = p->tris + 3 * A.tlist[k];
            for (int j = 0; j < 3; ++j)
                if (colors[t[j]] >= 0) used[colors[t[j]]] = 1;
        }
        for (int k = A.cptr[i]; k < A.cptr[i + 1]; ++k) {
            int c = A.clist[k];
            for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s)
                if (colors[p->wc_vert[s]] >= 0) used[colors[p->wc_vert[s]]] = 1;
        }
        int col = 0;
        while (used[col]) ++col;
        if (col >= 255) { adj_free(&A); return -4; }
        colors[i] = col;
        if (col + 1 > ncol) ncol = col + 1;
    }
    adj_free(&A);
    return ncol;
}

/* ------------------------------------------------------------------ */
/* Local energy, local system and the update                            */
/* ------------------------------------------------------------------ */
/* Energy of the terms involving vertex i with y_i replaced by yi: incident
 * triangles A0 Psi(F), incident weak constraints, the half-plane penalties,
 * the inertia and -yi . fext_i; magnitudes added to *absum. */
static double local_energy(const or2_problem* p, const or2_adj* A, const double* y, int i,
                           const double* yi, double* absum)
{
    double E = 0.0, ab = 0.0;
    for (int k = A->tptr[i]; k < A->tptr[i + 1]; ++k) {
        int e = A->tlist[k];
        const int32_t* t = p->tris + 3 * e;
        const double* g = A->dN + 6 * e;
        double F[4];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j) {
                    const double* yj = (t[j] == i) ? yi : y + 2 * t[j];
                    s += yj[a] * g[2 * j + b];
                }
                F[2 * a + b] = s;
            }
        double w = A->A0[e] * or2_psi(p->model, p->mu[e], p->lam[e], F);
        E += w;
        ab += fabs(w);
    }
    for (int k = A->cptr[i]; k < A->cptr[i + 1]; ++k) {
        int c = A->clist[k];
        double C[2];
        constraint_value(p, c, y, i, yi, C);
        const double* K = p->wc_K + 3 * c;
        double w = 0.5 * (K[0] * C[0] * C[0] + 2.0 * K[1] * C[0] * C[1] + K[2] * C[1] * C[1]);
        E += w;
        ab += fabs(w);
    }
    for (int q = 0; q < p->n_planes; ++q) {
        const double* pl = p->planes + 4 * q;
        double phi = plane_phi(pl, yi);
        if (phi < 0.0) {
            double w = 0.5 * pl[3] * phi * phi;
            E += w;
            ab += fabs(w);
        }
    }
    if (p->minert) {
        double d0 = yi[0] - p->xhat[2 * i], d1 = yi[1] - p->xhat[2 * i + 1];
        double w = 0.5 * p->minert[i] * (d0 * d0 + d1 * d1);
        E += w;
        ab += fabs(w);
    }
    double w = -(yi[0] * p->fext[2 * i] + yi[1] * p->fext[2 * i + 1]);
    E += w;
    ab += fabs(w);
    if (absum) *absum += ab;
    return E;
}

/* g_i = dE/dy_i and the modified nodal Hessian of Eq. (mod_hess), the
 * density of Eq. (mod_hess_dens) contracted with dN_i dN_i^T, plus the
 * exact second derivatives of the other terms: s_ci^2 K_c for a weak
 * constraint in which vertex i has weight s_ci, k n n^T for an active
 * half-plane, minert_i I for the inertia. */
static void local_system(const or2_problem* p, const or2_adj* A, const double* y, int i, double* gi,
                         double* Ai)
{
    gi[0] = -p->fext[2 * i];
    gi[1] = -p->fext[2 * i + 1];
    for (int k = 0; k < 4; ++k) Ai[k] = 0.0;
    for (int k = A->tptr[i]; k < A->tptr[i + 1]; ++k) {
        int e = A->tlist[k], slot = A->tslot[k];
        const int32_t* t = p->tris + 3 * e;
        const double* g = A->dN + 6 * e;
        const double* a = g + 2 * slot;
        double F[4], P[4], Ct[16], V = A->A0[e];
        deformation_gradient(y, t, g, F);
        or2_pk1(p->model, p->mu[e], p->lam[e], F, P);
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) gi[r] += V * P[2 * r + c] * a[c];
        or2_mod_hess_density(p->mu[e], p->lam[e], F, Ct);
        for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be) {
                double s = 0.0;
                for (int ga = 0; ga < 2; ++ga)
                    for (int de = 0; de < 2; ++de) s += Ct[((al * 2 + ga) * 2 + be) * 2 + de] * a[ga] * a[de];
                Ai[2 * al + be] += V * s;
            }
    }
    for (int k = A->cptr[i]; k < A->cptr[i + 1]; ++k) {
        int c = A->clist[k];
        double sci = p->wc_w[A->cpos[k]], C[2];
        constraint_value(p, c, y, i, NULL, C);
        const double* K = p->wc_K + 3 * c;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                gi[a] += sci * symK(K, a, b) * C[b];
                Ai[2 * a + b] += sci * sci * symK(K, a, b);
            }
    }
    for (int q = 0; q < p->n_planes; ++q) {
        const double* pl = p->planes + 4 * q;
        double phi = plane_phi(pl, y + 2 * i);
        if (phi < 0.0)
            for (int a = 0; a < 2; ++a) {
                gi[a] += pl[3] * phi * pl[a];
                for (int b = 0; b < 2; ++b) Ai[2 * a + b] += pl[3] * pl[a] * pl[b];
            }
    }
    if (p->minert)
        for (int a = 0; a < 2; ++a) {
            gi[a] += p->minert[i] * (y[2 * i + a] - p->xhat[2 * i + a]);
            Ai[2 * a + a] += p->minert[i];
        }
}

static double to_f32(double v) { return (double)(float)v; }

/* One modified-Newton step on vertex i from Delta = 0 (Eq. pbgn_dx with the
 * 2x2 system A_i Delta = -g_i), optionally halving the step until the local
 * energy does not increase (slack 8 u sum |summands|); a vertex with no
 * passing step keeps its position.  Returns the halvings, or -1 when
 * rejected. */
static int update_vertex(const or2_problem* p, const or2_adj* A, double* y, int i, const or2_opts* o)
{
    double gi[2], Ai[4];
    local_system(p, A, y, i, gi, Ai);
    double det = det2(Ai);
    if (!(det > 0.0)) return -1;
    double d[2] = {-(Ai[3] * gi[0] - Ai[1] * gi[1]) / det, -(-Ai[2] * gi[0] + Ai[0] * gi[1]) / det};
    double yi0[2] = {y[2 * i], y[2 * i + 1]};
    double alpha = 1.0;
    int halvings = 0;
    if (o->safeguard == OR2_SAFEGUARD_BACKTRACK) {
        const double u = 1.1102230246251565e-16; /* 2^-53 */
        double ab0 = 0.0;
        double E0 = local_energy(p, A, y, i, yi0, &ab0);
        for (;;) {
            double yt[2], ab1 = 0.0;
            for (int a = 0; a < 2; ++a) {
                yt[a] = yi0[a] + alpha * d[a];
                if (o->emulate_f32) yt[a] = to_f32(yt[a]);
            }
            double E1 = local_energy(p, A, y, i, yt, &ab1);
            if (E1 - E0 <= 8.0 * u * (ab0 + ab1)) break;
            if (halvings >= o->max_halvings) return -1;
            alpha *= 0.5;
            ++halvings;
        }
    }
    for (int a = 0; a < 2; ++a) {
        double v = yi0[a] + alpha * d[a];
        y[2 * i + a] = o->emulate_f32 ? to_f32(v) : v;
    }
    return halvings;
}

/* r_i = f_i(y) + fhat_i over free vertices (Eq. fem_qs, with the inertia
 * the force of the incremental potential) by scattering the element forces
 * -A0 P dN_j, the constraint forces -w_j K_c C_c, the half-plane forces
 * -k phi n and -minert_i (y_i - xhat_i); total energy of every term.
 * Returns ||r||_2, or -1 on a mesh error. */
double or2_residual(const or2_problem* p, const double* y, double* r_out /* nullable [nv][2] */,
                    double* energy_out)
{
    or2_adj A;
    if (adj_build(p, &A)) return -1.0;
    double* f = (double*)calloc((size_t)2 * p->nv + 1, sizeof(double));
    double E = 0.0;
    for (int e = 0; e < p->nt; ++e) {
        const int32_t* t = p->tris + 3 * e;
        const double* g = A.dN + 6 * e;
        double F[4], P[4];
        deformation_gradient(y, t, g, F);
        or2_pk1(p->model, p->mu[e], p->lam[e], F, P);
        E += A.A0[e] * or2_psi(p->model, p->mu[e], p->lam[e], F);
        for (int j = 0; j < 3; ++j)
            for (int r = 0; r < 2; ++r) f[2 * t[j] + r] -= A.A0[e] * (P[2 * r] * g[2 * j] + P[2 * r + 1] * g[2 * j + 1]);
    }
    for (int c = 0; c < p->n_wc; ++c) {
        double C[2];
        constraint_value(p, c, y, -1, NULL, C);
        const double* K = p->wc_K + 3 * c;
        double KC[2] = {K[0] * C[0] + K[1] * C[1], K[1] * C[0] + K[2] * C[1]};
        E += 0.5 * (C[0] * KC[0] + C[1] * KC[1]);
        for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s)
            for (int a = 0; a < 2; ++a) f[2 * p->wc_vert[s] + a] -= p->wc_w[s] * KC[a];
    }
    for (int i = 0; i < p->nv; ++i) {
        for (int q = 0; q < p->n_planes; ++q) {
            const double* pl = p->planes + 4 * q;
            double phi = plane_phi(pl, y + 2 * i);
            if (phi < 0.0) {
                E += 0.5 * pl[3] * phi * phi;
                for (int a = 0; a < 2; ++a) f[2 * i + a] -= pl[3] * phi * pl[a];
            }
        }
        if (p->minert) {
            double d0 = y[2 * i] - p->xhat[2 * i], d1 = y[2 * i + 1] - p->xhat[2 * i + 1];
            E += 0.5 * p->minert[i] * (d0 * d0 + d1 * d1);
            f[2 * i] -= p->minert[i] * d0;
            f[2 * i + 1] -= p->minert[i] * d1;
        }
    }
    double n2 = 0.0;
    for (int i = 0; i < p->nv; ++i) {
        E -= y[2 * i] * p->fext[2 * i] + y[2 * i + 1] * p->fext[2 * i + 1];
        for (int a = 0; a < 2; ++a) {
            double r = p->is_dir[i] ? 0.0 : f[2 * i + a] + p->fext[2 * i + a];
            if (r_out) r_out[2 * i + a] = r;
            n2 += r * r;
        }
    }
    free(f);
    adj_free(&A);
    if (energy_out) *energy_out = E;
    return sqrt(n2);
}

/* Sweeps over the colours in sequence with the optional Chebyshev / SOR
 * blend of Sec. "Acceleration Techniques" on the free vertices, FP64
 * residual every check_every sweeps (relative residuals into hist when
 * non-null).  x: initial iterate with Dirichlet rows set; receives the
 * result. */
int32_t or2_solve(const or2_problem* p, const int32_t* colors, double* x, const or2_opts* o,
                  or2_stats* st, double* hist)
{
    memset(st, 0, sizeof *st);
    or2_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    int nv = p->nv, ncol = 0;
    for (int i = 0; i < nv; ++i)
        if (colors[i] + 1 > ncol) ncol = colors[i] + 1;
    size_t nb = sizeof(double) * 2 * (size_t)(nv > 0 ? nv : 1);
    double* xl = (double*)malloc(nb);
    double* xlm1 = (double*)malloc(nb);
    memcpy(xlm1, x, sizeof(double) * 2 * (size_t)nv);
    double E = 0.0;
    double res0 = or2_residual(p, x, NULL, &E);
    st->res0 = st->res = res0;
    st->rel = res0 > 0 ? 1.0 : 0.0;
    st->energy = E;
    double omega = 1.0;
    int every = o->check_every > 0 ? o->check_every : 1, nh = 0;
    for (int l = 0; l < o->max_sweeps; ++l) {
        if (res0 == 0.0) { st->converged = 1; break; }
        memcpy(xl, x, sizeof(double) * 2 * (size_t)nv);
        for (int c = 0; c < ncol; ++c)
            for (int i = 0; i < nv; ++i) {
                if (colors[i] != c) continue;
                int h = update_vertex(p, &A, x, i, o);
                if (h < 0) st->rejected++;
                else st->halvings += h;
            }
        if (o->accel != OR2_ACCEL_NONE) {
            double w, gam;
            if (o->accel == OR2_ACCEL_CHEBYSHEV) {
                if (l < 2) omega = 1.0;
                else if (l == 2) omega = 2.0 / (2.0 - o->rho * o->rho);
                else omega = 4.0 / (4.0 - o->rho * o->rho * omega);
                w = omega;
                gam = o->gamma;
            } else {
                w = o->omega;
                gam = 1.0;
            }
            for (int i = 0; i < nv; ++i) {
                if (p->is_dir[i]) continue;
                for (int a = 0; a < 2; ++a) {
                    int k = 2 * i + a;
                    double v = o->accel == OR2_ACCEL_CHEBYSHEV
                                   ? w * (gam * (x[k] - xl[k]) + xl[k] - xlm1[k]) + xlm1[k]
                                   : w * (x[k] - xlm1[k]) + xlm1[k];
                    x[k] = o->emulate_f32 ? to_f32(v) : v;
                }
            }
            double* t = xlm1; xlm1 = xl; xl = t;
        }
        st->sweeps = l + 1;
        if ((l + 1) % every == 0 || l + 1 == o->max_sweeps) {
            double r = or2_residual(p, x, NULL, &E);
            st->res = r;
            st->rel = r / res0;
            st->energy = E;
            if (hist && (l + 1) % every == 0) hist[nh++] = st->rel;
            if (!isfinite(r)) break;
            if (st->rel <= o->rel_tol) { st->converged = 1; break; }
        }
    }
    free(xl);
    free(xlm1);
    adj_free(&A);
    return 0;
}

/* Energy change of each single-vertex update of one plain sweep, in sweep
 * order, into dE [n_free]; returns the number of updates. */
int32_t or2_sweep_energy_trace(const or2_problem* p, const int32_t* colors, double* x, const or2_opts* o,
                               double* dE)
{
    or2_adj A;
    if (adj_build(p, &A)) return -1;
    int ncol = 0, n = 0;
    for (int i = 0; i < p->nv; ++i)
        if (colors[i] + 1 > ncol) ncol = colors[i] + 1;
    for (int c = 0; c < ncol; ++c)
        for (int i = 0; i < p->nv; ++i) {
            if (colors[i] != c) continue;
            double E0, E1;
            or2_residual(p, x, NULL, &E0);
            update_vertex(p, &A, x, i, o);
            or2_residual(p, x, NULL, &E1);
            dE[n++] = E1 - E0;
        }
    adj_free(&A);
    return n;
}

/* ------------------------------------------------------------------ */
/* Adjoint: the true Hessian and the parameter gradients                */
/* ------------------------------------------------------------------ */
/* dP[L], the derivative of P(F) along L, for d = 2.  cof is linear in F
 * here (cof(F + L) = cof F + cof L), and det F has derivative cof F : L.
 *   Neo-Hookean: mu L + lhat (cof F : L) cof F + (lhat (J - 1) - mu) cof L
 *   corotated:   2 mu (L - dR[L]) + lambda (cof F : L) cof F
 *                + lambda (J - 1) cof L,
 * with R = [[c, -s], [s, c]] at the angle theta = atan2(b, a) of
 * (a, b) = (F00 + F11, F10 - F01) and dR = dtheta [[-s, -c], [c, -s]],
 * dtheta = (a (L10 - L01) - b (L00 + L11)) / (a^2 + b^2) (0 where a = b = 0,
 * the one configuration without a unique closest rotation). */
void or2_stress_diff(int model, double mu, double lam, const double* F, const double* L, double* dP)
{
    double C[4], CL[4], J = det2(F);
    cofactor2(F, C);
    cofactor2(L, CL);
    double cl = 0.0;
    for (int k = 0; k < 4; ++k) cl += C[k] * L[k];
    if (model == OR2_NEOHOOKEAN) {
        double lh = mu + lam;
        for (int k = 0; k < 4; ++k) dP[k] = mu * L[k] + lh * cl * C[k] + (lh * (J - 1.0) - mu) * CL[k];
        return;
    }
    double a = F[0] + F[3], b = F[2] - F[1], r2 = a * a + b * b;
    double R[4], dR[4] = {0.0, 0.0, 0.0, 0.0};
    or2_rotation(F, R);
    if (r2 > 0.0) {
        double dth = (a * (L[2] - L[1]) - b * (L[0] + L[3])) / r2;
        double c = R[0], s = R[2];
        dR[0] = -s * dth;
        dR[1] = -c * dth;
        dR[2] = c * dth;
        dR[3] = -s * dth;
    }
    for (int k = 0; k < 4; ++k) dP[k] = 2.0 * mu * (L[k] - dR[k]) + lam * cl * C[k] + lam * (J - 1.0) * CL[k];
}

/* out = H v for every vertex row, H the true Hessian of the total energy at
 * y (triangles through dP, weak constraints s_ci K_c C_c(v), active
 * half-planes k (n . v_i) n, inertia minert_i v_i); v is taken as zero on
 * Dirichlet vertices.  Returns 0, or < 0 on a mesh error. */
int32_t or2_hessian_apply(const or2_problem* p, const double* y, const double* v, double* out)
{
    or2_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    for (int k = 0; k < 2 * p->nv; ++k) out[k] = 0.0;
    for (int e = 0; e < p->nt; ++e) {
        const int32_t* t = p->tris + 3 * e;
        const double* g = A.dN + 6 * e;
        double F[4], L[4] = {0.0, 0.0, 0.0, 0.0}, dP[4];
        deformation_gradient(y, t, g, F);
        for (int j = 0; j < 3; ++j) {
            if (p->is_dir[t[j]]) continue;
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) L[2 * r + c] += v[2 * t[j] + r] * g[2 * j + c];
        }
        or2_stress_diff(p->model, p->mu[e], p->lam[e], F, L, dP);
        for (int j = 0; j < 3; ++j)
            for (int r = 0; r < 2; ++r)
                out[2 * t[j] + r] += A.A0[e] * (dP[2 * r] * g[2 * j] + dP[2 * r + 1] * g[2 * j + 1]);
    }
    for (int c = 0; c < p->n_wc; ++c) {
        double Cv[2] = {0.0, 0.0};
        for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s) {
            int u = p->wc_vert[s];
            if (p->is_dir[u]) continue;
            Cv[0] += p->wc_w[s] * v[2 * u];
            Cv[1] += p->wc_w[s] * v[2 * u + 1];
        }
        const double* K = p->wc_K + 3 * c;
        double KC[2] = {K[0] * Cv[0] + K[1] * Cv[1], K[1] * Cv[0] + K[2] * Cv[1]};
        for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s)
            for (int a = 0; a < 2; ++a) out[2 * p->wc_vert[s] + a] += p->wc_w[s] * KC[a];
    }
    for (int i = 0; i < p->nv; ++i) {
        if (p->is_dir[i]) continue;
        for (int q = 0; q < p->n_planes; ++q) {
            const double* pl = p->planes + 4 * q;
            if (plane_phi(pl, y + 2 * i) < 0.0) {
                double nv = pl[0] * v[2 * i] + pl[1] * v[2 * i + 1];
                out[2 * i] += pl[3] * nv * pl[0];
                out[2 * i + 1] += pl[3] * nv * pl[1];
            }
        }
        if (p->minert) {
            out[2 * i] += p->minert[i] * v[2 * i];
            out[2 * i + 1] += p->minert[i] * v[2 * i + 1];
        }
    }
    adj_free(&A);
    return 0;
}

/* Parameter gradients of L(x*(theta)) from the adjoint lam (H lam = dL/dx
 * on free vertices, zero on Dirichlet ones): with Lam_e = sum_j lam_j dN_j^T,
 *   dL/dmu_e     = -A0_e < dP/dmu, Lam_e >,
 *   dL/dlambda_e = -A0_e (J - 1) < cof F, Lam_e >,
 * dP/dmu = F + (J - 2) cof F (Neo-Hookean: P = mu F + (lhat (J - 1) - mu)
 * cof F with lhat = mu + lambda) or 2 (F - R) (corotated). */
int32_t or2_adjoint_gradients(const or2_problem* p, const double* y, const double* lam_v, double* dmu,
                              double* dlam)
{
    or2_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    for (int e = 0; e < p->nt; ++e) {
        const int32_t* t = p->tris + 3 * e;
        const double* g = A.dN + 6 * e;
        double F[4], C[4], L[4] = {0.0, 0.0, 0.0, 0.0};
        deformation_gradient(y, t, g, F);
        cofactor2(F, C);
        double J = det2(F);
        for (int j = 0; j < 3; ++j) {
            if (p->is_dir[t[j]]) continue;
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) L[2 * r + c] += lam_v[2 * t[j] + r] * g[2 * j + c];
        }
        double FL = 0.0, CL = 0.0;
        for (int k = 0; k < 4; ++k) {
            FL += F[k] * L[k];
            CL += C[k] * L[k];
        }
        double dPdmu;
        if (p->model == OR2_NEOHOOKEAN) {
            dPdmu = FL + (J - 2.0) * CL;
        } else {
            double R[4], RL = 0.0;
            or2_rotation(F, R);
            for (int k = 0; k < 4; ++k) RL += R[k] * L[k];
            dPdmu = 2.0 * (FL - RL);
        }
        dmu[e] = -A.A0[e] * dPdmu;
        dlam[e] = -A.A0[e] * (J - 1.0) * CL;
    }
    adj_free(&A);
    return 0;
}
