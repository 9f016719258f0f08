/*
 * pbng_oracle.c -- plain, serial FP64 reference for Position-Based Nonlinear
 * Gauss-Seidel (PBNG; Chen, Han, Chen & Teran, "Position-Based Nonlinear
 * Gauss-Seidel for Quasistatic Hyperelasticity", arXiv 2306.09021).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is built into oracle/liboracle.so and
 * is loaded by tests/, by __graft_entry__.smoke() and by the cpu_baseline leg
 * of bench.py -- nothing else.  It shares no code, header, table or helper
 * with the HIP library.  It is written for a reader checking it against the
 * paper, not for speed: every quantity is computed from its definition in
 * double precision, colours run in sequence and the vertices of one colour
 * run in ascending index (or, optionally, in an OpenMP loop over one colour,
 * which gives bit-identical results because same-coloured vertices share no
 * element or constraint).
 *
 * Section references are to the paper:
 *   Sec. "Equations" / "Constitutive Models"   Eq. (cor), (nh), (snh), (lame)
 *   Sec. "Discretization"                      Eq. (fem_qs), (pe_hat), (disc_pe)
 *   Sec. "Weak Constraints"                    PE^wc, C_c, K_c
 *   Sec. "Position-Based Nonlinear Gauss-Seidel"  Eq. (pbgn_update), (pbgn_dx)
 *   Sec. "Modified Hessian"                    Eq. (hess), (mod_hess_dens), (mod_hess)
 *   Sec. "Acceleration Techniques"             Chebyshev and SOR updates
 *   Sec. "Coloring and Parallelism"            node colouring with sets S_c
 *   Sec. "Position-Based Dynamics: Constraint-Based Nonlinear Gauss-Seidel"
 *                                              Eq. (fem_be), lumped mass m_ii
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_NEOHOOKEAN 0
#define OR_COROTATED 1
#define OR_STABLE_NEOHOOKEAN 2

#define OR_ACCEL_NONE 0
#define OR_ACCEL_CHEBYSHEV 1
#define OR_ACCEL_SOR 2

#define OR_SAFEGUARD_NONE 0
#define OR_SAFEGUARD_BACKTRACK 1

/* Problem, all arrays owned by the caller.  K_c is stored as the symmetric
 * 3x3 (xx, xy, xz, yy, yz, zz); a plane is (n_x, n_y, n_z, d, k) and adds
 * the penalty 1/2 k min(0, n.y - d)^2 to every vertex. */
typedef struct {
    int32_t nv, nt, model;
    const double* X;        /* [nv][3] rest positions           */
    const int32_t* tets;    /* [nt][4]                          */
    const double* mu;       /* [nt]                             */
    const double* lam;      /* [nt] Lame lambda                 */
    const double* fext;     /* [nv][3] lumped external force    */
    const uint8_t* is_dir;  /* [nv] 1 = Dirichlet               */
    int32_t n_wc;
    const int32_t* wc_ptr;  /* [n_wc + 1]                       */
    const int32_t* wc_vert; /* [nnz]                            */
    const double* wc_w;     /* [nnz] w0 - w1                    */
    const double* wc_K;     /* [n_wc][6]                        */
    int32_t n_planes;
    const double* planes;   /* [n_planes][5]                    */
    /* Backward-Euler inertia (Eq. fem_be written as the minimisation of the
     * incremental potential): when minert is not NULL the energy gains
     * sum_i 1/2 minert_i |y_i - xhat_i|^2, minert_i = m_ii / dt^2 (zero on
     * Dirichlet vertices), xhat = 2 x^n - x^{n-1}. */
    const double* minert;   /* [nv] or NULL                     */
    const double* xhat;     /* [nv][3]                          */
} or_problem;

typedef struct {
    int32_t max_sweeps;
    int32_t check_every;    /* residual every k sweeps (>= 1)   */
    double rel_tol;         /* stop when ||r|| / ||r0|| <= tol  */
    int32_t accel;
    double rho, gamma, omega;
    int32_t safeguard;
    int32_t max_halvings;
    double skip_tol;        /* skip a vertex whose |g| <= skip_tol (0 = off) */
    int32_t emulate_f32;    /* round every stored position to float */
    int32_t n_threads;      /* >1: OpenMP within one colour      */
} or_opts;

typedef struct {
    int32_t sweeps;
    int32_t converged;
    int64_t rejected;       /* safeguard: vertices left unchanged */
    int64_t halvings;       /* safeguard: total step halvings     */
    double res0, res, rel, energy;
} or_stats;

/* ------------------------------------------------------------------ */
/* Linear algebra on 3x3 row-major matrices M[3*r + c]                 */
/* ------------------------------------------------------------------ */
static double det3(const double* A)
{
    return A[0] * (A[4] * A[8] - A[5] * A[7])
         - A[1] * (A[3] * A[8] - A[5] * A[6])
         + A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* cof(F)_{ij} = (-1)^{i+j} det(minor_ij): the cofactor matrix, equal to
 * det(F) F^{-T} where F is invertible and defined for every F (Sec.
 * "Modified Hessian"). */
static void cofactor3(const double* F, double* C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            int r0 = (i + 1) % 3, r1 = (i + 2) % 3;
            int c0 = (j + 1) % 3, c1 = (j + 2) % 3;
            /* cyclic minors carry the (-1)^{i+j} sign automatically */
            C[3 * i + j] = F[3 * r0 + c0] * F[3 * r1 + c1] - F[3 * r0 + c1] * F[3 * r1 + c0];
        }
}

static void matmul3(const double* A, const double* B, double* C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

/* Inverse by the adjugate: A^{-1} = cof(A)^T / det(A). */
static int inv3(const double* A, double* Ai)
{
    double C[9];
    double d = det3(A);
    if (d == 0.0 || !isfinite(d)) return -1;
    cofactor3(A, C);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Ai[3 * i + j] = C[3 * j + i] / d;
    return 0;
}

/* ------------------------------------------------------------------ */
/* 3x3 SVD by one-sided (Hestenes) Jacobi, with the sign convention that  */
/* U, V are rotations and the smallest singular value carries the sign */
/* of det(F) (Irving et al. 2004; Stomakhin et al. 2012).               */
/* ------------------------------------------------------------------ */
static void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

void or_svd3(const double* F, double* U, double* sig, double* V)
{
    /* W holds the columns of F V; rotate pairs of columns until they are
     * mutually orthogonal. */
    double W[9], Vm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    memcpy(W, F, sizeof W);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double a = 0, b = 0, g = 0;
                for (int r = 0; r < 3; ++r) {
                    a += W[3 * r + p] * W[3 * r + p];
                    b += W[3 * r + q] * W[3 * r + q];
                    g += W[3 * r + p] * W[3 * r + q];
                }
                if (g == 0.0 || fabs(g) <= 1e-300) continue;
                double ratio = fabs(g) / sqrt(a * b);
                if (!(ratio > 1e-17)) continue;
                if (ratio > off) off = ratio;
                double zeta = (b - a) / (2.0 * g);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int r = 0; r < 3; ++r) {
                    double wp = W[3 * r + p], wq = W[3 * r + q];
                    W[3 * r + p] = c * wp - s * wq;
                    W[3 * r + q] = s * wp + c * wq;
                    double vp = Vm[3 * r + p], vq = Vm[3 * r + q];
                    Vm[3 * r + p] = c * vp - s * vq;
                    Vm[3 * r + q] = s * vp + c * vq;
                }
            }
        if (off <= 1e-16) break;
    }
    double s[3];
    for (int k = 0; k < 3; ++k)
        s[k] = sqrt(W[k] * W[k] + W[3 + k] * W[3 + k] + W[6 + k] * W[6 + k]);
    /* sort descending */
    int ord[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (s[ord[j]] > s[ord[i]]) { int t = ord[i]; ord[i] = ord[j]; ord[j] = t; }
    double Us[9], Vs[9], ss[3];
    for (int k = 0; k < 3; ++k) {
        int o = ord[k];
        ss[k] = s[o];
        for (int r = 0; r < 3; ++r) {
            Vs[3 * r + k] = Vm[3 * r + o];
            Us[3 * r + k] = ss[k] > 0 ? W[3 * r + o] / ss[k] : 0.0;
        }
    }
    /* complete U where singular values vanish */
    double smax = ss[0] > 0 ? ss[0] : 1.0;
    if (ss[1] <= 1e-300 * smax || ss[0] == 0.0) {
        if (ss[0] == 0.0) { memcpy(Us, Vs, sizeof Us); }
        else {
            double u0[3] = {Us[0], Us[3], Us[6]}, e[3] = {1, 0, 0}, u1[3], u2[3];
            if (fabs(u0[0]) > 0.9) { e[0] = 0; e[1] = 1; }
            cross3(u0, e, u1);
            double n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
            for (int r = 0; r < 3; ++r) u1[r] /= n1;
            cross3(u0, u1, u2);
            for (int r = 0; r < 3; ++r) { Us[3 * r + 1] = u1[r]; Us[3 * r + 2] = u2[r]; }
        }
    } else if (ss[2] <= 1e-300 * smax) {
        double u0[3] = {Us[0], Us[3], Us[6]}, u1[3] = {Us[1], Us[4], Us[7]}, u2[3];
        cross3(u0, u1, u2);
        for (int r = 0; r < 3; ++r) Us[3 * r + 2] = u2[r];
    }
    /* make V a rotation (flip its last column together with U's) */
    if (det3(Vs) < 0) {
        for (int r = 0; r < 3; ++r) { Vs[3 * r + 2] = -Vs[3 * r + 2]; Us[3 * r + 2] = -Us[3 * r + 2]; }
    }
    /* make U a rotation: the smallest singular value takes the sign */
    if (det3(Us) < 0) {
        for (int r = 0; r < 3; ++r) Us[3 * r + 2] = -Us[3 * r + 2];
        ss[2] = -ss[2];
    }
    memcpy(U, Us, sizeof Us);
    memcpy(V, Vs, sizeof Vs);
    memcpy(sig, ss, sizeof ss);
}

/* R(F) of the polar decomposition F = R S with det R = +1, R = U V^T. */
static void rotation_part(const double* F, double* R)
{
    double U[9], s[3], V[9], Vt[9];
    or_svd3(F, U, s, V);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Vt[3 * i + j] = V[3 * j + i];
    matmul3(U, Vt, R);
}

/* ------------------------------------------------------------------ */
/* Constitutive models, Sec. "Constitutive Models"                      */
/* ------------------------------------------------------------------ */
void or_lame(double E, double nu, double* mu, double* lam)
{
    /* Eq. (lame) */
    *mu = E / (2.0 * (1.0 + nu));
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

/* Psi(F).  Corotated, Eq. (cor): mu |F - R(F)|_F^2 + lambda/2 (det F - 1)^2.
 * Neo-Hookean, Eq. (nh): 1/2 mu |F|_F^2 + lhat/2 (det F - 1 - mu/lhat)^2,
 * lhat = mu + lambda.  Stable Neo-Hookean, Eq. (snh) with the Lame lambda on
 * its volume term (the printed equation lacks a factor there; with it the
 * rest state is stress free): 1/2 mu (|F|^2 - 3) + 1/2 lambda (det F - alpha)^2
 * - 1/2 mu log(1 + |F|^2), alpha = 1 + 3 mu / (4 lambda). */
double or_psi(int model, double mu, double lam, const double* F)
{
    double J = det3(F);
    if (model == OR_STABLE_NEOHOOKEAN) {
        double f2 = 0.0;
        for (int k = 0; k < 9; ++k) f2 += F[k] * F[k];
        double q = J - 1.0 - 0.75 * mu / lam;
        return 0.5 * mu * (f2 - 3.0) + 0.5 * lam * q * q - 0.5 * mu * log(1.0 + f2);
    }
    if (model == OR_NEOHOOKEAN) {
        double lh = mu + lam, f2 = 0.0;
        for (int k = 0; k < 9; ++k) f2 += F[k] * F[k];
        double q = J - 1.0 - mu / lh;
        return 0.5 * mu * f2 + 0.5 * lh * q * q;
    } else {
        double R[9], d2 = 0.0;
        rotation_part(F, R);
        for (int k = 0; k < 9; ++k) d2 += (F[k] - R[k]) * (F[k] - R[k]);
        return mu * d2 + 0.5 * lam * (J - 1.0) * (J - 1.0);
    }
}

/* P = dPsi/dF.  d det(F)/dF = cof(F); for the corotated model the term
 * d/dF |F - R(F)|^2 = 2 (F - R) (the standard result for the polar
 * rotation, valid with the signed-SVD convention). */
void or_pk1(int model, double mu, double lam, const double* F, double* P)
{
    double C[9];
    double J = det3(F);
    cofactor3(F, C);
    if (model == OR_STABLE_NEOHOOKEAN) {
        /* d/dF [-1/2 mu log(1 + |F|^2)] = -mu F / (1 + |F|^2) */
        double f2 = 0.0;
        for (int k = 0; k < 9; ++k) f2 += F[k] * F[k];
        double q = J - 1.0 - 0.75 * mu / lam;
        for (int k = 0; k < 9; ++k) P[k] = mu * (1.0 - 1.0 / (1.0 + f2)) * F[k] + lam * q * C[k];
    } else if (model == OR_NEOHOOKEAN) {
        double lh = mu + lam;
        double q = J - 1.0 - mu / lh;
        for (int k = 0; k < 9; ++k) P[k] = mu * F[k] + lh * q * C[k];
    } else {
        double R[9];
        rotation_part(F, R);
        for (int k = 0; k < 9; ++k) P[k] = 2.0 * mu * (F[k] - R[k]) + lam * (J - 1.0) * C[k];
    }
}

/* Neo-Hookean stress differential dP[dF] (the true Hessian density applied
 * to dF).  The cofactor is a quadratic function of F, so its directional
 * derivative is exactly (cof(F + dF) - cof(F - dF)) / 2. */
void or_nh_dpk1(double mu, double lam, const double* F, const double* dF, double* dP)
{
    double C[9], Cp[9], Cm[9], Fp[9], Fm[9];
    double lh = mu + lam;
    double J = det3(F);
    double q = J - 1.0 - mu / lh;
    cofactor3(F, C);
    for (int k = 0; k < 9; ++k) { Fp[k] = F[k] + dF[k]; Fm[k] = F[k] - dF[k]; }
    cofactor3(Fp, Cp);
    cofactor3(Fm, Cm);
    double dJ = 0.0;
    for (int k = 0; k < 9; ++k) dJ += C[k] * dF[k];
    for (int k = 0; k < 9; ++k)
        dP[k] = mu * dF[k] + lh * dJ * C[k] + lh * q * 0.5 * (Cp[k] - Cm[k]);
}

/* Stress differential dP[dF] for any model (the true Hessian density of
 * Eq. (hess) applied to dF).  The cofactor is quadratic in F, so its
 * derivative along dF is exactly (cof(F + dF) - cof(F - dF)) / 2, and
 * d det = cof(F) : dF.
 *   Neo-Hookean:        mu dF + lhat (cof:dF) cof + lhat (J - 1 - mu/lhat) dcof
 *   stable Neo-Hookean: mu (1 - 1/(1+|F|^2)) dF + 2 mu (F:dF)/(1+|F|^2)^2 F
 *                       + lambda (cof:dF) cof + lambda (J - alpha) dcof
 *   corotated:          2 mu (dF - dR) + lambda (cof:dF) cof + lambda (J - 1) dcof,
 * where, with F = R S (S symmetric), dR = R [w]_x and w solves
 * ((tr S) I - S) w = axial(R^T dF - dF^T R): the skew part of R^T dF equals
 * (W S + S W) / 2 for W = [w]_x, and W S + S W = [((tr S) I - S) w]_x. */
void or_dpk1(int model, double mu, double lam, const double* F, const double* dF, double* dP)
{
    double C[9], Cp[9], Cm[9], Fp[9], Fm[9];
    double J = det3(F);
    cofactor3(F, C);
    for (int k = 0; k < 9; ++k) { Fp[k] = F[k] + dF[k]; Fm[k] = F[k] - dF[k]; }
    cofactor3(Fp, Cp);
    cofactor3(Fm, Cm);
    double dJ = 0.0;
    for (int k = 0; k < 9; ++k) dJ += C[k] * dF[k];
    if (model == OR_NEOHOOKEAN) {
        or_nh_dpk1(mu, lam, F, dF, dP);
    } else if (model == OR_STABLE_NEOHOOKEAN) {
        double f2 = 0.0, fd = 0.0;
        for (int k = 0; k < 9; ++k) { f2 += F[k] * F[k]; fd += F[k] * dF[k]; }
        double q = J - 1.0 - 0.75 * mu / lam;
        double a = mu * (1.0 - 1.0 / (1.0 + f2)), b = 2.0 * mu * fd / ((1.0 + f2) * (1.0 + f2));
        for (int k = 0; k < 9; ++k)
            dP[k] = a * dF[k] + b * F[k] + lam * dJ * C[k] + lam * q * 0.5 * (Cp[k] - Cm[k]);
    } else {
        double R[9], S[9], M[9], Mi[9], W[9], w[3], om[3], Om[9], dR[9];
        rotation_part(F, R);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0, t = 0.0;
                for (int k = 0; k < 3; ++k) {
                    s += R[3 * k + i] * F[3 * k + j];    /* S = R^T F */
                    t += R[3 * k + i] * dF[3 * k + j];   /* R^T dF    */
                }
                S[3 * i + j] = s;
                W[3 * i + j] = t;
            }
        /* axial vector of R^T dF - (R^T dF)^T */
        w[0] = W[3 * 2 + 1] - W[3 * 1 + 2];
        w[1] = W[3 * 0 + 2] - W[3 * 2 + 0];
        w[2] = W[3 * 1 + 0] - W[3 * 0 + 1];
        double tr = S[0] + S[4] + S[8];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[3 * i + j] = (i == j ? tr : 0.0) - 0.5 * (S[3 * i + j] + S[3 * j + i]);
        if (inv3(M, Mi)) {
            for (int k = 0; k < 9; ++k) dP[k] = NAN;
            return;
        }
        for (int i = 0; i < 3; ++i) om[i] = Mi[3 * i] * w[0] + Mi[3 * i + 1] * w[1] + Mi[3 * i + 2] * w[2];
        Om[0] = 0.0;    Om[1] = -om[2]; Om[2] = om[1];
        Om[3] = om[2];  Om[4] = 0.0;    Om[5] = -om[0];
        Om[6] = -om[1]; Om[7] = om[0];  Om[8] = 0.0;
        matmul3(R, Om, dR);
        for (int k = 0; k < 9; ++k)
            dP[k] = 2.0 * mu * (dF[k] - dR[k]) + lam * dJ * C[k] + lam * (J - 1.0) * 0.5 * (Cp[k] - Cm[k]);
    }
}

/* Modified Hessian density, Eq. (mod_hess_dens), as the full fourth-order
 * tensor Ct[alpha][gamma][beta][delta] (index ((a*3+g)*3+b)*3+d):
 *   2 mu delta_ab delta_gd + lambda cof(F)_ag cof(F)_bd
 * (Lame lambda for every model). */
void or_mod_hess_density(double mu, double lam, const double* F, double* Ct)
{
    double C[9];
    cofactor3(F, C);
    for (int a = 0; a < 3; ++a)
        for (int g = 0; g < 3; ++g)
            for (int b = 0; b < 3; ++b)
                for (int d = 0; d < 3; ++d)
                    Ct[((a * 3 + g) * 3 + b) * 3 + d] =
                        2.0 * mu * (a == b) * (g == d) + lam * C[3 * a + g] * C[3 * b + d];
}

/* ------------------------------------------------------------------ */
/* Discretisation, Sec. "Discretization"                                */
/* ------------------------------------------------------------------ */
/* Per tet: dN[e][j][:] = dN_j/dX for the 4 vertices, V0[e] = rest volume.
 * With Dm = [X1 - X0, X2 - X0, X3 - X0], dN_j (j = 1..3) is row j-1 of Dm^{-1}
 * and dN_0 = -(dN_1 + dN_2 + dN_3).  Returns -1 if a tet has V0 <= 0. */
int or_prep(int32_t nv, int32_t nt, const double* X, const int32_t* tets,
            double* dN /* [nt][4][3] */, double* V0 /* [nt] */)
{
    for (int e = 0; e < nt; ++e) {
        const int32_t* t = tets + 4 * e;
        for (int j = 0; j < 4; ++j)
            if (t[j] < 0 || t[j] >= nv) return -2;
        double Dm[9], Dmi[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Dm[3 * r + c] = X[3 * t[c + 1] + r] - X[3 * t[0] + r];
        double v = det3(Dm) / 6.0;
        if (!(v > 0.0)) return -1;
        if (inv3(Dm, Dmi)) return -1;
        V0[e] = v;
        double* g = dN + 12 * e;
        for (int j = 1; j < 4; ++j)
            for (int c = 0; c < 3; ++c) g[3 * j + c] = Dmi[3 * (j - 1) + c];
        for (int c = 0; c < 3; ++c) g[c] = -(g[3 + c] + g[6 + c] + g[9 + c]);
    }
    return 0;
}

/* Lumped body force: fhat_i = int R0 g N_i dX = sum_{e containing i} R0 g V0_e / 4
 * (a linear basis function integrates to V0/4 over a tet). */
void or_body_force(int32_t nv, int32_t nt, const int32_t* tets, const double* V0,
                   double density, const double* grav, double* fext /* [nv][3], accumulated */)
{
    (void)nv;
    for (int e = 0; e < nt; ++e)
        for (int j = 0; j < 4; ++j)
            for (int c = 0; c < 3; ++c) fext[3 * tets[4 * e + j] + c] += density * grav[c] * V0[e] / 4.0;
}

/* Lumped mass of Eq. (fem_be): m_ii = int R0 N_i dX, which for linear tets
 * is R0 V0_e / 4 from every incident tet.  Accumulates into m[nv]. */
void or_lumped_mass(int32_t nv, int32_t nt, const int32_t* tets, const double* V0,
                    double density, double* m)
{
    (void)nv;
    for (int e = 0; e < nt; ++e)
        for (int j = 0; j < 4; ++j) m[tets[4 * e + j]] += density * V0[e] / 4.0;
}

/* Inertia term 1/2 minert_i |yi - xhat_i|^2 of vertex i (0 without inertia). */
static double inertia_energy(const or_problem* p, int i, const double* yi)
{
    if (!p->minert) return 0.0;
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d = yi[a] - p->xhat[3 * i + a];
        s += d * d;
    }
    return 0.5 * p->minert[i] * s;
}

/* F_e(y) = sum_j y_j dN_j^T. */
static void deformation_gradient(const double* y, const int32_t* t, const double* g, double* F)
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int j = 0; j < 4; ++j) s += y[3 * t[j] + a] * g[3 * j + b];
            F[3 * a + b] = s;
        }
}

/* ------------------------------------------------------------------ */
/* Internal adjacency: vertex -> incident tets (with local slot) and     */
/* vertex -> incident weak constraints (with position in the CSR).      */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t *tptr, *tlist, *tslot;
    int32_t *cptr, *clist, *cpos;
    double* dN;
    double* V0;
} or_adj;

static void adj_free(or_adj* A)
{
    free(A->tptr); free(A->tlist); free(A->tslot);
    free(A->cptr); free(A->clist); free(A->cpos);
    free(A->dN); free(A->V0);
    memset(A, 0, sizeof *A);
}

static int adj_build(const or_problem* p, or_adj* A)
{
    memset(A, 0, sizeof *A);
    int nv = p->nv, nt = p->nt;
    A->dN = (double*)malloc(sizeof(double) * 12 * (size_t)(nt > 0 ? nt : 1));
    A->V0 = (double*)malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
    int rc = or_prep(nv, nt, p->X, p->tets, A->dN, A->V0);
    if (rc) { adj_free(A); return rc; }
    A->tptr = (int32_t*)calloc((size_t)nv + 1, sizeof(int32_t));
    for (int e = 0; e < nt; ++e)
        for (int j = 0; j < 4; ++j) A->tptr[p->tets[4 * e + j] + 1]++;
    for (int i = 0; i < nv; ++i) A->tptr[i + 1] += A->tptr[i];
    A->tlist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(4 * nt + 1));
    A->tslot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(4 * nt + 1));
    int32_t* fill = (int32_t*)calloc((size_t)nv, sizeof(int32_t));
    for (int e = 0; e < nt; ++e)
        for (int j = 0; j < 4; ++j) {
            int v = p->tets[4 * e + j];
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
    memset(fill, 0, sizeof(int32_t) * (size_t)nv);
    for (int c = 0; c < p->n_wc; ++c)
        for (int k = p->wc_ptr[c]; k < p->wc_ptr[c + 1]; ++k) {
            int v = p->wc_vert[k];
            int s = A->cptr[v] + fill[v]++;
            A->clist[s] = c;
            A->cpos[s] = k;
        }
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Node colouring, Sec. "Coloring and Parallelism"                       */
/* ------------------------------------------------------------------ */
/* Vertices are visited in ascending index, Dirichlet vertices skipped
 * (colour -1).  A vertex takes the least colour not used by an already
 * coloured vertex that shares a tet or a weak constraint with it -- the
 * union of the used-colour sets S_c of its incident elements and
 * constraints.  Returns the number of colours, or < 0 on error. */
int32_t or_color(const or_problem* p, int32_t* colors)
{
    or_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    int nv = p->nv;
    int ncol = 0;
    int cap = 64;
    char* used = (char*)malloc((size_t)cap);
    for (int i = 0; i < nv; ++i) colors[i] = -1;
    for (int i = 0; i < nv; ++i) {
        if (p->is_dir[i]) continue;
        memset(used, 0, (size_t)cap);
        for (int k = A.tptr[i]; k < A.tptr[i + 1]; ++k) {
            const int32_t* t = p->tets + 4 * A.tlist[k];
            for (int j = 0; j < 4; ++j)
                if (colors[t[j]] >= 0) used[colors[t[j]]] = 1;
        }
        for (int k = A.cptr[i]; k < A.cptr[i + 1]; ++k) {
            int c = A.clist[k];
            for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s) {
                int v = p->wc_vert[s];
                if (colors[v] >= 0) used[colors[v]] = 1;
            }
        }
        int col = 0;
        while (col < cap && used[col]) ++col;
        if (col >= cap) {
            used = (char*)realloc(used, (size_t)cap * 2);
            cap *= 2;
        }
        colors[i] = col;
        if (col + 1 > ncol) ncol = col + 1;
    }
    free(used);
    adj_free(&A);
    return ncol;
}

/* Incremental recolouring (Sec. "Collision Coloring"): after new weak
 * constraints were added to p, the free vertices incident to them -- given
 * in `nodes`, processed in the order given -- each keep their colour from
 * `colors` if no other vertex sharing a tet or a weak constraint with them
 * uses it (the union of the colour sets S_c of their elements and
 * constraints, their own entry left out), and otherwise take the least
 * colour not in that union.  `colors` is updated in place, so later nodes
 * see earlier changes.  Returns the number of colours, or < 0 on error. */
int32_t or_recolor(const or_problem* p, int32_t n_nodes, const int32_t* nodes, int32_t* colors)
{
    or_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    int cap = 1;
    for (int i = 0; i < p->nv; ++i)
        if (colors[i] + 2 > cap) cap = colors[i] + 2;
    cap += n_nodes;
    char* used = (char*)malloc((size_t)cap);
    for (int k = 0; k < n_nodes; ++k) {
        int i = nodes[k];
        if (p->is_dir[i]) continue;
        memset(used, 0, (size_t)cap);
        for (int m = A.tptr[i]; m < A.tptr[i + 1]; ++m) {
            const int32_t* t = p->tets + 4 * A.tlist[m];
            for (int j = 0; j < 4; ++j)
                if (t[j] != i && colors[t[j]] >= 0) used[colors[t[j]]] = 1;
        }
        for (int m = A.cptr[i]; m < A.cptr[i + 1]; ++m) {
            int c = A.clist[m];
            for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s) {
                int v = p->wc_vert[s];
                if (v != i && colors[v] >= 0) used[colors[v]] = 1;
            }
        }
        if (colors[i] >= 0 && !used[colors[i]]) continue;
        int col = 0;
        while (used[col]) ++col;
        colors[i] = col;
    }
    int ncol = 0;
    for (int i = 0; i < p->nv; ++i)
        if (colors[i] + 1 > ncol) ncol = colors[i] + 1;
    free(used);
    adj_free(&A);
    return ncol;
}

/* ------------------------------------------------------------------ */
/* Energy, forces and the local step                                     */
/* ------------------------------------------------------------------ */
static double sym6(const double* K, int a, int b)
{
    static const int idx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    return K[idx[a][b]];
}

/* Local energy of the terms that involve vertex i, with y_i replaced by yi:
 * sum over incident tets of V0 Psi, incident weak constraints 1/2 C^T K C,
 * planes 1/2 k min(0, n.yi - d)^2, and -yi . fext_i.  The magnitudes of the
 * summands are added to *absum. */
static double local_energy(const or_problem* p, const or_adj* A, const double* y, int i,
                           const double* yi, double* absum)
{
    double E = 0.0, ab = 0.0;
    for (int k = A->tptr[i]; k < A->tptr[i + 1]; ++k) {
        int e = A->tlist[k];
        const int32_t* t = p->tets + 4 * e;
        const double* g = A->dN + 12 * e;
        double F[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int j = 0; j < 4; ++j) {
                    const double* yj = (t[j] == i) ? yi : y + 3 * t[j];
                    s += yj[a] * g[3 * j + b];
                }
                F[3 * a + b] = s;
            }
        double w = A->V0[e] * or_psi(p->model, p->mu[e], p->lam[e], F);
        E += w;
        ab += fabs(w);
    }
    for (int k = A->cptr[i]; k < A->cptr[i + 1]; ++k) {
        int c = A->clist[k];
        double C[3] = {0, 0, 0};
        for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s) {
            int v = p->wc_vert[s];
            const double* yv = (v == i) ? yi : y + 3 * v;
            for (int a = 0; a < 3; ++a) C[a] += p->wc_w[s] * yv[a];
        }
        double w = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) w += 0.5 * C[a] * sym6(p->wc_K + 6 * c, a, b) * C[b];
        E += w;
        ab += fabs(w);
    }
    for (int q = 0; q < p->n_planes; ++q) {
        const double* pl = p->planes + 5 * q;
        double phi = pl[0] * yi[0] + pl[1] * yi[1] + pl[2] * yi[2] - pl[3];
        if (phi < 0) {
            double w = 0.5 * pl[4] * phi * phi;
            E += w;
            ab += fabs(w);
        }
    }
    double w = -(yi[0] * p->fext[3 * i] + yi[1] * p->fext[3 * i + 1] + yi[2] * p->fext[3 * i + 2]);
    E += w;
    ab += fabs(w);
    w = inertia_energy(p, i, yi);
    E += w;
    ab += fabs(w);
    if (absum) *absum += ab;
    return E;
}

/* Gradient g_i = dE/dy_i (= -(f_i + fhat_i)) and the modified nodal
 * Hessian A_i of Eq. (mod_hess), contracting the fourth-order density of
 * Eq. (mod_hess_dens) with dN_i dN_i^T, plus (w0 - w1)^2 K_c for weak
 * constraints and k n n^T for active planes. */
static void local_system(const or_problem* p, const or_adj* A, const double* y, int i,
                         double* gi, double* Ai)
{
    for (int a = 0; a < 3; ++a) gi[a] = -p->fext[3 * i + a];
    for (int k = 0; k < 9; ++k) Ai[k] = 0.0;
    for (int k = A->tptr[i]; k < A->tptr[i + 1]; ++k) {
        int e = A->tlist[k], slot = A->tslot[k];
        const int32_t* t = p->tets + 4 * e;
        const double* g = A->dN + 12 * e;
        const double* a = g + 3 * slot;
        double F[9], P[9], Ct[81];
        double V = A->V0[e];
        deformation_gradient(y, t, g, F);
        or_pk1(p->model, p->mu[e], p->lam[e], F, P);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) gi[r] += V * P[3 * r + c] * a[c];
        or_mod_hess_density(p->mu[e], p->lam[e], F, Ct);
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be) {
                double s = 0.0;
                for (int ga = 0; ga < 3; ++ga)
                    for (int de = 0; de < 3; ++de)
                        s += Ct[((al * 3 + ga) * 3 + be) * 3 + de] * a[ga] * a[de];
                Ai[3 * al + be] += V * s;
            }
    }
    for (int k = A->cptr[i]; k < A->cptr[i + 1]; ++k) {
        int c = A->clist[k];
        double sci = p->wc_w[A->cpos[k]];
        double C[3] = {0, 0, 0};
        for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s)
            for (int a = 0; a < 3; ++a) C[a] += p->wc_w[s] * y[3 * p->wc_vert[s] + a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double Kab = sym6(p->wc_K + 6 * c, a, b);
                gi[a] += sci * Kab * C[b];
                Ai[3 * a + b] += sci * sci * Kab;
            }
    }
    for (int q = 0; q < p->n_planes; ++q) {
        const double* pl = p->planes + 5 * q;
        const double* yi = y + 3 * i;
        double phi = pl[0] * yi[0] + pl[1] * yi[1] + pl[2] * yi[2] - pl[3];
        if (phi < 0)
            for (int a = 0; a < 3; ++a) {
                gi[a] += pl[4] * phi * pl[a];
                for (int b = 0; b < 3; ++b) Ai[3 * a + b] += pl[4] * pl[a] * pl[b];
            }
    }
    if (p->minert)
        for (int a = 0; a < 3; ++a) {
            gi[a] += p->minert[i] * (y[3 * i + a] - p->xhat[3 * i + a]);
            Ai[3 * a + a] += p->minert[i];
        }
}

static double to_f32(double v) { return (double)(float)v; }

/* One sub-iterate of Eq. (pbgn_update)/(pbgn_dx): a single modified-Newton
 * step on vertex i from Delta = 0, optionally safeguarded by halving the
 * step until the local energy does not increase (beyond a round-off slack
 * of 8 u sum |summands|); if no step length passes, the vertex keeps its
 * position.  Returns the number of halvings, or -1 when rejected. */
static int update_vertex(const or_problem* p, const or_adj* A, double* y, int i,
                         const or_opts* o)
{
    double gi[3], Ai[9], Aiv[9], d[3];
    local_system(p, A, y, i, gi, Ai);
    if (o->skip_tol > 0.0 &&
        sqrt(gi[0] * gi[0] + gi[1] * gi[1] + gi[2] * gi[2]) <= o->skip_tol)
        return 0;
    if (inv3(Ai, Aiv)) return -1;
    for (int a = 0; a < 3; ++a)
        d[a] = -(Aiv[3 * a] * gi[0] + Aiv[3 * a + 1] * gi[1] + Aiv[3 * a + 2] * gi[2]);
    double yi0[3] = {y[3 * i], y[3 * i + 1], y[3 * i + 2]};
    double alpha = 1.0;
    int halvings = 0;
    if (o->safeguard == OR_SAFEGUARD_BACKTRACK) {
        const double u = 1.1102230246251565e-16; /* 2^-53 */
        double ab0 = 0.0;
        double E0 = local_energy(p, A, y, i, yi0, &ab0);
        for (;;) {
            double yt[3], ab1 = 0.0;
            for (int a = 0; a < 3; ++a) yt[a] = yi0[a] + alpha * d[a];
            if (o->emulate_f32)
                for (int a = 0; a < 3; ++a) yt[a] = to_f32(yt[a]);
            double E1 = local_energy(p, A, y, i, yt, &ab1);
            if (E1 - E0 <= 8.0 * u * (ab0 + ab1)) break;
            if (halvings >= o->max_halvings) return -1;
            alpha *= 0.5;
            ++halvings;
        }
    }
    for (int a = 0; a < 3; ++a) {
        double v = yi0[a] + alpha * d[a];
        y[3 * i + a] = o->emulate_f32 ? to_f32(v) : v;
    }
    return halvings;
}

/* Residual r_i = f_i(y) + fhat_i over free vertices (Eq. fem_qs), computed
 * by scattering the element forces -V0 P dN_j, and the total energy
 * PE(y) - y . fhat (Eq. pe_hat plus the plane penalty).  Returns ||r||_2. */
double or_residual(const or_problem* p, const double* y, double* r_out /* nullable [nv][3] */,
                   double* energy_out)
{
    or_adj A;
    if (adj_build(p, &A)) return -1.0;
    double* f = (double*)calloc((size_t)3 * p->nv, sizeof(double));
    double E = 0.0;
    for (int e = 0; e < p->nt; ++e) {
        const int32_t* t = p->tets + 4 * e;
        const double* g = A.dN + 12 * e;
        double F[9], P[9];
        deformation_gradient(y, t, g, F);
        or_pk1(p->model, p->mu[e], p->lam[e], F, P);
        E += A.V0[e] * or_psi(p->model, p->mu[e], p->lam[e], F);
        for (int j = 0; j < 4; ++j)
            for (int r = 0; r < 3; ++r) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c) s += P[3 * r + c] * g[3 * j + c];
                f[3 * t[j] + r] -= A.V0[e] * s;
            }
    }
    for (int c = 0; c < p->n_wc; ++c) {
        double C[3] = {0, 0, 0};
        for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s)
            for (int a = 0; a < 3; ++a) C[a] += p->wc_w[s] * y[3 * p->wc_vert[s] + a];
        double KC[3];
        for (int a = 0; a < 3; ++a) {
            KC[a] = 0.0;
            for (int b = 0; b < 3; ++b) KC[a] += sym6(p->wc_K + 6 * c, a, b) * C[b];
        }
        E += 0.5 * (C[0] * KC[0] + C[1] * KC[1] + C[2] * KC[2]);
        for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s)
            for (int a = 0; a < 3; ++a) f[3 * p->wc_vert[s] + a] -= p->wc_w[s] * KC[a];
    }
    for (int i = 0; i < p->nv; ++i) {
        for (int q = 0; q < p->n_planes; ++q) {
            const double* pl = p->planes + 5 * q;
            double phi = pl[0] * y[3 * i] + pl[1] * y[3 * i + 1] + pl[2] * y[3 * i + 2] - pl[3];
            if (phi < 0) {
                E += 0.5 * pl[4] * phi * phi;
                for (int a = 0; a < 3; ++a) f[3 * i + a] -= pl[4] * phi * pl[a];
            }
        }
        for (int a = 0; a < 3; ++a) E -= y[3 * i + a] * p->fext[3 * i + a];
        if (p->minert) {
            E += inertia_energy(p, i, y + 3 * i);
            for (int a = 0; a < 3; ++a) f[3 * i + a] -= p->minert[i] * (y[3 * i + a] - p->xhat[3 * i + a]);
        }
    }
    double n2 = 0.0;
    for (int i = 0; i < p->nv; ++i)
        for (int a = 0; a < 3; ++a) {
            double r = p->is_dir[i] ? 0.0 : f[3 * i + a] + p->fext[3 * i + a];
            if (r_out) r_out[3 * i + a] = r;
            n2 += r * r;
        }
    free(f);
    adj_free(&A);
    if (energy_out) *energy_out = E;
    return sqrt(n2);
}

/* Chebyshev weights, Sec. "Acceleration Techniques": omega_{l+1} = 1 for
 * l < 2, 2 / (2 - rho^2) for l = 2 and 4 / (4 - rho^2 omega_l) for l > 2.
 * Writes omega_1 .. omega_n into w[0 .. n-1]. */
void or_chebyshev_weights(double rho, int32_t n, double* w)
{
    double prev = 1.0;
    for (int l = 0; l < n; ++l) {
        double om;
        if (l < 2) om = 1.0;
        else if (l == 2) om = 2.0 / (2.0 - rho * rho);
        else om = 4.0 / (4.0 - rho * rho * prev);
        w[l] = om;
        prev = om;
    }
}

/* One Gauss-Seidel sweep over the colours in sequence, in place. */
static void sweep(const or_problem* p, const or_adj* A, const int32_t* colors, int32_t ncol,
                  const int32_t* order, const int32_t* cptr, double* y, const or_opts* o,
                  or_stats* st)
{
    (void)colors;
    for (int c = 0; c < ncol; ++c) {
        int64_t rej = 0, hal = 0;
        int lo = cptr[c], hi = cptr[c + 1];
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(+ : rej, hal) num_threads(o->n_threads > 1 ? o->n_threads : 1) if (o->n_threads > 1)
#endif
        for (int k = lo; k < hi; ++k) {
            int h = update_vertex(p, A, y, order[k], o);
            if (h < 0) ++rej;
            else hal += h;
        }
        st->rejected += rej;
        st->halvings += hal;
    }
}

/* Full solve: sweeps, optional Chebyshev / SOR blend across sweeps over the
 * free vertices, FP64 residual every check_every sweeps.  x holds the
 * initial iterate (Dirichlet rows already set) and receives the result.
 * If hist is non-null, the relative residual after each check is written
 * there (hist[k] after sweep (k + 1) * check_every). */
int32_t or_solve(const or_problem* p, const int32_t* colors, double* x, const or_opts* o,
                 or_stats* st, double* hist)
{
    memset(st, 0, sizeof *st);
    or_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    int nv = p->nv;
    int ncol = 0;
    for (int i = 0; i < nv; ++i)
        if (colors[i] + 1 > ncol) ncol = colors[i] + 1;
    int32_t* cptr = (int32_t*)calloc((size_t)ncol + 1, sizeof(int32_t));
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nv + 1));
    for (int i = 0; i < nv; ++i)
        if (colors[i] >= 0) cptr[colors[i] + 1]++;
    for (int c = 0; c < ncol; ++c) cptr[c + 1] += cptr[c];
    int32_t* fill = (int32_t*)calloc((size_t)ncol + 1, sizeof(int32_t));
    for (int i = 0; i < nv; ++i)
        if (colors[i] >= 0) order[cptr[colors[i]] + fill[colors[i]]++] = i;
    free(fill);

    double* xl = (double*)malloc(sizeof(double) * 3 * (size_t)nv);   /* x^l     */
    double* xlm1 = (double*)malloc(sizeof(double) * 3 * (size_t)nv); /* x^{l-1} */
    memcpy(xlm1, x, sizeof(double) * 3 * (size_t)nv);
    double E = 0.0;
    double res0 = or_residual(p, x, NULL, &E);
    st->res0 = res0;
    st->res = res0;
    st->rel = res0 > 0 ? 1.0 : 0.0;
    st->energy = E;
    double omega = 1.0;
    int every = o->check_every > 0 ? o->check_every : 1;
    int nh = 0;
    for (int l = 0; l < o->max_sweeps; ++l) {
        if (res0 == 0.0) { st->converged = 1; break; }
        memcpy(xl, x, sizeof(double) * 3 * (size_t)nv);
        sweep(p, &A, colors, ncol, order, cptr, x, o, st);  /* x := x_PBNG^{l+1} */
        if (o->accel != OR_ACCEL_NONE) {
            double w, gam;
            if (o->accel == OR_ACCEL_CHEBYSHEV) {
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
                for (int a = 0; a < 3; ++a) {
                    int k = 3 * i + a;
                    double v;
                    if (o->accel == OR_ACCEL_CHEBYSHEV)
                        v = w * (gam * (x[k] - xl[k]) + xl[k] - xlm1[k]) + xlm1[k];
                    else
                        v = w * (x[k] - xlm1[k]) + xlm1[k];
                    x[k] = o->emulate_f32 ? to_f32(v) : v;
                }
            }
            double* t = xlm1; xlm1 = xl; xl = t;   /* x^{l-1} := x^l */
        }
        st->sweeps = l + 1;
        if ((l + 1) % every == 0 || l + 1 == o->max_sweeps) {
            double r = or_residual(p, x, NULL, &E);
            st->res = r;
            st->rel = r / res0;
            st->energy = E;
            if (hist && (l + 1) % every == 0) hist[nh++] = st->rel;
            if (!isfinite(r)) break;
            if (st->rel <= o->rel_tol) { st->converged = 1; break; }
        }
    }
    free(xl); free(xlm1); free(cptr); free(order);
    adj_free(&A);
    return 0;
}

/* Energy change of every single-vertex update during one sweep (no blend):
 * dE[k] = E(after update k) - E(before update k) for the k-th update in
 * sweep order.  Used to check that the safeguard never increases the
 * energy. */
int32_t or_sweep_energy_trace(const or_problem* p, const int32_t* colors, double* x,
                              const or_opts* o, double* dE /* [n_free] */)
{
    or_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    int nv = p->nv, ncol = 0, n = 0;
    for (int i = 0; i < nv; ++i)
        if (colors[i] + 1 > ncol) ncol = colors[i] + 1;
    for (int c = 0; c < ncol; ++c)
        for (int i = 0; i < nv; ++i) {
            if (colors[i] != c) continue;
            double before[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
            double E0 = local_energy(p, &A, x, i, before, NULL);
            update_vertex(p, &A, x, i, o);
            double after[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
            double E1 = local_energy(p, &A, x, i, after, NULL);
            dE[n++] = E1 - E0;
        }
    adj_free(&A);
    return n;
}

/* The single-vertex update of Eq. (pbgn_dx) (with the safeguard of *o)
 * applied to each listed vertex, every one computed from the same
 * positions y (valid for vertices of one colour, which share no term).
 * out[k] receives the new position of verts[k]; y is not modified. */
int32_t or_update_vertices(const or_problem* p, const double* y, int32_t n, const int32_t* verts,
                           const or_opts* o, double* out)
{
    or_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    double* z = (double*)malloc(sizeof(double) * 3 * (size_t)p->nv);
    memcpy(z, y, sizeof(double) * 3 * (size_t)p->nv);
    for (int k = 0; k < n; ++k) {
        int i = verts[k];
        update_vertex(p, &A, z, i, o);
        for (int a = 0; a < 3; ++a) {
            out[3 * k + a] = z[3 * i + a];
            z[3 * i + a] = y[3 * i + a];
        }
    }
    free(z);
    adj_free(&A);
    return 0;
}

/* ------------------------------------------------------------------ */
/* True Hessian and adjoint gradient assembly                           */
/* ------------------------------------------------------------------ */
/* out = H v, with H = d^2 E / dy^2 at y, for every vertex (Dirichlet rows
 * included; callers restrict).  Element part: sum_e V0 dP_e[sum_j v_j dN_j^T]
 * dN_i (Eq. hess with the exact density); weak constraints: s_ci K_c
 * sum_j s_cj v_j; active planes: k n n^T v_i; inertia: minert_i v_i. */
int32_t or_hvp(const or_problem* p, const double* y, const double* v, double* out)
{
    or_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    memset(out, 0, sizeof(double) * 3 * (size_t)p->nv);
    for (int e = 0; e < p->nt; ++e) {
        const int32_t* t = p->tets + 4 * e;
        const double* g = A.dN + 12 * e;
        double F[9], dF[9], dP[9];
        deformation_gradient(y, t, g, F);
        deformation_gradient(v, t, g, dF);
        or_dpk1(p->model, p->mu[e], p->lam[e], F, dF, dP);
        for (int j = 0; j < 4; ++j)
            for (int r = 0; r < 3; ++r) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c) s += dP[3 * r + c] * g[3 * j + c];
                out[3 * t[j] + r] += A.V0[e] * s;
            }
    }
    for (int c = 0; c < p->n_wc; ++c) {
        double C[3] = {0, 0, 0};
        for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s)
            for (int a = 0; a < 3; ++a) C[a] += p->wc_w[s] * v[3 * p->wc_vert[s] + a];
        for (int s = p->wc_ptr[c]; s < p->wc_ptr[c + 1]; ++s)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    out[3 * p->wc_vert[s] + a] += p->wc_w[s] * sym6(p->wc_K + 6 * c, a, b) * C[b];
    }
    for (int i = 0; i < p->nv; ++i)
        for (int q = 0; q < p->n_planes; ++q) {
            const double* pl = p->planes + 5 * q;
            double phi = pl[0] * y[3 * i] + pl[1] * y[3 * i + 1] + pl[2] * y[3 * i + 2] - pl[3];
            if (phi < 0) {
                double nv_ = pl[0] * v[3 * i] + pl[1] * v[3 * i + 1] + pl[2] * v[3 * i + 2];
                for (int a = 0; a < 3; ++a) out[3 * i + a] += pl[4] * pl[a] * nv_;
            }
        }
    if (p->minert)
        for (int i = 0; i < p->nv; ++i)
            for (int a = 0; a < 3; ++a) out[3 * i + a] += p->minert[i] * v[3 * i + a];
    adj_free(&A);
    return 0;
}

/* Given the adjoint vector lam (zero on Dirichlet rows) solving H_FF lam =
 * dL/dx_F, the gradients of L(x*(theta)) follow from dL/dtheta =
 * -lam^T dg/dtheta with g = dE/dy_F:
 *   dL/dmu_e     = -V0 < dP/dmu,  Lam_e >
 *   dL/dlambda_e = -V0 < dP/dlam, Lam_e >,   dP/dlam = (J - 1) cof F (all models)
 *   dL/dx_k      = -(H lam)_k for Dirichlet vertices k
 * with dP/dmu = F + (J - 2) cof F (Neo-Hookean), 2 (F - R) (corotated) and
 * (1 - 1/(1+|F|^2)) F - 3/4 cof F (stable Neo-Hookean), and
 * Lam_e = sum_j lam_j dN_j^T.  Any output may be NULL. */
int32_t or_adjoint_gradients(const or_problem* p, const double* y, const double* lam,
                             double* dmu, double* dlam, double* dxd /* [nv][3] */)
{
    or_adj A;
    int rc = adj_build(p, &A);
    if (rc) return rc;
    for (int e = 0; e < p->nt; ++e) {
        const int32_t* t = p->tets + 4 * e;
        const double* g = A.dN + 12 * e;
        double F[9], L[9], C[9];
        deformation_gradient(y, t, g, F);
        deformation_gradient(lam, t, g, L);
        cofactor3(F, C);
        double J = det3(F);
        double Pm[9], R[9], f2 = 0.0;
        for (int k = 0; k < 9; ++k) f2 += F[k] * F[k];
        if (p->model == OR_COROTATED) rotation_part(F, R);
        for (int k = 0; k < 9; ++k) {
            if (p->model == OR_NEOHOOKEAN) Pm[k] = F[k] + (J - 2.0) * C[k];
            else if (p->model == OR_COROTATED) Pm[k] = 2.0 * (F[k] - R[k]);
            else Pm[k] = (1.0 - 1.0 / (1.0 + f2)) * F[k] - 0.75 * C[k];
        }
        double smu = 0.0, slam = 0.0;
        for (int k = 0; k < 9; ++k) {
            smu += Pm[k] * L[k];
            slam += (J - 1.0) * C[k] * L[k];
        }
        if (dmu) dmu[e] = -A.V0[e] * smu;
        if (dlam) dlam[e] = -A.V0[e] * slam;
    }
    if (dxd) {
        double* hl = (double*)malloc(sizeof(double) * 3 * (size_t)p->nv);
        rc = or_hvp(p, y, lam, hl);
        for (int i = 0; i < p->nv; ++i)
            for (int a = 0; a < 3; ++a) dxd[3 * i + a] = p->is_dir[i] ? -hl[3 * i + a] : 0.0;
        free(hl);
    }
    adj_free(&A);
    return rc;
}

/* Gradient of the energy, dE/dy for every vertex (no Dirichlet masking). */
int32_t or_energy_gradient(const or_problem* p, const double* y, double* grad)
{
    double* r = (double*)malloc(sizeof(double) * 3 * (size_t)p->nv);
    uint8_t* save = (uint8_t*)malloc((size_t)p->nv);
    or_problem q = *p;
    memset(save, 0, (size_t)p->nv);
    q.is_dir = save;
    double E;
    double n = or_residual(&q, y, r, &E);
    for (int k = 0; k < 3 * p->nv; ++k) grad[k] = -r[k];
    free(r);
    free(save);
    return n < 0 ? -1 : 0;
}

int32_t or_version(void) { return 1; }
