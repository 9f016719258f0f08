// Device-side small-matrix math for the PBNG kernels (gfx950).
//
// Matrices are kept as three column vectors because the cofactor of a 3x3
// matrix is formed column by column from cross products:
//   cof(F)[:,0] = F[:,1] x F[:,2],  cof(F)[:,1] = F[:,2] x F[:,0],
//   cof(F)[:,2] = F[:,0] x F[:,1],  det F = F[:,0] . cof(F)[:,0],
// which is defined for singular and inverted F (Sec. "Modified Hessian").
#pragma once

#include <hip/hip_runtime.h>

namespace pbng {

template <class R>
struct V3 {
    R x, y, z;
};

template <class R>
__device__ __forceinline__ V3<R> mk(R x, R y, R z) { return V3<R>{x, y, z}; }
template <class R>
__device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class R>
__device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R>
__device__ __forceinline__ V3<R> operator*(R s, V3<R> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class R>
__device__ __forceinline__ R dot(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class R>
__device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// a*s + b*t + c*u
template <class R>
__device__ __forceinline__ V3<R> comb(V3<R> a, R s, V3<R> b, R t, V3<R> c, R u)
{
    return {a.x * s + b.x * t + c.x * u, a.y * s + b.y * t + c.y * u, a.z * s + b.z * t + c.z * u};
}

// Single-instruction reciprocal, reciprocal square root and square root in
// float (about 1 ulp); correctly rounded operations in double.
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float abs_(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double abs_(double x) { return fabs(x); }

// Symmetric 3x3 stored as (xx, xy, xz, yy, yz, zz).
template <class R>
struct Sym {
    R xx, xy, xz, yy, yz, zz;
};

template <class R>
__device__ __forceinline__ void sym_add_outer(Sym<R>& A, R w, V3<R> c)
{
    V3<R> wc = w * c;
    A.xx += wc.x * c.x; A.xy += wc.x * c.y; A.xz += wc.x * c.z;
    A.yy += wc.y * c.y; A.yz += wc.y * c.z; A.zz += wc.z * c.z;
}
template <class R>
__device__ __forceinline__ V3<R> sym_mul(const Sym<R>& A, V3<R> v)
{
    return {A.xx * v.x + A.xy * v.y + A.xz * v.z, A.xy * v.x + A.yy * v.y + A.yz * v.z,
            A.xz * v.x + A.yz * v.y + A.zz * v.z};
}

// Solve A d = b for SPD A by Cholesky (A = L L^T).  Returns false if a
// pivot is not positive (never for the SPD modified Hessian unless the
// input is non-finite).
template <class R>
__device__ __forceinline__ bool chol_solve(const Sym<R>& A, V3<R> b, V3<R>& d)
{
    R l00 = A.xx;
    if (!(l00 > R(0))) return false;
    R i00 = rsq(l00);
    R l10 = A.xy * i00, l20 = A.xz * i00;
    R t11 = A.yy - l10 * l10;
    if (!(t11 > R(0))) return false;
    R i11 = rsq(t11);
    R l21 = (A.yz - l20 * l10) * i11;
    R t22 = A.zz - l20 * l20 - l21 * l21;
    if (!(t22 > R(0))) return false;
    R i22 = rsq(t22);
    // forward: L y = b
    R y0 = b.x * i00;
    R y1 = (b.y - l10 * y0) * i11;
    R y2 = (b.z - l20 * y0 - l21 * y1) * i22;
    // backward: L^T d = y
    R d2 = y2 * i22;
    R d1 = (y1 - l21 * d2) * i11;
    R d0 = (y0 - l10 * d1 - l20 * d2) * i00;
    d = {d0, d1, d2};
    return true;
}

// Deformation gradient of a visit from edge vectors.  The visit record of
// vertex i in tet e stores M = rows (dN_b, dN_c, dN_d) of the other three
// vertices; since the four shape-function gradients sum to zero,
// F = sum_j x_j dN_j^T = sum_{j != i} (x_j - x_i) dN_j^T, i.e. column k of F
// is e1 m0[k] + e2 m1[k] + e3 m2[k].
template <class R>
struct Cols {
    V3<R> c0, c1, c2;
};

template <class R>
__device__ __forceinline__ Cols<R> edge_F(V3<R> e1, V3<R> e2, V3<R> e3, const R* m)
{
    Cols<R> F;
    F.c0 = comb(e1, m[0], e2, m[3], e3, m[6]);
    F.c1 = comb(e1, m[1], e2, m[4], e3, m[7]);
    F.c2 = comb(e1, m[2], e2, m[5], e3, m[8]);
    return F;
}

template <class R>
__device__ __forceinline__ Cols<R> cofactor(const Cols<R>& F)
{
    return {cross(F.c1, F.c2), cross(F.c2, F.c0), cross(F.c0, F.c1)};
}

// F a for F given by columns.
template <class R>
__device__ __forceinline__ V3<R> apply(const Cols<R>& F, V3<R> a)
{
    return comb(F.c0, a.x, F.c1, a.y, F.c2, a.z);
}

template <class R>
__device__ __forceinline__ R frob2(const Cols<R>& F)
{
    return dot(F.c0, F.c0) + dot(F.c1, F.c1) + dot(F.c2, F.c2);
}

// ---------------------------------------------------------------------------
// Rotation part of the polar decomposition with det R = +1 (signed SVD
// convention of Irving et al. 2004 / Stomakhin et al. 2012), following the
// structure of McAdams et al. 2011, "Computing the singular value
// decomposition of 3x3 matrices with minimal branching and elementary
// floating point operations": (1) Jacobi eigen-analysis of the symmetric
// F^T F, accumulating V in SO(3); (2) B = F V with columns sorted by
// decreasing norm (a swap is paired with a sign flip so det V stays +1);
// (3) QR of B by three Givens rotations, B = U R with U in SO(3).  The
// diagonal of R holds the signed singular values (the last one takes the
// sign of det F).  Exact Jacobi rotations are used (not the quaternion
// approximations of the paper), with a fixed sweep count in float and a
// converged loop in double.
// ---------------------------------------------------------------------------
template <class R>
struct Polar {
    // rotation R = U V^T, kept factored: U as three Givens (c, s) pairs and V
    // as a full matrix (columns)
    Cols<R> V;
    R g1c, g1s, g2c, g2s, g3c, g3s;
    V3<R> sigma;   // signed singular values
};

template <class R>
__device__ __forceinline__ void jacobi_rot(R& app, R& aqq, R& apq, R& arp, R& arq, V3<R>& vp,
                                           V3<R>& vq)
{
    // Rotation angle from cot(2 theta) = (aqq - app) / (2 apq), written as
    // t = tan(theta) = sgn(d) h / (|d| + sqrt(d^2 + h^2)), d = aqq - app,
    // h = 2 apq: no division by a small apq.  Off-diagonal entries below
    // working precision relative to the diagonal are left alone.
    constexpr bool dbl = sizeof(R) == 8;
    const R rel = dbl ? R(1e-22) : R(1e-12);
    const R tiny = dbl ? R(1e-150) : R(1e-18);
    if (!(abs_(apq) > rel * (abs_(app) + abs_(aqq))) || !(abs_(apq) > tiny)) return;
    const R d = aqq - app, h = R(2) * apq;
    R t = (d >= R(0) ? h : -h) * rcp(abs_(d) + sqrt_(d * d + h * h));
    R c = rsq(R(1) + t * t);
    R s = t * c;
    app -= t * apq;
    aqq += t * apq;
    apq = R(0);
    R nrp = c * arp - s * arq;
    R nrq = s * arp + c * arq;
    arp = nrp;
    arq = nrq;
    V3<R> np = c * vp - s * vq;
    V3<R> nq = s * vp + c * vq;
    vp = np;
    vq = nq;
}

template <class R>
__device__ __forceinline__ void givens(R a, R b, R& c, R& s)
{
    R n2 = a * a + b * b;
    if (n2 > R(0)) {
        R in = rsq(n2);
        c = a * in;
        s = b * in;
    } else {
        c = R(1);
        s = R(0);
    }
}

template <class R>
__device__ __forceinline__ void polar(const Cols<R>& F, Polar<R>& out)
{
    // S = F^T F
    R s00 = dot(F.c0, F.c0), s01 = dot(F.c0, F.c1), s02 = dot(F.c0, F.c2);
    R s11 = dot(F.c1, F.c1), s12 = dot(F.c1, F.c2), s22 = dot(F.c2, F.c2);
    V3<R> v0 = mk<R>(1, 0, 0), v1 = mk<R>(0, 1, 0), v2 = mk<R>(0, 0, 1);
    constexpr bool dbl = sizeof(R) == 8;
    const int max_sweeps = dbl ? 12 : 5;
    // Cyclic sweeps until the off-diagonal part is below working precision
    // relative to the diagonal (|off| <= 3e-7 |diag| in float, 1e-17 in
    // double), tested per lane before every sweep: a converged lane is
    // masked off, so its result does not depend on the other lanes of its
    // wave, and the wave leaves the loop once all of its lanes converged.
    const R tol = dbl ? R(1e-34) : R(1e-13);
    bool act = true;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        const R off = s01 * s01 + s02 * s02 + s12 * s12;
        const R dia = s00 * s00 + s11 * s11 + s22 * s22;
        act = act && !(off <= tol * dia);
        if (!__any(act)) break;
        if (act) {
            // pair (0,1), remaining 2
            jacobi_rot(s00, s11, s01, s02, s12, v0, v1);
            // pair (0,2), remaining 1: a_rp = s01 (row 1, col 0), a_rq = s12
            jacobi_rot(s00, s22, s02, s01, s12, v0, v2);
            // pair (1,2), remaining 0
            jacobi_rot(s11, s22, s12, s01, s02, v1, v2);
        }
    }
    // B = F V, sorted by decreasing column norm
    V3<R> b0 = apply(F, v0), b1 = apply(F, v1), b2 = apply(F, v2);
    R n0 = dot(b0, b0), n1 = dot(b1, b1), n2 = dot(b2, b2);
    if (n0 < n1) {
        V3<R> t = b0; b0 = b1; b1 = R(-1) * t;
        t = v0; v0 = v1; v1 = R(-1) * t;
        R tn = n0; n0 = n1; n1 = tn;
    }
    if (n0 < n2) {
        V3<R> t = b0; b0 = b2; b2 = R(-1) * t;
        t = v0; v0 = v2; v2 = R(-1) * t;
        R tn = n0; n0 = n2; n2 = tn;
    }
    if (n1 < n2) {
        V3<R> t = b1; b1 = b2; b2 = R(-1) * t;
        t = v1; v1 = v2; v2 = R(-1) * t;
    }
    // QR by Givens on rows: zero (1,0), then (2,0), then (2,1).  Row r of B
    // is (b0[r], b1[r], b2[r]).
    R r0[3] = {b0.x, b1.x, b2.x}, r1[3] = {b0.y, b1.y, b2.y}, r2[3] = {b0.z, b1.z, b2.z};
    R c, s;
    givens(r0[0], r1[0], c, s);
    out.g1c = c; out.g1s = s;
    for (int k = 0; k < 3; ++k) {
        R a = r0[k], b = r1[k];
        r0[k] = c * a + s * b;
        r1[k] = -s * a + c * b;
    }
    givens(r0[0], r2[0], c, s);
    out.g2c = c; out.g2s = s;
    for (int k = 0; k < 3; ++k) {
        R a = r0[k], b = r2[k];
        r0[k] = c * a + s * b;
        r2[k] = -s * a + c * b;
    }
    givens(r1[1], r2[1], c, s);
    out.g3c = c; out.g3s = s;
    for (int k = 1; k < 3; ++k) {
        R a = r1[k], b = r2[k];
        r1[k] = c * a + s * b;
        r2[k] = -s * a + c * b;
    }
    out.sigma = mk(r0[0], r1[1], r2[2]);
    out.V.c0 = v0; out.V.c1 = v1; out.V.c2 = v2;
}

// R a = U (V^T a); U = G1^T G2^T G3^T applied right to left.
template <class R>
__device__ __forceinline__ V3<R> polar_apply(const Polar<R>& P, V3<R> a)
{
    R w0 = dot(P.V.c0, a), w1 = dot(P.V.c1, a), w2 = dot(P.V.c2, a);
    // G3^T on (1,2)
    R t1 = P.g3c * w1 - P.g3s * w2;
    R t2 = P.g3s * w1 + P.g3c * w2;
    w1 = t1; w2 = t2;
    // G2^T on (0,2)
    R t0 = P.g2c * w0 - P.g2s * w2;
    t2 = P.g2s * w0 + P.g2c * w2;
    w0 = t0; w2 = t2;
    // G1^T on (0,1)
    t0 = P.g1c * w0 - P.g1s * w1;
    t1 = P.g1s * w0 + P.g1c * w1;
    return mk(t0, t1, w2);
}

// Columns of the rotation R = U V^T (for the FP64 stress evaluation).
template <class R>
__device__ __forceinline__ Cols<R> polar_matrix(const Polar<R>& P)
{
    return {polar_apply(P, mk<R>(1, 0, 0)), polar_apply(P, mk<R>(0, 1, 0)),
            polar_apply(P, mk<R>(0, 0, 1))};
}

// Rotation of the polar decomposition by the scaled Newton iteration
// X <- (zeta X + (zeta X)^{-T}) / 2 with the Frobenius-norm scaling
// zeta = (|X^{-1}|_F / |X|_F)^{1/2} (Higham 1986, "Computing the polar
// decomposition - with applications").  It converges quadratically to the
// orthogonal polar factor, which for det F > 0 is the rotation of the signed
// convention above.  Once the iteration is in its quadratic regime the error
// left after a step is about half the square of that step's change, so a
// change below 3e-5 (float) or 1e-9 (double) in Frobenius norm ends it.
// Returns false when det F <= 0 (inverted or degenerate) or the iteration
// has not converged within its budget; the caller then takes the Jacobi/QR
// path.  Converged lanes are masked off, so a lane's result does not depend
// on the other lanes of its wave.
template <class R>
__device__ __forceinline__ bool polar_newton(const Cols<R>& F, Cols<R>& X)
{
    constexpr bool dbl = sizeof(R) == 8;
    const int iters = dbl ? 12 : 8;
    const R tol = dbl ? R(1e-18) : R(1e-9);
    const R tiny = dbl ? R(1e-200) : R(1e-30);
    X = F;
    bool act = true, ok = false;
    R dprev = R(1);
    for (int it = 0; it < iters; ++it) {
        if (!__any(act)) break;
        if (act) {
            const Cols<R> C = cofactor(X);
            const R det = dot(X.c0, C.c0);
            if (!(det > tiny)) {
                act = false;
            } else {
                // Frobenius scaling speeds up the first steps; once a step
                // changed X by less than 1e-2 the unscaled iteration is
                // already in its quadratic regime (Higham 1986), and the
                // scale factor's norms and roots are skipped.
                R zeta = R(1);
                if (dprev > R(1e-4)) {
                    const R q = sqrt_(frob2(C) * rcp(frob2(X)));   // |X^{-1}|_F det / |X|_F
                    zeta = sqrt_(q * rcp(det));
                }
                const R a = R(0.5) * zeta, b = R(0.5) * rcp(zeta * det);
                Cols<R> Y;
                Y.c0 = a * X.c0 + b * C.c0;
                Y.c1 = a * X.c1 + b * C.c1;
                Y.c2 = a * X.c2 + b * C.c2;
                const V3<R> d0 = Y.c0 - X.c0, d1 = Y.c1 - X.c1, d2 = Y.c2 - X.c2;
                const R d = dot(d0, d0) + dot(d1, d1) + dot(d2, d2);
                dprev = d;
                X = Y;
                if (d <= tol) {
                    act = false;
                    ok = true;
                }
            }
        }
    }
    return ok;
}

// Rotation R(F) with det R = +1: Newton where it applies, else Jacobi/QR.
template <class R>
__device__ __forceinline__ Cols<R> rotation_of(const Cols<R>& F)
{
    Cols<R> X;
    if (!polar_newton(F, X)) {
        Polar<R> pol;
        polar(F, pol);
        X = polar_matrix(pol);
    }
    return X;
}

}  // namespace pbng
