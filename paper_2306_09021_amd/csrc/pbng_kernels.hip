// HIP kernels of libpbng for gfx950 (MI355X).
//
// Hot path: one launch per colour phase.  A group of LANES lanes of a
// 64-wide wavefront owns one free vertex; lane l takes the vertex's visits
// l, l + LANES, ...  Per visit it forms F from the three gathered
// neighbour positions, the stress contribution V0 P(F) dN_i to the local
// gradient and the modified-Hessian contribution
//   V0 (2 mu |dN_i|^2 I + lambda (cof F dN_i)(cof F dN_i)^T)
// (Eq. mod_hess), then the group sums its partial results with a butterfly
// of cross-lane shuffles (every lane ends with the same bits), solves the
// SPD 3x3 system by Cholesky and takes the single modified-Newton step of
// Eq. pbgn_dx.  All work is FP32 (or FP64) vector ALU work on gathered
// data; there is no dense contraction to put on the matrix cores.
#include "pbng_device.hpp"
#include "pbng_internal.hpp"
#include "pbng_math.hpp"

#ifndef PBNG_KERNEL_SET
#define PBNG_KERNEL_SET 0
#endif

namespace pbng {

constexpr int kNeo = 0;
constexpr int kCor = 1;
constexpr int kSnh = 2;
// Neo-Hookean with one (mu, lambda) per instance: the 40-byte record form
// (internal model id; the public model is Neo-Hookean)
constexpr int kNeoU = 3;
template <int M>
constexpr bool is_nh = M == kNeo || M == kNeoU;
constexpr int kBlock = 256;

template <int LANES, class R>
__device__ __forceinline__ void lsum3(V3<R>& v)
{
    v.x = lsum<LANES>(v.x);
    v.y = lsum<LANES>(v.y);
    v.z = lsum<LANES>(v.z);
}

template <int LANES, class R>
__device__ __forceinline__ void lsum6(Sym<R>& s)
{
    s.xx = lsum<LANES>(s.xx);
    s.xy = lsum<LANES>(s.xy);
    s.xz = lsum<LANES>(s.xz);
    s.yy = lsum<LANES>(s.yy);
    s.yz = lsum<LANES>(s.yz);
    s.zz = lsum<LANES>(s.zz);
}

template <class P4>
__device__ __forceinline__ auto xyz(P4 p)
{
    using R = decltype(p.x);
    return V3<R>{p.x, p.y, p.z};
}

template <class R>
__device__ __forceinline__ typename R4t<R>::T pack4(V3<R> v)
{
    return typename R4t<R>::T{v.x, v.y, v.z, R(0)};
}

template <class R>
__device__ __forceinline__ Sym<R> sym_zero()
{
    return Sym<R>{R(0), R(0), R(0), R(0), R(0), R(0)};
}

template <class R>
__device__ __forceinline__ void sym_acc(Sym<R>& A, const Sym<R>& B)
{
    A.xx += B.xx; A.xy += B.xy; A.xz += B.xz; A.yy += B.yy; A.yz += B.yz; A.zz += B.zz;
}

template <class R>
__device__ __forceinline__ void sym_add_scaled(Sym<R>& A, R w, const R* K)
{
    A.xx += w * K[0]; A.xy += w * K[1]; A.xz += w * K[2];
    A.yy += w * K[3]; A.yz += w * K[4]; A.zz += w * K[5];
}

template <class R>
__device__ __forceinline__ V3<R> symK_mul(const R* K, V3<R> v)
{
    return {K[0] * v.x + K[1] * v.y + K[2] * v.z, K[1] * v.x + K[3] * v.y + K[4] * v.z,
            K[2] * v.x + K[4] * v.y + K[5] * v.z};
}

template <class T, class S>
__device__ __forceinline__ V3<T> cvt(V3<S> v)
{
    return V3<T>{T(v.x), T(v.y), T(v.z)};
}

// Edge vector x_j - x_i formed in the position precision PR, then rounded to
// the arithmetic precision R (with FP64 positions and FP32 arithmetic the
// edge keeps FP32 accuracy relative to the element size, not to |x|).
template <class R, class P4, class PR>
__device__ __forceinline__ V3<R> rel(P4 pj, V3<PR> xi)
{
    return cvt<R>(V3<PR>{PR(pj.x) - xi.x, PR(pj.y) - xi.y, PR(pj.z) - xi.z});
}

// Signed distance n . x - d of a position to a plane (n, d, k).
template <class R, class PR>
__device__ __forceinline__ R plane_phi(const R* pl, V3<PR> x)
{
    return R(PR(pl[0]) * x.x + PR(pl[1]) * x.y + PR(pl[2]) * x.z - PR(pl[3]));
}

// Corotated energy density times V0 from the rotation: with F = R S (S
// symmetric, signed singular values sigma), |F - R|^2 = |S - I|^2 =
// sum (sigma_i - 1)^2.
template <class R>
__device__ __forceinline__ R corot_energy(const Cols<R>& F, const Cols<R>& Rm, R J, R vm, R vl)
{
    const V3<R> d0 = F.c0 - Rm.c0, d1 = F.c1 - Rm.c1, d2 = F.c2 - Rm.c2;
    return vm * (dot(d0, d0) + dot(d1, d1) + dot(d2, d2)) + R(0.5) * vl * (J - R(1)) * (J - R(1));
}

// Stable Neo-Hookean energy density times V0 (Eq. snh with the Lame lambda
// on the volume term): with vm = V0 mu, vl = V0 lambda,
// 1/2 vm (|F|^2 - 3) + 1/2 vl (J - alpha)^2 - 1/2 vm log(1 + |F|^2),
// alpha = 1 + 3 mu / (4 lambda), i.e. vl (J - alpha) = vl (J - 1) - 3/4 vm.
template <class R>
__device__ __forceinline__ R snh_energy(const Cols<R>& F, R J, R vm, R vl)
{
    const R ic = frob2(F);
    const R q = vl * (J - R(1)) - R(0.75) * vm;
    return R(0.5) * vm * (ic - R(3)) + R(0.5) * q * q / vl - R(0.5) * vm * log(R(1) + ic);
}

// Stress differential dP[L] (the true Hessian density of Eq. hess applied
// to L) for the corotated and stable Neo-Hookean models, with (m, l) =
// (mu, lambda) or (V0 mu, V0 lambda), C = cof F, J = det F:
//   dcof[L] columns: L_1 x F_2 + F_1 x L_2, L_2 x F_0 + F_2 x L_0, L_0 x F_1 + F_0 x L_1
//   stable NH: m (1 - 1/(1+|F|^2)) L + 2 m (F:L)/(1+|F|^2)^2 F + l (C:L) C
//              + (l (J - 1) - 3/4 m) dcof[L]
//   corotated: 2 m (L - dR) + l (C:L) C + l (J - 1) dcof[L], with F = R S,
//              dR = R [w]x and ((tr S) I - S) w = axial(R^T L - L^T R).
template <class R, int MODEL>
__device__ __forceinline__ Cols<R> stress_diff(const Cols<R>& F, const Cols<R>& C, R J,
                                               const Cols<R>& L, R m, R l)
{
    const R cofL = dot(C.c0, L.c0) + dot(C.c1, L.c1) + dot(C.c2, L.c2);
    const V3<R> d0 = cross(L.c1, F.c2) + cross(F.c1, L.c2);
    const V3<R> d1 = cross(L.c2, F.c0) + cross(F.c2, L.c0);
    const V3<R> d2 = cross(L.c0, F.c1) + cross(F.c0, L.c1);
    const R lc = l * cofL;
    Cols<R> out;
    if constexpr (MODEL == kSnh) {
        const R den = R(1) + frob2(F);
        const R a = m * (R(1) - rcp(den));
        const R b = R(2) * m * (dot(F.c0, L.c0) + dot(F.c1, L.c1) + dot(F.c2, L.c2)) * rcp(den * den);
        const R q = l * (J - R(1)) - R(0.75) * m;
        out.c0 = a * L.c0 + b * F.c0 + lc * C.c0 + q * d0;
        out.c1 = a * L.c1 + b * F.c1 + lc * C.c1 + q * d1;
        out.c2 = a * L.c2 + b * F.c2 + lc * C.c2 + q * d2;
    } else {
        const Cols<R> Rm = rotation_of(F);
        // S = R^T F and R^T L (entry (i, j) = R_i . X_j for columns R_i, X_j)
        const R s00 = dot(Rm.c0, F.c0), s11 = dot(Rm.c1, F.c1), s22 = dot(Rm.c2, F.c2);
        const R s01 = R(0.5) * (dot(Rm.c0, F.c1) + dot(Rm.c1, F.c0));
        const R s02 = R(0.5) * (dot(Rm.c0, F.c2) + dot(Rm.c2, F.c0));
        const R s12 = R(0.5) * (dot(Rm.c1, F.c2) + dot(Rm.c2, F.c1));
        const V3<R> w = mk(dot(Rm.c2, L.c1) - dot(Rm.c1, L.c2), dot(Rm.c0, L.c2) - dot(Rm.c2, L.c0),
                           dot(Rm.c1, L.c0) - dot(Rm.c0, L.c1));
        const R tr = s00 + s11 + s22;
        // M = (tr S) I - S (symmetric): w_rot = cof(M) w / det M
        const R m00 = tr - s00, m11 = tr - s11, m22 = tr - s22;
        const R k00 = m11 * m22 - s12 * s12, k11 = m00 * m22 - s02 * s02, k22 = m00 * m11 - s01 * s01;
        const R k01 = s01 * m22 + s12 * s02;   // cofactors of M = [[m00,-s01,-s02],...]
        const R k02 = s01 * s12 + s02 * m11;
        const R k12 = m00 * s12 + s01 * s02;
        const R det = m00 * k00 - s01 * k01 - s02 * k02;
        const R id = rcp(det);
        const V3<R> om = id * mk(k00 * w.x + k01 * w.y + k02 * w.z, k01 * w.x + k11 * w.y + k12 * w.z,
                                 k02 * w.x + k12 * w.y + k22 * w.z);
        // dR = R [om]x: column j of [om]x is om x e_j
        const V3<R> dr0 = om.z * Rm.c1 - om.y * Rm.c2;   // R (0, om_z, -om_y)
        const V3<R> dr1 = om.x * Rm.c2 - om.z * Rm.c0;   // R (-om_z, 0, om_x)
        const V3<R> dr2 = om.y * Rm.c0 - om.x * Rm.c1;   // R (om_y, -om_x, 0)
        const R q = l * (J - R(1));
        out.c0 = (R(2) * m) * (L.c0 - dr0) + lc * C.c0 + q * d0;
        out.c1 = (R(2) * m) * (L.c1 - dr1) + lc * C.c1 + q * d1;
        out.c2 = (R(2) * m) * (L.c2 - dr2) + lc * C.c2 + q * d2;
    }
    return out;
}

// Raw record of one visit (loaded before any arithmetic so that the loads of
// several visits are in flight together).
//
// Corotated workspaces keep the three shape-function gradient rows m[9]: the
// polar decomposition needs F itself.  Neo-Hookean workspaces keep only what
// the step needs.  With D = [e1 e2 e3] the edge vectors x_j - x_i and M the
// matrix of rows m_1, m_2, m_3, F = D M, so
//   F dN_i     = sum_a alpha_a e_a,            alpha_a = m_a . dN_i
//   cof F dN_i = cof D (cof M dN_i) = sum_k beta_k X_k,
//                X_1 = e2 x e3, X_2 = e3 x e1, X_3 = e1 x e2,  beta = cof M dN_i
//   J = det F  = delta (e1 . X_1),              delta = det M
// and the record holds a = V0 mu alpha, V0 lambda, beta and delta.  Where
// every tet of an instance has the same (mu, lambda), |delta| = 1 / (6 V0)
// gives V0, so the record shrinks to V0 alpha, beta and delta (40 bytes in
// FP32) and V0 mu, V0 lambda come from the instance's parameters.
template <class R>
struct VisitRaw {
    int i1, i2, i3;
    R m[9];
    R vm, vl;
};

template <class R>
struct VisitNH {
    int i1, i2, i3;
    R vm, vl, delta;
    V3<R> a, beta;
};

template <class R>
__device__ __forceinline__ R vm_of(int4 j, const R* vmu, int k)
{
    if constexpr (sizeof(R) == 4) return __int_as_float(j.w);
    else return at(vmu, k);
}

template <class R, class A>
__device__ __forceinline__ VisitRaw<R> load_raw(const A& a, int k)
{
    VisitRaw<R> r;
    const int4 j = at(a.jv, k);
    const auto p = at(a.ma, k);
    const auto q = at(a.mb, k);
    const auto t = at(a.mc, k);
    r.i1 = j.x;
    r.i2 = j.y;
    r.i3 = j.z;
    r.m[0] = p.x; r.m[1] = p.y; r.m[2] = p.z; r.m[3] = p.w;
    r.m[4] = q.x; r.m[5] = q.y; r.m[6] = q.z; r.m[7] = q.w;
    r.m[8] = t.x;
    r.vl = t.y;
    r.vm = vm_of<R>(j, a.vmu, k);
    return r;
}

// Neo-Hookean record k; mu, lam are the instance's parameters (used by the
// 40-byte form only).
template <class R, int MODEL, class A>
__device__ __forceinline__ VisitNH<R> load_nh(const A& a, int k, R mu, R lam)
{
    VisitNH<R> r;
    const int4 j = at(a.jv, k);
    const auto p = at(a.ma, k);
    r.i1 = j.x;
    r.i2 = j.y;
    r.i3 = j.z;
    if constexpr (MODEL == kNeoU) {
        // jv.w (FP32) or vmu (FP64) = delta; ma = (V0 alpha, beta_1); mc = (beta_2, beta_3)
        const auto t = at(a.mc, k);
        const R delta = vm_of<R>(j, a.vmu, k);
        const R V0 = rcp(R(6) * abs_(delta));
        r.delta = delta;
        r.vm = mu * V0;
        r.vl = lam * V0;
        r.a = mu * mk(p.x, p.y, p.z);
        r.beta = mk(p.w, t.x, t.y);
    } else {
        const auto q = at(a.mb, k);
        r.a = mk(p.x, p.y, p.z);
        r.vl = p.w;
        r.beta = mk(q.x, q.y, q.z);
        r.delta = q.w;
        r.vm = vm_of<R>(j, a.vmu, k);
    }
    return r;
}

// Visit k of vertex at xi (corotated records): deformation gradient, own
// gradient a = dN_i, V0 mu, V0 lambda.
template <class R, class A, class PR>
__device__ __forceinline__ void load_visit(const A& a, int k, V3<PR> xi, Cols<R>& F, V3<R>& av,
                                           R& vm, R& vl)
{
    const VisitRaw<R> r = load_raw<R>(a, k);
    vm = r.vm;
    vl = r.vl;
    const V3<R> e1 = rel<R>(at(a.W, r.i1), xi);
    const V3<R> e2 = rel<R>(at(a.W, r.i2), xi);
    const V3<R> e3 = rel<R>(at(a.W, r.i3), xi);
    F = edge_F(e1, e2, e3, r.m);
    av = mk(-(r.m[0] + r.m[3] + r.m[6]), -(r.m[1] + r.m[4] + r.m[7]), -(r.m[2] + r.m[5] + r.m[8]));
}

// Per-vertex accumulators of the local gradient and Hessian pieces.
template <class R>
struct Acc {
    V3<R> g;     // elastic + weak-constraint gradient
    Sym<R> Aw;   // sum V0 lambda c c^T + sum s^2 K
    Sym<R> Cm;   // Neo-Hookean safeguard: sum V0 mu c c^T
    V3<R> gw;    // corotated / stable NH safeguard: quadratic (weak, inertia) part of g
    Sym<R> Kw;   // corotated / stable NH safeguard: its Hessian
    R E0, E0a;   // corotated / stable NH safeguard: elastic energy and sum of |terms|
};

// Neo-Hookean visit: V0 P dN_i with P = mu F + (lhat (J - 1) - mu) cof F,
// lhat = mu + lambda, and the V0 lambda c c^T part of the modified Hessian.
template <class R, bool SAFE>
__device__ __forceinline__ void visit_nh(Acc<R>& q, const VisitNH<R>& r, V3<R> e1, V3<R> e2, V3<R> e3)
{
    const V3<R> X1 = cross(e2, e3), X2 = cross(e3, e1), X3 = cross(e1, e2);
    const R J = r.delta * dot(e1, X1);
    const V3<R> c = comb(X1, r.beta.x, X2, r.beta.y, X3, r.beta.z);  // cof F dN_i
    const V3<R> p = comb(e1, r.a.x, e2, r.a.y, e3, r.a.z);           // V0 mu F dN_i
    sym_add_outer(q.Aw, r.vl, c);
    q.g = q.g + p + ((r.vm + r.vl) * (J - R(1)) - r.vm) * c;
    if (SAFE) sym_add_outer(q.Cm, r.vm, c);
}

// Corotated visit: V0 P dN_i with P = 2 mu (F - R) + lambda (J - 1) cof F.
template <class R, bool SAFE>
__device__ __forceinline__ void visit_cor(Acc<R>& q, const VisitRaw<R>& r, V3<R> e1, V3<R> e2, V3<R> e3)
{
    const Cols<R> F = edge_F(e1, e2, e3, r.m);
    const V3<R> av = mk(-(r.m[0] + r.m[3] + r.m[6]), -(r.m[1] + r.m[4] + r.m[7]),
                        -(r.m[2] + r.m[5] + r.m[8]));
    const Cols<R> C = cofactor(F);
    const R J = dot(F.c0, C.c0);
    const V3<R> c = apply(C, av);   // cof(F) dN_i
    const V3<R> p = apply(F, av);   // F dN_i
    const R vm = r.vm, vl = r.vl;
    sym_add_outer(q.Aw, vl, c);
    const Cols<R> Rm = rotation_of(F);
    const V3<R> ra = apply(Rm, av);
    q.g = q.g + (R(2) * vm) * (p - ra) + (vl * (J - R(1))) * c;
    if (SAFE) {
        const R e = corot_energy(F, Rm, J, vm, vl);
        q.E0 += e;
        q.E0a += abs_(e);
    }
}

// Stable Neo-Hookean visit: V0 P dN_i with
// P = mu (1 - 1/(1 + |F|^2)) F + (lambda (J - 1) - 3/4 mu) cof F.
template <class R, bool SAFE>
__device__ __forceinline__ void visit_snh(Acc<R>& q, const VisitRaw<R>& r, V3<R> e1, V3<R> e2, V3<R> e3)
{
    const Cols<R> F = edge_F(e1, e2, e3, r.m);
    const V3<R> av = mk(-(r.m[0] + r.m[3] + r.m[6]), -(r.m[1] + r.m[4] + r.m[7]),
                        -(r.m[2] + r.m[5] + r.m[8]));
    const Cols<R> C = cofactor(F);
    const R J = dot(F.c0, C.c0);
    const V3<R> c = apply(C, av);
    const V3<R> p = apply(F, av);
    const R vm = r.vm, vl = r.vl;
    sym_add_outer(q.Aw, vl, c);
    const R a = vm * (R(1) - rcp(R(1) + frob2(F)));
    q.g = q.g + a * p + (vl * (J - R(1)) - R(0.75) * vm) * c;
    if (SAFE) {
        const R e = snh_energy(F, J, vm, vl);
        q.E0 += e;
        q.E0a += abs_(e);
    }
}

template <class R, int MODEL, bool SAFE>
__device__ __forceinline__ void visit_full(Acc<R>& q, const VisitRaw<R>& r, V3<R> e1, V3<R> e2, V3<R> e3)
{
    if constexpr (MODEL == kSnh) visit_snh<R, SAFE>(q, r, e1, e2, e3);
    else visit_cor<R, SAFE>(q, r, e1, e2, e3);
}

// Visits of one lane: two per pass while any lane of the wave still has two,
// else one; the branch conditions are uniform over the wave, and lanes with
// fewer visits sit a visit out under the execution mask.  A lane without a
// second visit loads its first one twice and skips the second accumulation.
template <class R, int MODEL, bool SAFE, int LANES, class A, class PR>
__device__ __forceinline__ void lane_visits(const A& a, Acc<R>& q, int kb, int ke, int lane, V3<PR> xi,
                                            R imu, R ilam)
{
    for (int k = kb + lane; __any(k < ke); k += 2 * LANES) {
        const bool h0 = k < ke;
        const bool h1 = k + LANES < ke;
        const int k1 = h1 ? k + LANES : k;
        if constexpr (is_nh<MODEL>) {
            if (__any(h1)) {
                if (h0) {
                    const VisitNH<R> r0 = load_nh<R, MODEL>(a, k, imu, ilam);
                    const VisitNH<R> r1 = load_nh<R, MODEL>(a, k1, imu, ilam);
                    const auto p01 = at(a.W, r0.i1), p02 = at(a.W, r0.i2), p03 = at(a.W, r0.i3);
                    const auto p11 = at(a.W, r1.i1), p12 = at(a.W, r1.i2), p13 = at(a.W, r1.i3);
                    visit_nh<R, SAFE>(q, r0, rel<R>(p01, xi), rel<R>(p02, xi), rel<R>(p03, xi));
                    if (h1) visit_nh<R, SAFE>(q, r1, rel<R>(p11, xi), rel<R>(p12, xi), rel<R>(p13, xi));
                }
            } else if (h0) {
                const VisitNH<R> r0 = load_nh<R, MODEL>(a, k, imu, ilam);
                visit_nh<R, SAFE>(q, r0, rel<R>(at(a.W, r0.i1), xi), rel<R>(at(a.W, r0.i2), xi),
                                  rel<R>(at(a.W, r0.i3), xi));
            }
        } else {
            if (__any(h1)) {
                if (h0) {
                    const VisitRaw<R> r0 = load_raw<R>(a, k);
                    const VisitRaw<R> r1 = load_raw<R>(a, k1);
                    const auto p01 = at(a.W, r0.i1), p02 = at(a.W, r0.i2), p03 = at(a.W, r0.i3);
                    const auto p11 = at(a.W, r1.i1), p12 = at(a.W, r1.i2), p13 = at(a.W, r1.i3);
                    visit_full<R, MODEL, SAFE>(q, r0, rel<R>(p01, xi), rel<R>(p02, xi), rel<R>(p03, xi));
                    if (h1)
                        visit_full<R, MODEL, SAFE>(q, r1, rel<R>(p11, xi), rel<R>(p12, xi), rel<R>(p13, xi));
                }
            } else if (h0) {
                const VisitRaw<R> r0 = load_raw<R>(a, k);
                visit_full<R, MODEL, SAFE>(q, r0, rel<R>(at(a.W, r0.i1), xi), rel<R>(at(a.W, r0.i2), xi),
                                           rel<R>(at(a.W, r0.i3), xi));
            }
        }
    }
}

// GEN = 0: one instance without weak constraints, planes or inertia (no
// per-vertex instance lookup); GEN = 1: batched instances with per-instance
// activity flags, weak constraints, contact planes, recoloured vertices and
// inertia; GEN = 2: one instance whose only extra term is the inertia.
template <class R, class PR, int MODEL, int LANES, bool ACCEL, bool SAFE, int GEN>
__global__ __launch_bounds__(kBlock) void k_phase(SweepArgs<R, PR> a, int vbeg, int vend)
{
    using P4 = typename R4t<PR>::T;
    constexpr bool WC = GEN == 1;
    const int gid = xcd_block() * kBlock + threadIdx.x;
    int v = vbeg + gid / LANES;
    const int lane = gid & (LANES - 1);
    if (v >= vend) return;
    if (GEN == 1) {
        // vertices recoloured after new weak constraints (whole lane groups
        // return together)
        if (a.vlist && v >= a.list_from) v = at(a.vlist, v - a.list_from + a.list_beg);
        else if (a.pcol && at(a.pcol, v) != a.pcolor) return;
    }
    const int kb = at(a.vptr, v), ke = at(a.vptr, v + 1);
    const P4 xw = at(a.W, v);
    int inst = 0;
    if (GEN == 1 && a.vinst) {
        inst = at(a.vinst, v);
        if (!at(a.active, inst)) {
            if (ACCEL && lane == 0) *ptr_at(a.N, v) = xw;
            return;
        }
    }
    const V3<PR> xi = xyz(xw);

    Acc<R> q;
    q.g = mk<R>(0, 0, 0);
    q.Aw = sym_zero<R>();
    q.Cm = sym_zero<R>();
    q.gw = mk<R>(0, 0, 0);
    q.Kw = sym_zero<R>();
    q.E0 = R(0);
    q.E0a = R(0);

    // lane l takes visits kb + l, kb + l + LANES, ...
    R imu = R(0), ilam = R(0);
    if constexpr (MODEL == kNeoU) {
        imu = at(a.imu, inst);
        ilam = at(a.ilam, inst);
    }
    lane_visits<R, MODEL, SAFE, LANES>(a, q, kb, ke, lane, xi, imu, ilam);
    V3<R>& g = q.g;
    const R S = at(a.Sv, v);  // sum V0 mu |dN_i|^2 of the vertex
    Sym<R>& Aw = q.Aw;
    Sym<R>& Cm = q.Cm;
    V3<R>& gw = q.gw;
    Sym<R>& Kw = q.Kw;
    R& E0 = q.E0;
    R& E0a = q.E0a;
    if (WC) {
        for (int k = a.wvptr[v] + lane; k < a.wvptr[v + 1]; k += LANES) {
            const int cc = a.wv_c[k];
            const R s = a.wv_s[k];
            V3<PR> Cp = mk<PR>(0, 0, 0);
            for (int j = a.wc_ptr[cc]; j < a.wc_ptr[cc + 1]; ++j)
                Cp = Cp + PR(a.wc_w[j]) * xyz(a.W[a.wc_vert[j]]);
            const V3<R> Cc = cvt<R>(Cp);
            const R* K = a.wc_K + 6 * cc;
            const V3<R> gk = s * symK_mul(K, Cc);
            g = g + gk;
            sym_add_scaled(Aw, s * s, K);
            if (SAFE && !is_nh<MODEL>) {
                gw = gw + gk;
                sym_add_scaled(Kw, s * s, K);
            }
        }
    }
    if (LANES > 1) {
        lsum3<LANES>(g);
        lsum6<LANES>(Aw);
        if (SAFE && is_nh<MODEL>) lsum6<LANES>(Cm);
        if (SAFE && !is_nh<MODEL>) {
            E0 = lsum<LANES>(E0);
            E0a = lsum<LANES>(E0a);
            if (WC) {
                lsum3<LANES>(gw);
                lsum6<LANES>(Kw);
            }
        }
    }
    if (GEN != 0 && a.inert) {
        // backward-Euler inertia: 1/2 c |y_i - xhat_i|^2, c = m_ii / dt^2,
        // exactly quadratic (so it also joins the safeguard's exact part)
        const R c = at(a.inert, v);
        const V3<R> dx = cvt<R>(xi - xyz(at(a.xhat, v)));
        g = g + c * dx;
        Aw.xx += c;
        Aw.yy += c;
        Aw.zz += c;
        if (SAFE && !is_nh<MODEL>) {
            gw = gw + c * dx;
            Kw.xx += c;
            Kw.yy += c;
            Kw.zz += c;
        }
    }
    const V3<R> f = xyz(at(a.fext, v));
    const V3<R> gt = g - f;
    Sym<R> A = Aw;
    A.xx += R(2) * S;
    A.yy += R(2) * S;
    A.zz += R(2) * S;
    V3<R> gtot = gt;
    int pb = 0, pe = 0;
    if (WC) {
        pb = a.plane_ptr[inst];
        pe = a.plane_ptr[inst + 1];
        for (int q = pb; q < pe; ++q) {
            const R* pl = a.planes + 5 * q;
            const V3<R> n = mk(pl[0], pl[1], pl[2]);
            const R phi = plane_phi(pl, xi);
            if (phi < R(0)) {
                gtot = gtot + (pl[4] * phi) * n;
                sym_add_outer(A, pl[4], n);
            }
        }
    }
    V3<R> d;
    const bool ok = chol_solve(A, R(-1) * gtot, d);
    bool reject = !ok;
    R alpha = R(1);
    if (SAFE && ok) {
        const R u = sizeof(R) == 8 ? R(1.1102230246251565e-16) : R(5.9604644775390625e-08);
        R lin, quad;
        // Corotated: for any rotation Q, mu |F' - R(F')|^2 <= mu |F' - Q|^2
        // (R(F') is the closest rotation), so with Q = R(F) the local energy
        // is majorised by a quadratic in x_i whose gradient is g and whose
        // Hessian is the modified Hessian A (without planes).  The exact
        // evaluation below runs only when this bound does not already show
        // that the step decreases the energy.
        bool bound_ok = false;
        if constexpr (MODEL == kCor) {
            Sym<R> Ab = Aw;
            Ab.xx += R(2) * S;
            Ab.yy += R(2) * S;
            Ab.zz += R(2) * S;
            const R bl = dot(gt, d), bq = dot(d, sym_mul(Ab, d));
            R dE = bl + R(0.5) * bq;
            R ab = abs_(bl) + abs_(R(0.5) * bq);
            if (WC) {
                for (int q2 = pb; q2 < pe; ++q2) {
                    const R* pl = a.planes + 5 * q2;
                    const V3<R> n = mk(pl[0], pl[1], pl[2]);
                    const R phi0 = plane_phi(pl, xi);
                    const R phi1 = phi0 + dot(n, d);
                    const R e0 = phi0 < R(0) ? R(0.5) * pl[4] * phi0 * phi0 : R(0);
                    const R e1 = phi1 < R(0) ? R(0.5) * pl[4] * phi1 * phi1 : R(0);
                    // active planes are inside the quadratic; only the change
                    // of the penalty beyond it counts here
                    const R quad_pl = phi0 < R(0) ? R(0.5) * pl[4] * (phi1 * phi1 - phi0 * phi0) : R(0);
                    dE += (e1 - e0) - quad_pl;
                    ab += e0 + e1 + abs_(quad_pl);
                }
            }
            bound_ok = dE <= R(8) * u * ab;
        }
        if constexpr (is_nh<MODEL>) {
            // Along x_i + alpha d the Neo-Hookean energy of the incident tets
            // is exactly quadratic: |F|^2 is quadratic and det F affine in x_i
            // (a rank-one update), with Hessian sum V0 (mu |dN_i|^2 I + lhat
            // c c^T); weak constraints are quadratic with Hessian s^2 K.
            Sym<R> H = Aw;
            sym_acc(H, Cm);
            H.xx += S;
            H.yy += S;
            H.zz += S;
            lin = dot(gt, d);
            quad = dot(d, sym_mul(H, d));
        } else {
            lin = dot(gw - f, d);
            quad = dot(d, sym_mul(Kw, d));
        }
        int h = 0;
        for (; !bound_ok;) {
            R dE = alpha * lin + R(0.5) * alpha * alpha * quad;
            R ab = abs_(alpha * lin) + abs_(R(0.5) * alpha * alpha * quad);
            if (WC) {
                for (int q = pb; q < pe; ++q) {
                    const R* pl = a.planes + 5 * q;
                    const V3<R> n = mk(pl[0], pl[1], pl[2]);
                    const R phi0 = plane_phi(pl, xi);
                    const R phi1 = phi0 + alpha * dot(n, d);
                    const R e0 = phi0 < R(0) ? R(0.5) * pl[4] * phi0 * phi0 : R(0);
                    const R e1 = phi1 < R(0) ? R(0.5) * pl[4] * phi1 * phi1 : R(0);
                    dE += e1 - e0;
                    ab += e0 + e1;
                }
            }
            if constexpr (!is_nh<MODEL>) {
                // exact elastic energy of the incident tets at the trial point
                R E1 = R(0), E1a = R(0);
                for (int k = kb + lane; k < ke; k += LANES) {
                    Cols<R> F;
                    V3<R> av;
                    R vm, vl;
                    load_visit(a, k, xi, F, av, vm, vl);
                    const V3<R> ad = alpha * d;
                    F.c0 = F.c0 + av.x * ad;
                    F.c1 = F.c1 + av.y * ad;
                    F.c2 = F.c2 + av.z * ad;
                    const R J1 = dot(F.c0, cross(F.c1, F.c2));
                    R e;
                    if constexpr (MODEL == kCor) e = corot_energy(F, rotation_of(F), J1, vm, vl);
                    else e = snh_energy(F, J1, vm, vl);
                    E1 += e;
                    E1a += abs_(e);
                }
                if (LANES > 1) {
                    E1 = lsum<LANES>(E1);
                    E1a = lsum<LANES>(E1a);
                }
                dE += E1 - E0;
                ab += E0a + E1a;
            }
            if (dE <= R(8) * u * ab) break;
            if (h >= a.max_halvings) {
                reject = true;
                break;
            }
            alpha *= R(0.5);
            ++h;
        }
    }
    const V3<PR> xn = reject ? xi : xi + cvt<PR>(alpha * d);
    if (lane == 0) {
        if (reject) atomicAdd(ptr_at(a.rejected, inst), 1);
        if (ACCEL) {
            const V3<PR> xp = xyz(at(a.P, v));
            const V3<PR> b = a.omega * (a.gamma * (xn - xi) + xi - xp) + xp;
            *ptr_at(a.W, v) = pack4(xn);
            *ptr_at(a.P, v) = xw;
            *ptr_at(a.N, v) = pack4(b);
        } else {
            *ptr_at(a.W, v) = pack4(xn);
        }
    }
}

template <class R, class PR, int MODEL, int LANES, bool ACCEL, bool SAFE, int GEN>
static hipError_t launch_phase_t(const SweepArgs<R, PR>& a, int vbeg, int vend, hipStream_t s)
{
    const int64_t threads = int64_t(vend - vbeg) * LANES;
    if (threads <= 0) return hipSuccess;
    const int blocks = int((threads + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_phase<R, PR, MODEL, LANES, ACCEL, SAFE, GEN>), dim3(blocks), dim3(kBlock), 0,
                       s, a, vbeg, vend);
    return hipGetLastError();
}

template <class R, class PR, int MODEL, int LANES, int GEN>
static hipError_t dispatch_as(const SweepArgs<R, PR>& a, bool accel, bool safe, int vb, int ve, hipStream_t s)
{
    const int code = (accel ? 2 : 0) | (safe ? 1 : 0);
    switch (code) {
    case 0: return launch_phase_t<R, PR, MODEL, LANES, false, false, GEN>(a, vb, ve, s);
    case 1: return launch_phase_t<R, PR, MODEL, LANES, false, true, GEN>(a, vb, ve, s);
    case 2: return launch_phase_t<R, PR, MODEL, LANES, true, false, GEN>(a, vb, ve, s);
    default: return launch_phase_t<R, PR, MODEL, LANES, true, true, GEN>(a, vb, ve, s);
    }
}

template <class R, class PR, int MODEL, int LANES>
static hipError_t dispatch_flags(const SweepArgs<R, PR>& a, bool accel, bool safe, int mode, int vb,
                                 int ve, hipStream_t s)
{
    switch (mode) {
    case 0: return dispatch_as<R, PR, MODEL, LANES, 0>(a, accel, safe, vb, ve, s);
    case 1: return dispatch_as<R, PR, MODEL, LANES, 1>(a, accel, safe, vb, ve, s);
    case 2: return dispatch_as<R, PR, MODEL, LANES, 2>(a, accel, safe, vb, ve, s);
    default: return hipErrorInvalidValue;
    }
}

template <class R, class PR, int MODEL>
static hipError_t dispatch_lanes(const SweepArgs<R, PR>& a, int lanes, bool accel, bool safe,
                                 int mode, int vb, int ve, hipStream_t s)
{
    switch (lanes) {
    case 1: return dispatch_flags<R, PR, MODEL, 1>(a, accel, safe, mode, vb, ve, s);
    case 2: return dispatch_flags<R, PR, MODEL, 2>(a, accel, safe, mode, vb, ve, s);
    case 4: return dispatch_flags<R, PR, MODEL, 4>(a, accel, safe, mode, vb, ve, s);
    case 8: return dispatch_flags<R, PR, MODEL, 8>(a, accel, safe, mode, vb, ve, s);
    case 16: return dispatch_flags<R, PR, MODEL, 16>(a, accel, safe, mode, vb, ve, s);
    case 32: return dispatch_flags<R, PR, MODEL, 32>(a, accel, safe, mode, vb, ve, s);
    case 64: return dispatch_flags<R, PR, MODEL, 64>(a, accel, safe, mode, vb, ve, s);
    default: return hipErrorInvalidValue;
    }
}

template <class R, class PR>
hipError_t launch_phase(const SweepArgs<R, PR>& a, int model, int lanes, bool accel, bool safe,
                        int mode, int vbeg, int vend, hipStream_t s)
{
    if (model == kNeo) return dispatch_lanes<R, PR, kNeo>(a, lanes, accel, safe, mode, vbeg, vend, s);
    if (model == kNeoU) return dispatch_lanes<R, PR, kNeoU>(a, lanes, accel, safe, mode, vbeg, vend, s);
    if (model == kSnh) return dispatch_lanes<R, PR, kSnh>(a, lanes, accel, safe, mode, vbeg, vend, s);
    return dispatch_lanes<R, PR, kCor>(a, lanes, accel, safe, mode, vbeg, vend, s);
}

// ---------------------------------------------------------------------------
// Adjoint: block Gauss-Seidel on the true Hessian H lam = b (Neo-Hookean).
// (H lam)_i = sum_e V0 dP_e[Lam_e] dN_i + weak + active planes with
// Lam_e = sum_j lam_j dN_j^T and, for the Neo-Hookean P = mu F + (lhat (J-1)
// - mu) cof F,
//   dP[L] = mu L + lhat (cof F : L) cof F + (lhat (J-1) - mu) dcof[L],
//   dcof[L][:,k] = L[:,k+1] x F[:,k+2] + F[:,k+1] x L[:,k+2].
// The diagonal block is H_ii = sum_e V0 (mu |dN_i|^2 I + lhat c c^T) + weak
// + planes, c = cof F dN_i (along x_i alone the Neo-Hookean energy is
// exactly quadratic).  Each update: lam_i += H_ii^{-1} (b_i - (H lam)_i).
// The corotated and stable Neo-Hookean models take dP[L] from stress_diff
// and use the modified block A_ii = sum V0 (2 mu |dN_i|^2 I + lambda c c^T)
// in place of H_ii: A_ii bounds H_ii from above (for the corotated model A
// is the Hessian of a majoriser), so 2 A_ii - H_ii is positive definite and
// the block Gauss-Seidel iteration converges wherever H is.
// ---------------------------------------------------------------------------
template <class R, class PR, int MODEL, int LANES, bool ACCEL, bool WC>
__global__ __launch_bounds__(kBlock) void k_adj_phase(AdjArgs<R, PR> a, int vbeg, int vend)
{
    using P4 = typename R4t<PR>::T;
    const int gid = xcd_block() * kBlock + threadIdx.x;
    int v = vbeg + gid / LANES;
    const int lane = gid & (LANES - 1);
    if (v >= vend) return;
    if (WC) {
        if (a.vlist && v >= a.list_from) v = at(a.vlist, v - a.list_from + a.list_beg);
        else if (a.pcol && at(a.pcol, v) != a.pcolor) return;
    }
    const V3<PR> xi = xyz(at(a.X, v));
    const P4 lw = at(a.L, v);
    const V3<PR> li = xyz(lw);
    V3<R> r = mk<R>(0, 0, 0);
    Sym<R> Hc = sym_zero<R>();
    const int kb = at(a.vptr, v), ke = at(a.vptr, v + 1);
    // Per visit with the Neo-Hookean record (e_a, l_a edge vectors of x and
    // lambda, X_k = cof D columns): Lam dN_i = sum alpha_a l_a,
    // cof F : Lam = delta sum_k X_k . l_k and dcof[Lam] dN_i =
    // sum_k beta_k (derivative of X_k along l).
    R imu = R(0), ilam = R(0);
    if constexpr (MODEL == kNeoU) {
        const int q0 = at(a.vinst, v);   // batched workspaces need not take the WC path
        imu = at(a.imu, q0);
        ilam = at(a.ilam, q0);
    }
    if constexpr (!is_nh<MODEL>) {
        for (int k = kb + lane; k < ke; k += LANES) {
            const VisitRaw<R> q = load_raw<R>(a, k);
            const Cols<R> F = edge_F(rel<R>(at(a.X, q.i1), xi), rel<R>(at(a.X, q.i2), xi),
                                     rel<R>(at(a.X, q.i3), xi), q.m);
            const Cols<R> Lm = edge_F(rel<R>(at(a.L, q.i1), li), rel<R>(at(a.L, q.i2), li),
                                      rel<R>(at(a.L, q.i3), li), q.m);
            const V3<R> av = mk(-(q.m[0] + q.m[3] + q.m[6]), -(q.m[1] + q.m[4] + q.m[7]),
                                -(q.m[2] + q.m[5] + q.m[8]));
            const Cols<R> C = cofactor(F);
            const R J = dot(F.c0, C.c0);
            r = r + apply(stress_diff<R, MODEL>(F, C, J, Lm, q.vm, q.vl), av);
            sym_add_outer(Hc, q.vl, apply(C, av));
        }
    }
    for (int k = kb + lane; is_nh<MODEL> && k < ke; k += LANES) {
        const VisitNH<R> q = load_nh<R, MODEL>(a, k, imu, ilam);
        const V3<R> e1 = rel<R>(at(a.X, q.i1), xi), e2 = rel<R>(at(a.X, q.i2), xi),
                    e3 = rel<R>(at(a.X, q.i3), xi);
        const V3<R> l1 = rel<R>(at(a.L, q.i1), li), l2 = rel<R>(at(a.L, q.i2), li),
                    l3 = rel<R>(at(a.L, q.i3), li);
        const V3<R> X1 = cross(e2, e3), X2 = cross(e3, e1), X3 = cross(e1, e2);
        const R J = q.delta * dot(e1, X1);
        const V3<R> c = comb(X1, q.beta.x, X2, q.beta.y, X3, q.beta.z);
        const R vm = q.vm, vl = q.vl;
        const R lh = vm + vl;
        const R qq = lh * (J - R(1)) - vm;
        const R cofL = q.delta * (dot(X1, l1) + dot(X2, l2) + dot(X3, l3));
        const V3<R> d1 = cross(l2, e3) + cross(e2, l3);
        const V3<R> d2 = cross(l3, e1) + cross(e3, l1);
        const V3<R> d3 = cross(l1, e2) + cross(e1, l2);
        const V3<R> dca = comb(d1, q.beta.x, d2, q.beta.y, d3, q.beta.z);
        r = r + comb(l1, q.a.x, l2, q.a.y, l3, q.a.z) + (lh * cofL) * c + qq * dca;
        sym_add_outer(Hc, lh, c);
    }
    const R S = at(a.Sv, v);
    int inst = 0;
    if (WC) {
        inst = a.vinst[v];
        for (int k = a.wvptr[v] + lane; k < a.wvptr[v + 1]; k += LANES) {
            const int cc = a.wv_c[k];
            const R s = a.wv_s[k];
            V3<PR> Cl = mk<PR>(0, 0, 0);
            for (int j = a.wc_ptr[cc]; j < a.wc_ptr[cc + 1]; ++j)
                Cl = Cl + PR(a.wc_w[j]) * xyz(a.L[a.wc_vert[j]]);
            const R* K = a.wc_K + 6 * cc;
            r = r + s * symK_mul(K, cvt<R>(Cl));
            sym_add_scaled(Hc, s * s, K);
        }
    }
    if (LANES > 1) {
        lsum3<LANES>(r);
        lsum6<LANES>(Hc);
    }
    if (WC && a.inert) {
        const R c = at(a.inert, v);
        r = r + c * cvt<R>(li);
        Hc.xx += c;
        Hc.yy += c;
        Hc.zz += c;
    }
    const R Sd = is_nh<MODEL> ? S : R(2) * S;
    Hc.xx += Sd;
    Hc.yy += Sd;
    Hc.zz += Sd;
    if (WC) {
        for (int q = a.plane_ptr[inst]; q < a.plane_ptr[inst + 1]; ++q) {
            const R* pl = a.planes + 5 * q;
            const V3<R> n = mk(pl[0], pl[1], pl[2]);
            if (plane_phi(pl, xi) < R(0)) {
                r = r + (pl[4] * dot(n, cvt<R>(li))) * n;
                sym_add_outer(Hc, pl[4], n);
            }
        }
    }
    const V3<R> rho = cvt<R>(xyz(at(a.B, v))) - r;
    V3<R> dl;
    if (!chol_solve(Hc, rho, dl)) dl = mk<R>(0, 0, 0);
    const V3<PR> ln = li + cvt<PR>(dl);
    if (lane == 0) {
        if (ACCEL) {
            const V3<PR> lp = xyz(at(a.P, v));
            const V3<PR> b = a.omega * (a.gamma * (ln - li) + li - lp) + lp;
            *ptr_at(a.L, v) = pack4(ln);
            *ptr_at(a.P, v) = lw;
            *ptr_at(a.N, v) = pack4(b);
        } else {
            *ptr_at(a.L, v) = pack4(ln);
        }
    }
}

template <class R, class PR, int MODEL, int LANES, bool ACCEL, bool WC>
static hipError_t launch_adj_t(const AdjArgs<R, PR>& a, int vb, int ve, hipStream_t s)
{
    const int64_t threads = int64_t(ve - vb) * LANES;
    if (threads <= 0) return hipSuccess;
    const int blocks = int((threads + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_adj_phase<R, PR, MODEL, LANES, ACCEL, WC>), dim3(blocks), dim3(kBlock), 0,
                       s, a, vb, ve);
    return hipGetLastError();
}

template <class R, class PR, int MODEL, int LANES>
static hipError_t adj_flags(const AdjArgs<R, PR>& a, bool accel, bool wc, int vb, int ve,
                            hipStream_t s)
{
    if (accel) {
        return wc ? launch_adj_t<R, PR, MODEL, LANES, true, true>(a, vb, ve, s)
                  : launch_adj_t<R, PR, MODEL, LANES, true, false>(a, vb, ve, s);
    }
    return wc ? launch_adj_t<R, PR, MODEL, LANES, false, true>(a, vb, ve, s)
              : launch_adj_t<R, PR, MODEL, LANES, false, false>(a, vb, ve, s);
}

template <class R, class PR, int MODEL>
static hipError_t adj_lanes(const AdjArgs<R, PR>& a, int lanes, bool accel, bool wc, int vbeg,
                            int vend, hipStream_t s)
{
    switch (lanes) {
    case 1: return adj_flags<R, PR, MODEL, 1>(a, accel, wc, vbeg, vend, s);
    case 2: return adj_flags<R, PR, MODEL, 2>(a, accel, wc, vbeg, vend, s);
    case 4: return adj_flags<R, PR, MODEL, 4>(a, accel, wc, vbeg, vend, s);
    case 8: return adj_flags<R, PR, MODEL, 8>(a, accel, wc, vbeg, vend, s);
    case 16: return adj_flags<R, PR, MODEL, 16>(a, accel, wc, vbeg, vend, s);
    case 32: return adj_flags<R, PR, MODEL, 32>(a, accel, wc, vbeg, vend, s);
    case 64: return adj_flags<R, PR, MODEL, 64>(a, accel, wc, vbeg, vend, s);
    default: return hipErrorInvalidValue;
    }
}

template <class R, class PR>
hipError_t launch_adjoint_phase(const AdjArgs<R, PR>& a, int model, int lanes, bool accel, bool wc,
                                int vbeg, int vend, hipStream_t s)
{
    if (model == kNeo) return adj_lanes<R, PR, kNeo>(a, lanes, accel, wc, vbeg, vend, s);
    if (model == kNeoU) return adj_lanes<R, PR, kNeoU>(a, lanes, accel, wc, vbeg, vend, s);
    if (model == kSnh) return adj_lanes<R, PR, kSnh>(a, lanes, accel, wc, vbeg, vend, s);
    return adj_lanes<R, PR, kCor>(a, lanes, accel, wc, vbeg, vend, s);
}

// ---------------------------------------------------------------------------
// FP64 passes: residual r = f + fhat and energy (Eq. fem_qs, pe_hat), and
// the adjoint assembly.  Tet-centric stress into a per-tet buffer, then a
// vertex-centric gather in a fixed order: deterministic, no atomics.
// ---------------------------------------------------------------------------
template <class R4>
__device__ __forceinline__ V3<double> x64(R4 p)
{
    return mk<double>(double(p.x), double(p.y), double(p.z));
}

__device__ __forceinline__ V3<double> grad_of_slot(const TetGeo& G, int slot)
{
    if (slot == 0)
        return mk(-(G.dm[0] + G.dm[3] + G.dm[6]), -(G.dm[1] + G.dm[4] + G.dm[7]),
                  -(G.dm[2] + G.dm[5] + G.dm[8]));
    const double* r = G.dm + 3 * (slot - 1);
    return mk(r[0], r[1], r[2]);
}

// V0 P dN_j of a tet for its four vertices j (12 doubles, slot-major), so
// that a vertex gathers 3 doubles per incident tet.
__device__ __forceinline__ void store_slot_forces(double* o, const TetGeo& G, const Cols<double>& P)
{
#pragma unroll
    for (int slot = 0; slot < 4; ++slot) {
        const V3<double> f = G.V0 * apply(P, grad_of_slot(G, slot));
        o[3 * slot] = f.x;
        o[3 * slot + 1] = f.y;
        o[3 * slot + 2] = f.z;
    }
}

// sum over the visits of vertex v of the per-slot vectors in vp (rv = tet *
// 4 + slot indexes them directly), in a fixed order
template <class R>
__device__ __forceinline__ V3<double> gather_vp(const ResArgs<R>& a, int v)
{
    V3<double> s = mk(0.0, 0.0, 0.0);
    const int jb = a.rvptr[v], je = a.rvptr[v + 1];
#pragma unroll 4
    for (int j = jb; j < je; ++j) {
        const double* o = a.vp + 3 * int64_t(a.rv[j]);
        s = s + mk(o[0], o[1], o[2]);
    }
    return s;
}

template <class R>
__device__ __forceinline__ Cols<double> tet_F(const ResArgs<R>& a, int4 t, const TetGeo& G)
{
    const V3<double> x0 = x64(a.X[t.x]);
    return edge_F(x64(a.X[t.y]) - x0, x64(a.X[t.z]) - x0, x64(a.X[t.w]) - x0, G.dm);
}

template <class R, int MODEL>
__global__ __launch_bounds__(kBlock) void k_tet_stress(ResArgs<R> a)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= a.n_tets) return;
    const int4 t = a.tet[e];
    const TetGeo G = a.geo[e];
    const Cols<double> F = tet_F(a, t, G);
    const Cols<double> C = cofactor(F);
    const double J = dot(F.c0, C.c0);
    Cols<double> P;
    double psi;
    if constexpr (MODEL == kSnh) {
        const double a = G.mu * (1.0 - 1.0 / (1.0 + frob2(F)));
        const double q = G.lam * (J - 1.0) - 0.75 * G.mu;
        P.c0 = a * F.c0 + q * C.c0;
        P.c1 = a * F.c1 + q * C.c1;
        P.c2 = a * F.c2 + q * C.c2;
        psi = snh_energy(F, J, G.mu, G.lam);
    } else if constexpr (MODEL == kNeo) {
        const double lh = G.mu + G.lam;
        const double q = J - 1.0 - G.mu / lh;
        P.c0 = G.mu * F.c0 + (lh * q) * C.c0;
        P.c1 = G.mu * F.c1 + (lh * q) * C.c1;
        P.c2 = G.mu * F.c2 + (lh * q) * C.c2;
        psi = 0.5 * G.mu * frob2(F) + 0.5 * lh * q * q;
    } else {
        const Cols<double> Rm = rotation_of(F);
        const double w = G.lam * (J - 1.0);
        P.c0 = (2.0 * G.mu) * (F.c0 - Rm.c0) + w * C.c0;
        P.c1 = (2.0 * G.mu) * (F.c1 - Rm.c1) + w * C.c1;
        P.c2 = (2.0 * G.mu) * (F.c2 - Rm.c2) + w * C.c2;
        psi = corot_energy(F, Rm, J, G.mu, G.lam);
    }
    store_slot_forces(a.vp + 12 * int64_t(e), G, P);
    a.ebuf[a.tet_eidx[e]] = G.V0 * psi;
}

template <class R>
__device__ __forceinline__ V3<double> weak_force(const ResArgs<R>& a, int v,
                                                 const typename R4t<R>::T* Y)
{
    V3<double> s = mk(0.0, 0.0, 0.0);
    for (int k = a.wvptr[v]; k < a.wvptr[v + 1]; ++k) {
        const int c = a.wv_c[k];
        V3<double> C = mk(0.0, 0.0, 0.0);
        for (int j = a.wc_ptr[c]; j < a.wc_ptr[c + 1]; ++j)
            C = C + a.wc_w64[j] * x64(Y[a.wc_vert[j]]);
        s = s + a.wv_s64[k] * symK_mul(a.wc_K64 + 6 * c, C);
    }
    return s;
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_vertex_residual(ResArgs<R> a, double* rsq,
                                                            double* r_out)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.n_verts) return;
    const int v = a.vorder[k];
    const V3<double> xi = x64(a.X[v]);
    const V3<double> f = mk(a.fext64[3 * v], a.fext64[3 * v + 1], a.fext64[3 * v + 2]);
    double ev = -dot(xi, f);
    V3<double> gp = mk(0.0, 0.0, 0.0);
    const int inst = a.vinst_all[v];
    for (int q = a.plane_ptr[inst]; q < a.plane_ptr[inst + 1]; ++q) {
        const double* pl = a.planes64 + 5 * q;
        const V3<double> n = mk(pl[0], pl[1], pl[2]);
        const double phi = dot(n, xi) - pl[3];
        if (phi < 0.0) {
            ev += 0.5 * pl[4] * phi * phi;
            gp = gp + (pl[4] * phi) * n;
        }
    }
    V3<double> r = mk(0.0, 0.0, 0.0);
    if (v < a.n_free) {
        r = f - gp - gather_vp(a, v);
        if (a.n_wc > 0) r = r - weak_force(a, v, a.X);
        if (a.inert64) {
            // backward-Euler inertia 1/2 c |x - xhat|^2, c = m_ii / dt^2
            const double c = a.inert64[v];
            const double* xh = a.xhat64 + 3 * int64_t(v);
            const V3<double> d = xi - mk(xh[0], xh[1], xh[2]);
            r = r - c * d;
            ev += 0.5 * c * dot(d, d);
        }
    }
    a.ebuf[a.vert_eidx[k]] = ev;
    rsq[k] = dot(r, r);
    if (r_out) {
        double* o = r_out + 3 * int64_t(a.orig_of[v]);
        o[0] = r.x; o[1] = r.y; o[2] = r.z;
    }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_wc_energy(ResArgs<R> a)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.n_wc) return;
    V3<double> C = mk(0.0, 0.0, 0.0);
    for (int j = a.wc_ptr[c]; j < a.wc_ptr[c + 1]; ++j)
        C = C + a.wc_w64[j] * x64(a.X[a.wc_vert[j]]);
    a.ebuf[a.wc_eidx[c]] = 0.5 * dot(C, symK_mul(a.wc_K64 + 6 * c, C));
}

static inline int nblk(int64_t n) { return int((n + kBlock - 1) / kBlock); }

template <class R>
hipError_t launch_residual(const ResArgs<R>& a, double* rsq, double* r_out, hipStream_t s)
{
    if (a.n_tets > 0) {
        if (a.model == kNeo)
            hipLaunchKernelGGL((k_tet_stress<R, kNeo>), dim3(nblk(a.n_tets)), dim3(kBlock), 0, s, a);
        else if (a.model == kSnh)
            hipLaunchKernelGGL((k_tet_stress<R, kSnh>), dim3(nblk(a.n_tets)), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_tet_stress<R, kCor>), dim3(nblk(a.n_tets)), dim3(kBlock), 0, s, a);
    }
    if (a.n_wc > 0) hipLaunchKernelGGL((k_wc_energy<R>), dim3(nblk(a.n_wc)), dim3(kBlock), 0, s, a);
    if (a.n_verts > 0)
        hipLaunchKernelGGL((k_vertex_residual<R>), dim3(nblk(a.n_verts)), dim3(kBlock), 0, s, a,
                           rsq, r_out);
    return hipGetLastError();
}

// Adjoint assembly in FP64: per tet V0 dP[Lam] (into vp) and the parameter
// gradients; per vertex (H lam)_i, the adjoint residual b - H lam on free
// vertices and dL/dx_D = -(H lam)_k on Dirichlet vertices.
template <class R, int MODEL>
__global__ __launch_bounds__(kBlock) void k_tet_adjoint(ResArgs<R> a,
                                                        const typename R4t<R>::T* L,
                                                        double* dmu, double* dlam)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= a.n_tets) return;
    const int4 t = a.tet[e];
    const TetGeo G = a.geo[e];
    const Cols<double> F = tet_F(a, t, G);
    const V3<double> l0 = x64(L[t.x]);
    const Cols<double> Lm = edge_F(x64(L[t.y]) - l0, x64(L[t.z]) - l0, x64(L[t.w]) - l0, G.dm);
    const Cols<double> C = cofactor(F);
    const double J = dot(F.c0, C.c0);
    const double cofL = dot(C.c0, Lm.c0) + dot(C.c1, Lm.c1) + dot(C.c2, Lm.c2);
    const double FL = dot(F.c0, Lm.c0) + dot(F.c1, Lm.c1) + dot(F.c2, Lm.c2);
    Cols<double> dP;
    double dPdmu;   // <dP/dmu, Lam>
    if constexpr (MODEL == kNeo) {
        const double lh = G.mu + G.lam;
        const double qq = lh * (J - 1.0) - G.mu;
        dP.c0 = G.mu * Lm.c0 + (lh * cofL) * C.c0 + qq * (cross(Lm.c1, F.c2) + cross(F.c1, Lm.c2));
        dP.c1 = G.mu * Lm.c1 + (lh * cofL) * C.c1 + qq * (cross(Lm.c2, F.c0) + cross(F.c2, Lm.c0));
        dP.c2 = G.mu * Lm.c2 + (lh * cofL) * C.c2 + qq * (cross(Lm.c0, F.c1) + cross(F.c0, Lm.c1));
        // dP/dmu = F + (J - 2) cof F
        dPdmu = FL + (J - 2.0) * cofL;
    } else {
        dP = stress_diff<double, MODEL>(F, C, J, Lm, G.mu, G.lam);
        if constexpr (MODEL == kSnh) {
            // dP/dmu = (1 - 1/(1 + |F|^2)) F - 3/4 cof F
            dPdmu = (1.0 - 1.0 / (1.0 + frob2(F))) * FL - 0.75 * cofL;
        } else {
            // dP/dmu = 2 (F - R)
            const Cols<double> Rm = rotation_of(F);
            dPdmu = 2.0 * (FL - dot(Rm.c0, Lm.c0) - dot(Rm.c1, Lm.c1) - dot(Rm.c2, Lm.c2));
        }
    }
    store_slot_forces(a.vp + 12 * int64_t(e), G, dP);
    // dP/dlambda = (J - 1) cof F for every model
    if (dmu) dmu[e] = -G.V0 * dPdmu;
    if (dlam) dlam[e] = -G.V0 * (J - 1.0) * cofL;
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_vertex_adjoint(ResArgs<R> a,
                                                           const typename R4t<R>::T* L,
                                                           const typename R4t<R>::T* B,
                                                           double* rsq, double* dxd,
                                                           const int* dir_pos)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.n_verts) return;
    const int v = a.vorder[k];
    V3<double> hl = gather_vp(a, v);
    if (a.n_wc > 0) hl = hl + weak_force(a, v, L);
    const V3<double> xi = x64(a.X[v]);
    const V3<double> li = x64(L[v]);
    const int inst = a.vinst_all[v];
    for (int q = a.plane_ptr[inst]; q < a.plane_ptr[inst + 1]; ++q) {
        const double* pl = a.planes64 + 5 * q;
        const V3<double> n = mk(pl[0], pl[1], pl[2]);
        if (dot(n, xi) - pl[3] < 0.0) hl = hl + (pl[4] * dot(n, li)) * n;
    }
    if (v < a.n_free) {
        if (a.inert64) hl = hl + a.inert64[v] * li;
        const V3<double> r = x64(B[v]) - hl;
        rsq[k] = dot(r, r);
    } else {
        // x*_D = x_D, so dL/dx_D = (dL/dx)_D - (H lam)_D
        rsq[k] = 0.0;
        if (dxd) {
            const V3<double> g = x64(B[v]) - hl;
            double* o = dxd + 3 * int64_t(dir_pos[v - a.n_free]);
            o[0] = g.x; o[1] = g.y; o[2] = g.z;
        }
    }
}

template <class R>
hipError_t launch_adjoint_assembly(const ResArgs<R>& a, const typename R4t<R>::T* lam,
                                   const typename R4t<R>::T* b, double* rsq, double* dmu,
                                   double* dlam, double* dxd, const int* dir_pos, hipStream_t s)
{
    if (a.n_tets > 0) {
        if (a.model == kNeo)
            hipLaunchKernelGGL((k_tet_adjoint<R, kNeo>), dim3(nblk(a.n_tets)), dim3(kBlock), 0, s, a,
                               lam, dmu, dlam);
        else if (a.model == kSnh)
            hipLaunchKernelGGL((k_tet_adjoint<R, kSnh>), dim3(nblk(a.n_tets)), dim3(kBlock), 0, s, a,
                               lam, dmu, dlam);
        else
            hipLaunchKernelGGL((k_tet_adjoint<R, kCor>), dim3(nblk(a.n_tets)), dim3(kBlock), 0, s, a,
                               lam, dmu, dlam);
    }
    if (a.n_verts > 0)
        hipLaunchKernelGGL((k_vertex_adjoint<R>), dim3(nblk(a.n_verts)), dim3(kBlock), 0, s, a,
                           lam, b, rsq, dxd, dir_pos);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deterministic segmented sums: fixed per-thread strides and a fixed LDS
// tree, first per chunk, then per instance over its chunks.
// ---------------------------------------------------------------------------
#if PBNG_KERNEL_SET == 0
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(kBlock) void k_chunk_sum(const double* vals, const int64_t* cb,
                                                     const int64_t* ce, double* partial)
{
    __shared__ double sh[kBlock];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t i = cb[c] + threadIdx.x; i < ce[c]; i += kBlock) s += vals[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) partial[c] = t;
}

__global__ __launch_bounds__(kBlock) void k_inst_sum(const double* partial, const int* qptr,
                                                    double* out)
{
    __shared__ double sh[kBlock];
    const int q = blockIdx.x;
    double s = 0.0;
    for (int i = qptr[q] + threadIdx.x; i < qptr[q + 1]; i += kBlock) s += partial[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[q] = t;
}

hipError_t launch_segsum(const double* vals, const SegPlan& plan, int n_inst, double* out,
                         hipStream_t s)
{
    if (plan.n_chunks > 0)
        hipLaunchKernelGGL(k_chunk_sum, dim3(plan.n_chunks), dim3(kBlock), 0, s, vals, plan.cbeg,
                           plan.cend, plan.partial);
    hipLaunchKernelGGL(k_inst_sum, dim3(n_inst), dim3(kBlock), 0, s, plan.partial, plan.qptr, out);
    return hipGetLastError();
}

#endif

// ---------------------------------------------------------------------------
// Layout conversion and parameter updates
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(kBlock) void k_load(const R* x_user, const int* orig_of,
                                                 const typename R4t<R>::T* xd_int,
                                                 typename R4t<R>::T* d0, typename R4t<R>::T* d1,
                                                 typename R4t<R>::T* d2, int n_free, int n_verts)
{
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n_verts) return;
    typename R4t<R>::T val;
    if (v < n_free || xd_int == nullptr) {
        const int64_t o = orig_of[v];
        val = typename R4t<R>::T{x_user[3 * o], x_user[3 * o + 1], x_user[3 * o + 2], R(0)};
    } else {
        val = xd_int[v - n_free];
    }
    d0[v] = val;
    if (d1) d1[v] = val;
    if (d2) d2[v] = val;
}

template <class R>
hipError_t launch_load(const R* x_user, const int* orig_of, const typename R4t<R>::T* xd_int,
                       typename R4t<R>::T* d0, typename R4t<R>::T* d1, typename R4t<R>::T* d2,
                       int n_free, int n_verts, hipStream_t s)
{
    if (n_verts > 0)
        hipLaunchKernelGGL((k_load<R>), dim3(nblk(n_verts)), dim3(kBlock), 0, s, x_user, orig_of,
                           xd_int, d0, d1, d2, n_free, n_verts);
    return hipGetLastError();
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_load_vec(const R* v_user, const int* orig_of,
                                                     typename R4t<R>::T* dst, int n_free,
                                                     int n_verts)
{
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n_verts) return;
    (void)n_free;
    const int64_t o = orig_of[v];
    dst[v] = typename R4t<R>::T{v_user[3 * o], v_user[3 * o + 1], v_user[3 * o + 2], R(0)};
}

template <class R>
hipError_t launch_load_vec(const R* v_user, const int* orig_of, typename R4t<R>::T* dst,
                           int n_free, int n_verts, hipStream_t s)
{
    if (n_verts > 0)
        hipLaunchKernelGGL((k_load_vec<R>), dim3(nblk(n_verts)), dim3(kBlock), 0, s, v_user,
                           orig_of, dst, n_free, n_verts);
    return hipGetLastError();
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_store(const typename R4t<R>::T* src, const int* orig_of,
                                                  R* x_user, int n_verts)
{
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n_verts) return;
    const typename R4t<R>::T p = src[v];
    const int64_t o = orig_of[v];
    x_user[3 * o] = p.x;
    x_user[3 * o + 1] = p.y;
    x_user[3 * o + 2] = p.z;
}

template <class R>
hipError_t launch_store(const typename R4t<R>::T* src, const int* orig_of, R* x_user, int n_verts,
                        hipStream_t s)
{
    if (n_verts > 0)
        hipLaunchKernelGGL((k_store<R>), dim3(nblk(n_verts)), dim3(kBlock), 0, s, src, orig_of,
                           x_user, n_verts);
    return hipGetLastError();
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_store64(const typename R4t<R>::T* src,
                                                    const int* orig_of, double* x_user,
                                                    int n_verts)
{
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n_verts) return;
    const typename R4t<R>::T p = src[v];
    const int64_t o = orig_of[v];
    x_user[3 * o] = double(p.x);
    x_user[3 * o + 1] = double(p.y);
    x_user[3 * o + 2] = double(p.z);
}

template <class R>
hipError_t launch_store64(const typename R4t<R>::T* src, const int* orig_of, double* x_user,
                          int n_verts, hipStream_t s)
{
    if (n_verts > 0)
        hipLaunchKernelGGL((k_store64<R>), dim3(nblk(n_verts)), dim3(kBlock), 0, s, src, orig_of,
                           x_user, n_verts);
    return hipGetLastError();
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_copy4(const typename R4t<R>::T* src,
                                                  typename R4t<R>::T* dst, int n)
{
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v < n) dst[v] = src[v];
}

template <class R>
hipError_t launch_copy4(const typename R4t<R>::T* src, typename R4t<R>::T* dst, int n,
                        hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL((k_copy4<R>), dim3(nblk(n)), dim3(kBlock), 0, s, src, dst, n);
    return hipGetLastError();
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_set_geo(const double* mu, const double* lam,
                                                    TetGeo* geo, int n_tets)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= n_tets) return;
    geo[e].mu = mu[e];
    geo[e].lam = lam[e];
}

// Visit records of free vertex v from the FP64 tet geometry: one thread per
// vertex, visits in CSR order (rv = tet * 4 + slot of v), the other three
// vertices in increasing slot order as the host listed them in jv.xyz.
// Also the per-vertex sum S = sum V0 mu |dN_i|^2, in visit order.
template <class R>
__global__ __launch_bounds__(kBlock) void k_build_visits(VisitBuild<R> b)
{
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= b.n_free) return;
    double S = 0.0;
    for (int k = b.vptr[v]; k < b.vptr[v + 1]; ++k) {
        const int e = b.rv[k] >> 2, slot = b.rv[k] & 3;
        const TetGeo& G = b.geo[e];
        V3<double> m[3];
        int no = 0;
        for (int j = 0; j < 4; ++j) {
            if (j == slot) continue;
            m[no++] = grad_of_slot(G, j);
        }
        const V3<double> av = grad_of_slot(G, slot);
        const double vm = G.V0 * G.mu, vl = G.V0 * G.lam;
        S += vm * dot(av, av);
        if constexpr (sizeof(R) == 4) b.jv[k].w = __float_as_int(float(vm));
        else b.vmu[k] = vm;
        using R4 = typename R4t<R>::T;
        if (b.model == kNeo || b.model == kNeoU) {
            // rows of cof M are m2 x m3, m3 x m1, m1 x m2
            const V3<double> c1 = cross(m[1], m[2]), c2 = cross(m[2], m[0]), c3 = cross(m[0], m[1]);
            const double delta = dot(m[0], c1);
            if (b.model == kNeoU) {
                // 40-byte form: delta in jv.w (FP32) or vmu (FP64), V0 alpha, beta
                if constexpr (sizeof(R) == 4) b.jv[k].w = __float_as_int(float(delta));
                else b.vmu[k] = delta;
                b.ma[k] = R4{R(G.V0 * dot(m[0], av)), R(G.V0 * dot(m[1], av)), R(G.V0 * dot(m[2], av)),
                             R(dot(c1, av))};
                b.mc[k] = typename R2t<R>::T{R(dot(c2, av)), R(dot(c3, av))};
                continue;
            }
            b.ma[k] = R4{R(vm * dot(m[0], av)), R(vm * dot(m[1], av)), R(vm * dot(m[2], av)), R(vl)};
            b.mb[k] = R4{R(dot(c1, av)), R(dot(c2, av)), R(dot(c3, av)), R(delta)};
        } else {
            b.ma[k] = R4{R(m[0].x), R(m[0].y), R(m[0].z), R(m[1].x)};
            b.mb[k] = R4{R(m[1].y), R(m[1].z), R(m[2].x), R(m[2].y)};
            b.mc[k] = typename R2t<R>::T{R(m[2].z), R(vl)};
        }
    }
    b.Sv[v] = R(S);
}

#if PBNG_KERNEL_SET == 0
// Material flags (see launch_material_flags): one thread per tet, its
// instance found by bisection over the tet offsets.  NaN parameters count
// as violations.
__global__ __launch_bounds__(kBlock) void k_flags_one(int* flag)
{
    if (threadIdx.x < 2) flag[threadIdx.x] = 1;
}

__global__ __launch_bounds__(kBlock) void k_material_flags(const double* mu, const double* lam,
                                                           const int64_t* t_off, int n_inst, int n,
                                                           int* flag)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= n) return;
    if (!(lam[e] >= mu[e])) flag[0] = 0;
    int lo = 0, hi = n_inst;   // t_off[lo] <= e < t_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (t_off[mid] <= e) lo = mid;
        else hi = mid;
    }
    const int64_t f = t_off[lo];
    if (!(mu[e] == mu[f]) || !(lam[e] == lam[f])) flag[1] = 0;
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_inst_materials(const double* mu, const double* lam,
                                                           const int64_t* t_off, int n_inst, R* imu,
                                                           R* ilam)
{
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= n_inst) return;
    const bool has = t_off[q + 1] > t_off[q];
    imu[q] = has ? R(mu[t_off[q]]) : R(0);
    ilam[q] = has ? R(lam[t_off[q]]) : R(0);
}

template <class R>
hipError_t launch_material_flags(const double* mu, const double* lam, const int64_t* t_off, int n_inst,
                                 int n_tets, int* flag, R* imu, R* ilam, hipStream_t s)
{
    hipLaunchKernelGGL(k_flags_one, dim3(1), dim3(kBlock), 0, s, flag);
    if (n_tets > 0)
        hipLaunchKernelGGL(k_material_flags, dim3(nblk(n_tets)), dim3(kBlock), 0, s, mu, lam, t_off,
                           n_inst, n_tets, flag);
    if (n_inst > 0)
        hipLaunchKernelGGL((k_inst_materials<R>), dim3(nblk(n_inst)), dim3(kBlock), 0, s, mu, lam,
                           t_off, n_inst, imu, ilam);
    return hipGetLastError();
}
#endif

template <class R>
hipError_t launch_build_visits(const VisitBuild<R>& b, hipStream_t s)
{
    if (b.n_free > 0)
        hipLaunchKernelGGL((k_build_visits<R>), dim3(nblk(b.n_free)), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

template <class R>
hipError_t launch_set_materials(const double* mu, const double* lam, TetGeo* geo, int n_tets,
                                const VisitBuild<R>& b, hipStream_t s)
{
    if (n_tets > 0)
        hipLaunchKernelGGL((k_set_geo<R>), dim3(nblk(n_tets)), dim3(kBlock), 0, s, mu, lam, geo,
                           n_tets);
    return launch_build_visits<R>(b, s);
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_set_dirichlet(const double* xd, const int* dir_internal,
                                                          int nd, int n_free,
                                                          typename R4t<R>::T* xd_int)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= nd) return;
    xd_int[dir_internal[k] - n_free] =
        typename R4t<R>::T{R(xd[3 * k]), R(xd[3 * k + 1]), R(xd[3 * k + 2]), R(0)};
}

template <class R>
hipError_t launch_set_dirichlet(const double* xd, const int* dir_internal, int nd, int n_free,
                                typename R4t<R>::T* xd_int, hipStream_t s)
{
    if (nd > 0)
        hipLaunchKernelGGL((k_set_dirichlet<R>), dim3(nblk(nd)), dim3(kBlock), 0, s, xd,
                           dir_internal, nd, n_free, xd_int);
    return hipGetLastError();
}

// Explicit instantiations.  The library compiles this file once per
// PBNG_KERNEL_SET (0: FP32, 1: FP64, 2: FP32 arithmetic on FP64 positions)
// so the three sets build in parallel; set 0 also holds the shared helpers.
template <class R, class PR>
__global__ __launch_bounds__(kBlock) void k_set_inertia(const double* x_n, const double* x_prev,
                                                        const int* orig_of, const double* mass,
                                                        int n_free, double inv_dt2, R* inert,
                                                        typename R4t<PR>::T* xhat, double* inert64,
                                                        double* xhat64)
{
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n_free) return;
    const int64_t o = 3 * int64_t(orig_of[v]);
    double h[3];
    for (int c = 0; c < 3; ++c) h[c] = 2.0 * x_n[o + c] - x_prev[o + c];
    const double w = mass[v] * inv_dt2;
    inert[v] = R(w);
    xhat[v] = typename R4t<PR>::T{PR(h[0]), PR(h[1]), PR(h[2]), PR(0)};
    inert64[v] = w;
    for (int c = 0; c < 3; ++c) xhat64[3 * int64_t(v) + c] = h[c];
}

template <class R, class PR>
hipError_t launch_set_inertia(const double* x_n, const double* x_prev, const int* orig_of,
                              const double* mass, int n_free, double dt, R* inert,
                              typename R4t<PR>::T* xhat, double* inert64, double* xhat64,
                              hipStream_t s)
{
    if (n_free > 0)
        hipLaunchKernelGGL((k_set_inertia<R, PR>), dim3(nblk(n_free)), dim3(kBlock), 0, s, x_n,
                           x_prev, orig_of, mass, n_free, 1.0 / (dt * dt), inert, xhat, inert64,
                           xhat64);
    return hipGetLastError();
}

#define PBNG_INST_POS(R)                                                                          \
    template hipError_t launch_load<R>(const R*, const int*, const R4t<R>::T*, R4t<R>::T*,       \
                                       R4t<R>::T*, R4t<R>::T*, int, int, hipStream_t);           \
    template hipError_t launch_load_vec<R>(const R*, const int*, R4t<R>::T*, int, int,           \
                                           hipStream_t);                                          \
    template hipError_t launch_store<R>(const R4t<R>::T*, const int*, R*, int, hipStream_t);     \
    template hipError_t launch_copy4<R>(const R4t<R>::T*, R4t<R>::T*, int, hipStream_t);         \
    template hipError_t launch_store64<R>(const R4t<R>::T*, const int*, double*, int,            \
                                          hipStream_t);                                           \
    template hipError_t launch_set_dirichlet<R>(const double*, const int*, int, int, R4t<R>::T*, \
                                                hipStream_t);                                     \
    template hipError_t launch_residual<R>(const ResArgs<R>&, double*, double*, hipStream_t);    \
    template hipError_t launch_adjoint_assembly<R>(const ResArgs<R>&, const R4t<R>::T*,          \
                                                   const R4t<R>::T*, double*, double*, double*,   \
                                                   double*, const int*, hipStream_t);
#define PBNG_INST_SWEEP(R, PR)                                                                    \
    template hipError_t launch_phase<R, PR>(const SweepArgs<R, PR>&, int, int, bool, bool, int,   \
                                            int, int, hipStream_t);                               \
    template hipError_t launch_adjoint_phase<R, PR>(const AdjArgs<R, PR>&, int, int, bool, bool,  \
                                                    int, int, hipStream_t);                            \
    template hipError_t launch_set_inertia<R, PR>(const double*, const double*, const int*,       \
                                                  const double*, int, double, R*, R4t<PR>::T*,    \
                                                  double*, double*, hipStream_t);
#if PBNG_KERNEL_SET == 0
PBNG_INST_POS(float)
PBNG_INST_POS(double)
template hipError_t launch_set_materials<float>(const double*, const double*, TetGeo*, int,
                                                const VisitBuild<float>&, hipStream_t);
template hipError_t launch_set_materials<double>(const double*, const double*, TetGeo*, int,
                                                 const VisitBuild<double>&, hipStream_t);
template hipError_t launch_material_flags<float>(const double*, const double*, const int64_t*, int,
                                                 int, int*, float*, float*, hipStream_t);
template hipError_t launch_material_flags<double>(const double*, const double*, const int64_t*, int,
                                                  int, int*, double*, double*, hipStream_t);
template hipError_t launch_build_visits<float>(const VisitBuild<float>&, hipStream_t);
template hipError_t launch_build_visits<double>(const VisitBuild<double>&, hipStream_t);
PBNG_INST_SWEEP(float, float)
#elif PBNG_KERNEL_SET == 1
PBNG_INST_SWEEP(double, double)
#else
PBNG_INST_SWEEP(float, double)
#endif

}  // namespace pbng
