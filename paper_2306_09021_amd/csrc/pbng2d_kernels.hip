// HIP kernels of libpbng for planar problems (triangle meshes, d = 2).
//
// Same organisation as the tetrahedral hot path: one launch per colour
// phase, a group of LANES lanes of a 64-wide wavefront per free vertex,
// lane l taking the vertex's visits l, l + LANES, ...  Per visit the lane
// forms the 2x2 F from two gathered edge vectors, adds the stress term
// A0 P(F) dN_i to the local gradient and accumulates the pieces of the
// modified nodal matrix of Eq. (mod_hess) with d = 2,
//   A_i = sum A0 (2 mu |dN_i|^2 I + lambda c c^T),  c = cof(F) dN_i,
// the group sums its partial results with in-row data-parallel moves and
// solves the 2x2 SPD system in closed form (Eq. pbgn_dx).  Gather-bound
// vector ALU work; nothing here is a dense contraction.
#include "pbng2d.hpp"
#include "pbng_device.hpp"
#include "pbng_math.hpp"

namespace pbng {

namespace {

constexpr int kBlk = 256;

inline int nblocks(int64_t n) { return int((n + kBlk - 1) / kBlk); }

// Closest rotation R = [[c, -s], [s, c]] to the 2x2 F (maximiser of
// tr(R^T F)): (c, s) is (F00 + F11, F10 - F01) normalised, R = I when both
// vanish.
template <class R>
__device__ __forceinline__ void rot2(R f00, R f01, R f10, R f11, R& c, R& s)
{
    const R a = f00 + f11, b = f10 - f01;
    const R r2 = a * a + b * b;
    if (r2 > R(0)) {
        const R ir = rsq(r2);
        c = a * ir;
        s = b * ir;
    } else {
        c = R(1);
        s = R(0);
    }
}

template <class R, int MODEL, int LANES, bool ACCEL, bool SAFE, bool UNI>
__global__ __launch_bounds__(kBlk) void k2_phase(Sweep2Args<R> a, int vbeg, int vend)
{
    using R2 = typename R2t<R>::T;
    const int t = xcd_block() * kBlk + int(threadIdx.x);
    const int v = vbeg + t / LANES;
    const int lane = t & (LANES - 1);
    if (v >= vend) return;  // whole groups leave together (LANES divides 64)
    const R2 xi = at(a.W, v);
    const int kb = at(a.vptr, v), ke = at(a.vptr, v + 1);
    R gx = R(0), gy = R(0), s = R(0), lxx = R(0), lxy = R(0), lyy = R(0);
    R mxx = R(0), mxy = R(0), myy = R(0);
    for (int k = kb + lane; k < ke; k += LANES) {
        const int2 jk = at(a.jk, k);
        const auto g = at(a.gm, k);   // dN_j = (g.x, g.y), dN_k = (g.z, g.w)
        R2 w;                         // (A0 mu, A0 lambda)
        if constexpr (UNI) {
            const R A0 = R(0.5) / abs_(g.x * g.w - g.y * g.z);
            w.x = a.mu_u * A0;
            w.y = a.lam_u * A0;
        } else {
            w = at(a.vw, k);
        }
        const R2 xj = at(a.W, jk.x), xk = at(a.W, jk.y);
        const R e1x = xj.x - xi.x, e1y = xj.y - xi.y;
        const R e2x = xk.x - xi.x, e2y = xk.y - xi.y;
        const R f00 = e1x * g.x + e2x * g.z, f01 = e1x * g.y + e2x * g.w;
        const R f10 = e1y * g.x + e2y * g.z, f11 = e1y * g.y + e2y * g.w;
        const R ax = -(g.x + g.z), ay = -(g.y + g.w);  // dN_i
        const R J = f00 * f11 - f01 * f10;
        // c = cof(F) dN_i with cof(F) = [[f11, -f10], [-f01, f00]]
        const R cx = f11 * ax - f10 * ay, cy = f00 * ay - f01 * ax;
        const R fax = f00 * ax + f01 * ay, fay = f10 * ax + f11 * ay;
        s += w.x * (ax * ax + ay * ay);
        lxx += w.y * cx * cx;
        lxy += w.y * cx * cy;
        lyy += w.y * cy * cy;
        if constexpr (MODEL == kPlanarNeo) {
            // A0 lhat (J - 1 - mu / lhat) = A0 lhat (J - 1) - A0 mu
            const R q = (w.x + w.y) * (J - R(1)) - w.x;
            gx += w.x * fax + q * cx;
            gy += w.x * fay + q * cy;
            if (SAFE) {
                mxx += w.x * cx * cx;
                mxy += w.x * cx * cy;
                myy += w.x * cy * cy;
            }
        } else {
            R c, sn;
            rot2(f00, f01, f10, f11, c, sn);
            const R rax = c * ax - sn * ay, ray = sn * ax + c * ay;  // R dN_i
            const R q = w.y * (J - R(1));
            gx += R(2) * w.x * (fax - rax) + q * cx;
            gy += R(2) * w.x * (fay - ray) + q * cy;
        }
    }
    if (LANES > 1) {
        gx = lsum<LANES>(gx);
        gy = lsum<LANES>(gy);
        s = lsum<LANES>(s);
        lxx = lsum<LANES>(lxx);
        lxy = lsum<LANES>(lxy);
        lyy = lsum<LANES>(lyy);
        if (MODEL == kPlanarNeo && SAFE) {
            mxx = lsum<LANES>(mxx);
            mxy = lsum<LANES>(mxy);
            myy = lsum<LANES>(myy);
        }
    }
    const R2 f = at(a.fext, v);
    const R gtx = gx - f.x, gty = gy - f.y;
    const R Axx = R(2) * s + lxx, Axy = lxy, Ayy = R(2) * s + lyy;
    const R det = Axx * Ayy - Axy * Axy;
    bool reject = !(Axx > R(0) && det > R(0));
    R dx = R(0), dy = R(0), alpha = R(1);
    if (!reject) {
        const R id = R(1) / det;
        dx = -(Ayy * gtx - Axy * gty) * id;
        dy = -(Axx * gty - Axy * gtx) * id;
        if constexpr (SAFE && MODEL == kPlanarNeo) {
            // Along x_i + alpha d the Neo-Hookean local energy is exactly
            // E(0) + alpha g.d + alpha^2 / 2 d^T H d with
            // H = sum A0 (mu |dN_i|^2 I + lhat c c^T): |F|^2 is quadratic and
            // det F affine in x_i.
            const R hxx = s + lxx + mxx, hxy = lxy + mxy, hyy = s + lyy + myy;
            const R lin = gtx * dx + gty * dy;
            const R quad = dx * (hxx * dx + hxy * dy) + dy * (hxy * dx + hyy * dy);
            const R u = sizeof(R) == 8 ? R(1.1102230246251565e-16) : R(5.9604644775390625e-08);
            for (int h = 0;; ++h) {
                const R dE = alpha * lin + R(0.5) * alpha * alpha * quad;
                const R ab = abs_(alpha * lin) + abs_(R(0.5) * alpha * alpha * quad);
                if (dE <= R(8) * u * ab) break;
                if (h >= a.max_halvings) {
                    reject = true;
                    break;
                }
                alpha *= R(0.5);
            }
        }
    }
    if (lane == 0) {
        R2 xn = xi;
        if (!reject) {
            xn.x = xi.x + alpha * dx;
            xn.y = xi.y + alpha * dy;
        } else {
            atomicAdd(a.rejected, 1);
        }
        if (ACCEL) {
            const R2 xp = at(a.P, v);
            R2 b;
            b.x = a.omega * (a.gamma * (xn.x - xi.x) + xi.x - xp.x) + xp.x;
            b.y = a.omega * (a.gamma * (xn.y - xi.y) + xi.y - xp.y) + xp.y;
            *ptr_at(a.W, v) = xn;
            *ptr_at(a.P, v) = xi;
            *ptr_at(a.N, v) = b;
        } else {
            *ptr_at(a.W, v) = xn;
        }
    }
}

template <class R, int MODEL, int LANES, bool ACCEL, bool SAFE, bool UNI>
hipError_t phase_t(const Sweep2Args<R>& a, int vb, int ve, hipStream_t s)
{
    const int64_t threads = int64_t(ve - vb) * LANES;
    if (threads <= 0) return hipSuccess;
    hipLaunchKernelGGL((k2_phase<R, MODEL, LANES, ACCEL, SAFE, UNI>), dim3(nblocks(threads)), dim3(kBlk), 0, s,
                       a, vb, ve);
    return hipGetLastError();
}

template <class R, int MODEL, int LANES, bool UNI>
hipError_t phase_flags(const Sweep2Args<R>& a, bool accel, bool safe, int vb, int ve, hipStream_t s)
{
    // the corotated full step never raises the local energy: no safeguard
    if (MODEL == kPlanarCor) safe = false;
    if (accel)
        return safe ? phase_t<R, MODEL, LANES, true, true, UNI>(a, vb, ve, s)
                    : phase_t<R, MODEL, LANES, true, false, UNI>(a, vb, ve, s);
    return safe ? phase_t<R, MODEL, LANES, false, true, UNI>(a, vb, ve, s)
                : phase_t<R, MODEL, LANES, false, false, UNI>(a, vb, ve, s);
}

template <class R, int MODEL, bool UNI>
hipError_t phase_lanes(const Sweep2Args<R>& a, int lanes, bool accel, bool safe, int vb, int ve, hipStream_t s)
{
    switch (lanes) {
    case 1: return phase_flags<R, MODEL, 1, UNI>(a, accel, safe, vb, ve, s);
    case 2: return phase_flags<R, MODEL, 2, UNI>(a, accel, safe, vb, ve, s);
    case 4: return phase_flags<R, MODEL, 4, UNI>(a, accel, safe, vb, ve, s);
    case 8: return phase_flags<R, MODEL, 8, UNI>(a, accel, safe, vb, ve, s);
    case 16: return phase_flags<R, MODEL, 16, UNI>(a, accel, safe, vb, ve, s);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// FP64 residual and energy
// ---------------------------------------------------------------------------
template <class R2>
__device__ __forceinline__ double2 x64(R2 p)
{
    return double2{double(p.x), double(p.y)};
}

template <class R, int MODEL>
__global__ __launch_bounds__(kBlk) void k2_tri_stress(Res2Args<R> a)
{
    const int e = blockIdx.x * kBlk + int(threadIdx.x);
    if (e >= a.n_tris) return;
    const int4 t = a.tri[e];
    const TriGeo G = a.geo[e];
    const double2 x0 = x64(a.X[t.x]), x1 = x64(a.X[t.y]), x2 = x64(a.X[t.z]);
    const double e1x = x1.x - x0.x, e1y = x1.y - x0.y, e2x = x2.x - x0.x, e2y = x2.y - x0.y;
    const double f00 = e1x * G.g1x + e2x * G.g2x, f01 = e1x * G.g1y + e2x * G.g2y;
    const double f10 = e1y * G.g1x + e2y * G.g2x, f11 = e1y * G.g1y + e2y * G.g2y;
    const double J = f00 * f11 - f01 * f10;
    const double c00 = f11, c01 = -f10, c10 = -f01, c11 = f00;  // cof F
    double p00, p01, p10, p11, psi;
    if constexpr (MODEL == kPlanarNeo) {
        const double lh = G.mu + G.lam, q = J - 1.0 - G.mu / lh;
        p00 = G.mu * f00 + lh * q * c00;
        p01 = G.mu * f01 + lh * q * c01;
        p10 = G.mu * f10 + lh * q * c10;
        p11 = G.mu * f11 + lh * q * c11;
        psi = 0.5 * G.mu * (f00 * f00 + f01 * f01 + f10 * f10 + f11 * f11) + 0.5 * lh * q * q;
    } else {
        double c, sn;
        rot2(f00, f01, f10, f11, c, sn);
        const double d00 = f00 - c, d01 = f01 + sn, d10 = f10 - sn, d11 = f11 - c;  // F - R
        const double w = G.lam * (J - 1.0);
        p00 = 2.0 * G.mu * d00 + w * c00;
        p01 = 2.0 * G.mu * d01 + w * c01;
        p10 = 2.0 * G.mu * d10 + w * c10;
        p11 = 2.0 * G.mu * d11 + w * c11;
        psi = G.mu * (d00 * d00 + d01 * d01 + d10 * d10 + d11 * d11) + 0.5 * G.lam * (J - 1.0) * (J - 1.0);
    }
    const double gx[3] = {-(G.g1x + G.g2x), G.g1x, G.g2x};
    const double gy[3] = {-(G.g1y + G.g2y), G.g1y, G.g2y};
    double* o = a.vp + 6 * int64_t(e);
    for (int j = 0; j < 3; ++j) {
        o[2 * j] = G.A0 * (p00 * gx[j] + p01 * gy[j]);
        o[2 * j + 1] = G.A0 * (p10 * gx[j] + p11 * gy[j]);
    }
    a.ebuf[e] = G.A0 * psi;
}

template <class R>
__global__ __launch_bounds__(kBlk) void k2_vertex_residual(Res2Args<R> a, double* r_out)
{
    const int v = blockIdx.x * kBlk + int(threadIdx.x);
    if (v >= a.n_verts) return;
    const double2 xi = x64(a.X[v]);
    const double fx = a.fext64[2 * v], fy = a.fext64[2 * v + 1];
    double rx = 0.0, ry = 0.0;
    if (v < a.n_free) {
        rx = fx;
        ry = fy;
        for (int k = a.rvptr[v]; k < a.rvptr[v + 1]; ++k) {
            const double* p = a.vp + 2 * int64_t(a.rv[k]);
            rx -= p[0];
            ry -= p[1];
        }
    }
    a.ebuf[a.n_tris + v] = -(xi.x * fx + xi.y * fy);
    a.rsq[v] = rx * rx + ry * ry;
    if (r_out) {
        double* o = r_out + 2 * int64_t(a.orig_of[v]);
        o[0] = rx;
        o[1] = ry;
    }
}

// ---------------------------------------------------------------------------
// Layout conversion: free vertices from the caller array, Dirichlet vertices
// from the workspace's targets (or, with xd_int null, also from the caller)
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(kBlk) void k2_load(const R* x_user, const int* orig_of,
                                                const typename R2t<R>::T* xd_int, typename R2t<R>::T* d0,
                                                typename R2t<R>::T* d1, typename R2t<R>::T* d2, int n_free,
                                                int n_verts)
{
    const int v = blockIdx.x * kBlk + int(threadIdx.x);
    if (v >= n_verts) return;
    typename R2t<R>::T p;
    if (v < n_free || !xd_int) {
        const int o = orig_of[v];
        p.x = x_user[2 * int64_t(o)];
        p.y = x_user[2 * int64_t(o) + 1];
    } else {
        p = xd_int[v - n_free];
    }
    d0[v] = p;
    if (d1) d1[v] = p;
    if (d2) d2[v] = p;
}

template <class R>
__global__ __launch_bounds__(kBlk) void k2_store(const typename R2t<R>::T* src, const int* orig_of, R* x_user,
                                                 int n_verts)
{
    const int v = blockIdx.x * kBlk + int(threadIdx.x);
    if (v >= n_verts) return;
    const typename R2t<R>::T p = src[v];
    const int o = orig_of[v];
    x_user[2 * int64_t(o)] = p.x;
    x_user[2 * int64_t(o) + 1] = p.y;
}

}  // namespace

template <class R>
hipError_t launch_phase2(const Sweep2Args<R>& a, int model, int lanes, bool accel, bool safe, bool uniform,
                         int vbeg, int vend, hipStream_t s)
{
    if (uniform) {
        if (model == kPlanarNeo) return phase_lanes<R, kPlanarNeo, true>(a, lanes, accel, safe, vbeg, vend, s);
        return phase_lanes<R, kPlanarCor, true>(a, lanes, accel, safe, vbeg, vend, s);
    }
    if (model == kPlanarNeo) return phase_lanes<R, kPlanarNeo, false>(a, lanes, accel, safe, vbeg, vend, s);
    return phase_lanes<R, kPlanarCor, false>(a, lanes, accel, safe, vbeg, vend, s);
}

template <class R>
hipError_t launch_residual2(const Res2Args<R>& a, double* r_out, hipStream_t s)
{
    if (a.n_tris > 0) {
        if (a.model == kPlanarNeo)
            hipLaunchKernelGGL((k2_tri_stress<R, kPlanarNeo>), dim3(nblocks(a.n_tris)), dim3(kBlk), 0, s, a);
        else
            hipLaunchKernelGGL((k2_tri_stress<R, kPlanarCor>), dim3(nblocks(a.n_tris)), dim3(kBlk), 0, s, a);
    }
    if (a.n_verts > 0)
        hipLaunchKernelGGL((k2_vertex_residual<R>), dim3(nblocks(a.n_verts)), dim3(kBlk), 0, s, a, r_out);
    return hipGetLastError();
}

template <class R>
hipError_t launch_load2(const R* x_user, const int* orig_of, const typename R2t<R>::T* xd_int,
                        typename R2t<R>::T* d0, typename R2t<R>::T* d1, typename R2t<R>::T* d2, int n_free,
                        int n_verts, hipStream_t s)
{
    if (n_verts > 0)
        hipLaunchKernelGGL((k2_load<R>), dim3(nblocks(n_verts)), dim3(kBlk), 0, s, x_user, orig_of, xd_int, d0,
                           d1, d2, n_free, n_verts);
    return hipGetLastError();
}

template <class R>
hipError_t launch_store2(const typename R2t<R>::T* src, const int* orig_of, R* x_user, int n_verts,
                         hipStream_t s)
{
    if (n_verts > 0)
        hipLaunchKernelGGL((k2_store<R>), dim3(nblocks(n_verts)), dim3(kBlk), 0, s, src, orig_of, x_user,
                           n_verts);
    return hipGetLastError();
}

#define PBNG2D_INSTANTIATE(R)                                                                                  \
    template hipError_t launch_phase2<R>(const Sweep2Args<R>&, int, int, bool, bool, bool, int, int,          \
                                         hipStream_t);                                                        \
    template hipError_t launch_residual2<R>(const Res2Args<R>&, double*, hipStream_t);                       \
    template hipError_t launch_load2<R>(const R*, const int*, const R2t<R>::T*, R2t<R>::T*, R2t<R>::T*,       \
                                        R2t<R>::T*, int, int, hipStream_t);                                   \
    template hipError_t launch_store2<R>(const R2t<R>::T*, const int*, R*, int, hipStream_t);

PBNG2D_INSTANTIATE(float)
PBNG2D_INSTANTIATE(double)

}  // namespace pbng
