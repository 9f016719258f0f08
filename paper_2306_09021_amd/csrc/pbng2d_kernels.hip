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

// One visit of vertex i at position (xix, xiy): F = (x_j - x_i) dN_j^T +
// (x_k - x_i) dN_k^T, dN_i = -(dN_j + dN_k) and (A0 mu, A0 lambda).
template <class R>
struct Visit2 {
    R f00, f01, f10, f11, ax, ay, wm, wl;
};

template <class R, bool UNI>
__device__ __forceinline__ Visit2<R> visit2(const Sweep2Args<R>& a, int k, R xix, R xiy)
{
    using R2 = typename R2t<R>::T;
    Visit2<R> r;
    const int2 jk = at(a.jk, k);
    const auto g = at(a.gm, k);   // dN_j = (g.x, g.y), dN_k = (g.z, g.w)
    if constexpr (UNI) {
        const R A0 = R(0.5) / abs_(g.x * g.w - g.y * g.z);
        r.wm = a.mu_u * A0;
        r.wl = a.lam_u * A0;
    } else {
        const R2 w = at(a.vw, k);
        r.wm = w.x;
        r.wl = w.y;
    }
    const R2 xj = at(a.W, jk.x), xk = at(a.W, jk.y);
    const R e1x = xj.x - xix, e1y = xj.y - xiy;
    const R e2x = xk.x - xix, e2y = xk.y - xiy;
    r.f00 = e1x * g.x + e2x * g.z;
    r.f01 = e1x * g.y + e2x * g.w;
    r.f10 = e1y * g.x + e2y * g.z;
    r.f11 = e1y * g.y + e2y * g.w;
    r.ax = -(g.x + g.z);
    r.ay = -(g.y + g.w);
    return r;
}

// A0 Psi of Eq. (cor) with d = 2 for one visit.
template <class R>
__device__ __forceinline__ R cor_energy2(const Visit2<R>& q)
{
    R c, sn;
    rot2(q.f00, q.f01, q.f10, q.f11, c, sn);
    const R d00 = q.f00 - c, d01 = q.f01 + sn, d10 = q.f10 - sn, d11 = q.f11 - c;
    const R J = q.f00 * q.f11 - q.f01 * q.f10;
    return q.wm * (d00 * d00 + d01 * d01 + d10 * d10 + d11 * d11) + R(0.5) * q.wl * (J - R(1)) * (J - R(1));
}

// Penalty 1/2 k min(0, phi)^2 of half-plane q at (x, y).
template <class R>
__device__ __forceinline__ R plane_energy2(const Sweep2Args<R>& a, int q, R x, R y)
{
    const R phi = at(a.planes, 4 * q) * x + at(a.planes, 4 * q + 1) * y - at(a.planes, 4 * q + 2);
    return phi < R(0) ? R(0.5) * at(a.planes, 4 * q + 3) * phi * phi : R(0);
}

// EXTRA: the vertex's weak constraints (spread over the lanes like its
// visits), the half-planes and the inertia; each is an exact quadratic in
// x_i except the half-planes, which are evaluated exactly along the step.
template <class R, int MODEL, int LANES, bool ACCEL, bool SAFE, bool UNI, bool EXTRA>
__global__ __launch_bounds__(kBlk) void k2_phase(Sweep2Args<R> a, int vbeg, int vend)
{
    using R2 = typename R2t<R>::T;
    constexpr bool COR_EXACT = SAFE && EXTRA && MODEL == kPlanarCor;
    const int t = xcd_block() * kBlk + int(threadIdx.x);
    const int v = vbeg + t / LANES;
    const int lane = t & (LANES - 1);
    if (v >= vend) return;  // whole groups leave together (LANES divides 64)
    const R2 xi = at(a.W, v);
    const int kb = at(a.vptr, v), ke = at(a.vptr, v + 1);
    R gx = R(0), gy = R(0), s = R(0), lxx = R(0), lxy = R(0), lyy = R(0);
    R mxx = R(0), mxy = R(0), myy = R(0);
    R E0 = R(0), E0a = R(0);
    for (int k = kb + lane; k < ke; k += LANES) {
        const Visit2<R> q = visit2<R, UNI>(a, k, xi.x, xi.y);
        const R J = q.f00 * q.f11 - q.f01 * q.f10;
        // c = cof(F) dN_i with cof(F) = [[f11, -f10], [-f01, f00]]
        const R cx = q.f11 * q.ax - q.f10 * q.ay, cy = q.f00 * q.ay - q.f01 * q.ax;
        const R fax = q.f00 * q.ax + q.f01 * q.ay, fay = q.f10 * q.ax + q.f11 * q.ay;
        s += q.wm * (q.ax * q.ax + q.ay * q.ay);
        lxx += q.wl * cx * cx;
        lxy += q.wl * cx * cy;
        lyy += q.wl * cy * cy;
        if constexpr (MODEL == kPlanarNeo) {
            // A0 lhat (J - 1 - mu / lhat) = A0 lhat (J - 1) - A0 mu
            const R qq = (q.wm + q.wl) * (J - R(1)) - q.wm;
            gx += q.wm * fax + qq * cx;
            gy += q.wm * fay + qq * cy;
            if (SAFE) {
                mxx += q.wm * cx * cx;
                mxy += q.wm * cx * cy;
                myy += q.wm * cy * cy;
            }
        } else {
            R c, sn;
            rot2(q.f00, q.f01, q.f10, q.f11, c, sn);
            const R rax = c * q.ax - sn * q.ay, ray = sn * q.ax + c * q.ay;  // R dN_i
            const R qq = q.wl * (J - R(1));
            gx += R(2) * q.wm * (fax - rax) + qq * cx;
            gy += R(2) * q.wm * (fay - ray) + qq * cy;
            if constexpr (COR_EXACT) {
                const R e = cor_energy2(q);
                E0 += e;
                E0a += abs_(e);
            }
        }
    }
    // exact quadratic terms other than the elastic ones: gradient (qgx, qgy)
    // and Hessian (kxx, kxy, kyy)
    R qgx = R(0), qgy = R(0), kxx = R(0), kxy = R(0), kyy = R(0);
    if constexpr (EXTRA) {
        for (int k = at(a.wvptr, v) + lane; k < at(a.wvptr, v + 1); k += LANES) {
            const int c = at(a.wv_c, k);
            const R sc = at(a.wv_s, k);
            R Cx = R(0), Cy = R(0);
            for (int j = at(a.wc_ptr, c); j < at(a.wc_ptr, c + 1); ++j) {
                const R w = at(a.wc_w, j);
                const R2 p = at(a.W, at(a.wc_vert, j));
                Cx += w * p.x;
                Cy += w * p.y;
            }
            const R K0 = at(a.wc_K, 3 * c), K1 = at(a.wc_K, 3 * c + 1), K2 = at(a.wc_K, 3 * c + 2);
            qgx += sc * (K0 * Cx + K1 * Cy);
            qgy += sc * (K1 * Cx + K2 * Cy);
            kxx += sc * sc * K0;
            kxy += sc * sc * K1;
            kyy += sc * sc * K2;
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
        if (EXTRA) {
            qgx = lsum<LANES>(qgx);
            qgy = lsum<LANES>(qgy);
            kxx = lsum<LANES>(kxx);
            kxy = lsum<LANES>(kxy);
            kyy = lsum<LANES>(kyy);
        }
        if (COR_EXACT) {
            E0 = lsum<LANES>(E0);
            E0a = lsum<LANES>(E0a);
        }
    }
    if (EXTRA && a.inert) {
        // backward-Euler inertia 1/2 c |x_i - xhat_i|^2, c = m_ii / dt^2
        const R c = at(a.inert, v);
        const R2 xh = at(a.xhat, v);
        qgx += c * (xi.x - xh.x);
        qgy += c * (xi.y - xh.y);
        kxx += c;
        kyy += c;
    }
    const R2 f = at(a.fext, v);
    const R gtx = gx + qgx - f.x, gty = gy + qgy - f.y;
    R Axx = R(2) * s + lxx + kxx, Axy = lxy + kxy, Ayy = R(2) * s + lyy + kyy;
    R gsx = gtx, gsy = gty;  // with the active half-planes
    if constexpr (EXTRA) {
        for (int q = 0; q < a.n_planes; ++q) {
            const R nx = at(a.planes, 4 * q), ny = at(a.planes, 4 * q + 1), kp = at(a.planes, 4 * q + 3);
            const R phi = nx * xi.x + ny * xi.y - at(a.planes, 4 * q + 2);
            if (phi < R(0)) {
                gsx += kp * phi * nx;
                gsy += kp * phi * ny;
                Axx += kp * nx * nx;
                Axy += kp * nx * ny;
                Ayy += kp * ny * ny;
            }
        }
    }
    const R det = Axx * Ayy - Axy * Axy;
    bool reject = !(Axx > R(0) && det > R(0));
    R dx = R(0), dy = R(0), alpha = R(1);
    if (!reject) {
        const R id = R(1) / det;
        dx = -(Ayy * gsx - Axy * gsy) * id;
        dy = -(Axx * gsy - Axy * gsx) * id;
    }
    if (SAFE && !reject) {
        const R u = sizeof(R) == 8 ? R(1.1102230246251565e-16) : R(5.9604644775390625e-08);
        // change of the half-plane penalties when x_i moves by alpha d
        auto plane_change = [&](R al, R& dE, R& ab) {
            if constexpr (EXTRA) {
                for (int q = 0; q < a.n_planes; ++q) {
                    const R e0 = plane_energy2(a, q, xi.x, xi.y);
                    const R e1 = plane_energy2(a, q, xi.x + al * dx, xi.y + al * dy);
                    dE += e1 - e0;
                    ab += e0 + e1;
                }
            }
        };
        if constexpr (MODEL == kPlanarNeo) {
            // Along x_i + alpha d the Neo-Hookean local energy is exactly
            // E(0) + alpha g.d + alpha^2 / 2 d^T H d with
            // H = sum A0 (mu |dN_i|^2 I + lhat c c^T) (|F|^2 is quadratic and
            // det F affine in x_i) plus the exact quadratic terms; the
            // half-planes are evaluated exactly.
            const R hxx = s + lxx + mxx + kxx, hxy = lxy + mxy + kxy, hyy = s + lyy + myy + kyy;
            const R lin = gtx * dx + gty * dy;
            const R quad = dx * (hxx * dx + hxy * dy) + dy * (hxy * dx + hyy * dy);
            for (int h = 0;; ++h) {
                R dE = alpha * lin + R(0.5) * alpha * alpha * quad;
                R ab = abs_(alpha * lin) + abs_(R(0.5) * alpha * alpha * quad);
                plane_change(alpha, dE, ab);
                if (dE <= R(8) * u * ab) break;
                if (h >= a.max_halvings) {
                    reject = true;
                    break;
                }
                alpha *= R(0.5);
            }
        } else if constexpr (COR_EXACT) {
            // The corotated local energy is majorised by the quadratic with
            // gradient g and Hessian A (without the half-planes): mu
            // |F' - R(F')|^2 <= mu |F' - R(F)|^2.  Only a half-plane that
            // the step enters can raise the energy beyond it; when the bound
            // does not show a decrease, the energy is evaluated exactly.
            const R bl = gtx * dx + gty * dy;
            const R bxx = R(2) * s + lxx + kxx, bxy = lxy + kxy, byy = R(2) * s + lyy + kyy;
            const R bq = dx * (bxx * dx + bxy * dy) + dy * (bxy * dx + byy * dy);
            R dEb = bl + R(0.5) * bq, abb = abs_(bl) + abs_(R(0.5) * bq);
            for (int q = 0; q < a.n_planes; ++q) {
                const R nx = at(a.planes, 4 * q), ny = at(a.planes, 4 * q + 1), kp = at(a.planes, 4 * q + 3);
                const R phi0 = nx * xi.x + ny * xi.y - at(a.planes, 4 * q + 2);
                const R phi1 = phi0 + nx * dx + ny * dy;
                const R e0 = phi0 < R(0) ? R(0.5) * kp * phi0 * phi0 : R(0);
                const R e1 = phi1 < R(0) ? R(0.5) * kp * phi1 * phi1 : R(0);
                // an active half-plane is inside the quadratic already
                const R qpl = phi0 < R(0) ? R(0.5) * kp * (phi1 * phi1 - phi0 * phi0) : R(0);
                dEb += (e1 - e0) - qpl;
                abb += e0 + e1 + abs_(qpl);
            }
            if (!(dEb <= R(8) * u * abb)) {
                const R qlin = qgx * dx + qgy * dy;
                const R qquad = dx * (kxx * dx + kxy * dy) + dy * (kxy * dx + kyy * dy);
                const R flin = f.x * dx + f.y * dy;
                for (int h = 0;; ++h) {
                    R E1 = R(0), E1a = R(0);
                    for (int k = kb + lane; k < ke; k += LANES) {
                        const R e = cor_energy2(visit2<R, UNI>(a, k, xi.x + alpha * dx, xi.y + alpha * dy));
                        E1 += e;
                        E1a += abs_(e);
                    }
                    if (LANES > 1) {
                        E1 = lsum<LANES>(E1);
                        E1a = lsum<LANES>(E1a);
                    }
                    R dE = (E1 - E0) + alpha * (qlin - flin) + R(0.5) * alpha * alpha * qquad;
                    R ab = E0a + E1a + abs_(alpha * (qlin - flin)) + abs_(R(0.5) * alpha * alpha * qquad);
                    plane_change(alpha, dE, ab);
                    if (dE <= R(8) * u * ab) break;
                    if (h >= a.max_halvings) {
                        reject = true;
                        break;
                    }
                    alpha *= R(0.5);
                }
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

template <class R, int MODEL, int LANES, bool ACCEL, bool SAFE, bool UNI, bool EXTRA>
hipError_t phase_t(const Sweep2Args<R>& a, int vb, int ve, hipStream_t s)
{
    const int64_t threads = int64_t(ve - vb) * LANES;
    if (threads <= 0) return hipSuccess;
    hipLaunchKernelGGL((k2_phase<R, MODEL, LANES, ACCEL, SAFE, UNI, EXTRA>), dim3(nblocks(threads)), dim3(kBlk),
                       0, s, a, vb, ve);
    return hipGetLastError();
}

template <class R, int MODEL, int LANES, bool UNI, bool EXTRA>
hipError_t phase_flags(const Sweep2Args<R>& a, bool accel, bool safe, int vb, int ve, hipStream_t s)
{
    // the corotated full step never raises the local energy unless it
    // enters a half-plane: no safeguard without them
    if (MODEL == kPlanarCor && !(EXTRA && a.n_planes > 0)) safe = false;
    if (accel)
        return safe ? phase_t<R, MODEL, LANES, true, true, UNI, EXTRA>(a, vb, ve, s)
                    : phase_t<R, MODEL, LANES, true, false, UNI, EXTRA>(a, vb, ve, s);
    return safe ? phase_t<R, MODEL, LANES, false, true, UNI, EXTRA>(a, vb, ve, s)
                : phase_t<R, MODEL, LANES, false, false, UNI, EXTRA>(a, vb, ve, s);
}

template <class R, int MODEL, bool UNI, bool EXTRA>
hipError_t phase_lanes(const Sweep2Args<R>& a, int lanes, bool accel, bool safe, int vb, int ve, hipStream_t s)
{
    switch (lanes) {
    case 1: return phase_flags<R, MODEL, 1, UNI, EXTRA>(a, accel, safe, vb, ve, s);
    case 2: return phase_flags<R, MODEL, 2, UNI, EXTRA>(a, accel, safe, vb, ve, s);
    case 4: return phase_flags<R, MODEL, 4, UNI, EXTRA>(a, accel, safe, vb, ve, s);
    case 8: return phase_flags<R, MODEL, 8, UNI, EXTRA>(a, accel, safe, vb, ve, s);
    case 16: return phase_flags<R, MODEL, 16, UNI, EXTRA>(a, accel, safe, vb, ve, s);
    default: return hipErrorInvalidValue;
    }
}

template <class R, bool UNI, bool EXTRA>
hipError_t phase_models(const Sweep2Args<R>& a, int model, int lanes, bool accel, bool safe, int vb, int ve,
                        hipStream_t s)
{
    if (model == kPlanarNeo) return phase_lanes<R, kPlanarNeo, UNI, EXTRA>(a, lanes, accel, safe, vb, ve, s);
    return phase_lanes<R, kPlanarCor, UNI, EXTRA>(a, lanes, accel, safe, vb, ve, s);
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

// C_c = sum_j w_j x_{v_j} in FP64.
template <class R>
__device__ __forceinline__ double2 constraint_value2(const Res2Args<R>& a, int c)
{
    double2 C{0.0, 0.0};
    for (int j = a.wc_ptr[c]; j < a.wc_ptr[c + 1]; ++j) {
        const double2 p = x64(a.X[a.wc_vert[j]]);
        C.x += a.wc_w[j] * p.x;
        C.y += a.wc_w[j] * p.y;
    }
    return C;
}

// 1/2 C_c^T K_c C_c of every weak constraint into its energy slot.
template <class R>
__global__ __launch_bounds__(kBlk) void k2_wc_energy(Res2Args<R> a)
{
    const int c = blockIdx.x * kBlk + int(threadIdx.x);
    if (c >= a.n_wc) return;
    const double2 C = constraint_value2(a, c);
    const double* K = a.wc_K + 3 * int64_t(c);
    a.ebuf[a.n_tris + a.n_verts + c] = 0.5 * (K[0] * C.x * C.x + 2.0 * K[1] * C.x * C.y + K[2] * C.y * C.y);
}

template <class R>
__global__ __launch_bounds__(kBlk) void k2_vertex_residual(Res2Args<R> a, double* r_out)
{
    const int v = blockIdx.x * kBlk + int(threadIdx.x);
    if (v >= a.n_verts) return;
    const double2 xi = x64(a.X[v]);
    const double fx = a.fext64[2 * v], fy = a.fext64[2 * v + 1];
    double rx = 0.0, ry = 0.0, E = -(xi.x * fx + xi.y * fy);
    // half-plane penalties on every vertex
    double px = 0.0, py = 0.0;
    for (int q = 0; q < a.n_planes; ++q) {
        const double* pl = a.planes + 4 * q;
        const double phi = pl[0] * xi.x + pl[1] * xi.y - pl[2];
        if (phi < 0.0) {
            E += 0.5 * pl[3] * phi * phi;
            px += pl[3] * phi * pl[0];
            py += pl[3] * phi * pl[1];
        }
    }
    if (v < a.n_free) {
        rx = fx - px;
        ry = fy - py;
        for (int k = a.rvptr[v]; k < a.rvptr[v + 1]; ++k) {
            const double* p = a.vp + 2 * int64_t(a.rv[k]);
            rx -= p[0];
            ry -= p[1];
        }
        if (a.n_wc > 0)
            for (int k = a.wvptr[v]; k < a.wvptr[v + 1]; ++k) {
                const int c = a.wv_c[k];
                const double2 C = constraint_value2(a, c);
                const double* K = a.wc_K + 3 * int64_t(c);
                rx -= a.wv_s[k] * (K[0] * C.x + K[1] * C.y);
                ry -= a.wv_s[k] * (K[1] * C.x + K[2] * C.y);
            }
        if (a.inert) {
            const double c = a.inert[v];
            const double dx = xi.x - a.xhat[2 * v], dy = xi.y - a.xhat[2 * v + 1];
            E += 0.5 * c * (dx * dx + dy * dy);
            rx -= c * dx;
            ry -= c * dy;
        }
    }
    a.ebuf[a.n_tris + v] = E;
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

// ---------------------------------------------------------------------------
// Adjoint: block Gauss-Seidel on H lam = b, FP64 residual and gradients
// ---------------------------------------------------------------------------
// dP[Lam] for d = 2, scaled by the rest area through wm = A0 mu and
// wl = A0 lambda (cof is linear in F here: dcof[Lam] = cof Lam):
//   Neo-Hookean: wm Lam + lh (C:Lam) C + (lh (J - 1) - wm) cof Lam, lh = wm + wl
//   corotated:   2 wm (Lam - dR[Lam]) + wl (C:Lam) C + wl (J - 1) cof Lam,
// C = cof F, dR = dtheta [[-s, -c], [c, -s]] at the rotation angle theta of
// (a, b) = (F00 + F11, F10 - F01), dtheta = (a db - b da) / (a^2 + b^2).
template <class R, int MODEL>
__device__ __forceinline__ void stress_diff2(R f00, R f01, R f10, R f11, R l00, R l01, R l10, R l11, R wm, R wl,
                                             R& d00, R& d01, R& d10, R& d11)
{
    const R J = f00 * f11 - f01 * f10;
    const R cl = f11 * l00 - f10 * l01 - f01 * l10 + f00 * l11;   // C : Lam
    if constexpr (MODEL == kPlanarNeo) {
        const R lh = wm + wl, q = lh * (J - R(1)) - wm, p = lh * cl;
        d00 = wm * l00 + p * f11 + q * l11;
        d01 = wm * l01 - p * f10 - q * l10;
        d10 = wm * l10 - p * f01 - q * l01;
        d11 = wm * l11 + p * f00 + q * l00;
    } else {
        const R a = f00 + f11, b = f10 - f01, r2 = a * a + b * b;
        R c, sn;
        rot2(f00, f01, f10, f11, c, sn);
        const R dth = r2 > R(0) ? (a * (l10 - l01) - b * (l00 + l11)) / r2 : R(0);
        const R q = wl * (J - R(1)), p = wl * cl, m2 = R(2) * wm;
        d00 = m2 * (l00 + sn * dth) + p * f11 + q * l11;
        d01 = m2 * (l01 + c * dth) - p * f10 - q * l10;
        d10 = m2 * (l10 - c * dth) - p * f01 - q * l01;
        d11 = m2 * (l11 + sn * dth) + p * f00 + q * l00;
    }
}

// One block Gauss-Seidel update of lam_i: r_i = b_i - (H lam)_i with the
// current lam, lam_i += D_i^{-1} r_i, D_i the true diagonal block for
// Neo-Hookean (sum A0 (mu |dN_i|^2 I + lhat c c^T): in 2-D the cofactor
// term of H_ii vanishes) and the modified A_i for corotated, plus s^2 K,
// the active half-planes' k n n^T and the inertia.
template <class R, int MODEL, int LANES, bool ACCEL, bool UNI, bool EXTRA>
__global__ __launch_bounds__(kBlk) void k2_adj_phase(Adj2Args<R> a, int vbeg, int vend)
{
    using R2 = typename R2t<R>::T;
    const int t = xcd_block() * kBlk + int(threadIdx.x);
    const int v = vbeg + t / LANES;
    const int lane = t & (LANES - 1);
    if (v >= vend) return;
    const R2 xi = at(a.X, v), li = at(a.L, v);
    const int kb = at(a.vptr, v), ke = at(a.vptr, v + 1);
    R hx = R(0), hy = R(0), dxx = R(0), dxy = R(0), dyy = R(0);
    for (int k = kb + lane; k < ke; k += LANES) {
        const int2 jk = at(a.jk, k);
        const auto g = at(a.gm, k);
        R wm, wl;
        if constexpr (UNI) {
            const R A0 = R(0.5) / abs_(g.x * g.w - g.y * g.z);
            wm = a.mu_u * A0;
            wl = a.lam_u * A0;
        } else {
            const R2 w = at(a.vw, k);
            wm = w.x;
            wl = w.y;
        }
        const R2 xj = at(a.X, jk.x), xk = at(a.X, jk.y);
        const R2 lj = at(a.L, jk.x), lk = at(a.L, jk.y);
        const R e1x = xj.x - xi.x, e1y = xj.y - xi.y, e2x = xk.x - xi.x, e2y = xk.y - xi.y;
        const R f00 = e1x * g.x + e2x * g.z, f01 = e1x * g.y + e2x * g.w;
        const R f10 = e1y * g.x + e2y * g.z, f11 = e1y * g.y + e2y * g.w;
        const R m1x = lj.x - li.x, m1y = lj.y - li.y, m2x = lk.x - li.x, m2y = lk.y - li.y;
        const R l00 = m1x * g.x + m2x * g.z, l01 = m1x * g.y + m2x * g.w;
        const R l10 = m1y * g.x + m2y * g.z, l11 = m1y * g.y + m2y * g.w;
        const R ax = -(g.x + g.z), ay = -(g.y + g.w);
        R d00, d01, d10, d11;
        stress_diff2<R, MODEL>(f00, f01, f10, f11, l00, l01, l10, l11, wm, wl, d00, d01, d10, d11);
        hx += d00 * ax + d01 * ay;
        hy += d10 * ax + d11 * ay;
        const R cx = f11 * ax - f10 * ay, cy = f00 * ay - f01 * ax, sa = ax * ax + ay * ay;
        if constexpr (MODEL == kPlanarNeo) {
            const R lh = wm + wl;
            dxx += wm * sa + lh * cx * cx;
            dxy += lh * cx * cy;
            dyy += wm * sa + lh * cy * cy;
        } else {
            dxx += R(2) * wm * sa + wl * cx * cx;
            dxy += wl * cx * cy;
            dyy += R(2) * wm * sa + wl * cy * cy;
        }
    }
    if constexpr (EXTRA) {
        for (int k = at(a.wvptr, v) + lane; k < at(a.wvptr, v + 1); k += LANES) {
            const int c = at(a.wv_c, k);
            const R sc = at(a.wv_s, k);
            R Cx = R(0), Cy = R(0);
            for (int j = at(a.wc_ptr, c); j < at(a.wc_ptr, c + 1); ++j) {
                const R w = at(a.wc_w, j);
                const R2 p = at(a.L, at(a.wc_vert, j));
                Cx += w * p.x;
                Cy += w * p.y;
            }
            const R K0 = at(a.wc_K, 3 * c), K1 = at(a.wc_K, 3 * c + 1), K2 = at(a.wc_K, 3 * c + 2);
            hx += sc * (K0 * Cx + K1 * Cy);
            hy += sc * (K1 * Cx + K2 * Cy);
            dxx += sc * sc * K0;
            dxy += sc * sc * K1;
            dyy += sc * sc * K2;
        }
    }
    if (LANES > 1) {
        hx = lsum<LANES>(hx);
        hy = lsum<LANES>(hy);
        dxx = lsum<LANES>(dxx);
        dxy = lsum<LANES>(dxy);
        dyy = lsum<LANES>(dyy);
    }
    if constexpr (EXTRA) {
        for (int q = 0; q < a.n_planes; ++q) {
            const R nx = at(a.planes, 4 * q), ny = at(a.planes, 4 * q + 1), kp = at(a.planes, 4 * q + 3);
            if (nx * xi.x + ny * xi.y - at(a.planes, 4 * q + 2) < R(0)) {
                const R nl = kp * (nx * li.x + ny * li.y);
                hx += nl * nx;
                hy += nl * ny;
                dxx += kp * nx * nx;
                dxy += kp * nx * ny;
                dyy += kp * ny * ny;
            }
        }
        if (a.inert) {
            const R c = at(a.inert, v);
            hx += c * li.x;
            hy += c * li.y;
            dxx += c;
            dyy += c;
        }
    }
    if (lane != 0) return;
    const R2 b = at(a.B, v);
    const R rx = b.x - hx, ry = b.y - hy;
    const R det = dxx * dyy - dxy * dxy;
    R2 ln = li;
    if (dxx > R(0) && det > R(0)) {
        const R id = R(1) / det;
        ln.x = li.x + (dyy * rx - dxy * ry) * id;
        ln.y = li.y + (dxx * ry - dxy * rx) * id;
    }
    if (ACCEL) {
        const R2 lp = at(a.P, v);
        R2 bl;
        bl.x = a.omega * (a.gamma * (ln.x - li.x) + li.x - lp.x) + lp.x;
        bl.y = a.omega * (a.gamma * (ln.y - li.y) + li.y - lp.y) + lp.y;
        *ptr_at(a.L, v) = ln;
        *ptr_at(a.P, v) = li;
        *ptr_at(a.N, v) = bl;
    } else {
        *ptr_at(a.L, v) = ln;
    }
}

// FP64: per triangle the slot terms A0 dP[Lam_e] dN_j, and the gradients
// dL/dmu_e = -A0 <dP/dmu, Lam_e> (dP/dmu = F + (J - 2) C for Neo-Hookean,
// 2 (F - R) for corotated) and dL/dlambda_e = -A0 (J - 1) <C, Lam_e>.
template <class R, int MODEL>
__global__ __launch_bounds__(kBlk) void k2_tri_adjoint(Res2Args<R> a, const typename R2t<R>::T* L, double* dmu,
                                                       double* dlam)
{
    const int e = blockIdx.x * kBlk + int(threadIdx.x);
    if (e >= a.n_tris) return;
    const int4 t = a.tri[e];
    const TriGeo G = a.geo[e];
    const double2 x0 = x64(a.X[t.x]), x1 = x64(a.X[t.y]), x2 = x64(a.X[t.z]);
    const double2 l0 = x64(L[t.x]), l1 = x64(L[t.y]), l2 = x64(L[t.z]);
    const double e1x = x1.x - x0.x, e1y = x1.y - x0.y, e2x = x2.x - x0.x, e2y = x2.y - x0.y;
    const double f00 = e1x * G.g1x + e2x * G.g2x, f01 = e1x * G.g1y + e2x * G.g2y;
    const double f10 = e1y * G.g1x + e2y * G.g2x, f11 = e1y * G.g1y + e2y * G.g2y;
    const double m1x = l1.x - l0.x, m1y = l1.y - l0.y, m2x = l2.x - l0.x, m2y = l2.y - l0.y;
    const double l00 = m1x * G.g1x + m2x * G.g2x, l01 = m1x * G.g1y + m2x * G.g2y;
    const double l10 = m1y * G.g1x + m2y * G.g2x, l11 = m1y * G.g1y + m2y * G.g2y;
    double d00, d01, d10, d11;
    stress_diff2<double, MODEL>(f00, f01, f10, f11, l00, l01, l10, l11, G.A0 * G.mu, G.A0 * G.lam, d00, d01,
                                d10, d11);
    const double gx[3] = {-(G.g1x + G.g2x), G.g1x, G.g2x};
    const double gy[3] = {-(G.g1y + G.g2y), G.g1y, G.g2y};
    double* o = a.vp + 6 * int64_t(e);
    for (int j = 0; j < 3; ++j) {
        o[2 * j] = d00 * gx[j] + d01 * gy[j];
        o[2 * j + 1] = d10 * gx[j] + d11 * gy[j];
    }
    const double J = f00 * f11 - f01 * f10;
    const double CL = f11 * l00 - f10 * l01 - f01 * l10 + f00 * l11;
    const double FL = f00 * l00 + f01 * l01 + f10 * l10 + f11 * l11;
    if (dmu) {
        double dPdmu;
        if constexpr (MODEL == kPlanarNeo) {
            dPdmu = FL + (J - 2.0) * CL;
        } else {
            double c, sn;
            rot2(f00, f01, f10, f11, c, sn);
            dPdmu = 2.0 * (FL - (c * l00 - sn * l01 + sn * l10 + c * l11));
        }
        dmu[e] = -G.A0 * dPdmu;
    }
    if (dlam) dlam[e] = -G.A0 * (J - 1.0) * CL;
}

template <class R>
__global__ __launch_bounds__(kBlk) void k2_vertex_adjoint(Res2Args<R> a, const typename R2t<R>::T* L,
                                                          const typename R2t<R>::T* B, double* dxd,
                                                          const int* dir_pos)
{
    const int v = blockIdx.x * kBlk + int(threadIdx.x);
    if (v >= a.n_verts) return;
    double hx = 0.0, hy = 0.0;
    for (int k = a.rvptr[v]; k < a.rvptr[v + 1]; ++k) {
        const double* p = a.vp + 2 * int64_t(a.rv[k]);
        hx += p[0];
        hy += p[1];
    }
    if (a.n_wc > 0)
        for (int k = a.wvptr[v]; k < a.wvptr[v + 1]; ++k) {
            const int c = a.wv_c[k];
            double Cx = 0.0, Cy = 0.0;
            for (int j = a.wc_ptr[c]; j < a.wc_ptr[c + 1]; ++j) {
                const double2 p = x64(L[a.wc_vert[j]]);
                Cx += a.wc_w[j] * p.x;
                Cy += a.wc_w[j] * p.y;
            }
            const double* K = a.wc_K + 3 * int64_t(c);
            hx += a.wv_s[k] * (K[0] * Cx + K[1] * Cy);
            hy += a.wv_s[k] * (K[1] * Cx + K[2] * Cy);
        }
    const double2 b = x64(B[v]);
    if (v < a.n_free) {
        const double2 xi = x64(a.X[v]), li = x64(L[v]);
        for (int q = 0; q < a.n_planes; ++q) {
            const double* pl = a.planes + 4 * q;
            if (pl[0] * xi.x + pl[1] * xi.y - pl[2] < 0.0) {
                const double nl = pl[3] * (pl[0] * li.x + pl[1] * li.y);
                hx += nl * pl[0];
                hy += nl * pl[1];
            }
        }
        if (a.inert) {
            hx += a.inert[v] * li.x;
            hy += a.inert[v] * li.y;
        }
        a.rsq[v] = (b.x - hx) * (b.x - hx) + (b.y - hy) * (b.y - hy);
    } else {
        a.rsq[v] = 0.0;
        if (dxd) {
            const int pos = dir_pos[v - a.n_free];
            dxd[2 * int64_t(pos)] = b.x - hx;
            dxd[2 * int64_t(pos) + 1] = b.y - hy;
        }
    }
}

template <class R>
__global__ __launch_bounds__(kBlk) void k2_store64(const typename R2t<R>::T* src, const int* orig_of, double* out,
                                                   int n_verts)
{
    const int v = blockIdx.x * kBlk + int(threadIdx.x);
    if (v >= n_verts) return;
    const int64_t o = orig_of[v];
    out[2 * o] = double(src[v].x);
    out[2 * o + 1] = double(src[v].y);
}

template <class R, int MODEL, int LANES, bool UNI, bool EXTRA>
hipError_t adj_t(const Adj2Args<R>& a, bool accel, int vb, int ve, hipStream_t s)
{
    const int64_t threads = int64_t(ve - vb) * LANES;
    if (threads <= 0) return hipSuccess;
    if (accel)
        hipLaunchKernelGGL((k2_adj_phase<R, MODEL, LANES, true, UNI, EXTRA>), dim3(nblocks(threads)), dim3(kBlk),
                           0, s, a, vb, ve);
    else
        hipLaunchKernelGGL((k2_adj_phase<R, MODEL, LANES, false, UNI, EXTRA>), dim3(nblocks(threads)),
                           dim3(kBlk), 0, s, a, vb, ve);
    return hipGetLastError();
}

template <class R, int MODEL, bool UNI, bool EXTRA>
hipError_t adj_lanes(const Adj2Args<R>& a, int lanes, bool accel, int vb, int ve, hipStream_t s)
{
    switch (lanes) {
    case 1: return adj_t<R, MODEL, 1, UNI, EXTRA>(a, accel, vb, ve, s);
    case 2: return adj_t<R, MODEL, 2, UNI, EXTRA>(a, accel, vb, ve, s);
    case 4: return adj_t<R, MODEL, 4, UNI, EXTRA>(a, accel, vb, ve, s);
    case 8: return adj_t<R, MODEL, 8, UNI, EXTRA>(a, accel, vb, ve, s);
    case 16: return adj_t<R, MODEL, 16, UNI, EXTRA>(a, accel, vb, ve, s);
    default: return hipErrorInvalidValue;
    }
}

template <class R, bool UNI, bool EXTRA>
hipError_t adj_models(const Adj2Args<R>& a, int model, int lanes, bool accel, int vb, int ve, hipStream_t s)
{
    if (model == kPlanarNeo) return adj_lanes<R, kPlanarNeo, UNI, EXTRA>(a, lanes, accel, vb, ve, s);
    return adj_lanes<R, kPlanarCor, UNI, EXTRA>(a, lanes, accel, vb, ve, s);
}

template <class R>
__global__ __launch_bounds__(kBlk) void k2_xhat(const double* x_n, const double* x_prev, const int* orig_of,
                                                double* xhat64, typename R2t<R>::T* xhat, int n_free)
{
    const int v = blockIdx.x * kBlk + int(threadIdx.x);
    if (v >= n_free) return;
    const int64_t o = orig_of[v];
    const double hx = 2.0 * x_n[2 * o] - x_prev[2 * o], hy = 2.0 * x_n[2 * o + 1] - x_prev[2 * o + 1];
    xhat64[2 * int64_t(v)] = hx;
    xhat64[2 * int64_t(v) + 1] = hy;
    typename R2t<R>::T h;
    h.x = R(hx);
    h.y = R(hy);
    xhat[v] = h;
}

}  // namespace

template <class R>
hipError_t launch_xhat2(const double* x_n, const double* x_prev, const int* orig_of, double* xhat64,
                        typename R2t<R>::T* xhat, int n_free, hipStream_t s)
{
    if (n_free > 0)
        hipLaunchKernelGGL((k2_xhat<R>), dim3(nblocks(n_free)), dim3(kBlk), 0, s, x_n, x_prev, orig_of, xhat64,
                           xhat, n_free);
    return hipGetLastError();
}

template <class R>
hipError_t launch_adj_phase2(const Adj2Args<R>& a, int model, int lanes, bool accel, bool uniform, bool extra,
                             int vbeg, int vend, hipStream_t s)
{
    if (extra)
        return uniform ? adj_models<R, true, true>(a, model, lanes, accel, vbeg, vend, s)
                       : adj_models<R, false, true>(a, model, lanes, accel, vbeg, vend, s);
    return uniform ? adj_models<R, true, false>(a, model, lanes, accel, vbeg, vend, s)
                   : adj_models<R, false, false>(a, model, lanes, accel, vbeg, vend, s);
}

template <class R>
hipError_t launch_adjoint_residual2(const Res2Args<R>& a, const typename R2t<R>::T* L,
                                    const typename R2t<R>::T* B, double* dmu, double* dlam, double* dxd,
                                    const int* dir_pos, hipStream_t s)
{
    if (a.n_tris > 0) {
        if (a.model == kPlanarNeo)
            hipLaunchKernelGGL((k2_tri_adjoint<R, kPlanarNeo>), dim3(nblocks(a.n_tris)), dim3(kBlk), 0, s, a, L,
                               dmu, dlam);
        else
            hipLaunchKernelGGL((k2_tri_adjoint<R, kPlanarCor>), dim3(nblocks(a.n_tris)), dim3(kBlk), 0, s, a, L,
                               dmu, dlam);
    }
    if (a.n_verts > 0)
        hipLaunchKernelGGL((k2_vertex_adjoint<R>), dim3(nblocks(a.n_verts)), dim3(kBlk), 0, s, a, L, B, dxd,
                           dir_pos);
    return hipGetLastError();
}

template <class R>
hipError_t launch_store2_f64(const typename R2t<R>::T* src, const int* orig_of, double* out, int n_verts,
                             hipStream_t s)
{
    if (n_verts > 0)
        hipLaunchKernelGGL((k2_store64<R>), dim3(nblocks(n_verts)), dim3(kBlk), 0, s, src, orig_of, out, n_verts);
    return hipGetLastError();
}

template <class R>
hipError_t launch_phase2(const Sweep2Args<R>& a, int model, int lanes, bool accel, bool safe, bool uniform,
                         bool extra, int vbeg, int vend, hipStream_t s)
{
    if (extra)
        return uniform ? phase_models<R, true, true>(a, model, lanes, accel, safe, vbeg, vend, s)
                       : phase_models<R, false, true>(a, model, lanes, accel, safe, vbeg, vend, s);
    return uniform ? phase_models<R, true, false>(a, model, lanes, accel, safe, vbeg, vend, s)
                   : phase_models<R, false, false>(a, model, lanes, accel, safe, vbeg, vend, s);
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
    if (a.n_wc > 0) hipLaunchKernelGGL((k2_wc_energy<R>), dim3(nblocks(a.n_wc)), dim3(kBlk), 0, s, a);
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
    template hipError_t launch_phase2<R>(const Sweep2Args<R>&, int, int, bool, bool, bool, bool, int, int,    \
                                         hipStream_t);                                                        \
    template hipError_t launch_residual2<R>(const Res2Args<R>&, double*, hipStream_t);                       \
    template hipError_t launch_load2<R>(const R*, const int*, const R2t<R>::T*, R2t<R>::T*, R2t<R>::T*,       \
                                        R2t<R>::T*, int, int, hipStream_t);                                   \
    template hipError_t launch_store2<R>(const R2t<R>::T*, const int*, R*, int, hipStream_t);                \
    template hipError_t launch_xhat2<R>(const double*, const double*, const int*, double*, R2t<R>::T*, int,  \
                                        hipStream_t);                                                         \
    template hipError_t launch_adj_phase2<R>(const Adj2Args<R>&, int, int, bool, bool, bool, int, int,        \
                                             hipStream_t);                                                    \
    template hipError_t launch_adjoint_residual2<R>(const Res2Args<R>&, const R2t<R>::T*, const R2t<R>::T*,   \
                                                    double*, double*, double*, const int*, hipStream_t);      \
    template hipError_t launch_store2_f64<R>(const R2t<R>::T*, const int*, double*, int, hipStream_t);

PBNG2D_INSTANTIATE(float)
PBNG2D_INSTANTIATE(double)

}  // namespace pbng
