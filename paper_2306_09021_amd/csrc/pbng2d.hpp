// Internal layout of a planar (triangle-mesh) libpbng workspace and its
// kernel launchers.
//
// Vertex order on the device: free vertices first, grouped by colour, inside
// a colour by decreasing valence (incident triangles) and then by caller
// index; Dirichlet vertices follow in caller order.  Positions are R2
// (float2 / double2) in that order.
//
// Per-visit records (one per (free vertex i, incident triangle e), CSR by
// internal vertex through vptr), three packed streams indexed by visit k:
//   jk[k] = {j, k}            internal indices of the other two vertices
//   gm[k] = {dN_j, dN_k}      their rest-state shape-function gradients, so
//                             that F = (x_j - x_i) dN_j^T + (x_k - x_i) dN_k^T
//                             and dN_i = -(dN_j + dN_k)
//   vw[k] = {A0 mu, A0 lambda}
// 8 + 16 + 8 = 32 bytes per visit in float.  When every triangle has the
// same (mu, lambda) the workspace omits vw (24 bytes per visit): the rest
// area follows from the stored gradients, det[dN_j; dN_k] = 1 / (2 A0) for
// the cyclic pair (j, k) after i, and mu, lambda are kernel arguments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pbng_internal.hpp"

namespace pbng {

constexpr int kPlanarNeo = 0;
constexpr int kPlanarCor = 1;

// FP64 geometry of a triangle: rows dN_1, dN_2 of Dm^{-1}, rest area, Lame
// parameters.
struct TriGeo {
    double g1x, g1y, g2x, g2y;
    double A0, mu, lam;
};

template <class R>
struct Sweep2Args {
    using R2 = typename R2t<R>::T;
    using R4 = typename R4t<R>::T;
    R2* W;                  // working iterate (Gauss-Seidel, in place)
    R2* P;                  // x^{l-1}                (acceleration only)
    R2* N;                  // x^{l+1} being blended  (acceleration only)
    const int* vptr;        // [n_free + 1]
    const int2* jk;         // [n_visits]
    const R4* gm;
    const R2* vw;           // null with uniform materials
    const R2* fext;         // [n_free] lumped external force
    R mu_u, lam_u;          // the uniform (mu, lambda) when vw is null
    int* rejected;          // [1]
    R omega, gamma;
    int max_halvings;
    // weak constraints, contact half-planes and inertia (EXTRA kernels)
    const int* wvptr;       // [n_free + 1] constraints of each free vertex
    const int* wv_c;        // constraint index
    const R* wv_s;          // weight of the vertex in that constraint
    const int* wc_ptr;      // [n_wc + 1]
    const int* wc_vert;     // internal vertex indices
    const R* wc_w;
    const R* wc_K;          // [n_wc][3] (xx, xy, yy)
    const R* planes;        // [n_planes][4] (n_x, n_y, d, k)
    int n_planes;
    const R* inert;         // [n_free] m_ii / dt^2, or null
    const R2* xhat;         // [n_free] 2 x^n - x^{n-1}
};

// Adjoint (block Gauss-Seidel on H lam = b over the same colours): X the
// equilibrium, L the iterate (zero on Dirichlet rows), P / N the previous
// and blended iterates with the Chebyshev blend.  The visit, constraint,
// half-plane and inertia data are those of the sweep.
template <class R>
struct Adj2Args {
    using R2 = typename R2t<R>::T;
    using R4 = typename R4t<R>::T;
    const R2* X;
    R2* L;
    R2* P;
    R2* N;
    const R2* B;            // dL/dx, internal order
    const int* vptr;
    const int2* jk;
    const R4* gm;
    const R2* vw;           // null with uniform materials
    R mu_u, lam_u;
    const int* wvptr;
    const int* wv_c;
    const R* wv_s;
    const int* wc_ptr;
    const int* wc_vert;
    const R* wc_w;
    const R* wc_K;
    const R* planes;
    int n_planes;
    const R* inert;         // or null
    R omega, gamma;
};

// FP64 residual / energy: per triangle A0 P dN_j (vp) and A0 Psi, per
// vertex the force balance, -x . fhat, the half-plane penalties and the
// inertia, per weak constraint its energy.
template <class R>
struct Res2Args {
    using R2 = typename R2t<R>::T;
    const R2* X;            // internal order
    const int4* tri;        // [n_tris] internal vertex indices (w unused)
    const TriGeo* geo;
    double* vp;             // [n_tris][3][2]
    double* ebuf;           // [n_tris + n_verts + n_wc] energy summands
    const int* rvptr;       // [n_verts + 1] triangle slots of every vertex
    const int* rv;          // tri * 3 + slot
    const double* fext64;   // [n_verts][2] internal order
    const int* orig_of;     // [n_verts]
    double* rsq;            // [n_verts] squared residual per vertex
    int n_free, n_verts, n_tris, model;
    // weak constraints (ebuf[n_tris + n_verts + c] takes 1/2 C^T K C),
    // half-planes (every vertex) and inertia (free vertices, or null)
    const int* wvptr;       // [n_free + 1]
    const int* wv_c;
    const double* wv_s;
    const int* wc_ptr;      // [n_wc + 1]
    const int* wc_vert;     // internal
    const double* wc_w;
    const double* wc_K;     // [n_wc][3]
    int n_wc;
    const double* planes;   // [n_planes][4]
    int n_planes;
    const double* inert;    // [n_free] m_ii / dt^2, or null
    const double* xhat;     // [n_free][2]
};

// uniform: the 24-byte record form (a.vw null, a.mu_u / a.lam_u set);
// extra: weak constraints, half-planes or inertia present
template <class R>
hipError_t launch_phase2(const Sweep2Args<R>& a, int model, int lanes, bool accel, bool safe, bool uniform,
                         bool extra, int vbeg, int vend, hipStream_t s);
template <class R>
hipError_t launch_residual2(const Res2Args<R>& a, double* r_out, hipStream_t s);
template <class R>
hipError_t launch_adj_phase2(const Adj2Args<R>& a, int model, int lanes, bool accel, bool uniform, bool extra,
                             int vbeg, int vend, hipStream_t s);
// FP64 adjoint residual: vp <- A0 dP[Lam_e] dN_j per triangle (with
// dL/dmu_e, dL/dlambda_e when dmu / dlam are non-null), then per vertex
// H lam from its slots, constraints, half-planes and inertia; rsq[v] =
// |b_v - (H lam)_v|^2 on free rows, dxd[dir_pos[v - n_free]] = b_v -
// (H lam)_v on Dirichlet rows (dxd may be null).  The slots of every
// vertex (rvptr / rv) and the constraint CSR (wvptr) cover all vertices.
template <class R>
hipError_t launch_adjoint_residual2(const Res2Args<R>& a, const typename R2t<R>::T* L,
                                    const typename R2t<R>::T* B, double* dmu, double* dlam, double* dxd,
                                    const int* dir_pos, hipStream_t s);
// lam_out (caller order, double [n_verts][2]) from an internal iterate
template <class R>
hipError_t launch_store2_f64(const typename R2t<R>::T* src, const int* orig_of, double* out, int n_verts,
                             hipStream_t s);
template <class R>
hipError_t launch_load2(const R* x_user, const int* orig_of, const typename R2t<R>::T* xd_int,
                        typename R2t<R>::T* d0, typename R2t<R>::T* d1, typename R2t<R>::T* d2, int n_free,
                        int n_verts, hipStream_t s);
// xhat = 2 x^n - x^{n-1} of the free vertices (internal order) from caller
// order FP64 arrays, in FP64 and in the sweep precision
template <class R>
hipError_t launch_xhat2(const double* x_n, const double* x_prev, const int* orig_of, double* xhat64,
                        typename R2t<R>::T* xhat, int n_free, hipStream_t s);
template <class R>
hipError_t launch_store2(const typename R2t<R>::T* src, const int* orig_of, R* x_user, int n_verts,
                         hipStream_t s);

}  // namespace pbng
