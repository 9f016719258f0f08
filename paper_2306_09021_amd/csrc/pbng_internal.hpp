// Internal layout of a libpbng workspace and the kernel launchers.
//
// Vertex order on the device ("internal order"): all free vertices first,
// grouped by colour; inside a colour by instance, then by decreasing
// valence (number of incident tets), then by caller index.  Dirichlet
// vertices follow.  Same-coloured vertices share no tet or weak constraint,
// so the order inside a colour does not change any computed value.
//
// Per-visit records (one per (free vertex i, incident tet e) pair, CSR by
// internal vertex through vptr) are four packed streams indexed by visit k,
// so that a wave reads each stream with one wide, coalesced load per lane:
//   jv[k] = {j1, j2, j3, w}   internal indices of the other three vertices of
//                              e; in FP32 workspaces w holds the bits of V0 mu
//   ma[k] = {m0, m1, m2, m3}  m[9]: rows dN_j1, dN_j2, dN_j3 of the rest-state
//   mb[k] = {m4, m5, m6, m7}  shape-function gradients (so that
//   mc[k] = {m8, V0 lambda}   F = sum (x_j - x_i) dN_j^T)
//   vmu[k] = V0 mu             FP64 workspaces only
// In float: 16 + 16 + 16 + 8 = 56 bytes per visit.  Neo-Hookean workspaces
// store cof(M) dN_i and det M instead of m[9] (48 bytes), or, when every tet
// of an instance has the same (mu, lambda), V0 alpha, beta and delta (40
// bytes: jv, ma and mc, with delta in jv.w or vmu).  Kernels address every
// stream with 32-bit byte offsets; the host rejects workspaces whose streams
// exceed 4 GiB.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pbng {

template <class R>
struct R4t;
template <>
struct R4t<float> {
    using T = float4;
};
template <>
struct R4t<double> {
    using T = double4;
};
template <class R>
struct R2t;
template <>
struct R2t<float> {
    using T = float2;
};
template <>
struct R2t<double> {
    using T = double2;
};

// Geometry of a tet for the FP64 passes: Dm^{-1} (row-major), V0, mu, lambda.
struct TetGeo {
    double dm[9];
    double V0, mu, lam;
};

// R: arithmetic type of the sweep; PR: type of the stored positions (PR =
// double with R = float keeps an FP64 master copy of the iterate).
template <class R, class PR = R>
struct SweepArgs {
    using R4 = typename R4t<R>::T;
    using P4 = typename R4t<PR>::T;
    P4* W;                 // working iterate (Gauss-Seidel, in place)
    P4* P;                 // x^{l-1}                (acceleration only)
    P4* N;                 // x^{l+1} being blended  (acceleration only)
    using R2 = typename R2t<R>::T;
    const int* vptr;       // [n_free + 1]
    const int4* jv;        // [n_visits] packed visit records (see above)
    const R4* ma;
    const R4* mb;
    const R2* mc;
    const R* vmu;          // FP64 only
    const R* Sv;           // [n_free] sum V0 mu |dN_i|^2 per vertex
    const R* imu;          // [n_inst] mu, lambda of each instance (40-byte
    const R* ilam;         //          Neo-Hookean records only)
    const R4* fext;        // [n_free] lumped external force
    const int* vinst;      // [n_free] instance of each free vertex; null with one
                           // instance (instance 0, active whenever sweeps run)
    const int* active;     // [n_inst] 1 while the instance iterates
    const int* wvptr;      // [n_verts + 1] weak constraints per vertex
    const int* wv_c;
    const R* wv_s;         // w0 - w1 of this vertex in the constraint
    const int* wc_ptr;     // [n_wc + 1]
    const int* wc_vert;    // internal vertex indices
    const R* wc_w;
    const R* wc_K;         // [n_wc][6]
    const int* plane_ptr;  // [n_inst + 1]
    const R* planes;       // [n_planes][5]
    int* rejected;         // [n_inst]
    const R* inert;        // [n_free] m_ii / dt^2 (backward Euler), or null
    const P4* xhat;        // [n_free] 2 x^n - x^{n-1}
    // recoloured vertices (general kernel only): the launch slots
    // [vbeg, list_from) are the colour's home range, whose vertices v are
    // skipped when their current colour pcol[v] is not pcolor (pcol null:
    // none moved); slots v >= list_from (vlist non-null) take the vertex
    // vlist[v - list_from + list_beg] recoloured into pcolor
    const int* vlist;
    const int* pcol;
    int pcolor;
    int list_from, list_beg;
    PR omega, gamma;
    int max_halvings;
};

// FP64 residual / energy / adjoint assembly arguments.
template <class R>
struct ResArgs {
    using R4 = typename R4t<R>::T;
    const R4* X;            // positions, internal order
    const int4* tet;        // [n_tets] internal vertex indices
    const TetGeo* geo;      // [n_tets]
    double* vp;             // [n_tets][4][3] scratch: V0 P dN_j or V0 dP[Lam] dN_j
    double* ebuf;           // energy summands
    const int* tet_eidx;    // [n_tets] slot of each tet energy in ebuf
    const int* vorder;      // [n_verts] internal vertex at instance-major position k
    const int* vert_eidx;   // [n_verts] (by position k) slot in ebuf
    const int* rvptr;       // [n_verts + 1] visits of every vertex (internal order)
    const int* rv;          // tet * 4 + slot
    const double* fext64;   // [n_verts][3] internal order
    const int* vinst_all;   // [n_verts] internal order
    const int* wvptr;
    const int* wv_c;
    const double* wv_s64;
    const int* wc_ptr;
    const int* wc_vert;
    const double* wc_w64;
    const double* wc_K64;
    const int* wc_eidx;
    const int* plane_ptr;
    const double* planes64;
    const int* orig_of;     // [n_verts] caller index of each internal vertex
    const double* inert64;  // [n_free] m_ii / dt^2, or null
    const double* xhat64;   // [n_free][3]
    int n_free;
    int n_verts;
    int n_tets;
    int n_wc;
    int model;
};

// Deterministic segmented sums: chunk c covers [cbeg[c], cend[c]) of the
// value array; instance q owns chunks [qptr[q], qptr[q+1]).
struct SegPlan {
    int64_t* cbeg = nullptr;
    int64_t* cend = nullptr;
    int* qptr = nullptr;
    double* partial = nullptr;
    int n_chunks = 0;
};

// ---- launchers (pbng_kernels.hip) -------------------------------------
// launch_load: free vertices from the caller array, Dirichlet vertices from
// xd_int (or, when xd_int is null, also from the caller array).
// mode: 0 the single-instance kernel, 1 the general variant (batched
// instances, weak constraints, planes, recoloured vertices, inertia), 2 the
// single-instance kernel with the backward-Euler inertia term
template <class R, class PR>
hipError_t launch_phase(const SweepArgs<R, PR>& a, int model, int lanes, bool accel, bool safe,
                        int mode, int vbeg, int vend, hipStream_t s);
template <class R>
hipError_t launch_load(const R* x_user, const int* orig_of, const typename R4t<R>::T* xd_int,
                       typename R4t<R>::T* d0, typename R4t<R>::T* d1, typename R4t<R>::T* d2,
                       int n_free, int n_verts, hipStream_t s);
template <class R>
hipError_t launch_store(const typename R4t<R>::T* src, const int* orig_of, R* x_user, int n_verts,
                        hipStream_t s);
template <class R>
hipError_t launch_residual(const ResArgs<R>& a, double* rsq, double* r_out, hipStream_t s);
template <class R>
hipError_t launch_adjoint_assembly(const ResArgs<R>& a, const typename R4t<R>::T* lam,
                                   const typename R4t<R>::T* b, double* rsq, double* dmu,
                                   double* dlam, double* dxd, const int* dir_pos,
                                   hipStream_t s);
hipError_t launch_segsum(const double* vals, const SegPlan& plan, int n_inst, double* out,
                         hipStream_t s);
// Visit-record build from the FP64 tet geometry (at workspace creation and
// after every material update): jv[k].w or vmu[k], ma, mb, mc and the
// per-vertex sums Sv.
template <class R>
struct VisitBuild {
    const TetGeo* geo;
    const int* rv;         // tet * 4 + slot, CSR by internal vertex
    const int* vptr;       // [n_free + 1]
    int n_free;
    int model;
    int4* jv;
    typename R4t<R>::T* ma;
    typename R4t<R>::T* mb;
    typename R2t<R>::T* mc;  // corotated only
    R* vmu;                  // FP64 only
    R* Sv;                   // [n_free]
};
template <class R>
hipError_t launch_build_visits(const VisitBuild<R>& b, hipStream_t s);
// Material flags after an update: flag[0] = 1 if lambda >= mu in every
// tet, flag[1] = 1 if every instance has a single (mu, lambda); imu, ilam
// receive the parameters of each instance's first tet.  t_off: [n_inst + 1]
// tet offsets.
template <class R>
hipError_t launch_material_flags(const double* mu, const double* lam, const int64_t* t_off, int n_inst,
                                 int n_tets, int* flag, R* imu, R* ilam, hipStream_t s);
// Material update: TetGeo mu/lambda, then the visit records.
template <class R>
hipError_t launch_set_materials(const double* mu, const double* lam, TetGeo* geo, int n_tets,
                                const VisitBuild<R>& b, hipStream_t s);
template <class R>
hipError_t launch_set_dirichlet(const double* xd, const int* dir_internal, int nd, int n_free,
                                typename R4t<R>::T* xd_int, hipStream_t s);
template <class R>
hipError_t launch_store64(const typename R4t<R>::T* src, const int* orig_of, double* x_user,
                          int n_verts, hipStream_t s);
template <class R>
hipError_t launch_copy4(const typename R4t<R>::T* src, typename R4t<R>::T* dst, int n,
                        hipStream_t s);
template <class R>
hipError_t launch_load_vec(const R* v_user, const int* orig_of, typename R4t<R>::T* dst,
                           int n_free, int n_verts, hipStream_t s);

// Backward-Euler inertia: from caller-order x^n, x^{n-1} ([n_verts][3]
// double) and the lumped masses of the free vertices (internal order), the
// sweep's m/dt^2 and xhat = 2 x^n - x^{n-1} (R, PR) and their FP64 copies.
template <class R, class PR>
hipError_t launch_set_inertia(const double* x_n, const double* x_prev, const int* orig_of,
                              const double* mass, int n_free, double dt, R* inert,
                              typename R4t<PR>::T* xhat, double* inert64, double* xhat64,
                              hipStream_t s);

// Proximity detection (pbng_contacts.hip): the candidate surface vertices
// with their caller index, instance, connected part and Dirichlet flag.
struct ContactCand {
    int n;
    const int* caller;
    const int* inst;
    const int* body;
    const int* dir;
    int inst_bits;          // bits of the largest instance index (0 for one)
    int vert_bits;          // bits of the largest caller vertex index
};
struct DetectScratch {
    unsigned long long* keys_in;
    unsigned long long* keys_out;
    int* vals_in;
    int* vals_out;
    int2* pairs;
    unsigned long long* pkeys_in;
    unsigned long long* pkeys_out;
    int* count;
    void* tmp;
    size_t tmp_bytes;
};
// Pairs within r, sorted, with normals, into pairs_out [max_pairs][2] and
// normals_out [max_pairs][3]; *n_found = number of pairs (outputs written
// only when it does not exceed max_pairs).  Synchronises s.
template <class P>
hipError_t launch_detect(const P* x, const ContactCand& c, double r, int max_pairs, DetectScratch& w,
                         int* pairs_out, double* normals_out, int* n_found, hipStream_t s);
size_t detect_tmp_bytes(int n, int max_pairs);

// Adjoint block Gauss-Seidel phase: L holds lambda (internal order), B the
// right-hand side dL/dx (internal order, free vertices), X the equilibrium.
template <class R, class PR = R>
struct AdjArgs {
    using P4 = typename R4t<PR>::T;
    const P4* X;
    P4* L;                 // working adjoint iterate
    P4* P;                 // previous (acceleration)
    P4* N;                 // next (acceleration)
    const P4* B;
    using R4 = typename R4t<R>::T;
    using R2 = typename R2t<R>::T;
    const int* vptr;
    const int4* jv;
    const R4* ma;
    const R4* mb;
    const R2* mc;
    const R* vmu;          // FP64 only
    const R* Sv;
    const R* imu;
    const R* ilam;
    const int* vinst;
    const int* wvptr;
    const int* wv_c;
    const R* wv_s;
    const int* wc_ptr;
    const int* wc_vert;
    const R* wc_w;
    const R* wc_K;
    const int* plane_ptr;
    const R* planes;
    const R* inert;        // [n_free] m_ii / dt^2, or null
    const int* vlist;      // as in SweepArgs
    const int* pcol;
    int pcolor;
    int list_from, list_beg;
    PR omega, gamma;
};
template <class R, class PR>
hipError_t launch_adjoint_phase(const AdjArgs<R, PR>& a, int model, int lanes, bool accel, bool wc,
                                int vbeg, int vend, hipStream_t s);

}  // namespace pbng
