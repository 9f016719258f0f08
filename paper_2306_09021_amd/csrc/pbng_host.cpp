// libpbng host side: validation, node colouring, packing of the device
// layout, the solve / residual / adjoint drivers and the C ABI of
// include/pbng.h.  No C++ exception leaves this file.
#include "pbng.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "pbng_hostutil.hpp"
#include "pbng_internal.hpp"

using namespace pbng;

namespace {

bool finite_arr(const double* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

double det3(const double* A)
{
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// Rest-state data of one tet: Dm = [X1 - X0, X2 - X0, X3 - X0] (columns),
// V0 = det(Dm) / 6, and Dm^{-1} (row j-1 = dN_j for j = 1..3).
bool tet_rest(const double* X, const int32_t* t, double* dminv, double* V0)
{
    double Dm[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Dm[3 * r + c] = X[3 * t[c + 1] + r] - X[3 * t[0] + r];
    const double d = det3(Dm);
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    // inverse = adj / det, adj_ij = cof_ji
    double C[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int r0 = (i + 1) % 3, r1 = (i + 2) % 3, c0 = (j + 1) % 3, c1 = (j + 2) % 3;
            C[3 * i + j] = Dm[3 * r0 + c0] * Dm[3 * r1 + c1] - Dm[3 * r0 + c1] * Dm[3 * r1 + c0];
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dminv[3 * i + j] = C[3 * j + i] / d;
    *V0 = d / 6.0;
    return true;
}

// What the colouring reads: sizes (the vertex -> tet incidence holds
// 4 n_tets int32 entries), tet and weak-constraint vertex indices, the
// constraint CSR and the Dirichlet list.
void validate_topology(const pbng_problem* p, int q)
{
    if (p->n_verts <= 0 || p->n_tets < 0) fail(PBNG_EINVAL, "problem %d: bad sizes", q);
    if (p->n_tets >= (int64_t(1) << 29)) fail(PBNG_EINVAL, "problem %d: too many tets for 32-bit indices", q);
    if (p->n_tets > 0 && !p->tets) fail(PBNG_EINVAL, "problem %d: tets is null", q);
    for (int64_t e = 0; e < p->n_tets; ++e) {
        const int32_t* t = p->tets + 4 * e;
        for (int j = 0; j < 4; ++j) {
            if (t[j] < 0 || t[j] >= p->n_verts)
                fail(PBNG_EMESH, "problem %d: tet %lld has vertex %d out of range", q, (long long)e, t[j]);
            for (int k = 0; k < j; ++k)
                if (t[k] == t[j]) fail(PBNG_EMESH, "problem %d: tet %lld repeats a vertex", q, (long long)e);
        }
    }
    if (p->n_dirichlet < 0 || p->n_dirichlet > p->n_verts) fail(PBNG_EINVAL, "problem %d: bad n_dirichlet", q);
    if (p->n_dirichlet > 0) {
        if (!p->dirichlet_idx) fail(PBNG_EINVAL, "problem %d: dirichlet_idx is null", q);
        std::vector<char> seen(p->n_verts, 0);
        for (int k = 0; k < p->n_dirichlet; ++k) {
            const int v = p->dirichlet_idx[k];
            if (v < 0 || v >= p->n_verts) fail(PBNG_EINVAL, "problem %d: Dirichlet index %d out of range", q, v);
            if (seen[v]) fail(PBNG_EINVAL, "problem %d: Dirichlet index %d repeated", q, v);
            seen[v] = 1;
        }
    }
    if (p->n_wc < 0) fail(PBNG_EINVAL, "problem %d: bad n_wc", q);
    if (p->n_wc > 0) {
        if (!p->wc_ptr || !p->wc_vert) fail(PBNG_EINVAL, "problem %d: weak-constraint arrays are null", q);
        if (p->wc_ptr[0] != 0) fail(PBNG_EINVAL, "problem %d: wc_ptr[0] must be 0", q);
        for (int c = 0; c < p->n_wc; ++c)
            if (p->wc_ptr[c + 1] < p->wc_ptr[c]) fail(PBNG_EINVAL, "problem %d: wc_ptr not monotone", q);
        const int nnz = p->wc_ptr[p->n_wc];
        for (int k = 0; k < nnz; ++k)
            if (p->wc_vert[k] < 0 || p->wc_vert[k] >= p->n_verts) fail(PBNG_EMESH, "problem %d: weak-constraint vertex out of range", q);
        for (int c = 0; c < p->n_wc; ++c)
            for (int k = p->wc_ptr[c]; k < p->wc_ptr[c + 1]; ++k)
                for (int j = p->wc_ptr[c]; j < k; ++j)
                    if (p->wc_vert[j] == p->wc_vert[k]) fail(PBNG_EMESH, "problem %d: weak constraint %d repeats a vertex", q, c);
    }
}

void validate_problem(const pbng_problem* p, int q)
{
    if (!p) fail(PBNG_EINVAL, "problem %d: null", q);
    validate_topology(p, q);
    if (!p->rest_pos) fail(PBNG_EINVAL, "problem %d: rest_pos is null", q);
    if (p->model != PBNG_NEOHOOKEAN && p->model != PBNG_COROTATED && p->model != PBNG_STABLE_NEOHOOKEAN)
        fail(PBNG_EINVAL, "problem %d: unknown model %d", q, p->model);
    if (!finite_arr(p->rest_pos, 3ll * p->n_verts)) fail(PBNG_ENAN, "problem %d: non-finite rest_pos", q);
    const bool pt = p->mu_tet != nullptr || p->lambda_tet != nullptr;
    if (pt && (!p->mu_tet || !p->lambda_tet))
        fail(PBNG_EINVAL, "problem %d: mu_tet and lambda_tet must be given together", q);
    if (pt) {
        for (int64_t e = 0; e < p->n_tets; ++e) {
            if (!std::isfinite(p->mu_tet[e]) || !std::isfinite(p->lambda_tet[e]))
                fail(PBNG_ENAN, "problem %d: non-finite Lame parameter", q);
            if (!(p->mu_tet[e] > 0.0) || !(p->lambda_tet[e] > 0.0))
                fail(PBNG_EMATERIAL, "problem %d: tet %lld has mu or lambda <= 0", q, (long long)e);
        }
    } else {
        if (!std::isfinite(p->mu) || !std::isfinite(p->lambda))
            fail(PBNG_ENAN, "problem %d: non-finite Lame parameter", q);
        if (!(p->mu > 0.0) || !(p->lambda > 0.0))
            fail(PBNG_EMATERIAL, "problem %d: mu and lambda must be > 0", q);
    }
    if (!std::isfinite(p->density) || !finite_arr(p->gravity, 3))
        fail(PBNG_ENAN, "problem %d: non-finite body force", q);
    if (p->nodal_force && !finite_arr(p->nodal_force, 3ll * p->n_verts))
        fail(PBNG_ENAN, "problem %d: non-finite nodal_force", q);
    if (p->n_dirichlet > 0) {
        if (!p->dirichlet_x) fail(PBNG_EINVAL, "problem %d: dirichlet_x is null", q);
        if (!finite_arr(p->dirichlet_x, 3ll * p->n_dirichlet)) fail(PBNG_ENAN, "problem %d: non-finite Dirichlet target", q);
    }
    if (p->n_wc > 0) {
        if (!p->wc_w || !p->wc_K) fail(PBNG_EINVAL, "problem %d: weak-constraint arrays are null", q);
        const int nnz = p->wc_ptr[p->n_wc];
        if (!finite_arr(p->wc_w, nnz) || !finite_arr(p->wc_K, 6ll * p->n_wc)) fail(PBNG_ENAN, "problem %d: non-finite weak constraint", q);
    }
    if (p->n_planes < 0) fail(PBNG_EINVAL, "problem %d: bad n_planes", q);
    if (p->n_planes > 0) {
        if (!p->planes) fail(PBNG_EINVAL, "problem %d: planes is null", q);
        if (!finite_arr(p->planes, 5ll * p->n_planes)) fail(PBNG_ENAN, "problem %d: non-finite plane", q);
        for (int k = 0; k < p->n_planes; ++k)
            if (p->planes[5 * k + 4] < 0.0) fail(PBNG_EINVAL, "problem %d: plane stiffness < 0", q);
    }
}

// Vertex -> incident tets (ascending tet index, with local slot) and
// vertex -> incident weak constraints.
struct Incidence {
    std::vector<int> tptr, tlist, cptr, clist, cpos;
};

Incidence incidence(const pbng_problem* p)
{
    Incidence I;
    const int nv = p->n_verts;
    I.tptr.assign(nv + 1, 0);
    for (int64_t e = 0; e < p->n_tets; ++e)
        for (int j = 0; j < 4; ++j) I.tptr[p->tets[4 * e + j] + 1]++;
    for (int i = 0; i < nv; ++i) I.tptr[i + 1] += I.tptr[i];
    I.tlist.resize(I.tptr[nv]);
    std::vector<int> fill(I.tptr.begin(), I.tptr.end() - 1);
    for (int64_t e = 0; e < p->n_tets; ++e)
        for (int j = 0; j < 4; ++j) I.tlist[fill[p->tets[4 * e + j]]++] = int(4 * e + j);
    const int nnz = p->n_wc > 0 ? p->wc_ptr[p->n_wc] : 0;
    I.cptr.assign(nv + 1, 0);
    for (int k = 0; k < nnz; ++k) I.cptr[p->wc_vert[k] + 1]++;
    for (int i = 0; i < nv; ++i) I.cptr[i + 1] += I.cptr[i];
    I.clist.resize(nnz);
    I.cpos.resize(nnz);
    std::vector<int> f2(I.cptr.begin(), I.cptr.end() - 1);
    for (int c = 0; c < p->n_wc; ++c)
        for (int k = p->wc_ptr[c]; k < p->wc_ptr[c + 1]; ++k) {
            const int v = p->wc_vert[k];
            I.clist[f2[v]] = c;
            I.cpos[f2[v]] = k;
            f2[v]++;
        }
    return I;
}

std::vector<char> dirichlet_mask(const pbng_problem* p)
{
    std::vector<char> d(p->n_verts, 0);
    for (int k = 0; k < p->n_dirichlet; ++k) d[p->dirichlet_idx[k]] = 1;
    return d;
}

// Greedy node colouring with used-colour sets S_c held as 64-bit masks on
// every tet and weak constraint (Sec. "Coloring and Parallelism").
int color_instance(const pbng_problem* p, int32_t* colors)
{
    const Incidence I = incidence(p);
    const std::vector<char> dir = dirichlet_mask(p);
    std::vector<uint64_t> St(p->n_tets, 0), Sc(p->n_wc, 0);
    int ncol = 0;
    for (int i = 0; i < p->n_verts; ++i) {
        if (dir[i]) {
            colors[i] = -1;
            continue;
        }
        uint64_t used = 0;
        for (int k = I.tptr[i]; k < I.tptr[i + 1]; ++k) used |= St[I.tlist[k] >> 2];
        for (int k = I.cptr[i]; k < I.cptr[i + 1]; ++k) used |= Sc[I.clist[k]];
        if (used == ~uint64_t(0)) fail(PBNG_ECOLOR, "more than 64 colours needed at vertex %d", i);
        const int c = __builtin_ctzll(~used);
        colors[i] = c;
        ncol = std::max(ncol, c + 1);
        const uint64_t bit = uint64_t(1) << c;
        for (int k = I.tptr[i]; k < I.tptr[i + 1]; ++k) St[I.tlist[k] >> 2] |= bit;
        for (int k = I.cptr[i]; k < I.cptr[i + 1]; ++k) Sc[I.clist[k]] |= bit;
    }
    return ncol;
}

int check_colors(const pbng_problem* p, const int32_t* colors)
{
    const std::vector<char> dir = dirichlet_mask(p);
    int ncol = 0;
    for (int i = 0; i < p->n_verts; ++i) {
        if (dir[i]) {
            if (colors[i] != -1) fail(PBNG_ECOLOR, "Dirichlet vertex %d must have colour -1", i);
            continue;
        }
        if (colors[i] < 0 || colors[i] >= 64) fail(PBNG_ECOLOR, "vertex %d has colour %d outside [0, 64)", i, colors[i]);
        ncol = std::max(ncol, colors[i] + 1);
    }
    for (int64_t e = 0; e < p->n_tets; ++e) {
        uint64_t m = 0;
        for (int j = 0; j < 4; ++j) {
            const int c = colors[p->tets[4 * e + j]];
            if (c < 0) continue;
            if (m >> c & 1) fail(PBNG_ECOLOR, "tet %lld has two vertices of colour %d", (long long)e, c);
            m |= uint64_t(1) << c;
        }
    }
    for (int k = 0; k < p->n_wc; ++k) {
        uint64_t m = 0;
        for (int j = p->wc_ptr[k]; j < p->wc_ptr[k + 1]; ++j) {
            const int c = colors[p->wc_vert[j]];
            if (c < 0) continue;
            if (m >> c & 1) fail(PBNG_ECOLOR, "weak constraint %d has two vertices of colour %d", k, c);
            m |= uint64_t(1) << c;
        }
    }
    return ncol;
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace
// ---------------------------------------------------------------------------
struct pbng_workspace {
    int real = PBNG_F32;
    int model = PBNG_NEOHOOKEAN;
    int n_inst = 0;
    int64_t nv = 0, nt = 0, nfree = 0, nvis = 0, nvis_all = 0;
    int ncol = 0;
    int n_wc = 0, n_planes = 0, nd = 0;
    bool any_wc = false;
    // The safeguard cannot reject a step here (so the plain kernel gives the
    // same result): no contact planes, and either the corotated model (its
    // modified Hessian is the Hessian of a majoriser of the local energy) or
    // the Neo-Hookean model with lambda >= mu in every tet (then 2 A - H is
    // positive semidefinite and the full step always lowers the exactly
    // quadratic local energy).  Weak constraints are exact quadratics inside
    // A and do not change either argument.
    bool safeguard_inactive = false;
    // general sweep kernel: batched instances, weak constraints or planes
    // phase-kernel variant: 1 general (batched, weak constraints, planes,
    // recoloured vertices, whose phases need the list / colour checks even
    // after the contacts that moved them are removed), 2 one instance with
    // inertia only, 0 plain
    int kernel_mode() const { return (any_wc || n_inst > 1 || moved_any) ? 1 : (inertia ? 2 : 0); }
    int device = 0;
    std::vector<int> col_ptr;              // internal free-vertex range of each colour
    std::vector<int64_t> v_off, t_off;     // per instance
    std::vector<int> ncol_inst;
    std::vector<int64_t> nfree_inst;
    std::vector<int64_t> phase_bytes, phase_verts, phase_visits;
    std::vector<int> phase_lanes;          // automatic lanes per vertex of each colour
    double mean_valence = 0.0;

    // sweep data
    Dev W, P, N, Wres;
    Dev jv, ma, mb, mc, vmu, Sv, flag, vptr, fext, vinst, active, rejected;
    // model id of the sweep and adjoint kernels: the public model, or 3 for
    // Neo-Hookean workspaces whose instances each have one (mu, lambda)
    // (40-byte records; instance parameters in imu / ilam)
    int kmodel = PBNG_NEOHOOKEAN;
    Dev imu, ilam, t_off_dev;
    // host copies for re-installing weak constraints (static ones from the
    // problems, in internal vertex indices, plus dynamic contacts)
    std::vector<int> h_wc_ptr, h_wc_vert, h_wc_inst;
    std::vector<double> h_wc_w, h_wc_K;
    struct Contact {
        int a, b, inst;
        double K[6];
    };
    std::vector<Contact> contacts;
    std::vector<int> h_int_of, h_orig_of;
    // every installed constraint (static and dynamic, internal indices) and
    // the per-vertex CSR of the constraints of each vertex
    std::vector<int> h_all_wc_ptr, h_all_wc_vert, h_wvptr, h_wv_c;
    // current colouring (internal order, -1 on Dirichlet vertices), the
    // host incidence it is checked against, and the launch plan of a sweep:
    // per colour the home range (skipping vertices recoloured away) and
    // the list of vertices recoloured into it
    std::vector<int> h_color, h_rvptr, h_rv, h_vinst;
    std::vector<int4> h_tet;
    // one launch per colour: home range [hb, he) of internal free
    // vertices, then the slice [lb, le) of xlist (vertices recoloured into
    // the colour)
    struct PhaseSpec {
        int color, hb, he, lb, le;
    };
    std::vector<PhaseSpec> phases;
    bool moved_any = false;
    int ncol_dyn = 0;
    Dev pcol, xlist;
    Pinned stage;                          // staging of batched uploads (host, device)
    Dev ustage;
    // proximity detection: candidate surface vertices (built on first use)
    // and scratch sized for n_cand candidates and det_cap pairs
    int n_cand = -1;
    Dev cand_caller, cand_inst, cand_body, cand_dir;
    int det_cap = -1;
    Dev d_keys_in, d_keys_out, d_vals_in, d_vals_out, d_pairs, d_pkeys_in, d_pkeys_out, d_count, d_tmp;
    size_t d_tmp_bytes = 0;
    // backward-Euler inertia (off until pbng_workspace_set_inertia)
    bool inertia = false;
    Dev mass64, inert, xhat, inert64, xhat64;
    Dev wvptr, wv_c, wv_s, wc_ptr, wc_vert, wc_w, wc_K, plane_ptr, planes;
    // FP64 data
    Dev tet, geo, vp, ebuf, tet_eidx, vorder, vert_eidx, rvptr, rv, fext64, vinst_all;
    Dev wv_s64, wc_w64, wc_K64, wc_eidx, planes64, orig_of, rsq;
    Dev xd_int, dir_internal, dir_pos;
    Dev seg_r_cb, seg_r_ce, seg_r_q, seg_r_part, seg_e_cb, seg_e_ce, seg_e_q, seg_e_part;
    SegPlan plan_r, plan_e;
    Dev out_r, out_e;
    double* hbuf = nullptr;  // pinned [2 n_inst]
    int* hact = nullptr;     // pinned [n_inst]
    // adjoint
    Dev L, LP, LN, B;

    // acceleration state
    int64_t sweep_l = 0;
    double omega_l = 1.0;
    bool ring_valid = false;

    // captured steady-state sweeps (one HIP graph, replayed)
    hipGraphExec_t gexec = nullptr;
    struct GraphKey {
        void *W, *P, *N;
        double omega, gamma;
        int sweeps, accel, safe, lanes, max_halvings;
        hipStream_t stream;
        bool operator==(const GraphKey& o) const
        {
            return W == o.W && P == o.P && N == o.N && omega == o.omega && gamma == o.gamma &&
                   sweeps == o.sweeps && accel == o.accel && safe == o.safe && lanes == o.lanes &&
                   max_halvings == o.max_halvings && stream == o.stream;
        }
    } gkey{};
    uint64_t lanes_version = 0;   // bumped when the automatic lane table changes
    uint64_t gkey_lanes_version = ~uint64_t(0);

    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
    }
    ~pbng_workspace()
    {
        drop_graph();
        if (hbuf) (void)hipHostFree(hbuf);
        if (hact) (void)hipHostFree(hact);
    }
    // positions in FP64 (PBNG_F64, PBNG_MIXED); sweep arithmetic in FP64
    // only for PBNG_F64
    bool pos64() const { return real != PBNG_F32; }
    bool math64() const { return real == PBNG_F64; }
    size_t r4() const { return pos64() ? 32 : 16; }
};

namespace {

template <class R>
void upload_real(Dev& d, const std::vector<double>& v)
{
    std::vector<R> t(v.begin(), v.end());
    d.upload(t);
}

template <class R>
void stage_real(Uploader& up, Dev& d, const std::vector<double>& v)
{
    std::vector<R> t(v.begin(), v.end());
    up.add(d, t);
}

SegPlan make_plan(const std::vector<int64_t>& seg, Dev& cb, Dev& ce, Dev& qp, Dev& part, Uploader& up)
{
    const int64_t chunk = 4096;
    std::vector<int64_t> b, e;
    std::vector<int> q(seg.size(), 0);
    for (size_t i = 0; i + 1 < seg.size(); ++i) {
        q[i] = int(b.size());
        for (int64_t s = seg[i]; s < seg[i + 1]; s += chunk) {
            b.push_back(s);
            e.push_back(std::min(seg[i + 1], s + chunk));
        }
    }
    q.back() = int(b.size());
    up.add(cb, b);
    up.add(ce, e);
    up.add(qp, q);
    part.reserve(std::max<size_t>(1, b.size()) * sizeof(double));
    SegPlan P;
    P.cbeg = cb.as<int64_t>();
    P.cend = ce.as<int64_t>();
    P.qptr = qp.as<int>();
    P.partial = part.as<double>();
    P.n_chunks = int(b.size());
    return P;
}

// Record streams for the workspace's kernel model: 40-byte Neo-Hookean
// (jv, ma, mc), 48-byte Neo-Hookean (jv, ma, mb) or full (jv, ma, mb, mc);
// FP64 workspaces add vmu.
void alloc_records(pbng_workspace* ws)
{
    const size_t r = ws->math64() ? sizeof(double) : sizeof(float);
    const size_t nv = size_t(ws->nvis);
    const bool u = ws->kmodel == 3, nh = ws->kmodel == PBNG_NEOHOOKEAN;
    ws->ma.alloc(nv * 4 * r);
    ws->mb.alloc(u ? 0 : nv * 4 * r);
    ws->mc.alloc(nh ? 0 : nv * 2 * r);
    ws->vmu.alloc(ws->math64() ? nv * r : 0);
}

template <class R>
VisitBuild<R> visit_build(pbng_workspace* ws)
{
    VisitBuild<R> b;
    b.geo = ws->geo.as<TetGeo>();
    b.rv = ws->rv.as<int>();
    b.vptr = ws->vptr.as<int>();
    b.n_free = int(ws->nfree);
    b.model = ws->kmodel;
    b.jv = ws->jv.as<int4>();
    b.ma = ws->ma.as<typename R4t<R>::T>();
    b.mb = ws->mb.as<typename R4t<R>::T>();
    b.mc = ws->mc.as<typename R2t<R>::T>();
    b.vmu = ws->vmu.as<R>();
    b.Sv = ws->Sv.as<R>();
    return b;
}

// Visit records from the tet geometry; with material arrays, first the
// new mu and lambda into the geometry.
hipError_t build_visits(pbng_workspace* ws, const double* mu, const double* lam, hipStream_t s)
{
    if (ws->math64()) {
        if (mu) return launch_set_materials<double>(mu, lam, ws->geo.as<TetGeo>(), int(ws->nt),
                                                    visit_build<double>(ws), s);
        return launch_build_visits<double>(visit_build<double>(ws), s);
    }
    if (mu) return launch_set_materials<float>(mu, lam, ws->geo.as<TetGeo>(), int(ws->nt),
                                               visit_build<float>(ws), s);
    return launch_build_visits<float>(visit_build<float>(ws), s);
}

// Launch plan of a sweep from the current colouring: colour c runs its home
// range [col_ptr[c], col_ptr[c+1]) (vertices recoloured away are skipped on
// the device) and then, if any, the list of vertices recoloured into c.
void rebuild_phases(pbng_workspace* ws, Uploader& up)
{
    const int nf = int(ws->nfree);
    int ncol = ws->ncol;
    std::vector<std::vector<int>> moved_in;
    ws->moved_any = false;
    for (int c = 0; c < ws->ncol; ++c)
        for (int k = ws->col_ptr[c]; k < ws->col_ptr[c + 1]; ++k)
            if (ws->h_color[k] != c) {
                const int cn = ws->h_color[k];
                if (cn + 1 > int(moved_in.size())) moved_in.resize(cn + 1);
                moved_in[cn].push_back(k);
                ncol = std::max(ncol, cn + 1);
                ws->moved_any = true;
            }
    ws->ncol_dyn = ncol;
    ws->phases.clear();
    std::vector<int> list;
    for (int c = 0; c < ncol; ++c) {
        pbng_workspace::PhaseSpec ph{c, 0, 0, int(list.size()), int(list.size())};
        if (c < ws->ncol) {
            ph.hb = ws->col_ptr[c];
            ph.he = ws->col_ptr[c + 1];
        }
        if (c < int(moved_in.size())) {
            list.insert(list.end(), moved_in[c].begin(), moved_in[c].end());
            ph.le = int(list.size());
        }
        if (ph.he > ph.hb || ph.le > ph.lb) ws->phases.push_back(ph);
    }
    if (ws->moved_any) {
        std::vector<int> pc(ws->h_color.begin(), ws->h_color.begin() + nf);
        up.add(ws->pcol, pc);
        up.add(ws->xlist, list);
    }
}

// Incremental recolouring after new weak constraints (Sec. "Collision
// Coloring"): every free vertex incident to a dynamic constraint, in
// ascending caller index, keeps its colour unless another vertex sharing a
// tet or a weak constraint with it has that colour; then it takes the least
// colour none of them has.  Colours of vertices processed earlier count.
void recolor_contacts(pbng_workspace* ws)
{
    const int nf = int(ws->nfree);
    // the constraints of every vertex (static and dynamic) come from the
    // per-vertex CSR that install_constraints has just built
    std::vector<int> extra;
    for (const auto& ct : ws->contacts)
        for (int v : {ct.a, ct.b})
            if (v < nf) extra.push_back(v);
    std::sort(extra.begin(), extra.end(), [&](int x, int y) { return ws->h_orig_of[x] < ws->h_orig_of[y]; });
    extra.erase(std::unique(extra.begin(), extra.end()), extra.end());
    std::vector<char> used;
    for (int v : extra) {
        used.assign(used.size(), 0);
        auto mark = [&](int u) {
            const int c = ws->h_color[u];
            if (c < 0) return;
            if (c >= int(used.size())) used.resize(c + 1, 0);
            used[c] = 1;
        };
        for (int k = ws->h_rvptr[v]; k < ws->h_rvptr[v + 1]; ++k) {
            const int4 t = ws->h_tet[ws->h_rv[k] >> 2];
            for (int u : {t.x, t.y, t.z, t.w})
                if (u != v) mark(u);
        }
        for (int k = ws->h_wvptr[v]; k < ws->h_wvptr[v + 1]; ++k) {
            const int c = ws->h_wv_c[k];
            for (int m = ws->h_all_wc_ptr[c]; m < ws->h_all_wc_ptr[c + 1]; ++m) {
                const int u = ws->h_all_wc_vert[m];
                if (u != v) mark(u);
            }
        }
        const int cur = ws->h_color[v];
        if (cur >= 0 && (cur >= int(used.size()) || !used[cur])) continue;
        int c = 0;
        while (c < int(used.size()) && used[c]) ++c;
        ws->h_color[v] = c;
    }
}

// Weak constraints of the workspace: the static ones from the problems and
// the dynamic contacts (two members, weights +1 / -1), instance by
// instance: the global constraint list, the per-vertex CSR (constraint,
// weight), and the instance-major energy slots (tets, vertices,
// constraints of each instance) with their segmented-sum plan.
void install_constraints(pbng_workspace* ws, Uploader& up)
{
    const int n = ws->n_inst;
    const int64_t nv = ws->nv, nt = ws->nt;
    const int n_static = int(ws->h_wc_inst.size());
    std::vector<std::vector<int>> dyn_of(n);
    for (int k = 0; k < int(ws->contacts.size()); ++k) dyn_of[ws->contacts[k].inst].push_back(k);
    std::vector<std::vector<int>> stat_of(n);
    for (int c = 0; c < n_static; ++c) stat_of[ws->h_wc_inst[c]].push_back(c);
    std::vector<int> wc_ptr(1, 0), wc_vert, wvptr(nv + 1, 0), wv_c, wc_eidx;
    std::vector<double> wc_w, wc_K, wv_s;
    std::vector<int> tet_eidx(nt), vert_eidx(nv);
    std::vector<int64_t> seg_e(n + 1);
    int64_t eo = 0;
    for (int q = 0; q < n; ++q) {
        const int64_t vo = ws->v_off[q], to = ws->t_off[q];
        const int64_t ntq = ws->t_off[q + 1] - to, nvq = ws->v_off[q + 1] - vo;
        seg_e[q] = eo;
        for (int64_t e = 0; e < ntq; ++e) tet_eidx[to + e] = int(eo + e);
        for (int64_t i = 0; i < nvq; ++i) vert_eidx[vo + i] = int(eo + ntq + i);
        int64_t slot = eo + ntq + nvq;
        auto add = [&](const int* verts, const double* w, int m, const double* K) {
            for (int j = 0; j < m; ++j) {
                wc_vert.push_back(verts[j]);
                wc_w.push_back(w[j]);
            }
            wc_ptr.push_back(int(wc_vert.size()));
            for (int j = 0; j < 6; ++j) wc_K.push_back(K[j]);
            wc_eidx.push_back(int(slot++));
        };
        for (int c : stat_of[q])
            add(ws->h_wc_vert.data() + ws->h_wc_ptr[c], ws->h_wc_w.data() + ws->h_wc_ptr[c],
                ws->h_wc_ptr[c + 1] - ws->h_wc_ptr[c], ws->h_wc_K.data() + 6 * c);
        for (int k : dyn_of[q]) {
            const auto& ct = ws->contacts[k];
            const int verts[2] = {ct.a, ct.b};
            const double w[2] = {1.0, -1.0};
            add(verts, w, 2, ct.K);
        }
        eo = slot;
    }
    seg_e[n] = eo;
    // per-vertex CSR of (constraint, weight), constraints in ascending
    // order for every vertex (a stable counting pass over the members)
    const int n_all = int(wc_ptr.size()) - 1;
    for (int v : wc_vert) wvptr[v + 1]++;
    for (int64_t k = 0; k < nv; ++k) wvptr[k + 1] += wvptr[k];
    wv_c.resize(wc_vert.size());
    wv_s.resize(wc_vert.size());
    {
        std::vector<int> fill(wvptr.begin(), wvptr.end() - 1);
        for (int c = 0; c < n_all; ++c)
            for (int m = wc_ptr[c]; m < wc_ptr[c + 1]; ++m) {
                const int k = fill[wc_vert[m]]++;
                wv_c[k] = c;
                wv_s[k] = wc_w[m];
            }
    }
    ws->n_wc = n_all;
    ws->any_wc = ws->n_wc > 0 || ws->n_planes > 0;
    auto upR = [&](Dev& d, const std::vector<double>& v) {
        if (ws->math64()) stage_real<double>(up, d, v);
        else stage_real<float>(up, d, v);
    };
    up.add(ws->wvptr, wvptr);
    up.add(ws->wv_c, wv_c);
    upR(ws->wv_s, wv_s);
    up.add(ws->wc_ptr, wc_ptr);
    up.add(ws->wc_vert, wc_vert);
    upR(ws->wc_w, wc_w);
    upR(ws->wc_K, wc_K);
    up.add(ws->wv_s64, wv_s);
    up.add(ws->wc_w64, wc_w);
    up.add(ws->wc_K64, wc_K);
    up.add(ws->wc_eidx, wc_eidx);
    up.add(ws->tet_eidx, tet_eidx);
    up.add(ws->vert_eidx, vert_eidx);
    ws->ebuf.reserve(std::max<int64_t>(1, eo) * sizeof(double));
    ws->plan_e = make_plan(seg_e, ws->seg_e_cb, ws->seg_e_ce, ws->seg_e_q, ws->seg_e_part, up);
    // host copies for the recolouring (the uploader holds its own)
    ws->h_all_wc_ptr = std::move(wc_ptr);
    ws->h_all_wc_vert = std::move(wc_vert);
    ws->h_wvptr = std::move(wvptr);
    ws->h_wv_c = std::move(wv_c);
}

void build_workspace(pbng_workspace* ws, const pbng_problem* ps, int n, const int32_t* colors_in)
{
    ws->n_inst = n;
    ws->model = ps[0].model;
    ws->v_off.assign(n + 1, 0);
    ws->t_off.assign(n + 1, 0);
    std::vector<int64_t> c_off(n + 1, 0), p_off(n + 1, 0), d_off(n + 1, 0);
    for (int q = 0; q < n; ++q) {
        validate_problem(ps + q, q);
        if (ps[q].model != ws->model) fail(PBNG_EINVAL, "all instances of a workspace must use the same model");
        ws->v_off[q + 1] = ws->v_off[q] + ps[q].n_verts;
        ws->t_off[q + 1] = ws->t_off[q] + ps[q].n_tets;
        c_off[q + 1] = c_off[q] + ps[q].n_wc;
        p_off[q + 1] = p_off[q] + ps[q].n_planes;
        d_off[q + 1] = d_off[q] + ps[q].n_dirichlet;
    }
    const int64_t nv = ws->v_off[n], nt = ws->t_off[n];
    if (nv >= (int64_t(1) << 31) / 2 || nt >= (int64_t(1) << 29))
        fail(PBNG_EINVAL, "problem too large for 32-bit indices");
    ws->nv = nv;
    ws->nt = nt;
    ws->n_wc = int(c_off[n]);
    ws->n_planes = int(p_off[n]);
    ws->nd = int(d_off[n]);
    ws->any_wc = ws->n_wc > 0 || ws->n_planes > 0;

    // colours, rest data, loads
    std::vector<int32_t> colors(nv);
    std::vector<double> dminv(9 * nt), V0(nt), mu(nt), lam(nt);
    std::vector<double> fext(3 * nv, 0.0);
    std::vector<double> mass(nv, 0.0);
    std::vector<double> inst_mu, inst_lam;
    std::vector<char> isdir(nv, 0);
    std::vector<int> valence(nv, 0);
    std::vector<Incidence> inc(n);
    ws->ncol_inst.assign(n, 0);
    ws->nfree_inst.assign(n, 0);
    for (int q = 0; q < n; ++q) {
        const pbng_problem* p = ps + q;
        const int64_t vo = ws->v_off[q], to = ws->t_off[q];
        int nc;
        if (colors_in) {
            nc = check_colors(p, colors_in + vo);
            std::copy(colors_in + vo, colors_in + vo + p->n_verts, colors.begin() + vo);
        } else {
            nc = color_instance(p, colors.data() + vo);
        }
        ws->ncol_inst[q] = nc;
        ws->ncol = std::max(ws->ncol, nc);
        for (int64_t e = 0; e < p->n_tets; ++e) {
            if (!tet_rest(p->rest_pos, p->tets + 4 * e, &dminv[9 * (to + e)], &V0[to + e]))
                fail(PBNG_EMESH, "problem %d: tet %lld has rest volume <= 0", q, (long long)e);
            mu[to + e] = p->mu_tet ? p->mu_tet[e] : p->mu;
            lam[to + e] = p->mu_tet ? p->lambda_tet[e] : p->lambda;
            for (int j = 0; j < 4; ++j)
                for (int a = 0; a < 3; ++a)
                    fext[3 * (vo + p->tets[4 * e + j]) + a] += p->density * p->gravity[a] * V0[to + e] / 4.0;
            // lumped mass m_ii = R0 sum V0_e / 4 (Eq. fem_be), for inertia
            for (int j = 0; j < 4; ++j) mass[vo + p->tets[4 * e + j]] += p->density * V0[to + e] / 4.0;
        }
        if (p->nodal_force)
            for (int64_t i = 0; i < 3ll * p->n_verts; ++i) fext[3 * vo + i] += p->nodal_force[i];
        for (int k = 0; k < p->n_dirichlet; ++k) isdir[vo + p->dirichlet_idx[k]] = 1;
        inc[q] = incidence(p);
        for (int i = 0; i < p->n_verts; ++i) {
            valence[vo + i] = inc[q].tptr[i + 1] - inc[q].tptr[i];
            if (!isdir[vo + i]) ws->nfree_inst[q]++;
        }
    }
    if (ws->ncol > 64) fail(PBNG_ECOLOR, "more than 64 colours");
    {
        bool lam_ge_mu = true;
        for (int64_t e = 0; e < nt; ++e) lam_ge_mu = lam_ge_mu && lam[e] >= mu[e];
        // (the stable Neo-Hookean step has no such guarantee: its volume term
        // has a curvature along x_i that the modified Hessian does not bound)
        ws->safeguard_inactive = ws->n_planes == 0 &&
                                 (ws->model == PBNG_COROTATED || (ws->model == PBNG_NEOHOOKEAN && lam_ge_mu));
        bool uniform = true;
        for (int q = 0; q < n && uniform; ++q)
            for (int64_t e = ws->t_off[q] + 1; e < ws->t_off[q + 1]; ++e)
                if (mu[e] != mu[ws->t_off[q]] || lam[e] != lam[ws->t_off[q]]) {
                    uniform = false;
                    break;
                }
        ws->kmodel = (ws->model == PBNG_NEOHOOKEAN && uniform) ? 3 : ws->model;
        inst_mu.assign(n, 0.0);
        inst_lam.assign(n, 0.0);
        for (int q = 0; q < n; ++q)
            if (ws->t_off[q + 1] > ws->t_off[q]) {
                inst_mu[q] = mu[ws->t_off[q]];
                inst_lam[q] = lam[ws->t_off[q]];
            }
    }

    // internal order
    std::vector<int> inst_of(nv);
    for (int q = 0; q < n; ++q)
        for (int64_t i = ws->v_off[q]; i < ws->v_off[q + 1]; ++i) inst_of[i] = q;
    std::vector<int> order;
    order.reserve(nv);
    for (int64_t i = 0; i < nv; ++i)
        if (!isdir[i]) order.push_back(int(i));
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (colors[a] != colors[b]) return colors[a] < colors[b];
        if (inst_of[a] != inst_of[b]) return inst_of[a] < inst_of[b];
        if (valence[a] != valence[b]) return valence[a] > valence[b];
        return a < b;
    });
    const int64_t nfree = int64_t(order.size());
    ws->nfree = nfree;
    for (int64_t i = 0; i < nv; ++i)
        if (isdir[i]) order.push_back(int(i));
    std::vector<int> int_of(nv);
    for (int64_t k = 0; k < nv; ++k) int_of[order[k]] = int(k);
    ws->col_ptr.assign(ws->ncol + 1, 0);
    for (int64_t k = 0; k < nfree; ++k) ws->col_ptr[colors[order[k]] + 1]++;
    for (int c = 0; c < ws->ncol; ++c) ws->col_ptr[c + 1] += ws->col_ptr[c];

    // visits: free vertices first (their records drive the sweeps), then
    // Dirichlet vertices (FP64 gathers only)
    std::vector<int> rvptr(nv + 1, 0), rv;
    std::vector<int> J1, J2, J3;
    rv.reserve(4 * nt);
    for (int64_t k = 0; k < nv; ++k) {
        const int gv = order[k];
        const int q = inst_of[gv];
        const int64_t vo = ws->v_off[q], to = ws->t_off[q];
        const int li = int(gv - vo);
        const Incidence& I = inc[q];
        for (int s = I.tptr[li]; s < I.tptr[li + 1]; ++s) {
            const int64_t e = to + (I.tlist[s] >> 2);
            const int slot = I.tlist[s] & 3;
            rv.push_back(int(e * 4 + slot));
            if (k < nfree) {
                // the other three vertices in increasing slot order (the
                // device record build takes their gradients in this order)
                int others[3], no = 0;
                for (int j = 0; j < 4; ++j)
                    if (j != slot) others[no++] = int_of[vo + ps[q].tets[4 * (e - to) + j]];
                J1.push_back(others[0]);
                J2.push_back(others[1]);
                J3.push_back(others[2]);
            }
        }
        rvptr[k + 1] = int(rv.size());
    }
    ws->nvis = int64_t(J1.size());
    ws->nvis_all = int64_t(rv.size());
    ws->mean_valence = nfree > 0 ? double(ws->nvis) / double(nfree) : 0.0;

    // packed visit streams (jv.xyz here; the rest is built on the device
    // from the FP64 tet geometry)
    const size_t rec_max = ws->math64() ? sizeof(double4) : sizeof(float4);
    const size_t pos_max = ws->pos64() ? sizeof(double4) : sizeof(float4);
    if (double(ws->nvis) * rec_max >= 4294967296.0 || double(nv) * pos_max >= 4294967296.0)
        fail(PBNG_EUNSUPPORTED, "workspace too large: visit streams and position arrays must stay "
                                "under 4 GiB each");
    std::vector<int32_t> JV(4 * ws->nvis, 0);
    for (int64_t k = 0; k < ws->nvis; ++k) {
        JV[4 * k] = J1[k];
        JV[4 * k + 1] = J2[k];
        JV[4 * k + 2] = J3[k];
    }

    // algorithmic bytes per colour phase
    ws->phase_bytes.assign(ws->ncol, 0);
    ws->phase_verts.assign(ws->ncol, 0);
    ws->phase_visits.assign(ws->ncol, 0);
    {
        std::vector<int> mark(nv, -1);
        for (int c = 0; c < ws->ncol; ++c) {
            int64_t uniq = 0;
            const int64_t vis = int64_t(rvptr[ws->col_ptr[c + 1]]) - rvptr[ws->col_ptr[c]];
            for (int64_t k = rvptr[ws->col_ptr[c]]; k < rvptr[ws->col_ptr[c + 1]]; ++k)
                for (int o : {J1[k], J2[k], J3[k]})
                    if (mark[o] != c) {
                        mark[o] = c;
                        ++uniq;
                    }
            ws->phase_visits[c] = vis;
            ws->phase_verts[c] = ws->col_ptr[c + 1] - ws->col_ptr[c];
            ws->phase_bytes[c] = vis * 60 + ws->phase_verts[c] * 24 + uniq * 12;
        }
    }
    // lanes per vertex of a colour: the power of two covering half the mean
    // number of visits, so that a lane takes about two visits (measured best
    // on MI355X for valence 8 and 32 grids)
    ws->phase_lanes.assign(ws->ncol, 1);
    for (int c = 0; c < ws->ncol; ++c) {
        const double mv = ws->phase_verts[c] ? double(ws->phase_visits[c]) / ws->phase_verts[c] : 1.0;
        int L = 1;
        while (L < 64 && 2 * L < mv) L *= 2;
        ws->phase_lanes[c] = L;
    }

    // per-vertex arrays in internal order
    std::vector<double> fext_int(3 * nv), fext_free(4 * nfree, 0.0), mass_free(nfree);
    std::vector<int> vinst_all(nv), orig_of(nv);
    for (int64_t k = 0; k < nv; ++k) {
        const int gv = order[k];
        orig_of[k] = gv;
        if (k < nfree) mass_free[k] = mass[gv];
        vinst_all[k] = inst_of[gv];
        for (int a = 0; a < 3; ++a) fext_int[3 * k + a] = fext[3 * gv + a];
        if (k < nfree)
            for (int a = 0; a < 3; ++a) fext_free[4 * k + a] = fext[3 * gv + a];
    }

    // static weak constraints with internal members (installed, together
    // with any contacts, by install_constraints)
    ws->h_wc_ptr.assign(1, 0);
    ws->h_wc_vert.clear();
    ws->h_wc_w.clear();
    ws->h_wc_K.clear();
    ws->h_wc_inst.clear();
    for (int q = 0; q < n; ++q) {
        const pbng_problem* p = ps + q;
        for (int c = 0; c < p->n_wc; ++c) {
            for (int k = p->wc_ptr[c]; k < p->wc_ptr[c + 1]; ++k) {
                ws->h_wc_vert.push_back(int_of[ws->v_off[q] + p->wc_vert[k]]);
                ws->h_wc_w.push_back(p->wc_w[k]);
            }
            ws->h_wc_ptr.push_back(int(ws->h_wc_vert.size()));
            for (int j = 0; j < 6; ++j) ws->h_wc_K.push_back(p->wc_K[6 * c + j]);
            ws->h_wc_inst.push_back(q);
        }
    }
    ws->h_int_of = int_of;
    ws->h_orig_of = orig_of;
    ws->h_vinst = vinst_all;
    std::vector<int> plane_ptr(n + 1, 0);
    std::vector<double> planes;
    for (int q = 0; q < n; ++q) {
        for (int k = 0; k < 5 * ps[q].n_planes; ++k) planes.push_back(ps[q].planes[k]);
        plane_ptr[q + 1] = int(p_off[q + 1]);
    }

    // FP64 tet data and energy slots
    std::vector<int4> tet(nt);
    std::vector<TetGeo> geo(nt);
    std::vector<int> vorder(nv);
    std::vector<int64_t> seg_r(n + 1);
    for (int q = 0; q < n; ++q) {
        const pbng_problem* p = ps + q;
        const int64_t vo = ws->v_off[q], to = ws->t_off[q];
        seg_r[q] = vo;
        for (int64_t e = 0; e < p->n_tets; ++e) {
            const int32_t* t = p->tets + 4 * e;
            tet[to + e] = int4{int_of[vo + t[0]], int_of[vo + t[1]], int_of[vo + t[2]], int_of[vo + t[3]]};
            TetGeo& G = geo[to + e];
            for (int c = 0; c < 9; ++c) G.dm[c] = dminv[9 * (to + e) + c];
            G.V0 = V0[to + e];
            G.mu = mu[to + e];
            G.lam = lam[to + e];
        }
        for (int i = 0; i < p->n_verts; ++i) vorder[vo + i] = int_of[vo + i];
    }
    seg_r[n] = nv;

    // Dirichlet targets
    std::vector<int> dir_internal(ws->nd), dir_pos(nv - nfree);
    std::vector<double> xd_int(4 * (nv - nfree), 0.0);
    {
        int k = 0;
        for (int q = 0; q < n; ++q)
            for (int j = 0; j < ps[q].n_dirichlet; ++j, ++k) {
                const int iv = int_of[ws->v_off[q] + ps[q].dirichlet_idx[j]];
                dir_internal[k] = iv;
                dir_pos[iv - nfree] = k;
                for (int a = 0; a < 3; ++a) xd_int[4 * (iv - nfree) + a] = ps[q].dirichlet_x[3 * j + a];
            }
    }

    // upload (the first HIP call: everything above is host-side validation and packing)
    hipchk(hipGetDevice(&ws->device), "hipGetDevice");
    auto upR = [&](Dev& d, const std::vector<double>& v) {
        if (ws->math64()) upload_real<double>(d, v);
        else upload_real<float>(d, v);
    };
    auto upP = [&](Dev& d, const std::vector<double>& v) {
        if (ws->pos64()) upload_real<double>(d, v);
        else upload_real<float>(d, v);
    };
    std::vector<int> vptr_free(rvptr.begin(), rvptr.begin() + nfree + 1);
    ws->vptr.upload(vptr_free);
    ws->jv.upload(JV);
    alloc_records(ws);
    ws->Sv.alloc(size_t(nfree) * (ws->math64() ? sizeof(double) : sizeof(float)));
    upR(ws->imu, inst_mu);
    upR(ws->ilam, inst_lam);
    ws->t_off_dev.upload(ws->t_off);
    upR(ws->fext, fext_free);
    ws->mass64.upload(mass_free);
    std::vector<int> vinst_free(vinst_all.begin(), vinst_all.begin() + nfree);
    ws->vinst.upload(vinst_free);
    ws->active.alloc(n * sizeof(int));
    ws->rejected.alloc(n * sizeof(int));
    ws->plane_ptr.upload(plane_ptr);
    upR(ws->planes, planes);
    ws->tet.upload(tet);
    ws->h_tet = tet;
    ws->h_rvptr = rvptr;
    ws->h_rv = rv;
    ws->geo.upload(geo);
    ws->vp.alloc(std::max<int64_t>(1, nt) * 12 * sizeof(double));
    ws->vorder.upload(vorder);
    ws->rvptr.upload(rvptr);
    ws->rv.upload(rv);
    ws->fext64.upload(fext_int);
    ws->vinst_all.upload(vinst_all);
    ws->planes64.upload(planes);
    ws->orig_of.upload(orig_of);
    ws->rsq.alloc(std::max<int64_t>(1, nv) * sizeof(double));
    upP(ws->xd_int, xd_int);
    ws->dir_internal.upload(dir_internal);
    ws->dir_pos.upload(dir_pos);
    Uploader up;
    ws->plan_r = make_plan(seg_r, ws->seg_r_cb, ws->seg_r_ce, ws->seg_r_q, ws->seg_r_part, up);
    install_constraints(ws, up);
    up.flush(ws->stage, ws->ustage, nullptr);
    ws->out_r.alloc(n * sizeof(double));
    ws->out_e.alloc(n * sizeof(double));
    ws->W.alloc(nv * ws->r4());
    ws->Wres.alloc(nv * ws->r4());
    hipchk(hipHostMalloc((void**)&ws->hbuf, 2 * n * sizeof(double)), "hipHostMalloc");
    hipchk(hipHostMalloc((void**)&ws->hact, n * sizeof(int)), "hipHostMalloc");
    hipchk(hipDeviceSynchronize(), "upload");
    hipchk(build_visits(ws, nullptr, nullptr, nullptr), "visit records");
    hipchk(hipDeviceSynchronize(), "visit records");
    ws->h_color.assign(nv, -1);
    for (int c = 0; c < ws->ncol; ++c)
        for (int k = ws->col_ptr[c]; k < ws->col_ptr[c + 1]; ++k) ws->h_color[k] = c;
    rebuild_phases(ws, up);
    up.flush(ws->stage, ws->ustage, nullptr);
}

template <class R, class PR>
SweepArgs<R, PR> sweep_args(pbng_workspace* ws, double omega, double gamma, int max_halvings)
{
    using R4 = typename R4t<R>::T;
    using P4 = typename R4t<PR>::T;
    SweepArgs<R, PR> a;
    a.W = ws->W.as<P4>();
    a.P = ws->P.as<P4>();
    a.N = ws->N.as<P4>();
    a.vptr = ws->vptr.as<int>();
    a.jv = ws->jv.as<int4>();
    a.ma = ws->ma.as<typename R4t<R>::T>();
    a.mb = ws->mb.as<typename R4t<R>::T>();
    a.mc = ws->mc.as<typename R2t<R>::T>();
    a.vmu = ws->vmu.as<R>();
    a.Sv = ws->Sv.as<R>();
    a.imu = ws->imu.as<R>();
    a.ilam = ws->ilam.as<R>();
    a.fext = ws->fext.as<R4>();
    // one instance: no per-vertex instance lookup (the solve loops run
    // sweeps only while that instance is active)
    a.vinst = ws->n_inst > 1 ? ws->vinst.as<int>() : nullptr;
    a.active = ws->active.as<int>();
    a.wvptr = ws->wvptr.as<int>();
    a.wv_c = ws->wv_c.as<int>();
    a.wv_s = ws->wv_s.as<R>();
    a.wc_ptr = ws->wc_ptr.as<int>();
    a.wc_vert = ws->wc_vert.as<int>();
    a.wc_w = ws->wc_w.as<R>();
    a.wc_K = ws->wc_K.as<R>();
    a.plane_ptr = ws->plane_ptr.as<int>();
    a.planes = ws->planes.as<R>();
    a.rejected = ws->rejected.as<int>();
    a.inert = ws->inertia ? ws->inert.as<R>() : nullptr;
    a.xhat = ws->inertia ? ws->xhat.as<P4>() : nullptr;
    a.vlist = nullptr;
    a.pcol = nullptr;
    a.pcolor = 0;
    a.list_from = 0;
    a.list_beg = 0;
    a.omega = PR(omega);
    a.gamma = PR(gamma);
    a.max_halvings = max_halvings;
    return a;
}

template <class R>
ResArgs<R> res_args(pbng_workspace* ws, const void* X)
{
    using R4 = typename R4t<R>::T;
    ResArgs<R> a;
    a.X = static_cast<const R4*>(X);
    a.tet = ws->tet.as<int4>();
    a.geo = ws->geo.as<TetGeo>();
    a.vp = ws->vp.as<double>();
    a.ebuf = ws->ebuf.as<double>();
    a.tet_eidx = ws->tet_eidx.as<int>();
    a.vorder = ws->vorder.as<int>();
    a.vert_eidx = ws->vert_eidx.as<int>();
    a.rvptr = ws->rvptr.as<int>();
    a.rv = ws->rv.as<int>();
    a.fext64 = ws->fext64.as<double>();
    a.vinst_all = ws->vinst_all.as<int>();
    a.wvptr = ws->wvptr.as<int>();
    a.wv_c = ws->wv_c.as<int>();
    a.wv_s64 = ws->wv_s64.as<double>();
    a.wc_ptr = ws->wc_ptr.as<int>();
    a.wc_vert = ws->wc_vert.as<int>();
    a.wc_w64 = ws->wc_w64.as<double>();
    a.wc_K64 = ws->wc_K64.as<double>();
    a.wc_eidx = ws->wc_eidx.as<int>();
    a.plane_ptr = ws->plane_ptr.as<int>();
    a.planes64 = ws->planes64.as<double>();
    a.orig_of = ws->orig_of.as<int>();
    a.inert64 = ws->inertia ? ws->inert64.as<double>() : nullptr;
    a.xhat64 = ws->inertia ? ws->xhat64.as<double>() : nullptr;
    a.n_free = int(ws->nfree);
    a.n_verts = int(ws->nv);
    a.n_tets = int(ws->nt);
    a.n_wc = ws->n_wc;
    a.model = ws->model;
    return a;
}

// FP64 residual norms and energies of positions X (internal order) into
// ws->hbuf[0..n) and ws->hbuf[n..2n); synchronises the stream.
template <class R>
void residual_internal(pbng_workspace* ws, const void* X, double* r_out, hipStream_t s)
{
    const ResArgs<R> a = res_args<R>(ws, X);
    hipchk(launch_residual<R>(a, ws->rsq.as<double>(), r_out, s), "residual");
    hipchk(launch_segsum(ws->rsq.as<double>(), ws->plan_r, ws->n_inst, ws->out_r.as<double>(), s), "residual sum");
    hipchk(launch_segsum(ws->ebuf.as<double>(), ws->plan_e, ws->n_inst, ws->out_e.as<double>(), s), "energy sum");
    hipchk(hipMemcpyAsync(ws->hbuf, ws->out_r.p, ws->n_inst * sizeof(double), hipMemcpyDeviceToHost, s), "d2h");
    hipchk(hipMemcpyAsync(ws->hbuf + ws->n_inst, ws->out_e.p, ws->n_inst * sizeof(double), hipMemcpyDeviceToHost, s), "d2h");
    hipchk(hipStreamSynchronize(s), "sync");
    for (int q = 0; q < ws->n_inst; ++q) ws->hbuf[q] = std::sqrt(ws->hbuf[q]);
}

bool safe_effective(const pbng_workspace* ws, const pbng_solve_opts* o)
{
    return o->safeguard == PBNG_SAFEGUARD_BACKTRACK && !ws->safeguard_inactive;
}

// Lanes per vertex for colour c: the requested power of two, or (0) the
// workspace's automatic choice for that colour.
int pick_lanes(const pbng_workspace* ws, int requested, int c)
{
    if (requested == 0) return c >= 0 && c < ws->ncol ? ws->phase_lanes[c] : 8;
    if (requested == 1 || requested == 2 || requested == 4 || requested == 8 || requested == 16 ||
        requested == 32 || requested == 64)
        return requested;
    fail(PBNG_EINVAL, "lanes must be 0, 1, 2, 4, 8, 16, 32 or 64");
}

void check_solve_opts(const pbng_solve_opts* o)
{
    if (!o) fail(PBNG_EINVAL, "options are null");
    if (o->max_sweeps < 0 || o->check_every < 1) fail(PBNG_EINVAL, "max_sweeps must be >= 0 and check_every >= 1");
    if (o->accel < 0 || o->accel > 2) fail(PBNG_EINVAL, "unknown acceleration %d", o->accel);
    if (o->safeguard < 0 || o->safeguard > 1) fail(PBNG_EINVAL, "unknown safeguard %d", o->safeguard);
    if (o->max_halvings < 0 || o->max_halvings > 60) fail(PBNG_EINVAL, "max_halvings out of range");
    if (!std::isfinite(o->rel_tol) || o->rel_tol < 0) fail(PBNG_EINVAL, "rel_tol must be >= 0");
    if (o->accel == PBNG_ACCEL_CHEBYSHEV && !(o->rho > 0 && o->rho < 1 && o->gamma > 0))
        fail(PBNG_EINVAL, "Chebyshev needs 0 < rho < 1 and gamma > 0");
    if (o->accel == PBNG_ACCEL_SOR && !(o->omega > 0 && o->omega < 2)) fail(PBNG_EINVAL, "SOR needs 0 < omega < 2");
}

// Chebyshev weight for the sweep that produces x^{l+1} (Sec. "Acceleration
// Techniques"): 1 for l < 2, 2 / (2 - rho^2) for l = 2, 4 / (4 - rho^2
// omega_l) for l > 2.
double chebyshev_next(int64_t l, double rho, double prev)
{
    if (l < 2) return 1.0;
    if (l == 2) return 2.0 / (2.0 - rho * rho);
    return 4.0 / (4.0 - rho * rho * prev);
}

void ensure_ring(pbng_workspace* ws)
{
    if (!ws->P.p) ws->P.alloc(ws->nv * ws->r4());
    if (!ws->N.p) ws->N.alloc(ws->nv * ws->r4());
}

// Launch slots of one colour's phase (home range, then recoloured list)
// into the kernel arguments; returns the slot range [vb, ve).
template <class Args>
std::pair<int, int> phase_slots(const pbng_workspace* ws, const pbng_workspace::PhaseSpec& ph, Args& a)
{
    const bool has_list = ph.le > ph.lb;
    a.vlist = has_list ? ws->xlist.as<int>() : nullptr;
    a.pcol = ws->moved_any ? ws->pcol.as<int>() : nullptr;
    a.pcolor = ph.color;
    a.list_from = ph.he;
    a.list_beg = ph.lb;
    return {ph.hb, ph.he + (ph.le - ph.lb)};
}

template <class R, class PR>
void launch_sweep(pbng_workspace* ws, const pbng_solve_opts* o, double omega, double gamma, hipStream_t s)
{
    const bool accel = o->accel != PBNG_ACCEL_NONE;
    SweepArgs<R, PR> a = sweep_args<R, PR>(ws, omega, gamma, o->max_halvings);
    for (const auto& ph : ws->phases) {
        const auto [vb, ve] = phase_slots(ws, ph, a);
        hipchk(launch_phase<R, PR>(a, ws->kmodel, pick_lanes(ws, o->lanes, ph.color), accel,
                                   safe_effective(ws, o), ws->kernel_mode(), vb, ve, s),
               "sweep launch");
    }
    if (accel) std::swap(ws->W.p, ws->N.p);
}

// Replays `reps` times a HIP graph holding `S` sweeps with fixed blend
// weights (the steady state of the acceleration), capturing it first if the
// launch arguments changed.  S is even when the blend swaps buffers, so the
// buffer roles after a replay equal those at capture time.
template <class R, class PR>
void graph_sweeps(pbng_workspace* ws, const pbng_solve_opts* o, int S, int reps, double omega, double gamma,
                  hipStream_t s)
{
    const pbng_workspace::GraphKey key{ws->W.p, ws->P.p, ws->N.p, omega, gamma, S, o->accel, o->safeguard,
                                       o->lanes, o->max_halvings, s};
    if (!ws->gexec || !(ws->gkey == key) || ws->gkey_lanes_version != ws->lanes_version) {
        ws->drop_graph();
        hipchk(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "capture begin");
        try {
            for (int k = 0; k < S; ++k) launch_sweep<R, PR>(ws, o, omega, gamma, s);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        hipGraph_t g = nullptr;
        hipchk(hipStreamEndCapture(s, &g), "capture end");
        const hipError_t e = hipGraphInstantiate(&ws->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        hipchk(e, "graph instantiate");
        ws->gkey = key;
        ws->gkey_lanes_version = ws->lanes_version;
        // the capture ran the host-side buffer swaps S times: even S restores them
    }
    for (int r = 0; r < reps; ++r) hipchk(hipGraphLaunch(ws->gexec, s), "graph launch");
}

template <class R, class PR>
int32_t solve_t(pbng_workspace* ws, void* x, const pbng_solve_opts* o, pbng_stats* st, hipStream_t s)
{
    using R4 = typename R4t<PR>::T;
    const int n = ws->n_inst;
    const bool accel = o->accel != PBNG_ACCEL_NONE;
    pick_lanes(ws, o->lanes, 0);
    if (accel) ensure_ring(ws);
    const bool resume = o->resume && ws->ring_valid;
    if (!resume) {
        hipchk(launch_load<PR>(static_cast<const PR*>(x), ws->orig_of.as<int>(), ws->xd_int.as<R4>(),
                              ws->W.as<R4>(), accel ? ws->P.as<R4>() : nullptr,
                              accel ? ws->N.as<R4>() : nullptr, int(ws->nfree), int(ws->nv), s),
               "load");
        ws->sweep_l = 0;
        ws->omega_l = 1.0;
    } else {
        hipchk(launch_load<PR>(static_cast<const PR*>(x), ws->orig_of.as<int>(), ws->xd_int.as<R4>(),
                              ws->W.as<R4>(), nullptr, nullptr, int(ws->nfree), int(ws->nv), s),
               "load");
    }
    ws->ring_valid = accel;
    hipchk(hipMemsetAsync(ws->rejected.p, 0, n * sizeof(int), s), "memset");
    residual_internal<PR>(ws, ws->W.p, nullptr, s);
    std::vector<double> r0(ws->hbuf, ws->hbuf + n), rr(r0), en(ws->hbuf + n, ws->hbuf + 2 * n);
    std::vector<int> act(n, 1), sweeps(n, 0), conv(n, 0);
    std::vector<double> ttol(n, -1.0);
    for (int q = 0; q < n; ++q) {
        if (!std::isfinite(r0[q])) fail(PBNG_ENAN, "instance %d: non-finite initial residual", q);
        if (r0[q] == 0.0 || (o->rel_tol > 0 && r0[q] <= 0.0)) {
            act[q] = 0;
            conv[q] = 1;
            ttol[q] = 0.0;
        }
    }
    auto push_active = [&]() {
        for (int q = 0; q < n; ++q) ws->hact[q] = act[q];
        hipchk(hipMemcpyAsync(ws->active.p, ws->hact, n * sizeof(int), hipMemcpyHostToDevice, s), "h2d");
    };
    push_active();
    hipchk(hipStreamSynchronize(s), "sync");
    const double t0 = now_ms();
    int n_active = 0;
    for (int q = 0; q < n; ++q) n_active += act[q];
    bool nan = false;
    const bool accel_swaps = o->accel != PBNG_ACCEL_NONE;
    int S = o->sweeps_per_graph > 0 ? o->sweeps_per_graph : 0;
    if (accel_swaps && (S & 1)) ++S;
    if (s == nullptr) S = 0;  // the legacy null stream cannot be captured
    for (int sw = 0; sw < o->max_sweeps && n_active > 0;) {
        double omega = 1.0, gamma = 1.0;
        if (o->accel == PBNG_ACCEL_CHEBYSHEV) {
            omega = chebyshev_next(ws->sweep_l, o->rho, ws->omega_l);
            gamma = o->gamma;
        } else if (o->accel == PBNG_ACCEL_SOR) {
            omega = o->omega;
        }
        // sweeps until the next residual check
        const int next_check = std::min(o->max_sweeps, (sw / o->check_every + 1) * o->check_every);
        const int todo = next_check - sw;
        // blend weights at their fixed point in the position precision: a
        // block of sweeps can be replayed from one captured graph
        // (for Chebyshev only past the special weights of l < 3, where
        // omega_{l+1} = omega_l marks the fixed point of the recurrence)
        const bool steady = o->accel != PBNG_ACCEL_CHEBYSHEV || (ws->sweep_l >= 3 && omega == ws->omega_l);
        int done = 1;
        if (S > 0 && steady && ws->sweep_l > 0 && todo >= S) {
            const int reps = todo / S;
            graph_sweeps<R, PR>(ws, o, S, reps, omega, gamma, s);
            done = reps * S;
            ws->sweep_l += done - 1;
        } else {
            launch_sweep<R, PR>(ws, o, omega, gamma, s);
        }
        ws->omega_l = omega;
        ws->sweep_l++;
        sw += done;
        for (int q = 0; q < n; ++q) sweeps[q] += act[q] * done;
        if (sw % o->check_every == 0 || sw == o->max_sweeps) {
            residual_internal<PR>(ws, ws->W.p, nullptr, s);
            const double t = now_ms() - t0;
            bool changed = false;
            for (int q = 0; q < n; ++q) {
                if (!act[q]) continue;
                rr[q] = ws->hbuf[q];
                en[q] = ws->hbuf[n + q];
                if (!std::isfinite(rr[q])) {
                    nan = true;
                    act[q] = 0;
                    changed = true;
                    continue;
                }
                if (o->rel_tol > 0 && rr[q] <= o->rel_tol * r0[q]) {
                    conv[q] = 1;
                    ttol[q] = t;
                    act[q] = 0;
                    changed = true;
                }
            }
            if (changed) {
                n_active = 0;
                for (int q = 0; q < n; ++q) n_active += act[q];
                push_active();
            }
        }
    }
    hipchk(launch_store<PR>(ws->W.as<R4>(), ws->orig_of.as<int>(), static_cast<PR*>(x), int(ws->nv), s), "store");
    std::vector<int> rej(n);
    hipchk(hipMemcpyAsync(rej.data(), ws->rejected.p, n * sizeof(int), hipMemcpyDeviceToHost, s), "d2h");
    hipchk(hipStreamSynchronize(s), "sync");
    const double t_all = now_ms() - t0;
    bool all = true;
    for (int q = 0; q < n; ++q) {
        all = all && conv[q];
        if (st) {
            st[q].sweeps = sweeps[q];
            st[q].converged = conv[q];
            st[q].n_colors = ws->moved_any ? std::max(ws->ncol_inst[q], ws->ncol_dyn) : ws->ncol_inst[q];
            st[q].rejected = rej[q];
            st[q].residual0 = r0[q];
            st[q].residual = rr[q];
            st[q].rel_residual = r0[q] > 0 ? rr[q] / r0[q] : 0.0;
            st[q].energy = en[q];
            st[q].time_ms = t_all;
            st[q].time_to_tol_ms = ttol[q];
            st[q].vertex_updates = double(sweeps[q]) * double(ws->nfree_inst[q]);
        }
    }
    if (nan) fail(PBNG_ENAN, "iterate became non-finite");
    return all ? PBNG_OK : PBNG_NOT_CONVERGED;
}

template <class R, class PR>
AdjArgs<R, PR> adj_args(pbng_workspace* ws, double omega, double gamma)
{
    using P4 = typename R4t<PR>::T;
    AdjArgs<R, PR> a;
    a.X = ws->Wres.as<P4>();
    a.L = ws->L.as<P4>();
    a.P = ws->LP.as<P4>();
    a.N = ws->LN.as<P4>();
    a.B = ws->B.as<P4>();
    a.vptr = ws->vptr.as<int>();
    a.jv = ws->jv.as<int4>();
    a.ma = ws->ma.as<typename R4t<R>::T>();
    a.mb = ws->mb.as<typename R4t<R>::T>();
    a.mc = ws->mc.as<typename R2t<R>::T>();
    a.vmu = ws->vmu.as<R>();
    a.Sv = ws->Sv.as<R>();
    a.imu = ws->imu.as<R>();
    a.ilam = ws->ilam.as<R>();
    a.vinst = ws->vinst.as<int>();
    a.wvptr = ws->wvptr.as<int>();
    a.wv_c = ws->wv_c.as<int>();
    a.wv_s = ws->wv_s.as<R>();
    a.wc_ptr = ws->wc_ptr.as<int>();
    a.wc_vert = ws->wc_vert.as<int>();
    a.wc_w = ws->wc_w.as<R>();
    a.wc_K = ws->wc_K.as<R>();
    a.plane_ptr = ws->plane_ptr.as<int>();
    a.planes = ws->planes.as<R>();
    a.inert = ws->inertia ? ws->inert.as<R>() : nullptr;
    a.vlist = nullptr;
    a.pcol = nullptr;
    a.pcolor = 0;
    a.list_from = 0;
    a.list_beg = 0;
    a.omega = PR(omega);
    a.gamma = PR(gamma);
    return a;
}

template <class R>
void adjoint_check(pbng_workspace* ws, double* dmu, double* dlam, double* dxd, hipStream_t s)
{
    using R4 = typename R4t<R>::T;
    const ResArgs<R> a = res_args<R>(ws, ws->Wres.p);
    hipchk(launch_adjoint_assembly<R>(a, ws->L.as<R4>(), ws->B.as<R4>(), ws->rsq.as<double>(), dmu, dlam, dxd,
                                      ws->dir_pos.as<int>(), s),
           "adjoint assembly");
    hipchk(launch_segsum(ws->rsq.as<double>(), ws->plan_r, ws->n_inst, ws->out_r.as<double>(), s), "sum");
    hipchk(hipMemcpyAsync(ws->hbuf, ws->out_r.p, ws->n_inst * sizeof(double), hipMemcpyDeviceToHost, s), "d2h");
    hipchk(hipStreamSynchronize(s), "sync");
    for (int q = 0; q < ws->n_inst; ++q) ws->hbuf[q] = std::sqrt(ws->hbuf[q]);
}

template <class R, class PR>
int32_t adjoint_t(pbng_workspace* ws, const void* x_eq, const void* dLdx, double* dxd, double* dmu,
                  double* dlam, double* lam_out, const pbng_adjoint_opts* o, pbng_stats* st,
                  hipStream_t s)
{
    using R4 = typename R4t<PR>::T;
    const int n = ws->n_inst;
    const bool accel = o->accel == PBNG_ACCEL_CHEBYSHEV;
    pick_lanes(ws, o->lanes, 0);
    if (!ws->L.p) ws->L.alloc(ws->nv * ws->r4());
    if (!ws->B.p) ws->B.alloc(ws->nv * ws->r4());
    if (accel) {
        if (!ws->LP.p) ws->LP.alloc(ws->nv * ws->r4());
        if (!ws->LN.p) ws->LN.alloc(ws->nv * ws->r4());
    }
    hipchk(launch_load<PR>(static_cast<const PR*>(x_eq), ws->orig_of.as<int>(), nullptr, ws->Wres.as<R4>(), nullptr,
                          nullptr, int(ws->nfree), int(ws->nv), s),
           "load");
    hipchk(launch_load_vec<PR>(static_cast<const PR*>(dLdx), ws->orig_of.as<int>(), ws->B.as<R4>(), int(ws->nfree),
                              int(ws->nv), s),
           "load");
    hipchk(hipMemsetAsync(ws->L.p, 0, ws->nv * ws->r4(), s), "memset");
    if (accel) {
        hipchk(hipMemsetAsync(ws->LP.p, 0, ws->nv * ws->r4(), s), "memset");
        hipchk(hipMemsetAsync(ws->LN.p, 0, ws->nv * ws->r4(), s), "memset");
    }
    adjoint_check<PR>(ws, nullptr, nullptr, nullptr, s);
    std::vector<double> b0(ws->hbuf, ws->hbuf + n), rr(b0);
    std::vector<int> act(n, 1), sweeps(n, 0), conv(n, 0);
    int n_active = 0;
    for (int q = 0; q < n; ++q) {
        if (!std::isfinite(b0[q])) fail(PBNG_ENAN, "instance %d: non-finite dL/dx", q);
        if (b0[q] == 0.0) {
            act[q] = 0;
            conv[q] = 1;
        }
        n_active += act[q];
    }
    const double t0 = now_ms();
    double omega_prev = 1.0;
    for (int64_t sw = 0; sw < o->max_sweeps && n_active > 0; ++sw) {
        double omega = 1.0;
        if (accel) omega = chebyshev_next(sw, o->rho, omega_prev);
        omega_prev = omega;
        AdjArgs<R, PR> a = adj_args<R, PR>(ws, omega, accel ? o->gamma : 1.0);
        for (const auto& ph : ws->phases) {
            const auto [vb, ve] = phase_slots(ws, ph, a);
            hipchk(launch_adjoint_phase<R, PR>(a, ws->kmodel, pick_lanes(ws, o->lanes, ph.color), accel,
                                               ws->any_wc || ws->inertia || ws->moved_any, vb, ve, s),
                   "adjoint launch");
        }
        if (accel) std::swap(ws->L.p, ws->LN.p);
        for (int q = 0; q < n; ++q) sweeps[q] += act[q];
        if ((sw + 1) % o->check_every == 0 || sw + 1 == o->max_sweeps) {
            adjoint_check<PR>(ws, nullptr, nullptr, nullptr, s);
            n_active = 0;
            for (int q = 0; q < n; ++q) {
                if (!act[q]) continue;
                rr[q] = ws->hbuf[q];
                if (!std::isfinite(rr[q])) fail(PBNG_ENAN, "adjoint iterate became non-finite");
                if (o->rel_tol > 0 && rr[q] <= o->rel_tol * b0[q]) {
                    conv[q] = 1;
                    act[q] = 0;
                }
                n_active += act[q];
            }
        }
    }
    // final assembly with the gradients
    adjoint_check<PR>(ws, dmu, dlam, dxd, s);
    for (int q = 0; q < n; ++q) rr[q] = ws->hbuf[q];
    if (lam_out)
        hipchk(launch_store64<PR>(ws->L.as<R4>(), ws->orig_of.as<int>(), lam_out, int(ws->nv), s), "store");
    hipchk(hipStreamSynchronize(s), "sync");
    const double t_all = now_ms() - t0;
    bool all = true;
    for (int q = 0; q < n; ++q) {
        conv[q] = conv[q] || (o->rel_tol > 0 && rr[q] <= o->rel_tol * b0[q]) || b0[q] == 0.0;
        all = all && conv[q];
        if (st) {
            st[q] = pbng_stats{};
            st[q].sweeps = sweeps[q];
            st[q].converged = conv[q];
            st[q].n_colors = ws->moved_any ? std::max(ws->ncol_inst[q], ws->ncol_dyn) : ws->ncol_inst[q];
            st[q].residual0 = b0[q];
            st[q].residual = rr[q];
            st[q].rel_residual = b0[q] > 0 ? rr[q] / b0[q] : 0.0;
            st[q].time_ms = t_all;
            st[q].time_to_tol_ms = -1.0;
            st[q].vertex_updates = double(sweeps[q]) * double(ws->nfree_inst[q]);
        }
    }
    return all ? PBNG_OK : PBNG_NOT_CONVERGED;
}

void check_ws(const pbng_workspace* ws)
{
    if (!ws) fail(PBNG_EINVAL, "workspace is null");
}

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    Events()
    {
        hipchk(hipEventCreate(&a), "event");
        hipchk(hipEventCreate(&b), "event");
    }
    ~Events()
    {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    float ms()
    {
        hipchk(hipEventSynchronize(b), "event sync");
        float t = 0.f;
        hipchk(hipEventElapsedTime(&t, a, b), "event time");
        return t;
    }
};

// The launch of one colour (its home range and the list of vertices
// recoloured into it), with the blend weights 1.
template <class R, class PR>
void phase_t(pbng_workspace* ws, const pbng_solve_opts* o, int color, hipStream_t s)
{
    SweepArgs<R, PR> a = sweep_args<R, PR>(ws, 1.0, 1.0, o->max_halvings);
    for (const auto& ph : ws->phases) {
        if (ph.color != color) continue;
        const auto [vb, ve] = phase_slots(ws, ph, a);
        hipchk(launch_phase<R, PR>(a, ws->kmodel, pick_lanes(ws, o->lanes, color), o->accel != PBNG_ACCEL_NONE,
                                   safe_effective(ws, o), ws->kernel_mode(), vb, ve, s),
               "phase");
    }
}

// Measured choice of the lanes per vertex of every colour (the tile of the
// colour-phase kernel) and of the sweeps per captured graph.
template <class R, class PR>
void autotune_t(pbng_workspace* ws, const void* x, const pbng_solve_opts* o, pbng_solve_opts* tuned,
                hipStream_t s)
{
    using P4 = typename R4t<PR>::T;
    ensure_ring(ws);
    auto reload = [&]() {
        hipchk(launch_load<PR>(static_cast<const PR*>(x), ws->orig_of.as<int>(), ws->xd_int.as<P4>(), ws->W.as<P4>(),
                               ws->P.as<P4>(), ws->N.as<P4>(), int(ws->nfree), int(ws->nv), s),
               "load");
        for (int q = 0; q < ws->n_inst; ++q) ws->hact[q] = 1;
        hipchk(hipMemcpyAsync(ws->active.p, ws->hact, ws->n_inst * sizeof(int), hipMemcpyHostToDevice, s), "h2d");
        hipchk(hipMemsetAsync(ws->rejected.p, 0, ws->n_inst * sizeof(int), s), "memset");
    };
    reload();
    Events ev;
    pbng_solve_opts q = *o;
    q.lanes = 0;
    // Lanes per colour: each candidate is timed inside whole sweeps (the
    // other colours at their current choice), so that the caches see the
    // solve's mix of phases; the valence heuristic stays unless a candidate
    // beats it by more than timing noise.
    auto time_sweeps = [&]() {
        float t = 1e30f;
        for (int trial = 0; trial < 3; ++trial) {
            hipchk(hipEventRecord(ev.a, s), "record");
            for (int k = 0; k < 16; ++k) launch_sweep<R, PR>(ws, &q, 1.0, 1.0, s);
            hipchk(hipEventRecord(ev.b, s), "record");
            t = std::min(t, ev.ms());
        }
        return t;
    };
    for (int c = 0; c < ws->ncol; ++c) {
        const int vb = ws->col_ptr[c], ve = ws->col_ptr[c + 1];
        if (ve <= vb) continue;
        const double mv = double(ws->phase_visits[c]) / double(ve - vb);
        const int heur = ws->phase_lanes[c];
        int best = heur;
        float best_t = time_sweeps();
        for (int L = 1; L <= 64; L *= 2) {
            if (L == heur || L > 2 * mv + 1 || 16 * L < mv) continue;
            ws->phase_lanes[c] = L;
            const float t = time_sweeps();
            if (t < 0.98f * best_t) {
                best_t = t;
                best = L;
            }
        }
        ws->phase_lanes[c] = best;
    }
    ws->lanes_version++;
    // sweeps per graph: plain launches against replayed graphs
    const int n_sw = 64;
    int best_S = 0;
    float best_t = 1e30f;
    for (int S : {0, 2, 8, 32}) {
        q.sweeps_per_graph = S;
        float t = 1e30f;
        for (int trial = 0; trial < 2; ++trial) {
            reload();
            if (S > 0) graph_sweeps<R, PR>(ws, &q, S, 1, 1.0, 1.0, s);  // capture outside the timing
            hipchk(hipEventRecord(ev.a, s), "record");
            if (S == 0) {
                for (int k = 0; k < n_sw; ++k) launch_sweep<R, PR>(ws, &q, 1.0, 1.0, s);
            } else {
                graph_sweeps<R, PR>(ws, &q, S, n_sw / S, 1.0, 1.0, s);
            }
            hipchk(hipEventRecord(ev.b, s), "record");
            t = std::min(t, ev.ms());
        }
        // a graph must win by more than timing noise to be chosen
        if (S == 0 || t < 0.98f * best_t) {
            if (t < best_t || S == 0) {
                best_t = t;
                best_S = S;
            }
        }
    }
    ws->drop_graph();
    ws->ring_valid = false;
    hipchk(hipStreamSynchronize(s), "sync");
    *tuned = *o;
    tuned->lanes = 0;
    tuned->sweeps_per_graph = best_S;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int32_t pbng_version(void) { return PBNG_ABI_VERSION; }

const char* pbng_last_error(void) { return g_err.c_str(); }

int32_t pbng_lame(int64_t n, const double* E, const double* nu, double* mu_out, double* lambda_out)
{
    return guard([&] {
        if (n < 0 || (n > 0 && (!E || !nu || !mu_out || !lambda_out))) fail(PBNG_EINVAL, "null argument");
        for (int64_t i = 0; i < n; ++i) {
            if (!(E[i] > 0) || !(nu[i] > -1.0 && nu[i] < 0.5)) fail(PBNG_EINVAL, "need E > 0 and -1 < nu < 0.5");
            mu_out[i] = E[i] / (2.0 * (1.0 + nu[i]));
            lambda_out[i] = E[i] * nu[i] / ((1.0 + nu[i]) * (1.0 - 2.0 * nu[i]));
        }
        return PBNG_OK;
    });
}

int32_t pbng_default_solve_opts(pbng_solve_opts* o)
{
    return guard([&] {
        if (!o) fail(PBNG_EINVAL, "null options");
        *o = pbng_solve_opts{};
        o->max_sweeps = 1000;
        o->rel_tol = 1e-5;
        o->check_every = 10;
        o->accel = PBNG_ACCEL_NONE;
        o->rho = 0.95;
        o->gamma = 1.7;
        o->omega = 1.7;
        o->safeguard = PBNG_SAFEGUARD_BACKTRACK;
        o->max_halvings = 8;
        o->lanes = 0;
        o->sweeps_per_graph = 0;
        o->resume = 0;
        return PBNG_OK;
    });
}

int32_t pbng_default_adjoint_opts(pbng_adjoint_opts* o)
{
    return guard([&] {
        if (!o) fail(PBNG_EINVAL, "null options");
        *o = pbng_adjoint_opts{};
        o->max_sweeps = 5000;
        o->rel_tol = 1e-6;
        o->check_every = 20;
        o->accel = PBNG_ACCEL_CHEBYSHEV;
        o->rho = 0.95;
        o->gamma = 1.0;
        o->lanes = 0;
        return PBNG_OK;
    });
}

int32_t pbng_color(const pbng_problem* p, int32_t* colors_out, int32_t* n_colors_out)
{
    return guard([&] {
        if (!p || !colors_out || !n_colors_out) fail(PBNG_EINVAL, "null argument");
        validate_topology(p, 0);
        *n_colors_out = color_instance(p, colors_out);
        return PBNG_OK;
    });
}

int32_t pbng_workspace_create(const pbng_problem* p, int32_t n_problems, const int32_t* colors, int32_t real,
                              pbng_workspace** ws_out)
{
    return guard([&] {
        if (!p || !ws_out || n_problems <= 0) fail(PBNG_EINVAL, "null argument or n_problems <= 0");
        if (real != PBNG_F32 && real != PBNG_F64 && real != PBNG_MIXED)
            fail(PBNG_EINVAL, "real must be PBNG_F32, PBNG_F64 or PBNG_MIXED");
        *ws_out = nullptr;
        pbng_workspace* ws = new pbng_workspace;
        ws->real = real;
        try {
            build_workspace(ws, p, n_problems, colors);
        } catch (...) {
            delete ws;
            throw;
        }
        *ws_out = ws;
        return PBNG_OK;
    });
}

int32_t pbng_workspace_destroy(pbng_workspace* ws)
{
    return guard([&] {
        delete ws;
        return PBNG_OK;
    });
}

int32_t pbng_workspace_info(const pbng_workspace* ws, int64_t* n_verts, int64_t* n_tets, int64_t* n_free,
                            int32_t* n_colors, int64_t* n_visits, int32_t* n_instances)
{
    return guard([&] {
        check_ws(ws);
        if (n_verts) *n_verts = ws->nv;
        if (n_tets) *n_tets = ws->nt;
        if (n_free) *n_free = ws->nfree;
        if (n_colors) *n_colors = ws->ncol_dyn;
        if (n_visits) *n_visits = ws->nvis;
        if (n_instances) *n_instances = ws->n_inst;
        return PBNG_OK;
    });
}

int32_t pbng_workspace_set_materials(pbng_workspace* ws, const double* mu_dev, const double* lambda_dev,
                                     void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (!mu_dev || !lambda_dev) fail(PBNG_EINVAL, "null material arrays");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (ws->model == PBNG_NEOHOOKEAN) {
            // The Neo-Hookean step is a descent step without the safeguard
            // only while lambda >= mu in every tet, and the 40-byte records
            // need one (mu, lambda) per instance: re-check both on the device.
            if (!ws->flag.p) ws->flag.alloc(2 * sizeof(int));
            hipError_t e = ws->math64()
                               ? launch_material_flags<double>(mu_dev, lambda_dev, ws->t_off_dev.as<int64_t>(),
                                                               ws->n_inst, int(ws->nt), ws->flag.as<int>(),
                                                               ws->imu.as<double>(), ws->ilam.as<double>(), s)
                               : launch_material_flags<float>(mu_dev, lambda_dev, ws->t_off_dev.as<int64_t>(),
                                                              ws->n_inst, int(ws->nt), ws->flag.as<int>(),
                                                              ws->imu.as<float>(), ws->ilam.as<float>(), s);
            hipchk(e, "material check");
            int h[2] = {0, 0};
            hipchk(hipMemcpyAsync(h, ws->flag.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "material check");
            hipchk(hipStreamSynchronize(s), "material check");
            const bool was_inactive = ws->safeguard_inactive;
            ws->safeguard_inactive = ws->n_planes == 0 && h[0] != 0;
            // the safeguard decides the kernel variant a captured graph holds
            if (was_inactive != ws->safeguard_inactive) ws->drop_graph();
            const int km = h[1] ? 3 : PBNG_NEOHOOKEAN;
            if (km != ws->kmodel) {
                // the record form changes: new streams, new kernel variant
                ws->kmodel = km;
                alloc_records(ws);
                ws->drop_graph();
            }
        }
        hipchk(build_visits(ws, mu_dev, lambda_dev, s), "set materials");
        return PBNG_OK;
    });
}

int32_t pbng_workspace_set_dirichlet(pbng_workspace* ws, const double* xd_dev, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (ws->nd > 0 && !xd_dev) fail(PBNG_EINVAL, "null Dirichlet array");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (ws->pos64())
            hipchk(launch_set_dirichlet<double>(xd_dev, ws->dir_internal.as<int>(), ws->nd, int(ws->nfree),
                                                ws->xd_int.as<double4>(), s),
                   "set dirichlet");
        else
            hipchk(launch_set_dirichlet<float>(xd_dev, ws->dir_internal.as<int>(), ws->nd, int(ws->nfree),
                                               ws->xd_int.as<float4>(), s),
                   "set dirichlet");
        ws->ring_valid = false;
        return PBNG_OK;
    });
}

int32_t pbng_workspace_set_inertia(pbng_workspace* ws, double dt, const double* x_n_dev,
                                   const double* x_prev_dev, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (std::isnan(dt) || std::isinf(dt)) fail(PBNG_EINVAL, "time step must be finite");
        const bool was = ws->inertia;
        if (dt <= 0.0) {
            ws->inertia = false;
        } else {
            if (!x_n_dev || !x_prev_dev) fail(PBNG_EINVAL, "null x^n or x^{n-1} array");
            hipStream_t s = static_cast<hipStream_t>(hip_stream);
            const int nf = int(ws->nfree);
            if (!ws->inert.p) {
                ws->inert.alloc(size_t(nf) * (ws->math64() ? sizeof(double) : sizeof(float)));
                ws->xhat.alloc(size_t(nf) * ws->r4());
                ws->inert64.alloc(size_t(nf) * sizeof(double));
                ws->xhat64.alloc(size_t(nf) * 3 * sizeof(double));
            }
            hipError_t e;
            if (ws->real == PBNG_F64)
                e = launch_set_inertia<double, double>(x_n_dev, x_prev_dev, ws->orig_of.as<int>(),
                                                       ws->mass64.as<double>(), nf, dt, ws->inert.as<double>(),
                                                       ws->xhat.as<double4>(), ws->inert64.as<double>(),
                                                       ws->xhat64.as<double>(), s);
            else if (ws->real == PBNG_MIXED)
                e = launch_set_inertia<float, double>(x_n_dev, x_prev_dev, ws->orig_of.as<int>(),
                                                      ws->mass64.as<double>(), nf, dt, ws->inert.as<float>(),
                                                      ws->xhat.as<double4>(), ws->inert64.as<double>(),
                                                      ws->xhat64.as<double>(), s);
            else
                e = launch_set_inertia<float, float>(x_n_dev, x_prev_dev, ws->orig_of.as<int>(),
                                                     ws->mass64.as<double>(), nf, dt, ws->inert.as<float>(),
                                                     ws->xhat.as<float4>(), ws->inert64.as<double>(),
                                                     ws->xhat64.as<double>(), s);
            hipchk(e, "set inertia");
            ws->inertia = true;
        }
        // the kernel variant (and its arguments) changes with inertia on or off
        if (was != ws->inertia) ws->drop_graph();
        ws->ring_valid = false;
        return PBNG_OK;
    });
}

int32_t pbng_workspace_set_contacts(pbng_workspace* ws, int32_t n, const int32_t* pairs_dev,
                                    const double* normals_dev, double k_n, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (n < 0) fail(PBNG_EINVAL, "negative contact count");
        if (n > 0 && (!pairs_dev || !normals_dev)) fail(PBNG_EINVAL, "null contact arrays");
        if (n > 0 && !(k_n > 0.0 && std::isfinite(k_n))) fail(PBNG_EINVAL, "contact stiffness must be > 0");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        std::vector<int32_t> pr(2 * size_t(n));
        std::vector<double> nr(3 * size_t(n));
        if (n > 0) {
            hipchk(hipMemcpyAsync(pr.data(), pairs_dev, pr.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s), "d2h");
            hipchk(hipMemcpyAsync(nr.data(), normals_dev, nr.size() * sizeof(double), hipMemcpyDeviceToHost, s), "d2h");
            hipchk(hipStreamSynchronize(s), "sync");
        }
        std::vector<pbng_workspace::Contact> cts(n);
        for (int k = 0; k < n; ++k) {
            const int ga = pr[2 * k], gb = pr[2 * k + 1];
            if (ga < 0 || gb < 0 || ga >= ws->nv || gb >= ws->nv || ga == gb)
                fail(PBNG_EINVAL, "contact %d: bad vertex pair", k);
            const int a = ws->h_int_of[ga], b = ws->h_int_of[gb];
            if (ws->h_vinst[a] != ws->h_vinst[b]) fail(PBNG_EINVAL, "contact %d joins two instances", k);
            const double* v = nr.data() + 3 * k;
            const double len = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (!(len > 0.0) || !std::isfinite(len)) fail(PBNG_EINVAL, "contact %d: bad normal", k);
            const double nx = v[0] / len, ny = v[1] / len, nz = v[2] / len;
            cts[k].a = a;
            cts[k].b = b;
            cts[k].inst = ws->h_vinst[a];
            const double K[6] = {k_n * nx * nx, k_n * nx * ny, k_n * nx * nz, k_n * ny * ny, k_n * ny * nz, k_n * nz * nz};
            for (int j = 0; j < 6; ++j) cts[k].K[j] = K[j];
        }
        // the constraint arrays keep their allocations (Dev::reserve): no
        // queued work may still read them
        hipchk(hipDeviceSynchronize(), "contacts");
        ws->contacts = std::move(cts);
        Uploader up;
        install_constraints(ws, up);
        recolor_contacts(ws);
        rebuild_phases(ws, up);
        up.flush(ws->stage, ws->ustage, s);
        ws->drop_graph();
        ws->ring_valid = false;
        return PBNG_OK;
    });
}

// Candidates of the proximity detection: vertices of faces that belong to a
// single tet, with their caller index, instance, connected part (union-find
// over the tets) and Dirichlet flag.
void build_candidates(pbng_workspace* ws)
{
    const int nv = int(ws->nv);
    std::vector<int> parent(nv);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int i) {
        while (parent[i] != i) {
            parent[i] = parent[parent[i]];
            i = parent[i];
        }
        return i;
    };
    std::vector<std::array<int, 3>> faces;
    faces.reserve(4 * ws->h_tet.size());
    for (const int4& t : ws->h_tet) {
        const int v[4] = {t.x, t.y, t.z, t.w};
        for (int j = 1; j < 4; ++j) {
            const int a = find(v[0]), b = find(v[j]);
            if (a != b) parent[b] = a;
        }
        for (int skip = 0; skip < 4; ++skip) {
            std::array<int, 3> f;
            int m = 0;
            for (int j = 0; j < 4; ++j)
                if (j != skip) f[m++] = v[j];
            std::sort(f.begin(), f.end());
            faces.push_back(f);
        }
    }
    std::sort(faces.begin(), faces.end());
    std::vector<char> surf(nv, 0);
    for (size_t i = 0; i < faces.size();) {
        size_t j = i + 1;
        while (j < faces.size() && faces[j] == faces[i]) ++j;
        if (j - i == 1)
            for (int v : faces[i]) surf[v] = 1;
        i = j;
    }
    std::vector<int> caller, inst, body, dir;
    for (int v = 0; v < nv; ++v)
        if (surf[v]) {
            caller.push_back(ws->h_orig_of[v]);
            inst.push_back(ws->h_vinst[v]);
            body.push_back(find(v));
            dir.push_back(v >= ws->nfree ? 1 : 0);
        }
    ws->n_cand = int(caller.size());
    ws->cand_caller.upload(caller);
    ws->cand_inst.upload(inst);
    ws->cand_body.upload(body);
    ws->cand_dir.upload(dir);
}

int32_t pbng_detect_contacts(pbng_workspace* ws, const void* x_dev, double radius, int32_t max_pairs,
                             int32_t* pairs_dev, double* normals_dev, int32_t* n_found, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (!x_dev || !n_found) fail(PBNG_EINVAL, "null argument");
        if (!(radius > 0.0) || !std::isfinite(radius)) fail(PBNG_EINVAL, "radius must be > 0");
        if (max_pairs < 0 || (max_pairs > 0 && (!pairs_dev || !normals_dev)))
            fail(PBNG_EINVAL, "bad output arrays");
        if (ws->n_inst >= (1 << 18)) fail(PBNG_EUNSUPPORTED, "too many instances for detection");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (ws->n_cand < 0) build_candidates(ws);
        const int cap = std::max(max_pairs, 1);
        if (ws->det_cap < cap) {
            const int nc = std::max(ws->n_cand, 1);
            ws->d_keys_in.alloc(size_t(nc) * 8);
            ws->d_keys_out.alloc(size_t(nc) * 8);
            ws->d_vals_in.alloc(size_t(nc) * 4);
            ws->d_vals_out.alloc(size_t(nc) * 4);
            ws->d_pairs.alloc(size_t(cap) * 8);
            ws->d_pkeys_in.alloc(size_t(cap) * 8);
            ws->d_pkeys_out.alloc(size_t(cap) * 8);
            ws->d_count.alloc(sizeof(int));
            ws->d_tmp_bytes = detect_tmp_bytes(nc, cap);
            ws->d_tmp.alloc(ws->d_tmp_bytes);
            ws->det_cap = cap;
        }
        auto bits = [](int64_t v) {
            int b = 0;
            while (v > 0) {
                ++b;
                v >>= 1;
            }
            return b;
        };
        ContactCand c{ws->n_cand, ws->cand_caller.as<int>(), ws->cand_inst.as<int>(), ws->cand_body.as<int>(),
                      ws->cand_dir.as<int>(), bits(ws->n_inst - 1), std::max(1, bits(ws->nv - 1))};
        DetectScratch w{ws->d_keys_in.as<unsigned long long>(), ws->d_keys_out.as<unsigned long long>(),
                        ws->d_vals_in.as<int>(), ws->d_vals_out.as<int>(), ws->d_pairs.as<int2>(),
                        ws->d_pkeys_in.as<unsigned long long>(), ws->d_pkeys_out.as<unsigned long long>(),
                        ws->d_count.as<int>(), ws->d_tmp.p, ws->d_tmp_bytes};
        int nf = 0;
        hipError_t e = ws->pos64()
                           ? launch_detect<double>(static_cast<const double*>(x_dev), c, radius, max_pairs, w,
                                                   pairs_dev, normals_dev, &nf, s)
                           : launch_detect<float>(static_cast<const float*>(x_dev), c, radius, max_pairs, w,
                                                  pairs_dev, normals_dev, &nf, s);
        hipchk(e, "detect contacts");
        hipchk(hipStreamSynchronize(s), "detect contacts");
        *n_found = nf;
        if (nf > max_pairs) fail(PBNG_EINVAL, "found %d contacts, more than max_pairs = %d", nf, max_pairs);
        return PBNG_OK;
    });
}

int32_t pbng_workspace_colors(const pbng_workspace* ws, int32_t* colors_out)
{
    return guard([&] {
        check_ws(ws);
        if (!colors_out) fail(PBNG_EINVAL, "null colours array");
        for (int64_t k = 0; k < ws->nv; ++k) colors_out[ws->h_orig_of[k]] = ws->h_color[k];
        return PBNG_OK;
    });
}

int32_t pbng_solve(pbng_workspace* ws, void* x_inout, const pbng_solve_opts* o, pbng_stats* stats, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (!x_inout) fail(PBNG_EINVAL, "x_inout is null");
        check_solve_opts(o);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (ws->real == PBNG_F64) return solve_t<double, double>(ws, x_inout, o, stats, s);
        if (ws->real == PBNG_MIXED) return solve_t<float, double>(ws, x_inout, o, stats, s);
        return solve_t<float, float>(ws, x_inout, o, stats, s);
    });
}

int32_t pbng_residual(pbng_workspace* ws, const void* x, double* res_norm, double* energy, double* r_out,
                      void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (!x) fail(PBNG_EINVAL, "x is null");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (ws->pos64()) {
            hipchk(launch_load<double>(static_cast<const double*>(x), ws->orig_of.as<int>(), nullptr,
                                       ws->Wres.as<double4>(), nullptr, nullptr, int(ws->nfree), int(ws->nv), s),
                   "load");
            residual_internal<double>(ws, ws->Wres.p, r_out, s);
        } else {
            hipchk(launch_load<float>(static_cast<const float*>(x), ws->orig_of.as<int>(), nullptr,
                                      ws->Wres.as<float4>(), nullptr, nullptr, int(ws->nfree), int(ws->nv), s),
                   "load");
            residual_internal<float>(ws, ws->Wres.p, r_out, s);
        }
        for (int q = 0; q < ws->n_inst; ++q) {
            if (res_norm) res_norm[q] = ws->hbuf[q];
            if (energy) energy[q] = ws->hbuf[ws->n_inst + q];
        }
        return PBNG_OK;
    });
}

int32_t pbng_adjoint(pbng_workspace* ws, const void* x_eq, const void* dL_dx, double* dL_dxD, double* dL_dmu,
                     double* dL_dlambda, double* lam_out, const pbng_adjoint_opts* o, pbng_stats* stats,
                     void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (!x_eq || !dL_dx || !o) fail(PBNG_EINVAL, "null argument");
        if (o->max_sweeps < 0 || o->check_every < 1) fail(PBNG_EINVAL, "bad adjoint sweep counts");
        if (o->accel != PBNG_ACCEL_NONE && o->accel != PBNG_ACCEL_CHEBYSHEV)
            fail(PBNG_EINVAL, "adjoint acceleration must be none or Chebyshev");
        if (o->accel == PBNG_ACCEL_CHEBYSHEV && !(o->rho > 0 && o->rho < 1 && o->gamma > 0))
            fail(PBNG_EINVAL, "Chebyshev needs 0 < rho < 1 and gamma > 0");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (ws->real == PBNG_F64)
            return adjoint_t<double, double>(ws, x_eq, dL_dx, dL_dxD, dL_dmu, dL_dlambda, lam_out, o, stats, s);
        if (ws->real == PBNG_MIXED)
            return adjoint_t<float, double>(ws, x_eq, dL_dx, dL_dxD, dL_dmu, dL_dlambda, lam_out, o, stats, s);
        return adjoint_t<float, float>(ws, x_eq, dL_dx, dL_dxD, dL_dmu, dL_dlambda, lam_out, o, stats, s);
    });
}

int32_t pbng_load(pbng_workspace* ws, const void* x, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (!x) fail(PBNG_EINVAL, "x is null");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        ensure_ring(ws);
        if (ws->pos64())
            hipchk(launch_load<double>(static_cast<const double*>(x), ws->orig_of.as<int>(), ws->xd_int.as<double4>(),
                                       ws->W.as<double4>(), ws->P.as<double4>(), ws->N.as<double4>(),
                                       int(ws->nfree), int(ws->nv), s),
                   "load");
        else
            hipchk(launch_load<float>(static_cast<const float*>(x), ws->orig_of.as<int>(), ws->xd_int.as<float4>(),
                                      ws->W.as<float4>(), ws->P.as<float4>(), ws->N.as<float4>(), int(ws->nfree),
                                      int(ws->nv), s),
                   "load");
        hipchk(hipMemsetAsync(ws->rejected.p, 0, ws->n_inst * sizeof(int), s), "memset");
        for (int q = 0; q < ws->n_inst; ++q) ws->hact[q] = 1;
        hipchk(hipMemcpyAsync(ws->active.p, ws->hact, ws->n_inst * sizeof(int), hipMemcpyHostToDevice, s), "h2d");
        hipchk(hipStreamSynchronize(s), "sync");
        ws->sweep_l = 0;
        ws->omega_l = 1.0;
        ws->ring_valid = true;
        return PBNG_OK;
    });
}

int32_t pbng_store(pbng_workspace* ws, void* x, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        if (!x) fail(PBNG_EINVAL, "x is null");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (ws->pos64())
            hipchk(launch_store<double>(ws->W.as<double4>(), ws->orig_of.as<int>(), static_cast<double*>(x),
                                        int(ws->nv), s),
                   "store");
        else
            hipchk(launch_store<float>(ws->W.as<float4>(), ws->orig_of.as<int>(), static_cast<float*>(x), int(ws->nv),
                                       s),
                   "store");
        return PBNG_OK;
    });
}

int32_t pbng_sweeps(pbng_workspace* ws, int32_t n_sweeps, const pbng_solve_opts* o, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        check_solve_opts(o);
        if (!ws->ring_valid) fail(PBNG_EINVAL, "call pbng_load first");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        pick_lanes(ws, o->lanes, 0);
        for (int k = 0; k < n_sweeps; ++k) {
            double omega = 1.0, gamma = 1.0;
            if (o->accel == PBNG_ACCEL_CHEBYSHEV) {
                omega = chebyshev_next(ws->sweep_l, o->rho, ws->omega_l);
                gamma = o->gamma;
            } else if (o->accel == PBNG_ACCEL_SOR) {
                omega = o->omega;
            }
            if (ws->real == PBNG_F64) launch_sweep<double, double>(ws, o, omega, gamma, s);
            else if (ws->real == PBNG_MIXED) launch_sweep<float, double>(ws, o, omega, gamma, s);
            else launch_sweep<float, float>(ws, o, omega, gamma, s);
            ws->omega_l = omega;
            ws->sweep_l++;
        }
        return PBNG_OK;
    });
}

int32_t pbng_phase(pbng_workspace* ws, int32_t color, const pbng_solve_opts* o, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        check_solve_opts(o);
        if (!ws->ring_valid) fail(PBNG_EINVAL, "call pbng_load first");
        if (color < 0 || color >= ws->ncol_dyn) fail(PBNG_EINVAL, "colour out of range");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        // with acceleration the phase blends with omega = 1 and gamma = 1 and
        // does not advance the ring (measurement of the fused kernel only)
        if (ws->real == PBNG_F64) phase_t<double, double>(ws, o, color, s);
        else if (ws->real == PBNG_MIXED) phase_t<float, double>(ws, o, color, s);
        else phase_t<float, float>(ws, o, color, s);
        return PBNG_OK;
    });
}

int32_t pbng_autotune(pbng_workspace* ws, const void* x, const pbng_solve_opts* o, pbng_solve_opts* tuned,
                      int32_t* lanes_out, void* hip_stream)
{
    return guard([&] {
        check_ws(ws);
        check_solve_opts(o);
        if (!x || !tuned) fail(PBNG_EINVAL, "null argument");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (s == nullptr) fail(PBNG_EINVAL, "pbng_autotune needs a non-null stream (graphs are captured)");
        if (ws->real == PBNG_F64) autotune_t<double, double>(ws, x, o, tuned, s);
        else if (ws->real == PBNG_MIXED) autotune_t<float, double>(ws, x, o, tuned, s);
        else autotune_t<float, float>(ws, x, o, tuned, s);
        if (lanes_out)
            for (int c = 0; c < ws->ncol; ++c) lanes_out[c] = ws->phase_lanes[c];
        return PBNG_OK;
    });
}

int32_t pbng_phase_bytes(const pbng_workspace* ws, int32_t color, int64_t* bytes, int64_t* vertices,
                         int64_t* visits)
{
    return guard([&] {
        check_ws(ws);
        if (color < 0 || color >= ws->ncol_dyn) fail(PBNG_EINVAL, "colour out of range");
        // the figures of the colour's home range (as packed at creation)
        const bool home = color < ws->ncol;
        if (bytes) *bytes = home ? ws->phase_bytes[color] : 0;
        if (vertices) *vertices = home ? ws->phase_verts[color] : 0;
        if (visits) *visits = home ? ws->phase_visits[color] : 0;
        return PBNG_OK;
    });
}

}  // extern "C"
