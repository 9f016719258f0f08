// libpbng host side for planar problems (include/pbng2d.h): validation,
// node colouring, packing of the device layout of pbng2d.hpp and the solve
// and residual drivers.  No C++ exception leaves this file.
#include "pbng2d.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "pbng2d.hpp"
#include "pbng_hostutil.hpp"

using namespace pbng;

struct pbng2d_workspace {
    int real = PBNG_F32;
    int model = 0;
    int64_t nv = 0, nt = 0, nfree = 0, nvis = 0;
    int ncol = 0;
    bool uniform = false;           // one (mu, lambda): 24-byte records, no vw stream
    double mu_u = 0.0, lam_u = 0.0;
    std::vector<int> cptr;          // [ncol + 1] colour ranges, internal order
    std::vector<int> orig_h;        // internal -> caller
    std::vector<int> colors_h;      // caller order, -1 on Dirichlet vertices
    std::vector<int64_t> ph_bytes, ph_verts, ph_visits;
    Dev W, P, N, Wres;              // R2 [nv]
    Dev vptr, jk, gm, vw, fext, rejected;
    Dev tri, geo, vp, ebuf, rsq, rvptr, rv, fext64, orig_of, xd_int;
    Dev cb_r, ce_r, qp_r, part_r, cb_e, ce_e, qp_e, part_e, out;
    SegPlan plan_r, plan_e;
    double* hbuf = nullptr;         // pinned [2]
    int64_t sweep_l = 0;
    double omega_l = 1.0;
    // weak constraints (internal vertex indices; per free vertex CSR),
    // half-planes and inertia
    int n_wc = 0, n_planes = 0;
    bool inertia = false;
    std::vector<double> mass_h;     // lumped m_ii, internal order
    Dev wvptr, wv_c, wv_s, wv_s64, wc_ptr, wc_vert, wc_w, wc_w64, wc_K, wc_K64, planes, planes64;
    Dev inert, inert64, xhat, xhat64;
    // adjoint: equilibrium, iterate ring, right-hand side (internal order),
    // Dirichlet vertex -> its position in the caller's Dirichlet list
    Dev XA, LA, LPa, LNa, BA, dir_pos;
    bool extra() const { return n_wc > 0 || n_planes > 0 || inertia; }

    size_t r2() const { return real == PBNG_F64 ? 2 * sizeof(double) : 2 * sizeof(float); }
    ~pbng2d_workspace()
    {
        if (hbuf) (void)hipHostFree(hbuf);
    }
};

namespace {

bool finite_all(const double* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

// Rest shape-function gradients of triangle t: rows dN_1, dN_2 of Dm^{-1},
// Dm = [X1 - X0, X2 - X0]; returns the rest area det(Dm) / 2.
double tri_rest(const double* X, const int32_t* t, double* g1, double* g2)
{
    const double a = X[2 * t[1]] - X[2 * t[0]], b = X[2 * t[2]] - X[2 * t[0]];
    const double c = X[2 * t[1] + 1] - X[2 * t[0] + 1], d = X[2 * t[2] + 1] - X[2 * t[0] + 1];
    const double det = a * d - b * c;  // Dm = [[a, b], [c, d]]
    g1[0] = d / det;
    g1[1] = -b / det;
    g2[0] = -c / det;
    g2[1] = a / det;
    return 0.5 * det;
}

void validate2(const pbng2d_problem* p)
{
    if (!p) fail(PBNG_EINVAL, "problem is null");
    if (p->n_verts < 1 || p->n_tris < 1) fail(PBNG_EINVAL, "need at least one vertex and one triangle");
    // the vertex -> triangle incidence holds 3 n_tris int32 entries
    if (p->n_tris > INT32_MAX / 3) fail(PBNG_EUNSUPPORTED, "too many triangles for 32-bit indices");
    if (!p->rest_pos || !p->tris) fail(PBNG_EINVAL, "rest_pos and tris are required");
    if (p->model != PBNG_NEOHOOKEAN && p->model != PBNG_COROTATED) {
        if (p->model == PBNG_STABLE_NEOHOOKEAN)
            fail(PBNG_EUNSUPPORTED, "the stable Neo-Hookean model is not offered for triangle meshes");
        fail(PBNG_EINVAL, "unknown model %d", p->model);
    }
    if (!finite_all(p->rest_pos, 2 * int64_t(p->n_verts))) fail(PBNG_ENAN, "non-finite rest position");
    for (int e = 0; e < p->n_tris; ++e) {
        const int32_t* t = p->tris + 3 * e;
        for (int j = 0; j < 3; ++j)
            if (t[j] < 0 || t[j] >= p->n_verts) fail(PBNG_EMESH, "triangle %d: vertex index out of range", e);
        if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) fail(PBNG_EMESH, "triangle %d: repeated vertex", e);
        double g1[2], g2[2];
        if (!(tri_rest(p->rest_pos, t, g1, g2) > 0.0))
            fail(PBNG_EMESH, "triangle %d: rest area <= 0 (vertices must be counter-clockwise)", e);
    }
    for (int e = 0; e < p->n_tris; ++e) {
        const double mu = p->mu_tri ? p->mu_tri[e] : p->mu;
        const double la = p->lambda_tri ? p->lambda_tri[e] : p->lambda;
        if (!(std::isfinite(mu) && std::isfinite(la) && mu > 0.0 && la > 0.0))
            fail(PBNG_EMATERIAL, "triangle %d: need finite mu > 0 and lambda > 0", e);
    }
    if (!std::isfinite(p->density) || !std::isfinite(p->gravity[0]) || !std::isfinite(p->gravity[1]))
        fail(PBNG_ENAN, "non-finite body force");
    if (p->nodal_force && !finite_all(p->nodal_force, 2 * int64_t(p->n_verts)))
        fail(PBNG_ENAN, "non-finite nodal force");
    if (p->n_dirichlet < 0 || p->n_dirichlet > p->n_verts) fail(PBNG_EINVAL, "bad n_dirichlet");
    if (p->n_dirichlet > 0 && (!p->dirichlet_idx || !p->dirichlet_x)) fail(PBNG_EINVAL, "Dirichlet arrays are null");
    std::vector<char> seen(p->n_verts, 0);
    for (int k = 0; k < p->n_dirichlet; ++k) {
        const int i = p->dirichlet_idx[k];
        if (i < 0 || i >= p->n_verts) fail(PBNG_EMESH, "Dirichlet index out of range");
        if (seen[i]) fail(PBNG_EINVAL, "repeated Dirichlet vertex %d", i);
        seen[i] = 1;
    }
    if (p->n_dirichlet > 0 && !finite_all(p->dirichlet_x, 2 * int64_t(p->n_dirichlet)))
        fail(PBNG_ENAN, "non-finite Dirichlet target");
    if (p->n_wc < 0) fail(PBNG_EINVAL, "bad n_wc");
    if (p->n_wc > 0) {
        if (!p->wc_ptr || !p->wc_vert || !p->wc_w || !p->wc_K) fail(PBNG_EINVAL, "weak-constraint arrays are null");
        if (p->wc_ptr[0] != 0) fail(PBNG_EINVAL, "wc_ptr[0] must be 0");
        for (int c = 0; c < p->n_wc; ++c)
            if (p->wc_ptr[c + 1] < p->wc_ptr[c]) fail(PBNG_EINVAL, "wc_ptr not monotone");
        const int nnz = p->wc_ptr[p->n_wc];
        for (int k = 0; k < nnz; ++k)
            if (p->wc_vert[k] < 0 || p->wc_vert[k] >= p->n_verts) fail(PBNG_EMESH, "weak-constraint vertex out of range");
        for (int c = 0; c < p->n_wc; ++c)
            for (int k = p->wc_ptr[c]; k < p->wc_ptr[c + 1]; ++k)
                for (int j = p->wc_ptr[c]; j < k; ++j)
                    if (p->wc_vert[j] == p->wc_vert[k]) fail(PBNG_EMESH, "weak constraint %d repeats a vertex", c);
        if (!finite_all(p->wc_w, nnz) || !finite_all(p->wc_K, 3 * int64_t(p->n_wc)))
            fail(PBNG_ENAN, "non-finite weak constraint");
    }
    if (p->n_planes < 0) fail(PBNG_EINVAL, "bad n_planes");
    if (p->n_planes > 0) {
        if (!p->planes) fail(PBNG_EINVAL, "planes is null");
        if (!finite_all(p->planes, 4 * int64_t(p->n_planes))) fail(PBNG_ENAN, "non-finite half-plane");
        for (int q = 0; q < p->n_planes; ++q)
            if (p->planes[4 * q + 3] < 0.0) fail(PBNG_EINVAL, "half-plane stiffness < 0");
    }
}

struct Inc {
    std::vector<int> ptr, tri, slot;
    std::vector<int> cptr, clist, cpos;   // vertex -> weak constraints
};

Inc incidence2(const pbng2d_problem* p)
{
    Inc I;
    I.ptr.assign(p->n_verts + 1, 0);
    for (int e = 0; e < p->n_tris; ++e)
        for (int j = 0; j < 3; ++j) I.ptr[p->tris[3 * e + j] + 1]++;
    for (int i = 0; i < p->n_verts; ++i) I.ptr[i + 1] += I.ptr[i];
    I.tri.resize(3 * size_t(p->n_tris));
    I.slot.resize(3 * size_t(p->n_tris));
    std::vector<int> fill(p->n_verts, 0);
    for (int e = 0; e < p->n_tris; ++e)
        for (int j = 0; j < 3; ++j) {
            const int v = p->tris[3 * e + j];
            const int k = I.ptr[v] + fill[v]++;
            I.tri[k] = e;
            I.slot[k] = j;
        }
    const int nnz = p->n_wc > 0 ? p->wc_ptr[p->n_wc] : 0;
    I.cptr.assign(p->n_verts + 1, 0);
    for (int k = 0; k < nnz; ++k) I.cptr[p->wc_vert[k] + 1]++;
    for (int i = 0; i < p->n_verts; ++i) I.cptr[i + 1] += I.cptr[i];
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

std::vector<char> dir_mask(const pbng2d_problem* p)
{
    std::vector<char> d(p->n_verts, 0);
    for (int k = 0; k < p->n_dirichlet; ++k) d[p->dirichlet_idx[k]] = 1;
    return d;
}

int color2(const pbng2d_problem* p, const Inc& I, int32_t* colors)
{
    const std::vector<char> dir = dir_mask(p);
    int ncol = 0;
    for (int i = 0; i < p->n_verts; ++i) colors[i] = -1;
    for (int i = 0; i < p->n_verts; ++i) {
        if (dir[i]) continue;
        uint64_t used = 0;
        for (int k = I.ptr[i]; k < I.ptr[i + 1]; ++k) {
            const int32_t* t = p->tris + 3 * I.tri[k];
            for (int j = 0; j < 3; ++j)
                if (colors[t[j]] >= 0) used |= uint64_t(1) << colors[t[j]];
        }
        for (int k = I.cptr[i]; k < I.cptr[i + 1]; ++k) {
            const int c = I.clist[k];
            for (int m = p->wc_ptr[c]; m < p->wc_ptr[c + 1]; ++m)
                if (colors[p->wc_vert[m]] >= 0) used |= uint64_t(1) << colors[p->wc_vert[m]];
        }
        if (used == ~uint64_t(0)) fail(PBNG_ECOLOR, "more than 64 colours needed");
        int c = 0;
        while (used >> c & 1) ++c;
        colors[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

int check_colors2(const pbng2d_problem* p, const int32_t* colors)
{
    const std::vector<char> dir = dir_mask(p);
    int ncol = 0;
    for (int i = 0; i < p->n_verts; ++i) {
        if (dir[i] ? colors[i] != -1 : (colors[i] < 0 || colors[i] >= 64))
            fail(PBNG_ECOLOR, "vertex %d: colour %d invalid", i, colors[i]);
        ncol = std::max(ncol, colors[i] + 1);
    }
    for (int e = 0; e < p->n_tris; ++e) {
        const int32_t* t = p->tris + 3 * e;
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b)
                if (colors[t[a]] >= 0 && colors[t[a]] == colors[t[b]])
                    fail(PBNG_ECOLOR, "triangle %d: two vertices share colour %d", e, colors[t[a]]);
    }
    for (int c = 0; c < p->n_wc; ++c)
        for (int k = p->wc_ptr[c]; k < p->wc_ptr[c + 1]; ++k)
            for (int j = p->wc_ptr[c]; j < k; ++j) {
                const int ca = colors[p->wc_vert[j]], cb = colors[p->wc_vert[k]];
                if (ca >= 0 && ca == cb) fail(PBNG_ECOLOR, "weak constraint %d: two vertices share colour %d", c, ca);
            }
    return ncol;
}

SegPlan plan_range(int64_t n, Dev& cb, Dev& ce, Dev& qp, Dev& part)
{
    const int64_t chunk = 4096;
    std::vector<int64_t> b, e;
    for (int64_t s = 0; s < n; s += chunk) {
        b.push_back(s);
        e.push_back(std::min(n, s + chunk));
    }
    std::vector<int> q = {0, int(b.size())};
    cb.upload(b);
    ce.upload(e);
    qp.upload(q);
    part.alloc(std::max<size_t>(1, b.size()) * sizeof(double));
    SegPlan P;
    P.cbeg = cb.as<int64_t>();
    P.cend = ce.as<int64_t>();
    P.qptr = qp.as<int>();
    P.partial = part.as<double>();
    P.n_chunks = int(b.size());
    return P;
}

template <class R>
void pack(pbng2d_workspace* ws, const pbng2d_problem* p, const Inc& I, const std::vector<int>& int_of)
{
    using R2 = typename R2t<R>::T;
    using R4 = typename R4t<R>::T;
    const int64_t nf = ws->nfree, nv = ws->nv, nt = ws->nt;
    std::vector<int> vptr(nf + 1, 0);
    for (int64_t v = 0; v < nf; ++v) {
        const int o = ws->orig_h[v];
        vptr[v + 1] = vptr[v] + (I.ptr[o + 1] - I.ptr[o]);
    }
    ws->nvis = vptr[nf];
    std::vector<int2> jk(std::max<int64_t>(1, ws->nvis));
    std::vector<R4> gm(std::max<int64_t>(1, ws->nvis));
    std::vector<R2> vw(std::max<int64_t>(1, ws->nvis));
    std::vector<TriGeo> geo(nt);
    std::vector<int4> tri(nt);
    for (int64_t e = 0; e < nt; ++e) {
        const int32_t* t = p->tris + 3 * e;
        TriGeo G;
        double g1[2], g2[2];
        G.A0 = tri_rest(p->rest_pos, t, g1, g2);
        G.g1x = g1[0];
        G.g1y = g1[1];
        G.g2x = g2[0];
        G.g2y = g2[1];
        G.mu = p->mu_tri ? p->mu_tri[e] : p->mu;
        G.lam = p->lambda_tri ? p->lambda_tri[e] : p->lambda;
        geo[e] = G;
        tri[e] = int4{int_of[t[0]], int_of[t[1]], int_of[t[2]], 0};
    }
    for (int64_t v = 0; v < nf; ++v) {
        const int o = ws->orig_h[v];
        int k = vptr[v];
        for (int m = I.ptr[o]; m < I.ptr[o + 1]; ++m, ++k) {
            const int e = I.tri[m], s = I.slot[m];
            const int32_t* t = p->tris + 3 * e;
            const TriGeo& G = geo[e];
            const double gx[3] = {-(G.g1x + G.g2x), G.g1x, G.g2x};
            const double gy[3] = {-(G.g1y + G.g2y), G.g1y, G.g2y};
            const int j = (s + 1) % 3, l = (s + 2) % 3;
            jk[k] = int2{int_of[t[j]], int_of[t[l]]};
            gm[k] = R4{R(gx[j]), R(gy[j]), R(gx[l]), R(gy[l])};
            vw[k] = R2{R(G.A0 * G.mu), R(G.A0 * G.lam)};
        }
    }
    // lumped loads: R0 g A0 / 3 per incident triangle, then nodal forces
    std::vector<double> f(2 * nv, 0.0);
    for (int64_t e = 0; e < nt; ++e)
        for (int j = 0; j < 3; ++j)
            for (int c = 0; c < 2; ++c)
                f[2 * size_t(p->tris[3 * e + j]) + c] += p->density * p->gravity[c] * geo[e].A0 / 3.0;
    if (p->nodal_force)
        for (int64_t i = 0; i < 2 * nv; ++i) f[i] += p->nodal_force[i];
    std::vector<double> f64(2 * nv);
    std::vector<R2> fr(std::max<int64_t>(1, nf));
    for (int64_t v = 0; v < nv; ++v) {
        const int o = ws->orig_h[v];
        f64[2 * v] = f[2 * size_t(o)];
        f64[2 * v + 1] = f[2 * size_t(o) + 1];
        if (v < nf) fr[v] = R2{R(f64[2 * v]), R(f64[2 * v + 1])};
    }
    std::vector<R2> xd(std::max<int64_t>(1, nv - nf));
    {
        std::vector<int> pos(p->n_verts, -1);
        for (int k = 0; k < p->n_dirichlet; ++k) pos[p->dirichlet_idx[k]] = k;
        std::vector<int> dpos(std::max<int64_t>(1, nv - nf), 0);
        for (int64_t v = nf; v < nv; ++v) {
            const int k = pos[ws->orig_h[v]];
            xd[v - nf] = R2{R(p->dirichlet_x[2 * k]), R(p->dirichlet_x[2 * k + 1])};
            dpos[v - nf] = k;
        }
        ws->dir_pos.upload(dpos);
    }
    // weak constraints in internal indices, the per-free-vertex CSR of
    // (constraint, weight), half-planes and the lumped masses
    ws->n_wc = p->n_wc;
    ws->n_planes = p->n_planes;
    {
        const int nnz = p->n_wc > 0 ? p->wc_ptr[p->n_wc] : 0;
        std::vector<int> wcp(p->n_wc + 1, 0), wcv(std::max(1, nnz)), wvp(nv + 1, 0), wvc;
        std::vector<double> wcw(std::max(1, nnz)), wck(std::max<int64_t>(1, 3 * int64_t(p->n_wc))), wvs;
        if (p->n_wc > 0) std::copy(p->wc_ptr, p->wc_ptr + p->n_wc + 1, wcp.begin());
        for (int k = 0; k < nnz; ++k) {
            wcv[k] = int_of[p->wc_vert[k]];
            wcw[k] = p->wc_w[k];
        }
        for (int64_t k = 0; k < 3 * int64_t(p->n_wc); ++k) wck[k] = p->wc_K[k];
        for (int64_t v = 0; v < nv; ++v) {   // every vertex (the adjoint needs the Dirichlet rows)
            const int o = ws->orig_h[v];
            for (int m = I.cptr[o]; m < I.cptr[o + 1]; ++m) {
                wvc.push_back(I.clist[m]);
                wvs.push_back(p->wc_w[I.cpos[m]]);
            }
            wvp[v + 1] = int(wvc.size());
        }
        if (wvc.empty()) {
            wvc.push_back(0);
            wvs.push_back(0.0);
        }
        std::vector<double> pl(std::max<int64_t>(1, 4 * int64_t(p->n_planes)), 0.0);
        for (int64_t k = 0; k < 4 * int64_t(p->n_planes); ++k) pl[k] = p->planes[k];
        auto conv = [](const std::vector<double>& a) { return std::vector<R>(a.begin(), a.end()); };
        ws->wc_ptr.upload(wcp);
        ws->wc_vert.upload(wcv);
        ws->wc_w.upload(conv(wcw));
        ws->wc_w64.upload(wcw);
        ws->wc_K.upload(conv(wck));
        ws->wc_K64.upload(wck);
        ws->wvptr.upload(wvp);
        ws->wv_c.upload(wvc);
        ws->wv_s.upload(conv(wvs));
        ws->wv_s64.upload(wvs);
        ws->planes.upload(conv(pl));
        ws->planes64.upload(pl);
        // lumped mass of Eq. (fem_be) with d = 2: R0 A0 / 3 per incident triangle
        ws->mass_h.assign(nv, 0.0);
        for (int64_t e = 0; e < nt; ++e) {
            const int ids[3] = {tri[e].x, tri[e].y, tri[e].z};
            for (int j = 0; j < 3; ++j) ws->mass_h[ids[j]] += p->density * geo[e].A0 / 3.0;
        }
    }
    ws->vptr.upload(vptr);
    ws->jk.upload(jk);
    ws->gm.upload(gm);
    ws->uniform = true;
    for (int64_t e = 1; e < nt && ws->uniform; ++e)
        ws->uniform = geo[e].mu == geo[0].mu && geo[e].lam == geo[0].lam;
    ws->mu_u = geo[0].mu;
    ws->lam_u = geo[0].lam;
    if (!ws->uniform) ws->vw.upload(vw);
    ws->fext.upload(fr);
    // triangle slots (3 e + local index) of every vertex, internal order
    {
        std::vector<int> rvp(nv + 1, 0), rva;
        rva.reserve(3 * size_t(nt));
        for (int64_t v = 0; v < nv; ++v) {
            const int o = ws->orig_h[v];
            for (int m = I.ptr[o]; m < I.ptr[o + 1]; ++m) rva.push_back(3 * I.tri[m] + I.slot[m]);
            rvp[v + 1] = int(rva.size());
        }
        if (rva.empty()) rva.push_back(0);
        ws->rvptr.upload(rvp);
        ws->rv.upload(rva);
    }
    ws->geo.upload(geo);
    ws->tri.upload(tri);
    ws->fext64.upload(f64);
    ws->xd_int.upload(xd);
    ws->orig_of.upload(ws->orig_h);
    // algorithmic bytes per colour phase, defined on the full 32-byte record
    // (FP32 form; doubled floats in FP64) whether or not vw is streamed
    const int64_t fb = ws->real == PBNG_F64 ? 2 : 1;
    ws->ph_bytes.assign(ws->ncol, 0);
    ws->ph_verts.assign(ws->ncol, 0);
    ws->ph_visits.assign(ws->ncol, 0);
    std::vector<int> mark(nv, -1);
    for (int c = 0; c < ws->ncol; ++c) {
        int64_t uniq = 0, vis = 0;
        for (int v = ws->cptr[c]; v < ws->cptr[c + 1]; ++v)
            for (int k = vptr[v]; k < vptr[v + 1]; ++k) {
                ++vis;
                for (int q : {jk[k].x, jk[k].y})
                    if (mark[q] != c) {
                        mark[q] = c;
                        ++uniq;
                    }
            }
        const int64_t nverts = ws->cptr[c + 1] - ws->cptr[c];
        ws->ph_verts[c] = nverts;
        ws->ph_visits[c] = vis;
        ws->ph_bytes[c] = vis * (8 + 24 * fb) + nverts * (4 + 24 * fb) + uniq * 8 * fb;
    }
}

void build2(pbng2d_workspace* ws, const pbng2d_problem* p, const int32_t* colors_in, int real)
{
    validate2(p);
    if (real != PBNG_F32 && real != PBNG_F64) fail(PBNG_EINVAL, "real must be PBNG_F32 or PBNG_F64");
    ws->real = real;
    ws->model = p->model;
    ws->nv = p->n_verts;
    ws->nt = p->n_tris;
    const Inc I = incidence2(p);
    ws->colors_h.assign(p->n_verts, -1);
    if (colors_in) {
        ws->ncol = check_colors2(p, colors_in);
        std::copy(colors_in, colors_in + p->n_verts, ws->colors_h.begin());
    } else {
        ws->ncol = color2(p, I, ws->colors_h.data());
    }
    // internal order: free vertices by colour, decreasing valence, caller
    // index; then Dirichlet vertices by caller index
    std::vector<int> order(p->n_verts);
    std::iota(order.begin(), order.end(), 0);
    const std::vector<int>& col = ws->colors_h;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int ca = col[a] < 0 ? 1 << 20 : col[a], cb = col[b] < 0 ? 1 << 20 : col[b];
        if (ca != cb) return ca < cb;
        if (col[a] < 0) return a < b;
        const int va = I.ptr[a + 1] - I.ptr[a], vb = I.ptr[b + 1] - I.ptr[b];
        if (va != vb) return va > vb;
        return a < b;
    });
    ws->orig_h = order;
    std::vector<int> int_of(p->n_verts);
    for (int v = 0; v < p->n_verts; ++v) int_of[order[v]] = v;
    ws->nfree = 0;
    for (int i = 0; i < p->n_verts; ++i) ws->nfree += col[i] >= 0;
    ws->cptr.assign(ws->ncol + 1, 0);
    for (int i = 0; i < p->n_verts; ++i)
        if (col[i] >= 0) ws->cptr[col[i] + 1]++;
    for (int c = 0; c < ws->ncol; ++c) ws->cptr[c + 1] += ws->cptr[c];
    // kernels address the visit streams and positions through 32-bit byte
    // offsets: the largest stream (FP64 shape gradients, 32 B per visit, at
    // most three visits per triangle) and the FP64 positions must stay below 4 GiB
    if (int64_t(3) * ws->nt * int64_t(sizeof(double4)) >= (int64_t(1) << 32) ||
        ws->nv * int64_t(sizeof(double2)) >= (int64_t(1) << 32))
        fail(PBNG_EUNSUPPORTED, "mesh too large for 32-bit stream offsets");
    if (real == PBNG_F64) pack<double>(ws, p, I, int_of);
    else pack<float>(ws, p, I, int_of);
    ws->W.alloc(ws->nv * ws->r2());
    ws->Wres.alloc(ws->nv * ws->r2());
    ws->rejected.alloc(sizeof(int));
    ws->vp.alloc(6 * ws->nt * sizeof(double));
    ws->ebuf.alloc((ws->nt + ws->nv + ws->n_wc) * sizeof(double));
    ws->rsq.alloc(ws->nv * sizeof(double));
    ws->out.alloc(2 * sizeof(double));
    ws->plan_r = plan_range(ws->nv, ws->cb_r, ws->ce_r, ws->qp_r, ws->part_r);
    ws->plan_e = plan_range(ws->nt + ws->nv + ws->n_wc, ws->cb_e, ws->ce_e, ws->qp_e, ws->part_e);
    hipchk(hipHostMalloc(reinterpret_cast<void**>(&ws->hbuf), 2 * sizeof(double), hipHostMallocDefault),
           "pinned alloc");
}

template <class R>
Res2Args<R> res_args(pbng2d_workspace* ws, const void* X)
{
    Res2Args<R> a;
    a.X = static_cast<const typename R2t<R>::T*>(X);
    a.tri = ws->tri.as<int4>();
    a.geo = ws->geo.as<TriGeo>();
    a.vp = ws->vp.as<double>();
    a.ebuf = ws->ebuf.as<double>();
    a.rvptr = ws->rvptr.as<int>();
    a.rv = ws->rv.as<int>();
    a.fext64 = ws->fext64.as<double>();
    a.orig_of = ws->orig_of.as<int>();
    a.rsq = ws->rsq.as<double>();
    a.n_free = int(ws->nfree);
    a.n_verts = int(ws->nv);
    a.n_tris = int(ws->nt);
    a.model = ws->model;
    a.wvptr = ws->wvptr.as<int>();
    a.wv_c = ws->wv_c.as<int>();
    a.wv_s = ws->wv_s64.as<double>();
    a.wc_ptr = ws->wc_ptr.as<int>();
    a.wc_vert = ws->wc_vert.as<int>();
    a.wc_w = ws->wc_w64.as<double>();
    a.wc_K = ws->wc_K64.as<double>();
    a.n_wc = ws->n_wc;
    a.planes = ws->planes64.as<double>();
    a.n_planes = ws->n_planes;
    a.inert = ws->inertia ? ws->inert64.as<double>() : nullptr;
    a.xhat = ws->inertia ? ws->xhat64.as<double>() : nullptr;
    return a;
}

template <class R>
void residual2(pbng2d_workspace* ws, const void* X, double* r_out, hipStream_t s)
{
    const Res2Args<R> a = res_args<R>(ws, X);
    hipchk(launch_residual2<R>(a, r_out, s), "residual");
    double* out = ws->out.as<double>();
    hipchk(launch_segsum(ws->rsq.as<double>(), ws->plan_r, 1, out, s), "residual sum");
    hipchk(launch_segsum(ws->ebuf.as<double>(), ws->plan_e, 1, out + 1, s), "energy sum");
    hipchk(hipMemcpyAsync(ws->hbuf, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "d2h");
    hipchk(hipStreamSynchronize(s), "sync");
    ws->hbuf[0] = std::sqrt(ws->hbuf[0]);
}

void check_opts2(const pbng_solve_opts* o)
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
    if (!(o->lanes == 0 || o->lanes == 1 || o->lanes == 2 || o->lanes == 4 || o->lanes == 8 || o->lanes == 16))
        fail(PBNG_EINVAL, "planar lanes must be 0, 1, 2, 4, 8 or 16");
}

void ensure_ring2(pbng2d_workspace* ws)
{
    if (!ws->P.p) ws->P.alloc(ws->nv * ws->r2());
    if (!ws->N.p) ws->N.alloc(ws->nv * ws->r2());
}

template <class R>
void load_ring(pbng2d_workspace* ws, const void* x, bool accel, hipStream_t s)
{
    using R2 = typename R2t<R>::T;
    hipchk(launch_load2<R>(static_cast<const R*>(x), ws->orig_of.as<int>(), ws->xd_int.as<R2>(), ws->W.as<R2>(),
                           accel ? ws->P.as<R2>() : nullptr, accel ? ws->N.as<R2>() : nullptr, int(ws->nfree),
                           int(ws->nv), s),
           "load");
}

template <class R>
void sweep2(pbng2d_workspace* ws, const pbng_solve_opts* o, double omega, double gamma, hipStream_t s)
{
    using R2 = typename R2t<R>::T;
    using R4 = typename R4t<R>::T;
    const bool accel = o->accel != PBNG_ACCEL_NONE;
    Sweep2Args<R> a;
    a.W = ws->W.as<R2>();
    a.P = accel ? ws->P.as<R2>() : nullptr;
    a.N = accel ? ws->N.as<R2>() : nullptr;
    a.vptr = ws->vptr.as<int>();
    a.jk = ws->jk.as<int2>();
    a.gm = ws->gm.as<R4>();
    a.vw = ws->uniform ? nullptr : ws->vw.as<R2>();
    a.mu_u = R(ws->mu_u);
    a.lam_u = R(ws->lam_u);
    a.fext = ws->fext.as<R2>();
    a.rejected = ws->rejected.as<int>();
    a.omega = R(omega);
    a.gamma = R(gamma);
    a.max_halvings = o->max_halvings;
    a.wvptr = ws->wvptr.as<int>();
    a.wv_c = ws->wv_c.as<int>();
    a.wv_s = ws->wv_s.as<R>();
    a.wc_ptr = ws->wc_ptr.as<int>();
    a.wc_vert = ws->wc_vert.as<int>();
    a.wc_w = ws->wc_w.as<R>();
    a.wc_K = ws->wc_K.as<R>();
    a.planes = ws->planes.as<R>();
    a.n_planes = ws->n_planes;
    a.inert = ws->inertia ? ws->inert.as<R>() : nullptr;
    a.xhat = ws->inertia ? ws->xhat.as<R2>() : nullptr;
    const int lanes = o->lanes == 0 ? 4 : o->lanes;
    const bool safe = o->safeguard == PBNG_SAFEGUARD_BACKTRACK;
    for (int c = 0; c < ws->ncol; ++c)
        hipchk(launch_phase2<R>(a, ws->model, lanes, accel, safe, ws->uniform, ws->extra(), ws->cptr[c],
                                ws->cptr[c + 1], s),
               "phase launch");
    if (accel) std::swap(ws->W.p, ws->N.p);
}

double chebyshev_next2(int64_t l, double rho, double prev)
{
    if (l < 2) return 1.0;
    if (l == 2) return 2.0 / (2.0 - rho * rho);
    return 4.0 / (4.0 - rho * rho * prev);
}

double wall_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class R>
int32_t solve2(pbng2d_workspace* ws, void* x, const pbng_solve_opts* o, pbng_stats* st, hipStream_t s)
{
    using R2 = typename R2t<R>::T;
    const bool accel = o->accel != PBNG_ACCEL_NONE;
    if (accel) ensure_ring2(ws);
    load_ring<R>(ws, x, accel, s);
    ws->sweep_l = 0;
    ws->omega_l = 1.0;
    hipchk(hipMemsetAsync(ws->rejected.p, 0, sizeof(int), s), "memset");
    residual2<R>(ws, ws->W.p, nullptr, s);
    const double r0 = ws->hbuf[0];
    double rr = r0, en = ws->hbuf[1], ttol = -1.0;
    if (!std::isfinite(r0)) fail(PBNG_ENAN, "non-finite initial residual");
    bool conv = r0 == 0.0, nan = false;
    if (conv) ttol = 0.0;
    const double t0 = wall_ms();
    int sweeps = 0;
    for (int sw = 0; sw < o->max_sweeps && !conv; ++sw) {
        double omega = 1.0, gamma = 1.0;
        if (o->accel == PBNG_ACCEL_CHEBYSHEV) {
            omega = chebyshev_next2(ws->sweep_l, o->rho, ws->omega_l);
            gamma = o->gamma;
        } else if (o->accel == PBNG_ACCEL_SOR) {
            omega = o->omega;
        }
        sweep2<R>(ws, o, omega, gamma, s);
        ws->omega_l = omega;
        ws->sweep_l++;
        sweeps = sw + 1;
        if (sweeps % o->check_every == 0 || sweeps == o->max_sweeps) {
            residual2<R>(ws, ws->W.p, nullptr, s);
            rr = ws->hbuf[0];
            en = ws->hbuf[1];
            if (!std::isfinite(rr)) {
                nan = true;
                break;
            }
            if (o->rel_tol > 0 && rr <= o->rel_tol * r0) {
                conv = true;
                ttol = wall_ms() - t0;
            }
        }
    }
    hipchk(launch_store2<R>(ws->W.as<R2>(), ws->orig_of.as<int>(), static_cast<R*>(x), int(ws->nv), s), "store");
    int rej = 0;
    hipchk(hipMemcpyAsync(&rej, ws->rejected.p, sizeof(int), hipMemcpyDeviceToHost, s), "d2h");
    hipchk(hipStreamSynchronize(s), "sync");
    if (st) {
        st->sweeps = sweeps;
        st->converged = conv;
        st->n_colors = ws->ncol;
        st->rejected = rej;
        st->residual0 = r0;
        st->residual = rr;
        st->rel_residual = r0 > 0 ? rr / r0 : 0.0;
        st->energy = en;
        st->time_ms = wall_ms() - t0;
        st->time_to_tol_ms = ttol;
        st->vertex_updates = double(sweeps) * double(ws->nfree);
    }
    if (nan) fail(PBNG_ENAN, "iterate became non-finite");
    return conv ? PBNG_OK : PBNG_NOT_CONVERGED;
}

// ||b - H lam|| over free vertices (FP64) of the adjoint iterate in LA.
template <class R>
double adjoint_check2(pbng2d_workspace* ws, const Res2Args<R>& a, hipStream_t s)
{
    using R2 = typename R2t<R>::T;
    hipchk(launch_adjoint_residual2<R>(a, ws->LA.as<R2>(), ws->BA.as<R2>(), nullptr, nullptr, nullptr, nullptr, s),
           "adjoint residual");
    double* out = ws->out.as<double>();
    hipchk(launch_segsum(ws->rsq.as<double>(), ws->plan_r, 1, out, s), "adjoint residual sum");
    hipchk(hipMemcpyAsync(ws->hbuf, out, sizeof(double), hipMemcpyDeviceToHost, s), "d2h");
    hipchk(hipStreamSynchronize(s), "sync");
    return std::sqrt(ws->hbuf[0]);
}

// Block Gauss-Seidel on H lam = dL/dx (free rows) over the colours, with
// the Chebyshev blend on request, then dL/dx_D, dL/dmu, dL/dlambda and lam.
template <class R>
int32_t adjoint2(pbng2d_workspace* ws, const void* x_eq, const void* dL_dx, double* dxd, double* dmu,
                 double* dlam, double* lam_out, const pbng_adjoint_opts* o, pbng_stats* st, hipStream_t s)
{
    using R2 = typename R2t<R>::T;
    using R4 = typename R4t<R>::T;
    const int nv = int(ws->nv), nf = int(ws->nfree);
    const bool accel = o->accel == PBNG_ACCEL_CHEBYSHEV;
    const size_t bytes = size_t(std::max(nv, 1)) * ws->r2();
    for (Dev* d : {&ws->XA, &ws->LA, &ws->LPa, &ws->LNa, &ws->BA}) d->reserve(bytes);
    // caller order -> internal order, every row from the caller's arrays
    hipchk(launch_load2<R>(static_cast<const R*>(x_eq), ws->orig_of.as<int>(), nullptr, ws->XA.as<R2>(), nullptr,
                           nullptr, nf, nv, s),
           "load");
    hipchk(launch_load2<R>(static_cast<const R*>(dL_dx), ws->orig_of.as<int>(), nullptr, ws->BA.as<R2>(), nullptr,
                           nullptr, nf, nv, s),
           "load");
    for (Dev* d : {&ws->LA, &ws->LPa, &ws->LNa}) hipchk(hipMemsetAsync(d->p, 0, bytes, s), "memset");
    const Res2Args<R> ra = res_args<R>(ws, ws->XA.p);
    const double b0 = adjoint_check2<R>(ws, ra, s);   // lam = 0: ||b|| over free rows
    if (!std::isfinite(b0)) fail(PBNG_ENAN, "non-finite dL/dx");
    Adj2Args<R> a;
    a.X = ws->XA.as<R2>();
    a.B = ws->BA.as<R2>();
    a.vptr = ws->vptr.as<int>();
    a.jk = ws->jk.as<int2>();
    a.gm = ws->gm.as<R4>();
    a.vw = ws->uniform ? nullptr : ws->vw.as<R2>();
    a.mu_u = R(ws->mu_u);
    a.lam_u = R(ws->lam_u);
    a.wvptr = ws->wvptr.as<int>();
    a.wv_c = ws->wv_c.as<int>();
    a.wv_s = ws->wv_s.as<R>();
    a.wc_ptr = ws->wc_ptr.as<int>();
    a.wc_vert = ws->wc_vert.as<int>();
    a.wc_w = ws->wc_w.as<R>();
    a.wc_K = ws->wc_K.as<R>();
    a.planes = ws->planes.as<R>();
    a.n_planes = ws->n_planes;
    a.inert = ws->inertia ? ws->inert.as<R>() : nullptr;
    const int lanes = o->lanes == 0 ? 4 : o->lanes;
    double rr = b0, omega_prev = 1.0;
    bool conv = b0 == 0.0, nan = false;
    int sweeps = 0;
    const double t0 = wall_ms();
    for (int sw = 0; sw < o->max_sweeps && !conv; ++sw) {
        const double omega = accel ? chebyshev_next2(sw, o->rho, omega_prev) : 1.0;
        omega_prev = omega;
        a.L = ws->LA.as<R2>();
        a.P = ws->LPa.as<R2>();
        a.N = ws->LNa.as<R2>();
        a.omega = R(omega);
        a.gamma = R(accel ? o->gamma : 1.0);
        for (int c = 0; c < ws->ncol; ++c)
            hipchk(launch_adj_phase2<R>(a, ws->model, lanes, accel, ws->uniform, ws->extra(), ws->cptr[c],
                                        ws->cptr[c + 1], s),
                   "adjoint phase");
        if (accel) std::swap(ws->LA.p, ws->LNa.p);
        sweeps = sw + 1;
        if (sweeps % o->check_every == 0 || sweeps == o->max_sweeps) {
            rr = adjoint_check2<R>(ws, ra, s);
            if (!std::isfinite(rr)) {
                nan = true;
                break;
            }
            if (o->rel_tol > 0 && rr <= o->rel_tol * b0) conv = true;
        }
    }
    hipchk(launch_adjoint_residual2<R>(ra, ws->LA.as<R2>(), ws->BA.as<R2>(), dmu, dlam, dxd,
                                       ws->dir_pos.as<int>(), s),
           "adjoint gradients");
    if (lam_out) hipchk(launch_store2_f64<R>(ws->LA.as<R2>(), ws->orig_of.as<int>(), lam_out, nv, s), "store");
    hipchk(hipStreamSynchronize(s), "sync");
    if (st) {
        *st = pbng_stats{};
        st->sweeps = sweeps;
        st->converged = conv;
        st->n_colors = ws->ncol;
        st->residual0 = b0;
        st->residual = rr;
        st->rel_residual = b0 > 0 ? rr / b0 : 0.0;
        st->time_ms = wall_ms() - t0;
        st->vertex_updates = double(sweeps) * double(ws->nfree);
    }
    if (nan) fail(PBNG_ENAN, "adjoint iterate became non-finite");
    return conv ? PBNG_OK : PBNG_NOT_CONVERGED;
}

void check_ws2(const pbng2d_workspace* ws)
{
    if (!ws) fail(PBNG_EINVAL, "workspace is null");
}

}  // namespace

extern "C" {

int32_t pbng2d_color(const pbng2d_problem* p, int32_t* colors_out, int32_t* n_colors_out)
{
    return guard([&] {
        validate2(p);
        if (!colors_out) fail(PBNG_EINVAL, "colors_out is null");
        const Inc I = incidence2(p);
        const int n = color2(p, I, colors_out);
        if (n_colors_out) *n_colors_out = n;
        return PBNG_OK;
    });
}

int32_t pbng2d_workspace_create(const pbng2d_problem* p, const int32_t* colors, int32_t real,
                                pbng2d_workspace** ws_out)
{
    return guard([&] {
        if (!ws_out) fail(PBNG_EINVAL, "ws_out is null");
        *ws_out = nullptr;
        pbng2d_workspace* ws = new pbng2d_workspace;
        try {
            build2(ws, p, colors, real);
        } catch (...) {
            delete ws;
            throw;
        }
        *ws_out = ws;
        return PBNG_OK;
    });
}

int32_t pbng2d_workspace_destroy(pbng2d_workspace* ws)
{
    delete ws;
    return PBNG_OK;
}

int32_t pbng2d_workspace_info(const pbng2d_workspace* ws, int64_t* n_verts, int64_t* n_tris, int64_t* n_free,
                              int32_t* n_colors, int64_t* n_visits)
{
    return guard([&] {
        check_ws2(ws);
        if (n_verts) *n_verts = ws->nv;
        if (n_tris) *n_tris = ws->nt;
        if (n_free) *n_free = ws->nfree;
        if (n_colors) *n_colors = ws->ncol;
        if (n_visits) *n_visits = ws->nvis;
        return PBNG_OK;
    });
}

int32_t pbng2d_workspace_colors(const pbng2d_workspace* ws, int32_t* colors_out)
{
    return guard([&] {
        check_ws2(ws);
        if (!colors_out) fail(PBNG_EINVAL, "colors_out is null");
        std::copy(ws->colors_h.begin(), ws->colors_h.end(), colors_out);
        return PBNG_OK;
    });
}

int32_t pbng2d_solve(pbng2d_workspace* ws, void* x_inout, const pbng_solve_opts* o, pbng_stats* stats,
                     void* hip_stream)
{
    return guard([&] {
        check_ws2(ws);
        if (!x_inout) fail(PBNG_EINVAL, "x is null");
        check_opts2(o);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        return ws->real == PBNG_F64 ? solve2<double>(ws, x_inout, o, stats, s)
                                    : solve2<float>(ws, x_inout, o, stats, s);
    });
}

int32_t pbng2d_residual(pbng2d_workspace* ws, const void* x, double* res_norm, double* energy, double* r_out,
                        void* hip_stream)
{
    return guard([&] {
        check_ws2(ws);
        if (!x) fail(PBNG_EINVAL, "x is null");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (ws->real == PBNG_F64) {
            hipchk(launch_load2<double>(static_cast<const double*>(x), ws->orig_of.as<int>(), nullptr,
                                        ws->Wres.as<double2>(), nullptr, nullptr, int(ws->nfree), int(ws->nv), s),
                   "load");
            residual2<double>(ws, ws->Wres.p, r_out, s);
        } else {
            hipchk(launch_load2<float>(static_cast<const float*>(x), ws->orig_of.as<int>(), nullptr,
                                       ws->Wres.as<float2>(), nullptr, nullptr, int(ws->nfree), int(ws->nv), s),
                   "load");
            residual2<float>(ws, ws->Wres.p, r_out, s);
        }
        if (res_norm) *res_norm = ws->hbuf[0];
        if (energy) *energy = ws->hbuf[1];
        return PBNG_OK;
    });
}

int32_t pbng2d_adjoint(pbng2d_workspace* ws, const void* x_eq, const void* dL_dx, double* dL_dxD, double* dL_dmu,
                       double* dL_dlambda, double* lam_out, const pbng_adjoint_opts* o, pbng_stats* stats,
                       void* hip_stream)
{
    return guard([&] {
        check_ws2(ws);
        if (!x_eq || !dL_dx || !o) fail(PBNG_EINVAL, "null argument");
        if (o->max_sweeps < 0 || o->check_every < 1) fail(PBNG_EINVAL, "max_sweeps must be >= 0 and check_every >= 1");
        if (o->accel != PBNG_ACCEL_NONE && o->accel != PBNG_ACCEL_CHEBYSHEV)
            fail(PBNG_EINVAL, "the adjoint takes no acceleration or Chebyshev");
        if (o->accel == PBNG_ACCEL_CHEBYSHEV && !(o->rho > 0 && o->rho < 1 && o->gamma > 0))
            fail(PBNG_EINVAL, "Chebyshev needs 0 < rho < 1 and gamma > 0");
        if (!std::isfinite(o->rel_tol) || o->rel_tol < 0) fail(PBNG_EINVAL, "rel_tol must be >= 0");
        if (!(o->lanes == 0 || o->lanes == 1 || o->lanes == 2 || o->lanes == 4 || o->lanes == 8 || o->lanes == 16))
            fail(PBNG_EINVAL, "planar lanes must be 0, 1, 2, 4, 8 or 16");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        return ws->real == PBNG_F64
                   ? adjoint2<double>(ws, x_eq, dL_dx, dL_dxD, dL_dmu, dL_dlambda, lam_out, o, stats, s)
                   : adjoint2<float>(ws, x_eq, dL_dx, dL_dxD, dL_dmu, dL_dlambda, lam_out, o, stats, s);
    });
}

int32_t pbng2d_workspace_set_inertia(pbng2d_workspace* ws, double dt, const double* x_n_dev,
                                     const double* x_prev_dev, void* hip_stream)
{
    return guard([&] {
        check_ws2(ws);
        if (!std::isfinite(dt)) fail(PBNG_EINVAL, "non-finite dt");
        if (dt <= 0.0) {
            ws->inertia = false;
            return PBNG_OK;
        }
        if (!x_n_dev || !x_prev_dev) fail(PBNG_EINVAL, "null x_n or x_prev");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const int64_t nf = ws->nfree;
        std::vector<double> c64(std::max<int64_t>(1, nf), 0.0);
        for (int64_t v = 0; v < nf; ++v) c64[v] = ws->mass_h[v] / (dt * dt);
        // no queued work reads the old inertia arrays after this sync
        hipchk(hipStreamSynchronize(s), "sync");
        ws->inert64.upload(c64);
        if (ws->real == PBNG_F64) {
            ws->inert.upload(c64);
        } else {
            std::vector<float> c32(c64.begin(), c64.end());
            ws->inert.upload(c32);
        }
        if (!ws->xhat64.p) ws->xhat64.alloc(std::max<int64_t>(1, nf) * 2 * sizeof(double));
        if (!ws->xhat.p) ws->xhat.alloc(std::max<int64_t>(1, nf) * ws->r2());
        if (ws->real == PBNG_F64)
            hipchk(launch_xhat2<double>(x_n_dev, x_prev_dev, ws->orig_of.as<int>(), ws->xhat64.as<double>(),
                                        ws->xhat.as<double2>(), int(nf), s),
                   "inertia");
        else
            hipchk(launch_xhat2<float>(x_n_dev, x_prev_dev, ws->orig_of.as<int>(), ws->xhat64.as<double>(),
                                       ws->xhat.as<float2>(), int(nf), s),
                   "inertia");
        hipchk(hipStreamSynchronize(s), "inertia");
        ws->inertia = true;
        return PBNG_OK;
    });
}

int32_t pbng2d_load(pbng2d_workspace* ws, const void* x, void* hip_stream)
{
    return guard([&] {
        check_ws2(ws);
        if (!x) fail(PBNG_EINVAL, "x is null");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        ensure_ring2(ws);
        if (ws->real == PBNG_F64) load_ring<double>(ws, x, true, s);
        else load_ring<float>(ws, x, true, s);
        hipchk(hipMemsetAsync(ws->rejected.p, 0, sizeof(int), s), "memset");
        hipchk(hipStreamSynchronize(s), "sync");
        ws->sweep_l = 0;
        ws->omega_l = 1.0;
        return PBNG_OK;
    });
}

int32_t pbng2d_store(pbng2d_workspace* ws, void* x, void* hip_stream)
{
    return guard([&] {
        check_ws2(ws);
        if (!x) fail(PBNG_EINVAL, "x is null");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (ws->real == PBNG_F64)
            hipchk(launch_store2<double>(ws->W.as<double2>(), ws->orig_of.as<int>(), static_cast<double*>(x),
                                         int(ws->nv), s),
                   "store");
        else
            hipchk(launch_store2<float>(ws->W.as<float2>(), ws->orig_of.as<int>(), static_cast<float*>(x), int(ws->nv),
                                        s),
                   "store");
        hipchk(hipStreamSynchronize(s), "sync");
        return PBNG_OK;
    });
}

int32_t pbng2d_sweeps(pbng2d_workspace* ws, int32_t n_sweeps, const pbng_solve_opts* o, void* hip_stream)
{
    return guard([&] {
        check_ws2(ws);
        check_opts2(o);
        if (n_sweeps < 0) fail(PBNG_EINVAL, "n_sweeps must be >= 0");
        if (!ws->P.p) fail(PBNG_EINVAL, "call pbng2d_load first");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        for (int k = 0; k < n_sweeps; ++k) {
            double omega = 1.0, gamma = 1.0;
            if (o->accel == PBNG_ACCEL_CHEBYSHEV) {
                omega = chebyshev_next2(ws->sweep_l, o->rho, ws->omega_l);
                gamma = o->gamma;
            } else if (o->accel == PBNG_ACCEL_SOR) {
                omega = o->omega;
            }
            if (ws->real == PBNG_F64) sweep2<double>(ws, o, omega, gamma, s);
            else sweep2<float>(ws, o, omega, gamma, s);
            ws->omega_l = omega;
            ws->sweep_l++;
        }
        return PBNG_OK;
    });
}

int32_t pbng2d_phase_bytes(const pbng2d_workspace* ws, int32_t color, int64_t* bytes, int64_t* vertices,
                           int64_t* visits)
{
    return guard([&] {
        check_ws2(ws);
        if (color < 0 || color >= ws->ncol) fail(PBNG_EINVAL, "colour out of range");
        if (bytes) *bytes = ws->ph_bytes[color];
        if (vertices) *vertices = ws->ph_verts[color];
        if (visits) *visits = ws->ph_visits[color];
        return PBNG_OK;
    });
}

}  // extern "C"
