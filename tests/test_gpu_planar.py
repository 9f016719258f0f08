"""Planar (triangle-mesh) path on the GPU against the planar FP64 oracle:
whole solves in FP64 and FP32 with every blend, the lanes-per-vertex
variants, per-triangle materials and loads, safeguard decisions, the FP64
residual / energy, degenerate problems, and one sweep plus the residual
vector element by element at the full 1025 x 1025 size.

Tolerances: FP64 1e-10 relative after the same sweeps (the kernel forms F
from edge vectors, the oracle from positions: rounding-level differences);
FP32 1e-5 (float positions and arithmetic against the FP64 oracle); FP64
residual and energy 1e-10."""
import numpy as np
import pytest

from oracle import planar as P
from paper_2306_09021_amd import pbng2d
from paper_2306_09021_amd import scenarios as S

from .gpu_util import announce, host, rel_err, require_gpu, torch

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def dev2(x, real):
    dt = torch.float32 if real == "f32" else torch.float64
    return torch.tensor(np.asarray(x, np.float64).reshape(-1, 2), dtype=dt, device="cuda").contiguous()


def ws2(sc, real):
    return pbng2d.Workspace2D(pbng2d.problem_from_scenario(sc), real=real)


def both(sc, real, sweeps, **kw):
    ws = ws2(sc, real)
    op = P.make_problem(sc)
    col = ws.colors()
    xo, sto = P.solve(op, col, sc.initial_iterate(), max_sweeps=sweeps, **kw)
    x = dev2(sc.initial_iterate(), real)
    rc, st = ws.solve(x, max_sweeps=sweeps, rel_tol=0.0, check_every=sweeps, **kw)
    return host(x), xo, st, sto, ws


CASES = [dict(accel="none", safeguard="backtrack"),
         dict(accel="chebyshev", rho=0.9, gamma=1.2, safeguard="backtrack"),
         dict(accel="sor", omega=1.5, safeguard="none")]


@pytest.mark.parametrize("model", ["nh", "corotated"])
@pytest.mark.parametrize("real", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_solve_parity(model, real, case):
    kw = dict(CASES[case])
    if real == "f32":
        kw["safeguard"] = "none"   # FP32 and FP64 energy comparisons may differ at ties
    sc = S.stretched_square(41, model, 1.5, noise=0.3, seed=case + 1)
    announce("planar solve %s %s %s" % (model, real, kw))
    xg, xo, st, sto, ws = both(sc, real, 30, **kw)
    e = rel_err(xg, xo)
    print("rel err", e, "oracle rel residual", sto["rel"])
    assert e <= TOL[real]
    assert st["sweeps"] == 30 and st["n_colors"] == ws.n_colors


@pytest.mark.parametrize("diag", ["uniform", "alternate"])
def test_lanes_variants_agree(diag):
    sc = S.stretched_square(33, "nh", 1.4, diagonal=diag, noise=0.2, seed=5)
    announce("planar lanes %s" % diag)
    ws = ws2(sc, "f64")
    op = P.make_problem(sc)
    xo, _ = P.solve(op, ws.colors(), sc.initial_iterate(), max_sweeps=20, accel="chebyshev", rho=0.9,
                    gamma=1.0)
    for lanes in (1, 2, 4, 8, 16):
        x = dev2(sc.initial_iterate(), "f64")
        ws.solve(x, max_sweeps=20, rel_tol=0.0, check_every=20, accel="chebyshev", rho=0.9, gamma=1.0,
                 lanes=lanes)
        assert rel_err(host(x), xo) <= 1e-10, lanes


@pytest.mark.parametrize("model", ["nh", "corotated"])
@pytest.mark.parametrize("real", ["f64", "f32"])
def test_residual_and_energy(model, real):
    sc = S.stretched_square(29, model, 1.6, density=30.0, gravity=(0.5, -9.8))
    rng = np.random.default_rng(3)
    x = sc.initial_iterate() + 0.01 * rng.normal(size=(sc.n_verts, 2))
    x[sc.dirichlet_idx] = sc.dirichlet_x
    xr = x.astype(np.float32).astype(np.float64) if real == "f32" else x
    n_o, E_o, r_o = P.residual(P.make_problem(sc), xr)
    announce("planar residual %s %s" % (model, real))
    ws = ws2(sc, real)
    rn, E, r = ws.residual(dev2(xr, real), want_r=True)
    assert abs(rn - n_o) <= 1e-10 * n_o
    assert abs(E - E_o) <= 1e-10 * abs(E_o)
    assert np.abs(host(r) - r_o).max() <= 1e-10 * np.abs(r_o).max()


def test_per_triangle_materials_and_loads():
    sc = S.stretched_square(31, "nh", 1.3, noise=0.2, seed=7, density=100.0, gravity=(0.0, -9.8))
    rng = np.random.default_rng(9)
    sc.E = rng.uniform(5e3, 5e4, sc.n_tris)
    sc.nu = rng.uniform(0.2, 0.45, sc.n_tris)
    sc.nodal_force = 0.5 * rng.normal(size=(sc.n_verts, 2))
    announce("planar per-triangle materials f64")
    xg, xo, st, sto, _ = both(sc, "f64", 25, accel="chebyshev", rho=0.9, gamma=1.0)
    assert rel_err(xg, xo) <= 1e-10
    assert abs(st["residual"] - sto["res"]) <= 1e-8 * sto["res"]


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_safeguard_decisions_match(model):
    """A hard start (stretch 2.5 with heavy jitter).  Neo-Hookean with
    lambda < mu (nu = 0.05), where full steps can raise the local energy: the
    kernel halves exactly where the oracle does (with lambda >= mu the full
    step never does).  Corotated: the oracle never needs a halving (the
    modified matrix majorises the local energy) and the kernel takes every
    full step."""
    nu = 0.05 if model == "nh" else 0.45
    sc = S.stretched_square(25, model, 2.5, E=1e4, nu=nu, noise=0.6, seed=9)
    announce("planar safeguard %s f64" % model)
    xg, xo, st, sto, _ = both(sc, "f64", 15, accel="none", safeguard="backtrack")
    assert rel_err(xg, xo) <= 1e-10
    assert st["rejected"] == sto["rejected"]
    if model == "nh":
        assert sto["halvings"] > 0
    else:
        assert sto["halvings"] == 0 and sto["rejected"] == 0


def test_convergence_to_tolerance():
    sc = S.stretched_square(21, "corotated", 1.5)
    announce("planar convergence f64")
    ws = ws2(sc, "f64")
    x = dev2(sc.initial_iterate(), "f64")
    rc, st = ws.solve(x, max_sweeps=5000, rel_tol=1e-9, check_every=10, accel="chebyshev", rho=0.95,
                      gamma=1.0)
    assert rc == 0 and st["converged"] and st["rel_residual"] <= 1e-9
    n_o, _, _ = P.residual(P.make_problem(sc), host(x))
    assert n_o <= 1.01e-9 * st["residual0"]


def test_degenerate_problems():
    # every vertex prescribed: nothing to solve, zero residual
    X, T = S.square_mesh(4, 4, 1.0 / 3)
    idx = np.arange(16, dtype=np.int32)
    sc = S.Scenario2D("all_dir", X, T, "nh", np.asarray(1e3), np.asarray(0.3), idx, 1.1 * X, X)
    announce("planar all-Dirichlet")
    ws = ws2(sc, "f64")
    assert ws.n_free == 0 and ws.n_colors == 0
    x = dev2(sc.initial_iterate(), "f64")
    rc, st = ws.solve(x, max_sweeps=10, rel_tol=1e-8)
    assert rc == 0 and st["sweeps"] == 0 and st["residual0"] == 0.0
    assert np.array_equal(host(x), 1.1 * X)
    # a single free vertex in the middle of a 3 x 3 patch
    X, T = S.square_mesh(3, 3, 0.5)
    bnd = np.array([0, 1, 2, 3, 5, 6, 7, 8], np.int32)
    sc = S.Scenario2D("one_free", X, T, "corotated", np.asarray(1e3), np.asarray(0.3), bnd, X[bnd] * 1.2,
                      X + np.array([0.1, -0.05]))
    announce("planar single free vertex")
    xg, xo, st, sto, ws = both(sc, "f64", 200)
    assert ws.n_free == 1 and rel_err(xg, xo) <= 1e-12
    assert np.abs(xg[4] - 1.2 * X[4]).max() <= 1e-9   # the affine patch solution


@pytest.mark.parametrize("real", ["f32", "f64"])
def test_full_size_one_sweep_and_residual(real):
    """At the measured size (1025 x 1025 vertices, 2.1M triangles, NH) in the
    launch configuration the benchmark times: one GPU sweep against one
    oracle sweep over every vertex, and the FP64 residual vector."""
    sc = S.stretched_square(1025, "nh", 1.5, noise=0.2, seed=1)
    op = P.make_problem(sc)
    announce("planar full size one sweep %s" % real)
    ws = ws2(sc, real)
    x0 = sc.initial_iterate()
    xr = x0.astype(np.float32).astype(np.float64) if real == "f32" else x0
    xo, _ = P.solve(op, ws.colors(), xr, max_sweeps=1, safeguard="none")
    x = dev2(xr, real)
    ws.solve(x, max_sweeps=1, rel_tol=0.0, check_every=1, safeguard="none", accel="none")
    xg = host(x)
    d = np.abs(xg - xo).max(axis=1)
    scale = np.abs(xo - xr).max()
    assert d.max() <= (1e-10 if real == "f64" else 1e-5) * max(scale, 1e-3) + (0.0 if real == "f64" else 1e-6)
    rn, E, r = ws.residual(x, want_r=True)
    n_o, E_o, r_o = P.residual(op, xg)
    assert abs(rn - n_o) <= 1e-10 * n_o and abs(E - E_o) <= 1e-10 * abs(E_o)
    assert np.abs(host(r) - r_o).max() <= 1e-9 * np.abs(r_o).max()


@pytest.mark.parametrize("model", ["nh", "corotated"])
@pytest.mark.parametrize("real", ["f64", "f32"])
@pytest.mark.parametrize("accel", ["none", "chebyshev"])
def test_constraints_and_half_plane_parity(model, real, accel):
    """Weak constraints, a stiff ground half-plane and gravity: the full step
    overshoots into the half-plane, so the safeguard halves (the corotated
    kernel then evaluates its energy exactly)."""
    sc = S.planar_terms(17, model)
    kw = dict(accel=accel, rho=0.9, gamma=1.0, safeguard="backtrack")
    announce("planar terms %s %s %s" % (model, real, accel))
    xg, xo, st, sto, ws = both(sc, real, 30, **kw)
    e = rel_err(xg, xo)
    print("rel err", e, "oracle halvings", sto["halvings"], "rejected", sto["rejected"], st["rejected"])
    assert sto["halvings"] > 0
    assert e <= TOL[real]
    assert st["rejected"] == sto["rejected"]


@pytest.mark.parametrize("model", ["nh", "corotated"])
@pytest.mark.parametrize("real", ["f64", "f32"])
def test_backward_euler_frames_parity(model, real):
    """Four backward-Euler frames (dt = 1/100) of the same block: each frame
    sets xhat from the two previous frames on both sides, then 20 sweeps."""
    sc = S.planar_terms(13, model)
    announce("planar backward euler %s %s" % (model, real))
    ws = ws2(sc, real)
    op = P.make_problem(sc)
    col = ws.colors()
    dt = 0.01
    xo_prev = xo_n = sc.initial_iterate()
    xg_prev = xg_n = torch.tensor(sc.initial_iterate(), dtype=torch.float64, device="cuda")
    for frame in range(4):
        op.set_inertia(dt, xo_n, xo_prev)
        xo, sto = P.solve(op, col, xo_n, max_sweeps=20, safeguard="backtrack")
        ws.set_inertia(dt, xg_n, xg_prev)
        x = xg_n.clone().to(ws.dtype).contiguous()     # a copy: the solve works in place
        ws.solve(x, max_sweeps=20, rel_tol=0.0, check_every=20, safeguard="backtrack")
        e = rel_err(host(x), xo)
        print("frame", frame, "rel err", e, "halvings", sto["halvings"])
        assert e <= TOL[real] * (1 + frame)
        xo_prev, xo_n = xo_n, xo
        xg_prev, xg_n = xg_n, x.to(torch.float64).clone()
    ws.set_inertia(0.0)
    x = dev2(sc.initial_iterate(), real)
    ws.solve(x, max_sweeps=10, rel_tol=0.0, check_every=10, safeguard="backtrack")
    op.set_inertia(0.0)
    xo, _ = P.solve(op, col, sc.initial_iterate(), max_sweeps=10, safeguard="backtrack")
    assert rel_err(host(x), xo) <= TOL[real]      # inertia off: the quasistatic solve again


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_residual_and_energy_with_every_term(real):
    sc = S.planar_terms(13, "corotated")
    announce("planar residual all terms %s" % real)
    ws = ws2(sc, real)
    op = P.make_problem(sc)
    rng = np.random.default_rng(3)
    x0 = sc.initial_iterate() + 0.01 * rng.normal(size=(sc.n_verts, 2))
    x0[sc.dirichlet_idx] = sc.dirichlet_x
    x = dev2(x0, real)
    xh = host(x)                                     # the positions as stored (float in f32)
    xn = torch.tensor(xh + 0.003, dtype=torch.float64, device="cuda")
    xp = torch.tensor(xh - 0.001, dtype=torch.float64, device="cuda")
    ws.set_inertia(0.02, xn, xp)
    op.set_inertia(0.02, host(xn), host(xp))
    rn, en, r = ws.residual(x, want_r=True)
    ro, eo, rvo = P.residual(op, xh)
    assert abs(rn - ro) <= 1e-10 * ro
    assert abs(en - eo) <= 1e-10 * max(1.0, abs(eo))
    assert np.abs(host(r) - rvo).max() <= 1e-10 * np.abs(rvo).max()


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_full_size_terms_one_sweep_and_residual(real):
    """The measured planar-terms workload at full size (1025 x 1025 hanging
    block, 2000 springs and 666 three-vertex constraints, ground half-plane,
    inertia): one GPU sweep against one oracle sweep over every vertex (the
    safeguard on in FP64; off in FP32, where float and double energy tests
    could decide a tie differently), then the FP64 residual vector."""
    sc = S.planar_terms(1025, "nh", n_springs=2000)
    op = P.make_problem(sc)
    announce("planar terms full size one sweep %s" % real)
    ws = ws2(sc, real)
    x0 = sc.initial_iterate()
    xr = x0.astype(np.float32).astype(np.float64) if real == "f32" else x0
    xp = xr.copy()
    xp[:, 1] += 0.001                        # moving down at 0.1 m/s with dt = 0.01
    op.set_inertia(0.01, xr, xp)
    ws.set_inertia(0.01, torch.tensor(xr, device="cuda"), torch.tensor(xp, device="cuda"))
    sg = "backtrack" if real == "f64" else "none"
    xo, sto = P.solve(op, ws.colors(), xr, max_sweeps=1, safeguard=sg)
    x = dev2(xr, real)
    ws.solve(x, max_sweeps=1, rel_tol=0.0, check_every=1, safeguard=sg, accel="chebyshev", rho=0.9, gamma=1.0)
    xg = host(x)
    d = np.abs(xg - xo).max(axis=1)
    scale = np.abs(xo - xr).max()
    print("max diff", d.max(), "scale", scale, "oracle halvings", sto["halvings"])
    assert d.max() <= (1e-10 if real == "f64" else 1e-5) * max(scale, 1e-3) + (0.0 if real == "f64" else 1e-6)
    rn, E, r = ws.residual(x, want_r=True)
    n_o, E_o, r_o = P.residual(op, xg)
    assert abs(rn - n_o) <= 1e-10 * n_o and abs(E - E_o) <= 1e-10 * abs(E_o)
    assert np.abs(host(r) - r_o).max() <= 1e-9 * np.abs(r_o).max()


@pytest.mark.parametrize("model", ["nh", "corotated"])
@pytest.mark.parametrize("lanes", [1, 2, 8, 16])
def test_terms_per_triangle_materials_and_lanes(model, lanes):
    """The extra terms with per-triangle Lame parameters (the 32-byte record
    form) and every lane count (the weak constraints of a vertex are spread
    over its lanes like its visits), safeguard on, FP64."""
    sc = S.planar_terms(17, model)
    rng = np.random.default_rng(9)
    sc.E = np.exp(rng.uniform(np.log(3e3), np.log(3e4), sc.n_tris))
    sc.nu = rng.uniform(0.2, 0.45, sc.n_tris)
    announce("planar terms per-triangle %s lanes=%d" % (model, lanes))
    ws = ws2(sc, "f64")
    op = P.make_problem(sc)
    op.set_inertia(0.02, sc.initial_iterate(), sc.initial_iterate())
    x0 = torch.tensor(sc.initial_iterate(), dtype=torch.float64, device="cuda")
    ws.set_inertia(0.02, x0, x0)
    xo, sto = P.solve(op, ws.colors(), sc.initial_iterate(), max_sweeps=25, safeguard="backtrack")
    x = dev2(sc.initial_iterate(), "f64")
    ws.solve(x, max_sweeps=25, rel_tol=0.0, check_every=25, safeguard="backtrack", lanes=lanes)
    e = rel_err(host(x), xo)
    print("rel err", e, "halvings", sto["halvings"])
    assert e <= 1e-10


def test_terms_degenerate_cases():
    """Edge cases of the extra terms: a constraint whose members are all
    Dirichlet (energy only), a free vertex that no triangle touches held by
    a spring alone (its A_i is s^2 K), a half-plane with k = 0 (no effect),
    and inertia on a vertex of zero lumped mass (no effect)."""
    X, T = S.square_mesh(6, 6, 0.2)
    X = np.vstack([X, [[3.0, 3.0]]])               # vertex 36: no triangle
    n = X.shape[0]
    top = np.nonzero(X[:36, 1] > 1.0 - 1e-12)[0]
    didx = np.concatenate([top, [0, 1]]).astype(np.int32)      # 0, 1: bottom corner pinned too
    rng = np.random.default_rng(4)
    x0 = X + 0.01 * rng.normal(size=X.shape)
    x0[didx] = X[didx]
    f = np.zeros((n, 2))
    f[36] = [0.5, -0.25]
    sc = S.Scenario2D(name="terms_edge", rest_pos=X, tris=T, model="nh", E=np.asarray(1e3), nu=np.asarray(0.3),
                      dirichlet_idx=didx, dirichlet_x=X[didx].copy(), x0=x0, density=10.0, gravity=(0.0, -9.8),
                      nodal_force=f,
                      wc_ptr=np.array([0, 2, 4, 6], np.int32),
                      wc_vert=np.array([0, 1, 36, 35, 12, 20], np.int32),   # all-Dirichlet; lone vertex; inner spring
                      wc_w=np.array([1.0, -1.0, 1.0, -1.0, 1.0, -1.0]),
                      wc_K=np.array([[50.0, 0.0, 50.0], [80.0, 10.0, 40.0], [30.0, 0.0, 30.0]]),
                      planes=np.array([[0.0, 1.0, 0.5, 0.0]]))
    announce("planar terms degenerate cases")
    for real in ("f64", "f32"):
        ws = ws2(sc, real)
        op = P.make_problem(sc)
        xn = torch.tensor(sc.initial_iterate(), dtype=torch.float64, device="cuda")
        ws.set_inertia(0.05, xn, xn)
        op.set_inertia(0.05, sc.initial_iterate(), sc.initial_iterate())
        assert op.mass[36] == 0.0
        xo, sto = P.solve(op, ws.colors(), sc.initial_iterate(), max_sweeps=20, safeguard="backtrack")
        x = dev2(sc.initial_iterate(), real)
        rc, st = ws.solve(x, max_sweeps=20, rel_tol=0.0, check_every=20, safeguard="backtrack")
        assert st["rejected"] == sto["rejected"] == 0
        assert rel_err(host(x), xo) <= TOL[real]
        rn, en = ws.residual(x)
        ro, eo, _ = P.residual(op, host(x))
        assert abs(rn - ro) <= 1e-10 * max(1.0, ro) and abs(en - eo) <= 1e-10 * max(1.0, abs(eo))


def _adjoint_case(kind, model):
    if kind == "square":
        sc = S.stretched_square(9, model, 1.3, noise=0.2, seed=2)
        sc.nodal_force = 2.0 * np.random.default_rng(4).normal(size=(sc.n_verts, 2))
    else:
        sc = S.planar_terms(9, model, n_springs=6, k_ground=300.0)
    op = P.make_problem(sc)
    if kind == "terms":
        op.set_inertia(0.05, sc.initial_iterate(), sc.initial_iterate())
    x = P.newton_equilibrium(op, sc.initial_iterate())
    rng = np.random.default_rng(11)
    b = rng.normal(size=x.shape)
    return sc, op, x, b


@pytest.mark.parametrize("kind", ["square", "terms"])
@pytest.mark.parametrize("model", ["nh", "corotated"])
@pytest.mark.parametrize("real,tol", [("f64", 1e-8), ("f32", 1e-4)])
@pytest.mark.parametrize("accel", ["none", "chebyshev"])
def test_adjoint_matches_the_dense_solve(kind, model, real, tol, accel):
    """pbng2d_adjoint at a Newton equilibrium against the oracle's dense
    adjoint: lam, dL/dx_D, dL/dmu and dL/dlambda (with the extra terms:
    springs, the ground half-plane and inertia)."""
    sc, op, x, b = _adjoint_case(kind, model)
    announce("planar adjoint %s %s %s %s" % (kind, model, real, accel))
    lam_o, xd_o, dmu_o, dlam_o = P.adjoint(op, x, b)
    ws = ws2(sc, real)
    if kind == "terms":
        x0 = torch.tensor(sc.initial_iterate(), dtype=torch.float64, device="cuda")
        ws.set_inertia(0.05, x0, x0.clone())
    rc, out, st = ws.adjoint(dev2(x, real), dev2(b, real), max_sweeps=20000, rel_tol=1e-12 if real == "f64" else 1e-6,
                             check_every=50, accel=accel, rho=0.9, gamma=1.0)
    print("sweeps", st["sweeps"], "rel", st["rel_residual"])
    assert rc == 0
    for g, o_ in ((out["lam_vec"], lam_o), (out["xd"], xd_o), (out["mu"], dmu_o), (out["lam"], dlam_o)):
        gg = host(g)
        assert np.abs(gg - o_).max() <= tol * np.abs(o_).max(), (np.abs(gg - o_).max(), np.abs(o_).max())


@pytest.mark.parametrize("real,fb", [("f32", 1), ("f64", 2)])
def test_phase_bytes_follow_their_definition(real, fb):
    """pbng2d_phase_bytes recomputed from the mesh and the colouring: per
    visit 8 + 24 fb bytes, per updated vertex 4 + 24 fb, per distinct other
    vertex of the visited triangles 8 fb (fb = 1 in FP32, 2 in FP64)."""
    sc = S.stretched_square(17, "nh", 1.3, diagonal="alternate")
    ws = ws2(sc, real)
    col = ws.colors()
    for c in range(ws.n_colors):
        verts = np.nonzero(col == c)[0]
        vis = 0
        others = set()
        for t in sc.tris:
            for v in t:
                if col[v] == c:
                    vis += 1
                    others.update(int(u) for u in t if u != v)
        b, nv_, nvis = ws.phase_bytes(c)
        assert (nv_, nvis) == (verts.size, vis)
        assert b == nvis * (8 + 24 * fb) + nv_ * (4 + 24 * fb) + len(others) * 8 * fb
