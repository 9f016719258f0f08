"""Pins for the oracle's discretisation, colouring, sweep, acceleration and
adjoint, against closed forms, special cases with known answers, brute force
on tiny meshes and the numbers the paper prints."""
import json
import os

import numpy as np
import pytest
import scipy.optimize

import oracle as O
from oracle import dense as D
from paper_2306_09021_amd import scenarios as S

HERE = os.path.dirname(os.path.abspath(__file__))
RNG = np.random.default_rng(99)


def small_twist(n=4, model="nh", twist=30.0, stretch=1.1, noise=0.05, seed=3):
    sc = S.twist_box(n, model, 1e4, 0.3, twist, stretch, noise, seed=seed)
    return sc


def with_extras(sc, seed=7):
    """Adds gravity, a weak spring, an anisotropic weak constraint, a ground
    plane and a nodal load to a scenario, for tests that must cover every
    energy term."""
    rng = np.random.default_rng(seed)
    sc.density = 1000.0
    sc.gravity = (0.0, -9.8, 0.5)
    free = np.setdiff1d(np.arange(sc.n_verts), sc.dirichlet_idx)
    a, b, c = rng.choice(free, 3, replace=False)
    d = sc.dirichlet_idx[0]
    K_iso = [300.0, 0, 0, 300.0, 0, 300.0]
    n = np.array([0.3, 0.9, 0.3])
    n /= np.linalg.norm(n)
    Kn = 500.0 * np.outer(n, n) + 20.0 * (np.eye(3) - np.outer(n, n))
    K_an = [Kn[0, 0], Kn[0, 1], Kn[0, 2], Kn[1, 1], Kn[1, 2], Kn[2, 2]]
    sc.wc_ptr = np.array([0, 2, 5], np.int32)
    sc.wc_vert = np.array([a, d, b, c, a], np.int32)
    sc.wc_w = np.array([1.0, -1.0, 0.6, 0.4, -1.0])
    sc.wc_K = np.array([K_iso, K_an])
    ymin = sc.x0[:, 1].min()
    sc.planes = np.array([[0.0, 1.0, 0.0, ymin + 0.2, 2e3]])
    sc.nodal_force = rng.normal(size=(sc.n_verts, 3)) * 0.1
    return sc


# ---------------------------------------------------------------------------
# colouring
# ---------------------------------------------------------------------------
def check_valid_coloring(op, col):
    for t in op.tets:
        cs = [col[v] for v in t if col[v] >= 0]
        assert len(cs) == len(set(cs))
    for c in range(op.wc_ptr.size - 1):
        vs = op.wc_vert[op.wc_ptr[c]:op.wc_ptr[c + 1]]
        cs = [col[v] for v in vs if col[v] >= 0]
        assert len(cs) == len(set(cs))
    assert np.all(col[op.is_dir == 1] == -1)
    assert np.all(col[op.is_dir == 0] >= 0)


def test_paper_box_counts_and_colors():
    """Table 1 / Table 3: the N^3 boxes have the printed vertex and element
    counts and 5 particle colours."""
    with open(os.path.join(HERE, "golden", "paper_box_counts.json")) as f:
        rows = json.load(f)["boxes"]

    def printed(s):
        return float(s[:-1]) * 1000.0

    for row in rows:
        n = row["n"]
        X, T = S.box_mesh(n, n, n, 1.0 / (n - 1))
        pv, pe = printed(row["vertices_printed"]), printed(row["elements_printed"])
        # printed counts are rounded to the shown digits
        assert abs(X.shape[0] - pv) <= 0.05 * pv
        assert abs(T.shape[0] - pe) <= 0.02 * pe
        if n <= 64:
            for pinned in (False, True):
                sc = S.Scenario(name="box", rest_pos=X, tets=T, model="nh", E=np.asarray(1e4),
                                nu=np.asarray(0.3),
                                dirichlet_idx=(np.nonzero(np.isclose(X[:, 1], 0) | np.isclose(X[:, 1], 1))[0]
                                               .astype(np.int32) if pinned else np.zeros(0, np.int32)),
                                dirichlet_x=np.zeros((0, 3)), x0=X)
                sc.dirichlet_x = X[sc.dirichlet_idx]
                op = O.make_problem(sc)
                col, nc = O.color(op)
                assert nc == row["particle_colors"]
                if n <= 16:
                    check_valid_coloring(op, col)


def test_coloring_small_cases_by_hand():
    # a single tet: four distinct colours 0..3 in index order
    sc = S.Scenario(name="tet", rest_pos=np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]),
                    tets=np.array([[0, 1, 2, 3]], np.int32), model="nh", E=np.asarray(1.0),
                    nu=np.asarray(0.3), dirichlet_idx=np.zeros(0, np.int32),
                    dirichlet_x=np.zeros((0, 3)), x0=np.zeros((4, 3)))
    col, n = O.color(O.make_problem(sc))
    assert list(col) == [0, 1, 2, 3] and n == 4
    # Dirichlet vertex 1 is skipped and gets -1
    sc.dirichlet_idx = np.array([1], np.int32)
    sc.dirichlet_x = sc.rest_pos[[1]]
    col, n = O.color(O.make_problem(sc))
    assert list(col) == [0, -1, 1, 2] and n == 3


def test_weak_constraints_add_coloring_edges():
    sc = with_extras(small_twist(4))
    op = O.make_problem(sc)
    col, _ = O.color(op)
    check_valid_coloring(op, col)


# ---------------------------------------------------------------------------
# forces and energy
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_residual_is_minus_energy_gradient(model):
    """r_i = f_i + fhat_i = -dE/dy_i (Eq. fem_qs), checked by central
    differences of the total energy over every term (tets, weak constraints,
    plane penalty, gravity, nodal loads)."""
    sc = with_extras(small_twist(4, model))
    op = O.make_problem(sc)
    x = sc.initial_iterate() + 0.02 * RNG.normal(size=(sc.n_verts, 3))
    x[sc.dirichlet_idx] = sc.dirichlet_x
    _, _, r = O.residual(op, x)
    h = 1e-6
    free = np.nonzero(op.is_dir == 0)[0]
    for i in RNG.choice(free, 8, replace=False):
        for a in range(3):
            xp = x.copy()
            xm = x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = (O.residual(op, xp)[1] - O.residual(op, xm)[1]) / (2 * h)
            assert abs(fd + r[i, a]) <= 1e-6 * max(1.0, np.abs(r).max())


def test_body_force_lumping():
    """Lumped gravity sums to the total weight R0 g Vol."""
    X, T = S.box_mesh(5, 4, 3, (0.25, 0.3, 0.5))
    sc = S.Scenario(name="b", rest_pos=X, tets=T, model="nh", E=np.asarray(1.0), nu=np.asarray(0.3),
                    dirichlet_idx=np.zeros(0, np.int32), dirichlet_x=np.zeros((0, 3)), x0=X,
                    density=7.0, gravity=(0.0, -9.8, 2.0))
    op = O.make_problem(sc)
    vol = 1.0 * 0.9 * 1.0
    assert np.allclose(op.fext.sum(0), 7.0 * np.array([0.0, -9.8, 2.0]) * vol, rtol=1e-12)
    assert abs(op.V0.sum() - vol) < 1e-12


@pytest.mark.parametrize("model", ["nh", "corotated", "snh"])
def test_hessian_vector_product_matches_gradient_differences(model):
    sc = with_extras(small_twist(4, model))
    op = O.make_problem(sc)
    x = sc.initial_iterate()
    v = RNG.normal(size=x.shape)
    h = 1e-6
    fd = (O.energy_gradient(op, x + h * v) - O.energy_gradient(op, x - h * v)) / (2 * h)
    Hv = O.hvp(op, x, v)
    assert np.abs(fd - Hv).max() <= 1e-6 * np.abs(Hv).max()


# ---------------------------------------------------------------------------
# the Gauss-Seidel iteration
# ---------------------------------------------------------------------------
def test_spring_and_load_exact_after_one_update():
    """One free vertex tied to a Dirichlet anchor by a zero-rest-length
    spring with stiffness K and loaded by f: the equilibrium x = a + K^{-1} f
    is reached by a single modified-Newton update (the local problem is
    quadratic and A = K)."""
    for K6 in ([50.0, 0, 0, 50.0, 0, 50.0], [80.0, 10.0, -5.0, 60.0, 3.0, 40.0]):
        a = np.array([0.1, 2.0, -0.3])
        f = np.array([0.5, -9.8, 1.25])
        sc = S.Scenario(name="spring", rest_pos=np.array([a, a + 1.0]), tets=np.zeros((0, 4), np.int32),
                        model="nh", E=np.asarray(1.0), nu=np.asarray(0.3),
                        dirichlet_idx=np.array([0], np.int32), dirichlet_x=a[None, :],
                        x0=np.array([a, [3.0, -1.0, 7.0]]), nodal_force=np.array([[0, 0, 0], f]),
                        wc_ptr=np.array([0, 2], np.int32), wc_vert=np.array([1, 0], np.int32),
                        wc_w=np.array([1.0, -1.0]), wc_K=np.array([K6]))
        op = O.make_problem(sc)
        col, n = O.color(op)
        assert n == 1
        x, st = O.solve(op, col, sc.initial_iterate(), max_sweeps=1)
        K = np.array([[K6[0], K6[1], K6[2]], [K6[1], K6[3], K6[4]], [K6[2], K6[4], K6[5]]])
        assert np.allclose(x[1], a + np.linalg.solve(K, f), rtol=0, atol=1e-13)
        assert st["rel"] < 1e-12


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_affine_patch(model):
    """Every boundary vertex moved by x = A X + b with homogeneous material:
    the affine field is the exact equilibrium, and the iteration reaches it."""
    n = 5
    X, T = S.box_mesh(n, n, n, 1.0 / (n - 1))
    bnd = np.nonzero((np.isclose(X, 0) | np.isclose(X, 1)).any(1))[0].astype(np.int32)
    A = np.eye(3) + np.array([[0.1, 0.2, -0.05], [0.0, -0.15, 0.1], [0.05, 0.0, 0.2]])
    b = np.array([0.3, -0.2, 0.1])
    xa = X @ A.T + b
    sc = S.Scenario(name="patch", rest_pos=X, tets=T, model=model, E=np.asarray(1e4),
                    nu=np.asarray(0.3), dirichlet_idx=bnd, dirichlet_x=xa[bnd],
                    x0=X + 0.02 * RNG.normal(size=X.shape))
    op = O.make_problem(sc)
    r, _, _ = O.residual(op, xa)
    assert r < 1e-9
    col, _ = O.color(op)
    x, st = O.solve(op, col, sc.initial_iterate(), max_sweeps=3000, rel_tol=1e-12, check_every=10)
    assert st["converged"]
    assert np.abs(x - xa).max() < 1e-9


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_single_free_vertex_matches_minimizer(model):
    """With one free vertex PBNG is a 3-DOF modified Newton method: it must
    converge to the minimiser of the total energy in that vertex."""
    n = 3
    X, T = S.box_mesh(n, n, n, 0.5)
    centre = 13
    bnd = np.setdiff1d(np.arange(27), [centre]).astype(np.int32)
    xd = X.copy()
    xd[:, 1] *= 1.2
    xd += 0.05 * np.random.default_rng(5).normal(size=X.shape)
    sc = S.Scenario(name="one", rest_pos=X, tets=T, model=model, E=np.asarray(1e4),
                    nu=np.asarray(0.3), dirichlet_idx=bnd, dirichlet_x=xd[bnd], x0=X.copy(),
                    density=1000.0, gravity=(0.0, -9.8, 0.0))
    op = O.make_problem(sc)
    col, nc = O.color(op)
    assert nc == 1
    x, st = O.solve(op, col, sc.initial_iterate(), max_sweeps=200, rel_tol=1e-14)

    def energy(y):
        z = sc.initial_iterate()
        z[centre] = y
        return O.residual(op, z)[1]

    def grad(y):
        z = sc.initial_iterate()
        z[centre] = y
        return O.energy_gradient(op, z)[centre]

    res = scipy.optimize.minimize(energy, X[centre], jac=grad, method="BFGS",
                                  options=dict(gtol=1e-10, maxiter=1000))
    assert np.abs(x[centre] - res.x).max() < 1e-8


@pytest.mark.parametrize("model", ["nh", "corotated", "snh"])
def test_equilibrium_matches_dense_newton(model):
    sc = small_twist(4, model, twist=25.0, stretch=1.1, noise=0.0)
    sc.density, sc.gravity = 100.0, (0.0, -9.8, 0.0)
    op = O.make_problem(sc)
    col, _ = O.color(op)
    x, st = O.solve(op, col, sc.initial_iterate(), max_sweeps=20000, rel_tol=1e-13,
                    check_every=20, accel="chebyshev", rho=0.9, gamma=1.0)
    assert st["converged"], st
    xn, it, rel = D.newton(op, sc.initial_iterate(), tol=1e-13)
    assert rel < 1e-12
    assert np.linalg.norm(x - xn) / np.linalg.norm(xn) < 1e-9


def test_linear_elastic_limit():
    """Tiny Dirichlet displacements: the nonlinear equilibrium matches the
    small-strain solve of Eq. (le) with the same Lame parameters."""
    n = 4
    X, T = S.box_mesh(n, n, n, 1.0 / (n - 1))
    bot = np.nonzero(np.isclose(X[:, 1], 0))[0]
    top = np.nonzero(np.isclose(X[:, 1], 1))[0]
    bnd = np.concatenate([bot, top]).astype(np.int32)
    eps = 1e-6
    ud = np.zeros_like(X)
    ud[top] = eps * np.array([0.3, 1.0, -0.4])
    ud[top, 0] += eps * 0.5 * X[top, 2]
    for model in ("nh", "corotated"):
        sc = S.Scenario(name="le", rest_pos=X, tets=T, model=model, E=np.asarray(1e5),
                        nu=np.asarray(0.45), dirichlet_idx=bnd, dirichlet_x=X[bnd] + ud[bnd],
                        x0=X.copy())
        op = O.make_problem(sc)
        col, _ = O.color(op)
        x, st = O.solve(op, col, sc.initial_iterate(), max_sweeps=20000, rel_tol=1e-9,
                        check_every=20, accel="chebyshev", rho=0.9, gamma=1.0)
        assert st["converged"]
        u = (x - X).reshape(-1)
        K = D.linear_fem_stiffness(X, T, op.mu, op.lam)
        fr = np.setdiff1d(np.arange(X.shape[0]), bnd)
        fd = (3 * fr[:, None] + np.arange(3)).reshape(-1)
        dd = (3 * bnd[:, None] + np.arange(3)).reshape(-1)
        ul = np.zeros_like(u)
        ul[dd] = ud[bnd].reshape(-1)
        ul[fd] = np.linalg.solve(K[np.ix_(fd, fd)], -K[np.ix_(fd, dd)] @ ul[dd])
        assert np.linalg.norm(u[fd] - ul[fd]) <= 1e-5 * np.linalg.norm(ul[fd])


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_safeguard_never_increases_local_energy(model):
    sc = small_twist(5, model, twist=90.0, stretch=1.3, noise=0.01)
    op = O.make_problem(sc)
    col, _ = O.color(op)
    x = sc.initial_iterate()
    worst = 0.0
    for _ in range(5):
        dE, x = O.sweep_energy_trace(op, col, x, safeguard="backtrack")
        _, E, _ = O.residual(op, x)
        worst = max(worst, dE.max() / max(1.0, abs(E)))
    assert worst <= 1e-13


def test_acceleration_first_steps():
    """Chebyshev: omega_1 = 1 and x^{-1} = x^0, so the first accelerated
    iterate is x^0 + gamma (x_PBNG - x^0).  SOR with x^{-1} = x^0 gives
    x^0 + omega (x_PBNG - x^0)."""
    sc = small_twist(4, "nh")
    op = O.make_problem(sc)
    col, _ = O.color(op)
    x0 = sc.initial_iterate()
    xp, _ = O.solve(op, col, x0, max_sweeps=1)
    xc, _ = O.solve(op, col, x0, max_sweeps=1, accel="chebyshev", gamma=1.7, rho=0.95)
    xs, _ = O.solve(op, col, x0, max_sweeps=1, accel="sor", omega=1.6)
    assert np.allclose(xc, x0 + 1.7 * (xp - x0), rtol=0, atol=1e-14)
    assert np.allclose(xs, x0 + 1.6 * (xp - x0), rtol=0, atol=1e-14)


def test_openmp_within_colour_is_bit_identical():
    sc = small_twist(6, "corotated", twist=60.0)
    op = O.make_problem(sc)
    col, _ = O.color(op)
    x1, _ = O.solve(op, col, sc.initial_iterate(), max_sweeps=5, n_threads=1)
    x4, _ = O.solve(op, col, sc.initial_iterate(), max_sweeps=5, n_threads=4)
    assert np.array_equal(x1, x4)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
def _adjoint_case(seed=11, model="nh"):
    rng = np.random.default_rng(seed)
    sc = S.random_cube(rng, 4, model, 1e4, 0.3, 15.0, 0.9, 1.1, "adj")
    op = O.make_problem(sc)
    op.mu = op.mu * np.exp(0.2 * rng.normal(size=op.nt))
    op.lam = op.lam * np.exp(0.2 * rng.normal(size=op.nt))
    target = sc.rest_pos + 0.05 * rng.normal(size=sc.rest_pos.shape)
    return sc, op, target


def _loss_at(op, sc, target, mu, lam, xd):
    op2 = O.OracleProblem(**{**op.__dict__, "mu": np.ascontiguousarray(mu),
                             "lam": np.ascontiguousarray(lam),
                             "dirichlet_x": np.ascontiguousarray(xd)})
    x, it, rel = D.newton(op2, sc.initial_iterate(), tol=1e-14)
    free = op.is_dir == 0
    return float(((x - target)[free] ** 2).sum()), x


@pytest.mark.parametrize("model", ["nh", "corotated", "snh"])
def test_adjoint_gradients_match_central_differences(model):
    """dL/dtheta from H lam = dL/dx (dense solve) and the gradient-assembly
    formulas, against FP64 central differences of L(x*(theta)) with Newton
    re-solves, on random directions in (x_D, log mu, log lambda)."""
    sc, op, target = _adjoint_case(model=model)
    free = op.is_dir == 0
    L0, x = _loss_at(op, sc, target, op.mu, op.lam, op.dirichlet_x)
    dLdx = np.where(free[:, None], 2.0 * (x - target), 0.0)
    lam_vec = D.adjoint_dense(op, x, dLdx)
    dmu, dla, dxd = O.adjoint_gradients(op, x, lam_vec)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(4):
        vx = rng.normal(size=op.dirichlet_x.shape)
        vm = rng.normal(size=op.nt)
        vl = rng.normal(size=op.nt)
        s = np.sqrt((vx ** 2).sum() + (vm ** 2).sum() + (vl ** 2).sum())
        vx, vm, vl = vx / s, vm / s, vl / s
        Lp, _ = _loss_at(op, sc, target, op.mu * np.exp(h * vm), op.lam * np.exp(h * vl),
                         op.dirichlet_x + h * vx)
        Lm, _ = _loss_at(op, sc, target, op.mu * np.exp(-h * vm), op.lam * np.exp(-h * vl),
                         op.dirichlet_x - h * vx)
        fd = (Lp - Lm) / (2 * h)
        an = float((dxd[op.dirichlet_idx] * vx).sum() + (dmu * op.mu * vm).sum()
                   + (dla * op.lam * vl).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3 * abs(L0)), (fd, an)


@pytest.mark.parametrize("model", ["nh", "corotated", "snh"])
def test_adjoint_parameter_gradients_by_linearity(model):
    """The energy gradient g is linear in (mu, lambda); so dg/dmu_e is exact
    by a difference quotient and dL/dmu_e = -lam^T dg/dmu_e (brute force over
    every tet of a tiny mesh)."""
    sc, op, target = _adjoint_case(seed=5, model=model)
    x, _, _ = D.newton(op, sc.initial_iterate(), tol=1e-13)
    lam_vec = RNG.normal(size=x.shape) * (op.is_dir == 0)[:, None]
    dmu, dla, _ = O.adjoint_gradients(op, x, lam_vec)
    g0 = O.energy_gradient(op, x)
    for e in RNG.choice(op.nt, 10, replace=False):
        for which, ref in (("mu", dmu), ("lam", dla)):
            arr = getattr(op, which).copy()
            arr[e] += 1.0
            op2 = O.OracleProblem(**{**op.__dict__, which: arr})
            dg = O.energy_gradient(op2, x) - g0
            assert abs(-(lam_vec * dg).sum() - ref[e]) <= 1e-9 * max(1.0, abs(ref[e]))


def test_safeguard_is_inactive_where_the_step_is_a_descent_step():
    """The corotated modified Hessian is the Hessian of a majoriser of the
    local energy, and for Neo-Hookean with lambda >= mu the full step is a
    descent step of the exactly quadratic local energy: the backtracking
    safeguard never halves.  With lambda < mu (nu = 0.1) it does."""
    for model, nu in (("corotated", 0.3), ("corotated", 0.45), ("nh", 0.3), ("nh", 0.45)):
        sc = S.twist_box(6, model, 1e4, nu, 90.0, 1.3, 0.01, seed=6)
        op = O.make_problem(sc)
        col, _ = O.color(op)
        _, st = O.solve(op, col, sc.initial_iterate(), max_sweeps=30, safeguard="backtrack")
        assert st["halvings"] == 0 and st["rejected"] == 0, (model, nu, st)
    sc = S.twist_box(6, "nh", 1e4, 0.05, 90.0, 2.0, 0.01, seed=6)
    op = O.make_problem(sc)
    col, _ = O.color(op)
    _, st = O.solve(op, col, sc.initial_iterate(), max_sweeps=30, safeguard="backtrack")
    assert st["halvings"] > 0
