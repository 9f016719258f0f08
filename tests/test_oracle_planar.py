"""Pins of the planar (d = 2) oracle against facts that do not come from it:

* the plane-strain reduction: with F = diag(F2, 1) the 3-D densities of
  Eq. (nh) and (cor) (the pinned 3-D oracle, an independent code with an
  SVD-based rotation) equal the planar ones up to the constant 1/2 mu of
  the Neo-Hookean |F|^2 term; the first Piola-Kirchhoff stress and the
  modified Hessian density of Eq. (mod_hess_dens) are their in-plane blocks;
* the closest rotation by brute-force maximisation over the angle, and the
  polar factor U V^T of numpy's SVD;
* the linearisation at rest, which must be planar isotropic linear
  elasticity 2 mu sym(H) + lambda tr(H) I (the reason for lhat = mu +
  lambda in Eq. nh);
* exact shape-function gradients on affine fields, and the total area;
* the residual as minus the central-difference gradient of the energy;
* the patch test: with every boundary vertex on an affine map the affine
  field is the exact discrete equilibrium, whatever the interior mesh;
* the equilibrium of an independent Newton solve with a finite-difference
  Hessian;
* an independent greedy colouring, safeguard monotonicity, and the blends
  that reduce to the plain iteration up to rounding (SOR omega = 1;
  Chebyshev rho = 0, gamma = 1)."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle as O
from oracle import planar as P
from paper_2306_09021_amd import scenarios as S

RNG = np.random.default_rng(77)
MODELS = ["nh", "corotated"]


def rand_F2(det_sign=1, scale=0.4):
    while True:
        F = np.eye(2) + scale * RNG.normal(size=(2, 2))
        if np.sign(np.linalg.det(F)) == det_sign and abs(np.linalg.det(F)) > 0.1:
            return F


def embed(F2):
    F = np.eye(3)
    F[:2, :2] = F2
    return F


@pytest.mark.parametrize("model", MODELS)
def test_plane_strain_reduction_of_the_3d_densities(model):
    mu, lam = 3.7, 11.2
    m2, m3 = P.MODEL[model], O.MODEL[model]
    c0 = 0.5 * mu if model == "nh" else 0.0
    for _ in range(20):
        F2 = rand_F2()
        F3 = embed(F2)
        e2, e3 = P.psi(m2, mu, lam, F2), O.psi(m3, mu, lam, F3)
        assert abs(e2 - (e3 - c0)) <= 1e-12 * max(1.0, abs(e3))
        P2, P3 = P.pk1(m2, mu, lam, F2), O.pk1(m3, mu, lam, F3)
        assert np.abs(P2 - P3[:2, :2]).max() <= 1e-12 * max(1.0, np.abs(P3).max())
        C2, C3 = P.mod_hess_density(mu, lam, F2), O.mod_hess_density(mu, lam, F3)
        assert np.abs(C2 - C3[:2, :2, :2, :2]).max() <= 1e-12 * np.abs(C3).max()


@pytest.mark.parametrize("det_sign", [1, -1])
def test_closest_rotation_by_brute_force(det_sign):
    for _ in range(10):
        F = rand_F2(det_sign, 0.8)
        R = P.rotation(F)
        assert np.abs(R.T @ R - np.eye(2)).max() <= 1e-14 and np.linalg.det(R) > 0
        f = lambda t: -(np.cos(t) * (F[0, 0] + F[1, 1]) + np.sin(t) * (F[1, 0] - F[0, 1]))
        ts = np.linspace(-np.pi, np.pi, 3601)
        t0 = ts[np.argmin([f(t) for t in ts])]
        t = minimize_scalar(f, bounds=(t0 - 0.01, t0 + 0.01), method="bounded",
                            options={"xatol": 1e-12}).x
        Rb = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
        assert np.abs(R - Rb).max() <= 1e-7
        if det_sign > 0:
            U, s, Vt = np.linalg.svd(F)
            assert np.abs(R - U @ Vt).max() <= 1e-13


@pytest.mark.parametrize("model", MODELS)
def test_linearisation_at_rest_is_isotropic_linear_elasticity(model):
    mu, lam = 2.0, 5.0
    m = P.MODEL[model]
    h = 1e-6
    for _ in range(5):
        H = RNG.normal(size=(2, 2))
        dP = (P.pk1(m, mu, lam, np.eye(2) + h * H) - P.pk1(m, mu, lam, np.eye(2) - h * H)) / (2 * h)
        lin = mu * (H + H.T) + lam * np.trace(H) * np.eye(2)
        assert np.abs(dP - lin).max() <= 1e-7 * np.abs(lin).max()


@pytest.mark.parametrize("model", MODELS)
def test_rest_state_is_stress_free_and_energy_rotation_invariant(model):
    m = P.MODEL[model]
    for _ in range(5):
        t = RNG.uniform(-np.pi, np.pi)
        Q = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
        assert np.abs(P.pk1(m, 1.3, 4.0, Q)).max() <= 1e-14
        F = rand_F2()
        assert abs(P.psi(m, 1.3, 4.0, Q @ F) - P.psi(m, 1.3, 4.0, F)) <= 1e-13


def jittered_square(n=7, model="nh", diag="alternate", seed=3):
    X, T = S.square_mesh(n, n, 1.0 / (n - 1), diag)
    rng = np.random.default_rng(seed)
    col, row = np.arange(n * n) % n, np.arange(n * n) // n
    inner = (col > 0) & (col < n - 1) & (row > 0) & (row < n - 1)
    X[inner] += 0.25 / (n - 1) * rng.uniform(-1, 1, size=(inner.sum(), 2))
    bnd = np.nonzero(~inner)[0].astype(np.int32)
    return X, T, bnd


def test_shape_gradients_are_exact_on_affine_fields():
    X, T, _ = jittered_square(8)
    sc = S.Scenario2D("p", X, T, "nh", np.asarray(1.0), np.asarray(0.3), np.zeros(0, np.int32),
                      np.zeros((0, 2)), X)
    op = P.make_problem(sc)
    assert abs(op.A0.sum() - 1.0) <= 1e-14
    assert np.abs(op.dN.sum(axis=1)).max() <= 1e-12
    A = RNG.normal(size=(2, 2))
    y = X @ A.T + RNG.normal(size=2)
    F = np.einsum("ejc,ejd->ecd", y[T], op.dN)       # F_e = sum_j y_j dN_j^T
    assert np.abs(F - A[None]).max() <= 1e-12


@pytest.mark.parametrize("model", MODELS)
def test_residual_is_minus_energy_gradient(model):
    X, T, bnd = jittered_square(6, model)
    sc = S.Scenario2D("p", X, T, model, np.asarray(1e3), np.asarray(0.35), bnd, X[bnd], X,
                      density=10.0, gravity=(0.3, -9.8))
    op = P.make_problem(sc)
    y = X + 0.05 * RNG.normal(size=X.shape)
    y[bnd] = X[bnd]
    _, _, r = P.residual(op, y)
    h = 1e-6
    free = np.nonzero(op.is_dir == 0)[0]
    for i in RNG.choice(free, 6, replace=False):
        for a in range(2):
            yp, ym = y.copy(), y.copy()
            yp[i, a] += h
            ym[i, a] -= h
            fd = (P.residual(op, yp)[1] - P.residual(op, ym)[1]) / (2 * h)
            assert abs(fd + r[i, a]) <= 1e-6 * max(1.0, np.abs(r).max())
    assert np.all(r[bnd] == 0.0)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("diag", ["uniform", "alternate"])
def test_patch_test_reaches_the_affine_field(model, diag):
    X, T, bnd = jittered_square(9, model, diag)
    A = np.array([[1.3, 0.2], [-0.1, 0.8]])
    b = np.array([0.05, -0.02])
    xd = X[bnd] @ A.T + b
    sc = S.Scenario2D("patch", X, T, model, np.asarray(1e3), np.asarray(0.3), bnd, xd, X)
    op = P.make_problem(sc)
    col, _ = P.color(op)
    x, st = P.solve(op, col, sc.initial_iterate(), max_sweeps=5000, rel_tol=1e-13, check_every=10,
                    accel="chebyshev", rho=0.9, gamma=1.0)
    assert st["converged"], st
    assert np.abs(x - (X @ A.T + b)).max() <= 1e-11


def fd_newton(op, x0, tol=1e-13, iters=30):
    """Newton on the free DOFs with the Hessian from central differences of
    the oracle's residual (so no Hessian code of the oracle is involved) and
    a backtracking line search on the total energy."""
    x = x0.copy()
    free = np.nonzero(op.is_dir == 0)[0]
    dofs = (2 * free[:, None] + np.arange(2)[None]).reshape(-1)
    r0 = P.residual(op, x)[0]
    for _ in range(iters):
        n, _, r = P.residual(op, x)
        if n <= tol * r0:
            break
        H = np.zeros((dofs.size, dofs.size))
        h = 1e-7
        for k, d in enumerate(dofs):
            xp, xm = x.reshape(-1).copy(), x.reshape(-1).copy()
            xp[d] += h
            xm[d] -= h
            H[:, k] = -(P.residual(op, xp.reshape(-1, 2))[2].reshape(-1)[dofs]
                        - P.residual(op, xm.reshape(-1, 2))[2].reshape(-1)[dofs]) / (2 * h)
        step = np.linalg.solve(0.5 * (H + H.T), r.reshape(-1)[dofs])
        E0, t = P.residual(op, x)[1], 1.0
        while t > 1e-8:                      # backtracking on the total energy
            xt = x.copy()
            xt.reshape(-1)[dofs] += t * step
            if P.residual(op, xt)[1] <= E0 + 1e-12 * abs(E0):
                break
            t *= 0.5
        x = xt
    return x, P.residual(op, x)[0] / r0


@pytest.mark.parametrize("model", MODELS)
def test_solve_reaches_the_newton_equilibrium(model):
    sc = S.stretched_square(7, model, 1.4, E=1e3, nu=0.3, diagonal="uniform", density=50.0,
                            gravity=(0.0, -9.8), noise=0.2, seed=4)
    op = P.make_problem(sc)
    xn, rel = fd_newton(op, sc.initial_iterate())
    assert rel <= 1e-11
    col, _ = P.color(op)
    x, st = P.solve(op, col, sc.initial_iterate(), max_sweeps=20000, rel_tol=1e-13, check_every=10,
                    accel="chebyshev", rho=0.9, gamma=1.0)
    assert st["converged"], st
    assert np.linalg.norm(x - xn) / np.linalg.norm(xn) <= 1e-10


def test_colouring_is_the_greedy_one():
    for diag in ("uniform", "alternate"):
        sc = S.stretched_square(12, "nh", 1.2, diagonal=diag)
        op = P.make_problem(sc)
        col, nc = P.color(op)
        nbrs = [set() for _ in range(op.nv)]
        for t in op.tris:
            for a in t:
                nbrs[a].update(int(b) for b in t if b != a)
        ref = -np.ones(op.nv, np.int64)
        for i in range(op.nv):
            if op.is_dir[i]:
                continue
            used = {ref[j] for j in nbrs[i] if ref[j] >= 0}
            ref[i] = min(c for c in range(len(used) + 1) if c not in used)
        assert np.array_equal(col, ref)
        assert nc == ref.max() + 1
        for t in op.tris:
            c = [col[v] for v in t if col[v] >= 0]
            assert len(c) == len(set(c))


@pytest.mark.parametrize("model", MODELS)
def test_safeguard_never_increases_the_energy(model):
    sc = S.stretched_square(10, model, 2.5, E=1e4, nu=0.45, noise=0.6, seed=9)
    op = P.make_problem(sc)
    col, _ = P.color(op)
    x = sc.initial_iterate()
    worst = 0.0
    for _ in range(4):
        dE, x = P.sweep_energy_trace(op, col, x, safeguard="backtrack")
        worst = max(worst, dE.max() / max(1.0, abs(P.residual(op, x)[1])))
    assert worst <= 1e-13


@pytest.mark.parametrize("kw", [dict(accel="sor", omega=1.0), dict(accel="chebyshev", rho=0.0, gamma=1.0)])
def test_blends_that_reduce_to_the_plain_iteration(kw):
    sc = S.stretched_square(9, "corotated", 1.6, noise=0.3, seed=2)
    op = P.make_problem(sc)
    col, _ = P.color(op)
    a, _ = P.solve(op, col, sc.initial_iterate(), max_sweeps=25)
    b, _ = P.solve(op, col, sc.initial_iterate(), max_sweeps=25, **kw)
    # equal up to the rounding of (x_P - x) + x
    assert np.abs(a - b).max() <= 1e-13
    c, _ = P.solve(op, col, sc.initial_iterate(), max_sweeps=25, accel="sor", omega=1.5)
    assert np.abs(a - c).max() > 1e-6


def test_modified_density_is_spd_for_every_F():
    """Eq. (mod_hess_dens) with d = 2 as a 4 x 4 matrix on vec(dF): SPD for
    regular, inverted, rank-one and zero F (mu, lambda > 0)."""
    mats = [rand_F2(1), rand_F2(-1), np.outer(RNG.normal(size=2), RNG.normal(size=2)), np.zeros((2, 2))]
    for F in mats:
        C = P.mod_hess_density(2.0, 7.0, F).reshape(4, 4)
        assert np.abs(C - C.T).max() <= 1e-14 * np.abs(C).max()
        assert np.linalg.eigvalsh(C).min() >= 2 * 2.0 * (1 - 1e-12)   # >= 2 mu


def test_energies_at_rotations():
    """The corotated energy vanishes on rotations; the Neo-Hookean one is its
    constant rest value 1/2 mu d + 1/2 lhat (mu / lhat)^2 there."""
    mu, lam = 1.7, 3.1
    lh = mu + lam
    for _ in range(5):
        t = RNG.uniform(-np.pi, np.pi)
        Q = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
        assert abs(P.psi(P.COROTATED, mu, lam, Q)) <= 1e-14
        assert abs(P.psi(P.NEOHOOKEAN, mu, lam, Q) - (mu + 0.5 * lh * (mu / lh) ** 2)) <= 1e-13
