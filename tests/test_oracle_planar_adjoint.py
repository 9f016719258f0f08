"""Pins of the planar (d = 2) oracle's adjoint pieces, against facts that do
not come from them:

* dP[L] against central differences of the pinned first Piola-Kirchhoff
  stress P (both models, the corotated one away from a = b = 0);
* H v against central differences of the pinned residual (minus the energy
  gradient) with every term present: elements, weak constraints, active
  half-planes and inertia;
* the symmetry w^T H v = v^T H w of the true Hessian;
* the gradients dL/dmu_e, dL/dlambda_e and dL/dx_D of L(x*) = 1/2 |x* - t|^2
  over free vertices against central differences of L through equilibria
  re-solved by Newton's method."""
import numpy as np
import pytest

from oracle import planar as P
from paper_2306_09021_amd import scenarios as S

RNG = np.random.default_rng(123)


def rand_F(scale=0.3):
    while True:
        F = np.eye(2) + scale * RNG.normal(size=(2, 2))
        if np.linalg.det(F) > 0.2:
            return F


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_stress_diff_is_the_derivative_of_P(model):
    m = P.MODEL[model]
    mu, lam = 2.5, 7.0
    h = 1e-6
    for _ in range(20):
        F, L = rand_F(), RNG.normal(size=(2, 2))
        fd = (P.pk1(m, mu, lam, F + h * L) - P.pk1(m, mu, lam, F - h * L)) / (2 * h)
        dP = P.stress_diff(m, mu, lam, F, L)
        assert np.abs(dP - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def _terms_problem(model, seed=3):
    sc = S.planar_terms(7, model, seed=seed, n_springs=6, k_ground=300.0)
    op = P.make_problem(sc)
    rng = np.random.default_rng(seed)
    x = sc.initial_iterate() + 0.02 * rng.normal(size=(sc.n_verts, 2))
    x[sc.dirichlet_idx] = sc.dirichlet_x
    x[:, 1] -= 0.01                            # a few vertices inside the half-plane
    x[sc.dirichlet_idx] = sc.dirichlet_x
    op.set_inertia(0.05, x + 0.003, x - 0.002)
    return sc, op, x


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_hessian_apply_is_the_residual_derivative(model):
    sc, op, x = _terms_problem(model)
    phi = x[:, 1] + 0.02
    free = op.is_dir == 0
    assert (phi[free] < 0).any() and (phi[free] > 0).any()      # active and inactive half-plane rows
    assert np.abs(phi).min() > 1e-4                              # no row at the kink
    h = 1e-7
    for _ in range(3):
        v = RNG.normal(size=x.shape)
        v[~free] = 0.0
        Hv = P.hessian_apply(op, x, v)
        rp = P.residual(op, x + h * v)[2]
        rm = P.residual(op, x - h * v)[2]
        fd = -(rp - rm) / (2 * h)
        assert np.abs(Hv[free] - fd[free]).max() <= 1e-6 * np.abs(fd[free]).max()


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_hessian_is_symmetric(model):
    sc, op, x = _terms_problem(model, seed=5)
    free = op.is_dir == 0
    v, w = RNG.normal(size=x.shape), RNG.normal(size=x.shape)
    v[~free] = 0.0
    w[~free] = 0.0
    a = np.sum(w * P.hessian_apply(op, x, v))
    b = np.sum(v * P.hessian_apply(op, x, w))
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_gradients_match_finite_differences_through_equilibria(model):
    sc = S.stretched_square(6, model, 1.3, noise=0.2, seed=2)
    sc.nodal_force = 2.0 * np.random.default_rng(4).normal(size=(sc.n_verts, 2))
    mu0, lam0 = P.make_problem(sc).mu.copy(), P.make_problem(sc).lam.copy()
    t = sc.rest_pos + 0.05 * np.random.default_rng(6).normal(size=sc.rest_pos.shape)

    def loss(mu=mu0, lam=lam0, xd=None):
        s2 = sc
        if xd is not None:
            s2 = S.Scenario2D(**{**sc.__dict__, "dirichlet_x": xd})
        op = P.make_problem(s2, mu=mu, lam=lam)
        x = P.newton_equilibrium(op, s2.initial_iterate())
        free = op.is_dir == 0
        return 0.5 * np.sum((x[free] - t[free]) ** 2), x, op

    L0, x, op = loss()
    free = op.is_dir == 0
    b = np.zeros_like(x)
    b[free] = x[free] - t[free]
    lam, dxd, dmu, dlam = P.adjoint(op, x, b)
    h = 1e-6
    for e in (0, 7, 23, 40):
        for arr, g in ((mu0, dmu), (lam0, dlam)):
            ep = arr.copy()
            em = arr.copy()
            ep[e] *= 1 + h
            em[e] *= 1 - h
            kw_p = {"mu": ep} if arr is mu0 else {"lam": ep}
            kw_m = {"mu": em} if arr is mu0 else {"lam": em}
            fd = (loss(**kw_p)[0] - loss(**kw_m)[0]) / (2 * h * arr[e])
            assert abs(g[e] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max())
    for k in (0, 3, 8):
        for a in range(2):
            xp = sc.dirichlet_x.copy()
            xm = sc.dirichlet_x.copy()
            xp[k, a] += h
            xm[k, a] -= h
            fd = (loss(xd=xp)[0] - loss(xd=xm)[0]) / (2 * h)
            assert abs(dxd[k, a] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(dxd).max())
