"""Pins of the oracle's backward-Euler inertia (Eq. fem_be minimised as an
incremental potential, lumped mass m_ii = int R0 N_i) against facts that do
not come from the oracle: exact mass sums, the exact free-fall step of a
rigid body, central differences, an independent dense Newton solve and
energy monotonicity."""
import numpy as np
import pytest

import oracle as O
from oracle import dense as D
from paper_2306_09021_amd import scenarios as S

from .test_oracle_solve import small_twist, with_extras

RNG = np.random.default_rng(2024)


def free_box(n=4, model="nh", density=1000.0, gravity=(0.0, -9.8, 0.0)):
    """A box with no Dirichlet vertex at all (inertia alone makes the
    incremental potential strictly convex)."""
    X, T = S.box_mesh(n, n, n, 1.0 / (n - 1))
    return S.Scenario(name="free", rest_pos=X, tets=T, model=model, E=np.asarray(1e4),
                      nu=np.asarray(0.3), dirichlet_idx=np.zeros(0, np.int32),
                      dirichlet_x=np.zeros((0, 3)), x0=X.copy(), density=density,
                      gravity=gravity)


def test_lumped_mass_sums_to_total_mass():
    """m_ii = R0 sum V0_e / 4: the masses sum to R0 times the volume, and a
    single right tet gives each vertex R0 / 24."""
    X, T = S.box_mesh(5, 4, 3, (0.25, 0.3, 0.5))
    sc = S.Scenario(name="m", rest_pos=X, tets=T, model="nh", E=np.asarray(1.0),
                    nu=np.asarray(0.3), dirichlet_idx=np.zeros(0, np.int32),
                    dirichlet_x=np.zeros((0, 3)), x0=X, density=7.0)
    op = O.make_problem(sc)
    assert abs(op.mass.sum() - 7.0 * 1.0 * 0.9 * 1.0) < 1e-12
    X1 = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    sc1 = S.Scenario(name="t", rest_pos=X1, tets=np.array([[0, 1, 2, 3]], np.int32), model="nh",
                     E=np.asarray(1.0), nu=np.asarray(0.3), dirichlet_idx=np.zeros(0, np.int32),
                     dirichlet_x=np.zeros((0, 3)), x0=X1, density=3.0)
    assert np.allclose(O.make_problem(sc1).mass, 3.0 / 24.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_free_fall_step_is_exact(model):
    """A rigid body translating with velocity v under gravity g: the
    incremental potential is minimised by the rigid translation
    y = xhat + dt^2 g (elastic energy is zero there and nonnegative
    elsewhere; the inertia term is strictly convex), with lumped gravity
    f_i = m_i g."""
    sc = free_box(4, model)
    op = O.make_problem(sc)
    dt = 1e-2
    v = np.array([0.3, -0.1, 0.2])
    c = np.array([0.05, 0.1, -0.02])
    x_n = sc.rest_pos + c
    x_prev = x_n - dt * v
    op.set_inertia(dt, x_n, x_prev)
    col, _ = O.color(op)
    y0 = x_n + 1e-3 * RNG.normal(size=x_n.shape)
    y, st = O.solve(op, col, y0, max_sweeps=500, rel_tol=1e-14, check_every=5, accel="none")
    exact = x_n + dt * v + dt * dt * np.asarray(sc.gravity)
    assert np.abs(y - exact).max() <= 1e-11
    assert st["converged"]


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_inertia_residual_is_minus_energy_gradient(model):
    """r_i = f_i + fhat_i - m_ii / dt^2 (y_i - xhat_i) = -dE/dy_i, checked by
    central differences of the energy with every term present."""
    sc = with_extras(small_twist(4, model))
    op = O.make_problem(sc)
    x_n = sc.initial_iterate() + 0.01 * RNG.normal(size=(sc.n_verts, 3))
    x_prev = x_n - 0.01 * RNG.normal(size=x_n.shape)
    op.set_inertia(5e-3, x_n, x_prev)
    x = x_n + 0.02 * RNG.normal(size=x_n.shape)
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


def test_inertia_hessian_vector_product():
    """The Hessian-vector product gains m_ii / dt^2 v_i: against central
    differences of the analytic gradient."""
    sc = with_extras(small_twist(4, "nh"))
    op = O.make_problem(sc)
    x = sc.initial_iterate()
    op.set_inertia(1e-2, x, x - 1e-3)
    v = RNG.normal(size=x.shape)
    h = 1e-6
    fd = (O.energy_gradient(op, x + h * v) - O.energy_gradient(op, x - h * v)) / (2 * h)
    Hv = O.hvp(op, x, v)
    assert np.abs(fd - Hv).max() <= 1e-6 * np.abs(Hv).max()


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_backward_euler_step_matches_dense_newton(model):
    """One backward-Euler step of a pinned, twisted box under gravity: the
    PBNG iteration on the incremental potential reaches the minimiser that an
    independent dense Newton solve finds."""
    sc = small_twist(4, model, twist=25.0, stretch=1.1, noise=0.0)
    sc.density, sc.gravity = 100.0, (0.0, -9.8, 0.0)
    op = O.make_problem(sc)
    x_n = sc.initial_iterate()
    x_prev = x_n.copy()
    x_prev[op.is_dir == 0] -= 1e-2 * np.array([0.0, 1.0, 0.5])
    op.set_inertia(2e-2, x_n, x_prev)
    col, _ = O.color(op)
    x, st = O.solve(op, col, x_n, max_sweeps=20000, rel_tol=1e-13, check_every=20,
                    accel="chebyshev", rho=0.9, gamma=1.0)
    assert st["converged"], st
    xn, it, rel = D.newton(op, x_n, tol=1e-13)
    assert rel < 1e-12
    assert np.linalg.norm(x - xn) / np.linalg.norm(xn) < 1e-9


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_inertia_safeguard_never_increases_local_energy(model):
    sc = small_twist(5, model, twist=90.0, stretch=1.3, noise=0.01)
    sc.density = 500.0
    op = O.make_problem(sc)
    x = sc.initial_iterate()
    op.set_inertia(1e-2, x, x)
    col, _ = O.color(op)
    worst = 0.0
    for _ in range(5):
        dE, x = O.sweep_energy_trace(op, col, x, safeguard="backtrack")
        _, E, _ = O.residual(op, x)
        worst = max(worst, dE.max() / max(1.0, abs(E)))
    assert worst <= 1e-13


def test_inertia_off_restores_quasistatics():
    sc = small_twist(4, "nh")
    sc.density = 100.0
    op = O.make_problem(sc)
    x = sc.initial_iterate()
    r0 = O.residual(op, x)
    op.set_inertia(1e-2, x, x - 0.1)
    assert O.residual(op, x)[0] != r0[0]
    op.set_inertia(0.0)
    assert O.residual(op, x)[0] == r0[0]
