"""Pins for the oracle's constitutive layer (Sec. "Constitutive Models",
"Modified Hessian", "Lame Coefficients"), checked against facts the paper and
the mathematics fix rather than against the oracle's own formulas."""
import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(1234)
MODELS = [O.NEOHOOKEAN, O.COROTATED, O.STABLE_NEOHOOKEAN]


def rand_rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def rand_F(rng, inverted=False):
    F = np.eye(3) + 0.4 * rng.normal(size=(3, 3))
    if inverted and np.linalg.det(F) > 0:
        F[:, 0] *= -1
    return F


def test_lame_closed_form():
    # Eq. (lame) at E = 1e4, nu = 0.3: mu = 1e4 / 2.6 = 50000/13,
    # lambda = 3000 / 0.52 = 75000/13 (exact rationals).
    mu, lam = O.lame(1e4, 0.3)
    assert abs(mu - 50000.0 / 13.0) < 1e-9
    assert abs(lam - 75000.0 / 13.0) < 1e-9
    # nu = 0.45, E = 1e5: mu = 1e5/2.9, lambda = 45000/(1.45*0.1)
    mu, lam = O.lame(1e5, 0.45)
    assert abs(mu - 1e5 / 2.9) < 1e-8
    assert abs(lam - 45000.0 / 0.145) < 1e-6


@pytest.mark.parametrize("model", MODELS)
def test_zero_stress_at_rest(model):
    mu, lam = O.lame(1e4, 0.3)
    P = O.pk1(model, mu, lam, np.eye(3))
    assert np.abs(P).max() < 1e-10 * mu
    # also at any rotation: both models are rotation invariant and stress free there
    Q = rand_rot(RNG)
    P = O.pk1(model, mu, lam, Q)
    assert np.abs(P).max() < 1e-9 * mu


def test_corotated_energy_zero_on_rotations_and_nonnegative():
    mu, lam = O.lame(1e4, 0.3)
    for _ in range(20):
        Q = rand_rot(RNG)
        assert abs(O.psi(O.COROTATED, mu, lam, Q)) < 1e-9 * mu
        F = rand_F(RNG, inverted=bool(RNG.integers(2)))
        assert O.psi(O.COROTATED, mu, lam, F) >= 0.0


def test_neohookean_minimum_at_rest():
    # Psi_nh(I) = 3 mu / 2 + mu^2 / (2 lhat) and I is a stationary point.
    mu, lam = O.lame(1e4, 0.3)
    lh = mu + lam
    assert abs(O.psi(O.NEOHOOKEAN, mu, lam, np.eye(3)) - (1.5 * mu + mu * mu / (2 * lh))) < 1e-8
    for _ in range(20):
        F = np.eye(3) + 1e-3 * RNG.normal(size=(3, 3))
        assert O.psi(O.NEOHOOKEAN, mu, lam, F) > O.psi(O.NEOHOOKEAN, mu, lam, np.eye(3))


@pytest.mark.parametrize("model", MODELS)
def test_rotation_invariance(model):
    mu, lam = O.lame(1e5, 0.45)
    for _ in range(25):
        F = rand_F(RNG, inverted=bool(RNG.integers(2)))
        Q = rand_rot(RNG)
        e0 = O.psi(model, mu, lam, F)
        e1 = O.psi(model, mu, lam, Q @ F)
        assert abs(e0 - e1) <= 1e-10 * max(1.0, abs(e0))
        P0 = O.pk1(model, mu, lam, F)
        P1 = O.pk1(model, mu, lam, Q @ F)
        assert np.abs(Q @ P0 - P1).max() <= 1e-9 * max(1.0, np.abs(P0).max())


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("inverted", [False, True])
def test_stress_is_energy_derivative(model, inverted):
    """Central differences of Psi against P, relative error <= 1e-7."""
    mu, lam = O.lame(1e4, 0.3)
    h = 1e-6
    for _ in range(10):
        F = rand_F(RNG, inverted)
        P = O.pk1(model, mu, lam, F)
        fd = np.zeros((3, 3))
        for a in range(3):
            for b in range(3):
                E = np.zeros((3, 3))
                E[a, b] = h
                fd[a, b] = (O.psi(model, mu, lam, F + E) - O.psi(model, mu, lam, F - E)) / (2 * h)
        assert np.abs(fd - P).max() <= 1e-7 * max(1.0, np.abs(P).max())


def test_neohookean_stress_differential():
    mu, lam = O.lame(1e5, 0.45)
    h = 1e-6
    for inverted in (False, True):
        for _ in range(10):
            F = rand_F(RNG, inverted)
            dF = RNG.normal(size=(3, 3))
            dP = O.nh_dpk1(mu, lam, F, dF)
            fd = (O.pk1(O.NEOHOOKEAN, mu, lam, F + h * dF)
                  - O.pk1(O.NEOHOOKEAN, mu, lam, F - h * dF)) / (2 * h)
            assert np.abs(fd - dP).max() <= 1e-7 * max(1.0, np.abs(dP).max())


def test_modified_hessian_density_is_spd():
    """Eq. (mod_hess_dens) is SPD for every F: regular, inverted, singular."""
    mu, lam = O.lame(1e5, 0.45)
    cases = [rand_F(RNG, False) for _ in range(10)] + [rand_F(RNG, True) for _ in range(10)]
    S = rand_F(RNG)
    S[:, 2] = S[:, 0] + S[:, 1]             # singular
    cases += [S, np.zeros((3, 3))]
    for F in cases:
        Ct = O.mod_hess_density(mu, lam, F).reshape(9, 9)   # [(a g), (b d)]
        assert np.abs(Ct - Ct.T).max() <= 1e-9 * np.abs(Ct).max()
        w = np.linalg.eigvalsh(Ct)
        assert w.min() >= 2 * mu * (1 - 1e-12)


@pytest.mark.parametrize("model", [O.NEOHOOKEAN, O.COROTATED])
def test_lame_consistency_at_rest(model):
    """Sec. "Lame Coefficients": at F = I the Hessian of Psi matches linear
    elasticity, Eq. (le), whose second variation for a symmetric dF is
    2 mu |dF|^2 + lambda tr(dF)^2; the modified density matches it too."""
    E, nu = 1e5, 0.45
    mu, lam = O.lame(E, nu)
    h = 1e-5
    for _ in range(10):
        A = RNG.normal(size=(3, 3))
        dF = 0.5 * (A + A.T)
        # second variation by central differences of P
        dP = (O.pk1(model, mu, lam, np.eye(3) + h * dF)
              - O.pk1(model, mu, lam, np.eye(3) - h * dF)) / (2 * h)
        q = float((dP * dF).sum())
        le = 2 * mu * float((dF * dF).sum()) + lam * np.trace(dF) ** 2
        assert abs(q - le) <= 1e-6 * le
        Ct = O.mod_hess_density(mu, lam, np.eye(3))
        qt = float(np.einsum("agbd,ag,bd->", Ct, dF, dF))
        assert abs(qt - le) <= 1e-10 * le


def test_stable_neohookean_at_rest():
    """Eq. (snh) with lambda on the volume term: Psi(I) = 9 mu^2 / (32 lambda)
    - mu log 2 (|I|^2 = 3, det I - alpha = -3 mu / (4 lambda)), and its
    second variation on a symmetric dF, worked out by hand from the Taylor
    series of |F|^2, det F and log(1 + |F|^2) about I, is
    (3/2) mu |dF|^2 + (lambda - 5 mu / 8) tr(dF)^2 (the printed model is not
    Lame-consistent without a rescaling of mu and lambda, which the paper
    does not give)."""
    mu, lam = O.lame(1e5, 0.45)
    assert abs(O.psi(O.STABLE_NEOHOOKEAN, mu, lam, np.eye(3))
               - (9 * mu * mu / (32 * lam) - mu * np.log(2.0))) <= 1e-9 * mu
    h = 1e-5
    for _ in range(10):
        A = RNG.normal(size=(3, 3))
        dF = 0.5 * (A + A.T)
        dP = (O.pk1(O.STABLE_NEOHOOKEAN, mu, lam, np.eye(3) + h * dF)
              - O.pk1(O.STABLE_NEOHOOKEAN, mu, lam, np.eye(3) - h * dF)) / (2 * h)
        q = float((dP * dF).sum())
        ref = 1.5 * mu * float((dF * dF).sum()) + (lam - 0.625 * mu) * np.trace(dF) ** 2
        assert abs(q - ref) <= 1e-6 * abs(ref)


@pytest.mark.parametrize("model", MODELS)
def test_stress_differential_all_models(model):
    """dP[dF] (the true Hessian density) against central differences of P,
    including inverted F for the Neo-Hookean models; for the corotated model
    F is kept away from the inversion where dR is singular."""
    mu, lam = O.lame(1e5, 0.45)
    h = 1e-6
    for inverted in (False, True):
        if inverted and model == O.COROTATED:
            continue
        for _ in range(10):
            F = rand_F(RNG, inverted)
            dF = RNG.normal(size=(3, 3))
            dP = O.dpk1(model, mu, lam, F, dF)
            fd = (O.pk1(model, mu, lam, F + h * dF) - O.pk1(model, mu, lam, F - h * dF)) / (2 * h)
            assert np.abs(fd - dP).max() <= 1e-7 * max(1.0, np.abs(dP).max())


def test_corotated_stress_differential_is_symmetric():
    """The Hessian density of a hyperelastic energy is symmetric:
    dF2 : dP[dF1] = dF1 : dP[dF2]."""
    mu, lam = O.lame(1e4, 0.3)
    for _ in range(10):
        F = rand_F(RNG)
        A, B = RNG.normal(size=(3, 3)), RNG.normal(size=(3, 3))
        a = float((B * O.dpk1(O.COROTATED, mu, lam, F, A)).sum())
        b = float((A * O.dpk1(O.COROTATED, mu, lam, F, B)).sum())
        assert abs(a - b) <= 1e-10 * max(abs(a), 1.0)


def test_signed_svd_against_library():
    """The oracle's 3x3 SVD matches numpy's singular values; U, V are
    rotations; the smallest singular value carries the sign of det F."""
    for inverted in (False, True):
        for _ in range(50):
            F = rand_F(RNG, inverted)
            U, s, V = O.svd3(F)
            ref = np.linalg.svd(F, compute_uv=False)
            assert np.allclose(np.abs(s), ref, rtol=1e-12, atol=1e-14)
            assert abs(np.linalg.det(U) - 1) < 1e-12 and abs(np.linalg.det(V) - 1) < 1e-12
            assert np.allclose(U @ np.diag(s) @ V.T, F, atol=1e-13)
            assert (s[2] < 0) == (np.linalg.det(F) < 0)
    # rank-deficient inputs still give rotations and reconstruct F
    for F in (np.diag([2.0, 1.0, 0.0]), np.zeros((3, 3)), np.outer([1, 2, 3], [0, 1, 1.0])):
        U, s, V = O.svd3(F)
        assert abs(np.linalg.det(U) - 1) < 1e-12 and abs(np.linalg.det(V) - 1) < 1e-12
        assert np.allclose(U @ np.diag(s) @ V.T, F, atol=1e-13)


def test_corotated_rotation_is_closest_rotation():
    """R(F) maximises tr(R^T F) over SO(3), so |F - R| <= |F - Q| for all Q."""
    mu, lam = 1.0, 0.0
    for _ in range(20):
        F = rand_F(RNG, inverted=bool(RNG.integers(2)))
        e = O.psi(O.COROTATED, mu, lam, F)
        for _ in range(20):
            Q = rand_rot(RNG)
            assert e <= np.sum((F - Q) ** 2) + 1e-12


def test_chebyshev_weights():
    """Sec. "Acceleration Techniques": omega_1 = omega_2 = 1, omega_3 =
    2/(2 - rho^2), then omega_{l+1} = 4/(4 - rho^2 omega_l), which converges
    to the fixed point 2 (1 - sqrt(1 - rho^2)) / rho^2."""
    for rho in (0.95, 0.995):
        w = O.chebyshev_weights(rho, 4000)
        assert w[0] == 1.0 and w[1] == 1.0
        assert abs(w[2] - 2.0 / (2.0 - rho * rho)) < 1e-15
        lim = 2.0 * (1.0 - np.sqrt(1.0 - rho * rho)) / (rho * rho)
        assert abs(w[-1] - lim) < 1e-12
        assert np.all(np.diff(w[2:]) <= 0)     # non-increasing towards the limit
    # rho = 0.95 hand values: omega_3 = 2/1.0975, omega_4 = 4/(4 - 0.9025 omega_3)
    w = O.chebyshev_weights(0.95, 4)
    assert abs(w[2] - 1.822323462415) < 1e-12
    assert abs(w[3] - 1.698259187621) < 1e-12
