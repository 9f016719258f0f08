"""Pins of the planar (d = 2) oracle's weak constraints (Sec. "Weak
Constraints"), contact half-planes and backward-Euler inertia (Eq. fem_be
as the incremental potential), against facts that do not come from it:

* the embedding into the pinned 3-D oracle, an independent code: a planar
  problem made only of these terms and nodal loads is a 3-D problem whose
  z components are decoupled (K_c block diagonal with K_zz > 0, normals
  with n_z = 0, no load along z), so the same sweeps give the same x, y;
* closed forms: one vertex on a spring to an anchor rests at a + K^{-1} f,
  one vertex pressed into a half-plane at depth f / k, one vertex with only
  inertia and a load at xhat + f / minert (each reached by one local step,
  whose energy is then exactly quadratic);
* the lumped masses add up to R0 times the total area, and a free-falling
  unconstrained vertex advances by one backward-Euler step
  x^{n+1} = 2 x^n - x^{n-1} + dt^2 g;
* the residual as minus the central-difference gradient of the total energy
  with every term present, and an independent greedy colouring that counts
  the constraints' colour sets."""
import numpy as np
import pytest

import oracle as O
from oracle import planar as P
from paper_2306_09021_amd import scenarios as S

RNG = np.random.default_rng(91)


def _tri_free(n_pts):
    """n_pts free points scattered in [-1, 1]^2 plus, far away, one pinned
    triangle (the planar problem needs no triangle at the free points)."""
    X = np.zeros((n_pts + 3, 2))
    X[:n_pts] = RNG.uniform(-1.0, 1.0, size=(n_pts, 2))
    X[n_pts:] = [[10.0, 10.0], [11.0, 10.0], [10.0, 11.0]]
    tris = np.array([[n_pts, n_pts + 1, n_pts + 2]], np.int32)
    didx = np.arange(n_pts, n_pts + 3, dtype=np.int32)
    return X, tris, didx


def _scen2(X, tris, didx, x0, **kw):
    return S.Scenario2D(name="terms", rest_pos=X, tris=tris, model="nh", E=np.asarray(1e3),
                        nu=np.asarray(0.3), dirichlet_idx=didx, dirichlet_x=X[didx].copy(), x0=x0, **kw)


def _embed(sc2, K3zz=7.0):
    """The 3-D scenario of a planar one without elastic elements at its free
    vertices: z = 0 everywhere, K_c gains a decoupled K_zz, planes n_z = 0."""
    n = sc2.n_verts
    X3 = np.zeros((n, 3))
    X3[:, :2] = sc2.rest_pos
    x3 = np.zeros((n, 3))
    x3[:, :2] = sc2.x0
    K2 = np.asarray(sc2.wc_K).reshape(-1, 3)
    K3 = np.zeros((K2.shape[0], 6))
    K3[:, 0], K3[:, 1], K3[:, 3], K3[:, 5] = K2[:, 0], K2[:, 1], K2[:, 2], K3zz
    pl2 = np.asarray(sc2.planes).reshape(-1, 4)
    pl3 = np.zeros((pl2.shape[0], 5))
    pl3[:, 0], pl3[:, 1], pl3[:, 3], pl3[:, 4] = pl2[:, 0], pl2[:, 1], pl2[:, 2], pl2[:, 3]
    f3 = None
    if sc2.nodal_force is not None:
        f3 = np.zeros((n, 3))
        f3[:, :2] = sc2.nodal_force
    xd = np.zeros((sc2.dirichlet_idx.size, 3))
    xd[:, :2] = sc2.dirichlet_x
    return S.Scenario(name="terms3", rest_pos=X3, tets=np.zeros((0, 4), np.int32), model="nh",
                      E=np.asarray(1e3), nu=np.asarray(0.3), dirichlet_idx=sc2.dirichlet_idx,
                      dirichlet_x=xd, x0=x3, nodal_force=f3, wc_ptr=sc2.wc_ptr, wc_vert=sc2.wc_vert,
                      wc_w=sc2.wc_w, wc_K=K3, planes=pl3)


def _random_terms(n_pts=12, n_wc=10, with_planes=True, seed=0):
    rng = np.random.default_rng(seed)
    X, tris, didx = _tri_free(n_pts)
    n = X.shape[0]
    ptr, vert, w, K = [0], [], [], []
    for _ in range(n_wc):
        m = int(rng.integers(2, 4))
        vs = rng.choice(n_pts + 1, size=m, replace=False)       # may include a pinned vertex
        vs = np.where(vs == n_pts, n_pts + 1, vs)
        vert += list(vs)
        w += list(rng.uniform(-1.0, 1.0, size=m))
        ptr.append(len(vert))
        a, b = rng.uniform(5.0, 20.0, 2)
        c = rng.uniform(-0.4, 0.4) * np.sqrt(a * b)
        K.append([a, c, b])
    # a soft spring from every free vertex to a pinned one: in the 3-D
    # embedding each free vertex then has stiffness along z (its K_zz)
    for v in range(n_pts):
        vert += [v, n_pts]
        w += [1.0, -1.0]
        ptr.append(len(vert))
        K.append([0.5, 0.0, 0.5])
    planes = np.zeros((0, 4))
    if with_planes:
        t = rng.uniform(0, 2 * np.pi, 2)
        planes = np.array([[np.cos(t[0]), np.sin(t[0]), -0.3, 40.0], [np.cos(t[1]), np.sin(t[1]), -0.5, 25.0]])
    x0 = X + 0.2 * rng.normal(size=X.shape)
    x0[didx] = X[didx]
    f = rng.normal(size=(n, 2))
    return _scen2(X, tris, didx, x0, nodal_force=f, wc_ptr=np.array(ptr, np.int32),
                  wc_vert=np.array(vert, np.int32), wc_w=np.array(w), wc_K=np.array(K), planes=planes)


@pytest.mark.parametrize("with_planes", [False, True])
@pytest.mark.parametrize("inertia", [False, True])
def test_embedding_into_the_3d_oracle(with_planes, inertia):
    sc2 = _random_terms(with_planes=with_planes, seed=3 + 2 * with_planes + inertia)
    sc3 = _embed(sc2)
    op2, op3 = P.make_problem(sc2), O.make_problem(sc3)
    if inertia:
        dt = 0.05
        xn2 = sc2.initial_iterate() + 0.01 * RNG.normal(size=(sc2.n_verts, 2))
        xp2 = sc2.initial_iterate()
        m = np.zeros(sc2.n_verts)
        m[: sc2.n_verts - 3] = RNG.uniform(0.5, 2.0, sc2.n_verts - 3)
        op2.mass = m.copy()
        op3.mass = m.copy()
        op2.set_inertia(dt, xn2, xp2)
        xn3, xp3 = np.zeros((sc2.n_verts, 3)), np.zeros((sc2.n_verts, 3))
        xn3[:, :2], xp3[:, :2] = xn2, xp2
        op3.set_inertia(dt, xn3, xp3)
    c2, n2 = P.color(op2)
    c3, n3 = O.color(op3)
    assert n2 == n3 and np.array_equal(c2, c3)
    x2, st2 = P.solve(op2, c2, sc2.initial_iterate(), max_sweeps=25, safeguard="backtrack")
    x3, st3 = O.solve(op3, c3, sc3.initial_iterate(), max_sweeps=25, safeguard="backtrack")
    assert np.abs(x3[:, 2]).max() == 0.0
    assert np.abs(x2 - x3[:, :2]).max() <= 1e-12 * max(1.0, np.abs(x3).max())
    r2, e2, _ = P.residual(op2, x2)
    r3, e3, _ = O.residual(op3, x3)
    assert abs(r2 - r3) <= 1e-10 * max(1.0, r3)
    # energies up to the constant of the pinned triangle (absent in 3-D)
    e20 = P.residual(op2, sc2.initial_iterate())[1]
    e30 = O.residual(op3, sc3.initial_iterate())[1]
    assert abs((e2 - e20) - (e3 - e30)) <= 1e-10 * max(1.0, abs(e30))


def test_spring_to_anchor_closed_form():
    X, tris, didx = _tri_free(1)
    a = X[didx[0]]
    K = np.array([[30.0, 4.0], [4.0, 12.0]])
    f = np.array([1.5, -2.25])
    forces = np.zeros_like(X)
    forces[0] = f
    x0 = X.copy()
    x0[0] = [3.0, -7.0]
    sc = _scen2(X, tris, didx, x0, nodal_force=forces, wc_ptr=np.array([0, 2], np.int32),
                wc_vert=np.array([0, didx[0]], np.int32), wc_w=np.array([1.0, -1.0]),
                wc_K=np.array([[K[0, 0], K[0, 1], K[1, 1]]]))
    op = P.make_problem(sc)
    c, _ = P.color(op)
    x, st = P.solve(op, c, sc.initial_iterate(), max_sweeps=1, safeguard="backtrack")
    assert np.allclose(x[0], a + np.linalg.solve(K, f), rtol=0, atol=1e-13)
    assert P.residual(op, x)[0] <= 1e-12


def test_half_plane_rest_depth_closed_form():
    """A vertex pushed into a half-plane (normal n) and held along the
    tangent t by a spring kappa t t^T to an anchor a: it rests at depth
    phi = -g / k with t . y = t . a (one local step: the energy is quadratic
    once phi < 0)."""
    X, tris, didx = _tri_free(1)
    k, g, kappa = 250.0, 3.0, 40.0
    nrm, tang = np.array([0.6, 0.8]), np.array([-0.8, 0.6])
    d = 0.4
    a = X[didx[0]]
    forces = np.zeros_like(X)
    forces[0] = -g * nrm                          # pushes into the half-plane
    x0 = X.copy()
    x0[0] = d * nrm + 1.7 * tang - 0.05 * nrm     # already inside (phi < 0)
    Kt = kappa * np.outer(tang, tang)
    sc = _scen2(X, tris, didx, x0, nodal_force=forces, planes=np.array([[nrm[0], nrm[1], d, k]]),
                wc_ptr=np.array([0, 2], np.int32), wc_vert=np.array([0, didx[0]], np.int32),
                wc_w=np.array([1.0, -1.0]), wc_K=np.array([[Kt[0, 0], Kt[0, 1], Kt[1, 1]]]))
    op = P.make_problem(sc)
    c, _ = P.color(op)
    x, st = P.solve(op, c, sc.initial_iterate(), max_sweeps=1, safeguard="backtrack")
    assert st["rejected"] == 0
    assert abs((nrm @ x[0] - d) - (-g / k)) <= 1e-14
    assert abs(tang @ x[0] - tang @ a) <= 1e-13


def test_inertia_only_closed_form_and_free_fall():
    X, tris, didx = _tri_free(1)
    f = np.array([0.7, -9.8])
    forces = np.zeros_like(X)
    forces[0] = f
    sc = _scen2(X, tris, didx, X.copy(), nodal_force=forces)
    op = P.make_problem(sc)
    m = np.zeros(X.shape[0])
    m[0] = 2.5
    op.mass = m
    dt = 0.02
    xn, xp = X.copy(), X.copy()
    xn[0] += [0.01, 0.03]
    op.set_inertia(dt, xn, xp)
    c, _ = P.color(op)
    x, _ = P.solve(op, c, xn, max_sweeps=1, safeguard="backtrack")
    xhat = 2 * xn[0] - xp[0]
    assert np.allclose(x[0], xhat + f / (m[0] / dt ** 2), rtol=0, atol=1e-14)
    # the same with the load as gravity on a massive vertex: one backward-Euler step
    grav = np.array([0.0, -9.81])
    forces[0] = m[0] * grav
    op.fext = np.ascontiguousarray(forces)
    x, _ = P.solve(op, c, xn, max_sweeps=1, safeguard="backtrack")
    assert np.allclose(x[0], 2 * xn[0] - xp[0] + dt ** 2 * grav, rtol=0, atol=1e-14)


def test_lumped_masses_add_up_to_the_total_mass():
    sc = S.stretched_square(9, "nh", 1.2, density=3.5)
    X, T = sc.rest_pos, sc.tris
    e1, e2 = X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]).sum()
    op = P.make_problem(sc)
    assert abs(op.mass.sum() - 3.5 * area) <= 1e-13
    assert abs(area - 1.0) <= 1e-13
    # interior vertex of the uniform mesh: six triangles of area h^2 / 2
    h = 1.0 / 8
    assert abs(op.mass[4 + 9 * 4] - 3.5 * 6 * (0.5 * h * h) / 3) <= 1e-15


@pytest.mark.parametrize("model", ["nh", "corotated"])
def test_residual_is_minus_energy_gradient_with_every_term(model):
    sc = S.stretched_square(5, model, 1.3, noise=0.3, seed=4)
    n = sc.n_verts
    rng = np.random.default_rng(8)
    ptr, vert, w, K = [0], [], [], []
    for _ in range(6):
        vs = rng.choice(n, size=3, replace=False)
        vert += list(vs)
        w += list(rng.uniform(-1, 1, 3))
        ptr.append(len(vert))
        K.append([50.0, 10.0, 30.0])
    sc.wc_ptr, sc.wc_vert, sc.wc_w, sc.wc_K = (np.array(ptr, np.int32), np.array(vert, np.int32),
                                              np.array(w), np.array(K))
    sc.planes = np.array([[0.0, 1.0, 0.3, 500.0], [-1.0, 0.0, -0.9, 300.0]])
    sc.density = 2.0
    op = P.make_problem(sc)
    x = sc.initial_iterate() + 0.05 * rng.normal(size=(n, 2))
    x[sc.dirichlet_idx] = sc.dirichlet_x
    op.set_inertia(0.1, x + 0.01, x - 0.02)
    _, _, r = P.residual(op, x)
    assert (np.array([[0, 1] @ xi - 0.3 for xi in x]) < 0).any()      # a plane is active
    h = 1e-6
    free = np.setdiff1d(np.arange(n), sc.dirichlet_idx)
    for i in free[:10]:
        for a in range(2):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (P.residual(op, xp)[1] - P.residual(op, xm)[1]) / (2 * h)
            assert abs(r[i, a] + g) <= 1e-6 * max(1.0, abs(g))


def test_colouring_counts_the_constraints():
    sc = _random_terms(n_pts=20, n_wc=15, seed=5)
    op = P.make_problem(sc)
    c, ncol = P.color(op)
    # independent greedy: ascending index, least colour not used by an
    # already coloured vertex sharing a triangle or a constraint
    n = sc.n_verts
    nb = [set() for _ in range(n)]
    for t in sc.tris:
        for a in t:
            nb[a].update(int(b) for b in t if b != a)
    for k in range(sc.wc_ptr.size - 1):
        m = sc.wc_vert[sc.wc_ptr[k]:sc.wc_ptr[k + 1]]
        for a in m:
            nb[a].update(int(b) for b in m if b != a)
    ref = -np.ones(n, np.int64)
    dset = set(sc.dirichlet_idx.tolist())
    for i in range(n):
        if i in dset:
            continue
        used = {ref[j] for j in nb[i] if ref[j] >= 0}
        col = 0
        while col in used:
            col += 1
        ref[i] = col
    assert np.array_equal(c, ref) and ncol == ref.max() + 1
