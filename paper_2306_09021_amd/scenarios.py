"""Seeded synthetic inputs for the PBNG solver and its oracle.

This module only builds *inputs*: rest meshes, material constants in (E, nu)
form, Dirichlet targets, initial iterates, weak-constraint lists and loss
targets.  It contains none of the solver's arithmetic (no deformation
gradients, stresses, Lame conversion or colouring), so both the HIP library
and the FP64 oracle can be fed from it without sharing any method code.

Mesh convention (the paper's box examples, Tables 1 and 3, are N^3 vertex
grids; every hexahedral cell is split into 5 tetrahedra):

* vertex index = i + nx * (j + ny * k), x <- i, y <- j (up), z <- k;
* cell (i, j, k) with (i + j + k) even uses the central tet
  {000, 110, 101, 011} plus the four corner tets at 100, 010, 001, 111;
  odd cells use the mirrored split, so face diagonals of neighbouring cells
  agree and the mesh is conforming;
* every tet is stored with positive rest volume.

All random draws use ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

NEOHOOKEAN = "nh"
COROTATED = "corotated"

# corner offsets of a unit cell, bit order (dx, dy, dz)
_CORNERS = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)],
                    dtype=np.int64)  # index = dx + 2 dy + 4 dz


def _cidx(s: str) -> int:
    return int(s[0]) + 2 * int(s[1]) + 4 * int(s[2])


def _split(central: List[str], corners: List[str]) -> List[List[int]]:
    tets = [[_cidx(c) for c in central]]
    cen = [_CORNERS[_cidx(c)] for c in central]
    for corner in corners:
        p = _CORNERS[_cidx(corner)]
        # the three central vertices at cube-edge distance 1 from this corner
        nb = [_cidx(c) for c, q in zip(central, cen) if np.abs(q - p).sum() == 1]
        assert len(nb) == 3
        tets.append([_cidx(corner)] + nb)
    return tets


_EVEN = _split(["000", "110", "101", "011"], ["100", "010", "001", "111"])
_ODD = _split(["100", "010", "001", "111"], ["000", "110", "101", "011"])


def _orient(pattern: List[List[int]]) -> np.ndarray:
    out = []
    for t in pattern:
        p = _CORNERS[t].astype(np.float64)
        d = np.stack([p[1] - p[0], p[2] - p[0], p[3] - p[0]], axis=1)
        if np.linalg.det(d) < 0:
            t = [t[0], t[2], t[1], t[3]]
        out.append(t)
    return np.array(out, dtype=np.int64)


_EVEN_O = _orient(_EVEN)
_ODD_O = _orient(_ODD)


def box_mesh(nx: int, ny: int, nz: int, h=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    """Vertex grid nx*ny*nz with spacing h, every cell split into 5 tets.

    Returns (rest_pos float64 [n, 3], tets int32 [m, 4]).
    """
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # vertex index = i + nx (j + ny k): build in that order
    ii = i.transpose(2, 1, 0).reshape(-1)
    jj = j.transpose(2, 1, 0).reshape(-1)
    kk = k.transpose(2, 1, 0).reshape(-1)
    X = np.stack([origin[0] + hx * ii, origin[1] + hy * jj, origin[2] + hz * kk], axis=1)
    X = X.astype(np.float64)
    if nx < 2 or ny < 2 or nz < 2:
        return X, np.zeros((0, 4), np.int32)
    ci, cj, ck = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1),
                             indexing="ij")
    ci = ci.transpose(2, 1, 0).reshape(-1)
    cj = cj.transpose(2, 1, 0).reshape(-1)
    ck = ck.transpose(2, 1, 0).reshape(-1)
    base = ci + nx * (cj + ny * ck)
    off = _CORNERS[:, 0] + nx * (_CORNERS[:, 1] + ny * _CORNERS[:, 2])  # [8]
    parity = (ci + cj + ck) % 2
    pat = np.where(parity[:, None, None] == 0, _EVEN_O[None], _ODD_O[None])  # [c,5,4]
    tets = base[:, None, None] + off[pat]
    return X, tets.reshape(-1, 4).astype(np.int32)


@dataclass
class Scenario:
    """One problem instance, in the paper's problem-statement terms."""
    name: str
    rest_pos: np.ndarray                 # float64 [n, 3]
    tets: np.ndarray                     # int32 [m, 4]
    model: str                           # "nh" or "corotated"
    E: np.ndarray                        # float64 scalar array or [m]
    nu: np.ndarray                       # float64 scalar array or [m]
    dirichlet_idx: np.ndarray            # int32 [nd]
    dirichlet_x: np.ndarray              # float64 [nd, 3]
    x0: np.ndarray                       # float64 [n, 3] initial iterate
    density: float = 0.0
    gravity: tuple = (0.0, 0.0, 0.0)
    nodal_force: Optional[np.ndarray] = None   # float64 [n, 3] extra lumped load
    wc_ptr: np.ndarray = field(default_factory=lambda: np.zeros(1, np.int32))
    wc_vert: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    wc_w: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float64))
    wc_K: np.ndarray = field(default_factory=lambda: np.zeros((0, 6), np.float64))
    planes: np.ndarray = field(default_factory=lambda: np.zeros((0, 5), np.float64))
    solve: dict = field(default_factory=dict)
    loss_target: Optional[np.ndarray] = None   # float64 [n, 3] (differentiable config)

    @property
    def n_verts(self) -> int:
        return int(self.rest_pos.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_free(self) -> int:
        return self.n_verts - int(np.unique(self.dirichlet_idx).size)

    def initial_iterate(self) -> np.ndarray:
        x = self.x0.copy()
        x[self.dirichlet_idx] = self.dirichlet_x
        return x


def _rot_about_axis(axis, angle):
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def _layer(X, n_axis_vals, axis, value):
    return np.nonzero(np.isclose(X[:, axis], value))[0].astype(np.int32)


def twist_box(n: int = 10, model: str = COROTATED, E: float = 1e4, nu: float = 0.3,
              twist_deg: float = 90.0, stretch: float = 1.3, noise: float = 0.01,
              seed: int = 1, sweeps: int = 200) -> Scenario:
    """Unit cube of n^3 vertices: bottom face (y = 0) pinned at rest; top face
    (y = 1) stretched by `stretch` in y and twisted by `twist_deg` about the
    vertical line x = z = 0.5 (right-handed about +y).  Free vertices start
    at rest plus U[-noise*h, noise*h]^3 (seeded)."""
    h = 1.0 / (n - 1)
    X, T = box_mesh(n, n, n, h)
    bot = _layer(X, n, 1, 0.0)
    top = _layer(X, n, 1, 1.0)
    R = _rot_about_axis([0, 1, 0], math.radians(twist_deg))
    c = np.array([0.5, 0.0, 0.5])
    xt = X[top].copy()
    xt[:, 1] = 0.0
    xt = c + (xt - c) @ R.T
    xt[:, 1] = stretch * X[top, 1]
    rng = np.random.default_rng(seed)
    x0 = X + rng.uniform(-noise * h, noise * h, size=X.shape)
    didx = np.concatenate([bot, top]).astype(np.int32)
    dx = np.concatenate([X[bot], xt])
    return Scenario(name=f"twist_box_{n}", rest_pos=X, tets=T, model=model,
                    E=np.asarray(E, np.float64), nu=np.asarray(nu, np.float64),
                    dirichlet_idx=didx, dirichlet_x=dx, x0=x0,
                    solve=dict(accel="none", max_sweeps=sweeps, safeguard="backtrack",
                               real="f64", rel_tol=0.0))


def paper_box_frames(n: int, model: str = COROTATED, n_frames: int = 60, E: float = 1e5,
                     nu: float = 0.3, density: float = 10.0, twist_deg: float = 90.0,
                     stretch: float = 1.5):
    """The paper's stretching block (Sec. "Examples", "Stretching Block"):
    unit cube of n^3 vertices (n = 32, 64, 128 give the 32K/150K, 260K/1250K
    and 2097K/10242K meshes of Table 3), R0 = 10, E = 1e5, nu = 0.3, no
    gravity, both end faces (y = 0 and y = 1) clamped and moved in opposite
    directions: at frame k of n_frames each is twisted by +-k/n_frames of
    twist_deg / 2 about the vertical line x = z = 0.5 and pulled apart so the
    height is 1 + k/n_frames (stretch - 1).  Returns the scenario (targets of
    frame 1, start at rest) and the Dirichlet targets of frames 1..n_frames."""
    h = 1.0 / (n - 1)
    X, T = box_mesh(n, n, n, h)
    bot = _layer(X, n, 1, 0.0)
    top = _layer(X, n, 1, 1.0)
    didx = np.concatenate([bot, top]).astype(np.int32)
    c = np.array([0.5, 0.0, 0.5])
    frames = []
    for k in range(1, n_frames + 1):
        t = k / n_frames
        out = []
        for idx, sgn in ((bot, -1.0), (top, 1.0)):
            R = _rot_about_axis([0, 1, 0], sgn * t * math.radians(twist_deg) / 2.0)
            xt = X[idx].copy()
            xt[:, 1] = 0.0
            xt = c + (xt - c) @ R.T
            xt[:, 1] = X[idx, 1] + sgn * 0.5 * t * (stretch - 1.0)
            out.append(xt)
        frames.append(np.concatenate(out))
    sc = Scenario(name=f"paper_box_{n}", rest_pos=X, tets=T, model=model,
                  E=np.asarray(E, np.float64), nu=np.asarray(nu, np.float64),
                  dirichlet_idx=didx, dirichlet_x=frames[0], x0=X.copy(), density=density)
    return sc, frames


def two_blocks(n: int = 8, gap: float = 0.02, model: str = COROTATED, E: float = 1000.0,
               nu: float = 0.3, density: float = 10.0, drive: float = 0.1) -> Scenario:
    """The paper's two colliding blocks (Sec. "Collisions", "Two Blocks
    Colliding"): two unit cubes of n^3 vertices side by side along x with a
    gap, one instance with two connected parts, R0 = 10, E = 1000.  The outer
    face of each block is clamped; the right block's is moved by `drive`
    toward the left block.  Starts at rest."""
    h = 1.0 / (n - 1)
    X1, T1 = box_mesh(n, n, n, h)
    X2 = X1 + np.array([1.0 + gap, 0.0, 0.0])
    X = np.concatenate([X1, X2])
    T = np.concatenate([T1, T1 + X1.shape[0]]).astype(np.int32)
    left = _layer(X1, n, 0, 0.0)
    right = _layer(X2, n, 0, 2.0 + gap) + X1.shape[0]
    didx = np.concatenate([left, right]).astype(np.int32)
    dx = np.concatenate([X[left], X[right] - np.array([drive, 0.0, 0.0])])
    return Scenario(name=f"two_blocks_{n}", rest_pos=X, tets=T, model=model,
                    E=np.asarray(E, np.float64), nu=np.asarray(nu, np.float64),
                    dirichlet_idx=didx, dirichlet_x=dx, x0=X.copy(), density=density)


def icosphere(subdiv: int):
    """Unit icosphere: vertices [n, 3] on the sphere and outward-oriented
    (counter-clockwise seen from outside) triangles [m, 3]; each
    subdivision splits every triangle into four at the normalised edge
    midpoints (12 vertices and 20 faces, then 42 / 80, 162 / 320, ...)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        mid = {}

        def m(a, b):
            k = (min(a, b), max(a, b))
            if k not in mid:
                v = V[a] + V[b]
                V.append(v / np.linalg.norm(v))
                mid[k] = len(V) - 1
            return mid[k]
        F = [f for (a, b, c) in F for f in ((a, m(a, b), m(c, a)), (b, m(b, c), m(a, b)),
                                            (c, m(c, a), m(b, c)), (m(a, b), m(b, c), m(c, a)))]
    return np.array(V), np.array(F, np.int32)


def hedgehog(subdiv: int = 2, model: str = NEOHOOKEAN, E: float = 1e4, nu: float = 0.3,
             seed: int = 11, squeeze: float = 0.8, jitter: float = 0.02) -> Scenario:
    """One free vertex of high valence: vertex 0 at the centre of a unit
    icosphere, one tet per sphere triangle (20 * 4^subdiv tets, all
    incident to vertex 0).  The lower half of the sphere is prescribed,
    squeezed along y by `squeeze`; the rest starts jittered (seeded)."""
    V, F = icosphere(subdiv)
    X = np.vstack([np.zeros((1, 3)), V])
    # (centre, a, b, c) with (a, b, c) counter-clockwise seen from outside
    # has det[Xa - X0, Xb - X0, Xc - X0] > 0: positive rest volume
    tets = np.concatenate([np.zeros((F.shape[0], 1), np.int32), F + 1], axis=1).astype(np.int32)
    rng = np.random.default_rng(seed)
    low = np.nonzero(X[:, 1] < -0.2)[0].astype(np.int32)
    xd = X[low] * np.array([1.0, squeeze, 1.0])
    x0 = X + jitter * rng.uniform(-1.0, 1.0, X.shape)
    x0[low] = xd
    return Scenario(name="hedgehog_%d" % subdiv, rest_pos=X, tets=tets, model=model, E=np.asarray(E),
                    nu=np.asarray(nu), dirichlet_idx=low, dirichlet_x=xd, x0=x0)


def clique_chain(n: int = 64, seed: int = 12) -> Scenario:
    """n free vertices on a line and a Dirichlet anchor (vertex n), no tets:
    one weak constraint binds all n + 1 (weights 1 and -n, K = I), so the
    free vertices take n different colours; springs (K = 10 I, weights
    +1 / -1) join consecutive vertices and vertex 0 to the anchor; seeded
    normal nodal forces and a jittered start."""
    rng = np.random.default_rng(seed)
    X = np.zeros((n + 1, 3))
    X[:, 0] = np.arange(n + 1, dtype=float)
    w = np.ones(n + 1)
    w[n] = -float(n)
    ptr, vert, wts, K = [0, n + 1], list(range(n + 1)), list(w), [[1.0, 0, 0, 1.0, 0, 1.0]]
    for a, b in [(j, j + 1) for j in range(n - 1)] + [(0, n)]:
        vert += [a, b]
        wts += [1.0, -1.0]
        ptr.append(len(vert))
        K.append([10.0, 0, 0, 10.0, 0, 10.0])
    x0 = X + 0.1 * rng.uniform(-1.0, 1.0, X.shape)
    x0[n] = X[n]
    return Scenario(name="clique_chain_%d" % n, rest_pos=X, tets=np.zeros((0, 4), np.int32), model=NEOHOOKEAN,
                    E=np.asarray(1e4), nu=np.asarray(0.3), dirichlet_idx=np.array([n], np.int32),
                    dirichlet_x=X[n:].copy(), x0=x0, nodal_force=rng.normal(size=X.shape),
                    wc_ptr=np.array(ptr, np.int32), wc_vert=np.array(vert, np.int32),
                    wc_w=np.array(wts), wc_K=np.array(K))


def config_plain_f64() -> Scenario:
    """Plain PBNG in FP64: 10^3-vertex unit cube (3,645 tets), fixed-corotated,
    E = 1e4, nu = 0.3, bottom pinned, top stretched 1.3x and twisted 90 deg,
    interior noise 0.01 h (seed 1), 200 sweeps, no acceleration."""
    s = twist_box(10, COROTATED, 1e4, 0.3, 90.0, 1.3, 0.01, seed=1, sweeps=200)
    s.name = "plain_f64_cube10_corot"
    return s


def gravity_beam(nx: int = 128, ny: int = 32, nz: int = 32, h: float = 1.0 / 31,
                 E: float = 1e5, nu: float = 0.45, density: float = 1000.0,
                 g: float = 9.8, model: str = NEOHOOKEAN) -> Scenario:
    """Cantilever beam under gravity: face x = 0 pinned, body force (0, -g, 0)
    at the given density, starting from rest."""
    X, T = box_mesh(nx, ny, nz, h)
    pin = _layer(X, nx, 0, 0.0)
    return Scenario(name=f"beam_{nx}x{ny}x{nz}", rest_pos=X, tets=T, model=model,
                    E=np.asarray(E, np.float64), nu=np.asarray(nu, np.float64),
                    dirichlet_idx=pin, dirichlet_x=X[pin].copy(), x0=X.copy(),
                    density=density, gravity=(0.0, -g, 0.0),
                    solve=dict(accel="chebyshev", rho=0.995, gamma=1.6, max_sweeps=2000,
                               rel_tol=1e-5, safeguard="backtrack", real="f32"))


def config_beam_f32() -> Scenario:
    """Plain PBNG, FP32 sweeps: 128x32x32-vertex beam (131,072 vertices,
    610,235 tets), Neo-Hookean E = 1e5, nu = 0.45, gravity at density 1000,
    x = 0 face pinned, Chebyshev rho = 0.995 with relaxation 1.6, to 1e-5
    relative residual or 2000 sweeps."""
    s = gravity_beam()
    s.name = "beam_128x32x32_nh"
    return s


def random_cube(rng: np.random.Generator, n: int, model: str, E: float, nu: float,
                max_angle_deg: float, scale_lo: float, scale_hi: float, name: str) -> Scenario:
    """Unit cube of n^3 vertices, bottom pinned at rest, top face mapped by
    x = c_t + s R (X - c_t), c_t = (0.5, 1, 0.5), R about a uniformly random
    axis by U[0, max_angle], s ~ U[scale_lo, scale_hi].  Starts at rest."""
    X, T = box_mesh(n, n, n, 1.0 / (n - 1))
    bot = _layer(X, n, 1, 0.0)
    top = _layer(X, n, 1, 1.0)
    axis = rng.normal(size=3)
    angle = math.radians(rng.uniform(0.0, max_angle_deg))
    s = rng.uniform(scale_lo, scale_hi)
    R = _rot_about_axis(axis, angle)
    ct = np.array([0.5, 1.0, 0.5])
    xt = ct + s * (X[top] - ct) @ R.T
    didx = np.concatenate([bot, top]).astype(np.int32)
    dx = np.concatenate([X[bot], xt])
    return Scenario(name=name, rest_pos=X, tets=T, model=model,
                    E=np.asarray(E, np.float64), nu=np.asarray(nu, np.float64),
                    dirichlet_idx=didx, dirichlet_x=dx, x0=X.copy())


def config_batched(n_instances: int = 256, seed: int = 4, n_lo: int = 4, n_hi: int = 32):
    """Batched FP32: cubes with n ~ U{n_lo..n_hi} vertices per side,
    fixed-corotated, E log-uniform [1e3, 1e5], nu ~ U[0.3, 0.48], top face
    rotated by up to 60 deg about a random axis and scaled by U[0.7, 1.4]."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n_instances):
        n = int(rng.integers(n_lo, n_hi + 1))
        E = float(10.0 ** rng.uniform(3.0, 5.0))
        nu = float(rng.uniform(0.3, 0.48))
        sc = random_cube(rng, n, COROTATED, E, nu, 60.0, 0.7, 1.4, f"batched_{q}_n{n}")
        sc.solve = dict(accel="chebyshev", rho=0.95, gamma=1.7, max_sweeps=20000,
                        rel_tol=1e-5, safeguard="backtrack", real="f32")
        out.append(sc)
    return out


def config_differentiable(n_instances: int = 64, seed: int = 5, n: int = 32):
    """Differentiable FP32: cubes of n^3 vertices, Neo-Hookean with per-tet
    (E, nu) = (1e4, 0.3), top face rotated by up to 15 deg and scaled by
    U[0.9, 1.1].  Each instance carries a loss target T_i = X_i + u(X_i),
    u(X) = sum_k 0.05 d_k sin(2 pi w_k . X + phi_k), d_k unit, w_k ~ U[-2, 2]^3,
    phi_k ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n_instances):
        sc = random_cube(rng, n, NEOHOOKEAN, 1e4, 0.3, 15.0, 0.9, 1.1, f"diff_{q}_n{n}")
        sc.E = np.full(sc.n_tets, 1e4)
        sc.nu = np.full(sc.n_tets, 0.3)
        u = np.zeros_like(sc.rest_pos)
        for _ in range(3):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            w = rng.uniform(-2.0, 2.0, size=3)
            phi = rng.uniform(0.0, 2 * math.pi)
            u += 0.05 * np.outer(np.sin(2 * math.pi * sc.rest_pos @ w + phi), d)
        sc.loss_target = sc.rest_pos + u
        sc.solve = dict(accel="chebyshev", rho=0.95, gamma=1.7, max_sweeps=20000,
                        rel_tol=1e-6, safeguard="backtrack", real="f32")
        out.append(sc)
    return out


def surface_vertices(tets: np.ndarray) -> np.ndarray:
    """Vertices on faces that belong to exactly one tet."""
    f = np.concatenate([tets[:, [0, 1, 2]], tets[:, [0, 1, 3]],
                        tets[:, [0, 2, 3]], tets[:, [1, 2, 3]]])
    f = np.sort(f, axis=1)
    uniq, cnt = np.unique(f, axis=0, return_counts=True)
    return np.unique(uniq[cnt == 1].reshape(-1)).astype(np.int32)


def ellipsoid_mesh(center, semi, n_target: int):
    """Lattice of spacing h = (4/3 pi abc / n_target)^(1/3); keep hex cells
    whose 8 corners lie inside the ellipsoid; 5-tet split; drop unused
    vertices."""
    a, b, c = semi
    h = (4.0 / 3.0 * math.pi * a * b * c / n_target) ** (1.0 / 3.0)
    n = [int(math.floor(2 * s / h)) + 2 for s in semi]
    origin = np.asarray(center) - np.array([(n[0] - 1) * h, (n[1] - 1) * h, (n[2] - 1) * h]) / 2
    X, T = box_mesh(n[0], n[1], n[2], h, origin)
    inside = (((X - center) / np.asarray(semi)) ** 2).sum(1) <= 1.0
    # a cell survives if all 8 corners are inside; its 5 tets are consecutive
    keep = inside[T].all(1).reshape(-1, 5).all(1)
    T = T.reshape(-1, 5, 4)[keep].reshape(-1, 4)
    used = np.unique(T)
    remap = -np.ones(X.shape[0], np.int64)
    remap[used] = np.arange(used.size)
    return X[used], remap[T].astype(np.int32)


def config_muscles(seed: int = 3, n_meshes: int = 8, n_target: int = 40000,
                   bind_frac: float = 0.05, bind_dist: float = 0.02) -> Scenario:
    """Muscle-like FP32 stand-in: 8 ellipsoidal tet meshes in a row along x
    (semi-axes U[0.5, 2]^3 sorted so z is the longest, neighbours overlapping
    by 0.05), per-tet E log-uniform [1e3, 1e5], nu = 0.45, Neo-Hookean;
    isotropic zero-rest-length binding springs (k = 1e4) on a seeded 5% of
    cross-mesh surface-vertex pairs closer than 0.02; a ground plane with
    contact stiffness 1e5 at min_y + 0.05; both z end caps (|z - c_z| >= 0.9 c)
    translated by seeded vectors of length U[0, 0.2]; Chebyshev rho = 0.95,
    relaxation 1.7, 1000 sweeps."""
    rng = np.random.default_rng(seed)
    Xs, Ts, Es, dids, dxs = [], [], [], [], []
    surf = []
    base = 0
    cx_prev, a_prev = None, None
    for k in range(n_meshes):
        semi = np.sort(rng.uniform(0.5, 2.0, size=3))  # z longest
        a = semi[0]
        cx = 0.0 if cx_prev is None else cx_prev + a_prev + a - 0.05
        center = np.array([cx, 0.0, 0.0])
        X, T = ellipsoid_mesh(center, semi, n_target)
        E = 10.0 ** rng.uniform(3.0, 5.0, size=T.shape[0])
        cz = semi[2]
        cap = np.abs(X[:, 2] - center[2]) >= 0.9 * cz
        capidx = np.nonzero(cap)[0]
        lo = capidx[X[capidx, 2] < center[2]]
        hi = capidx[X[capidx, 2] >= center[2]]
        dx = X.copy()
        for part in (lo, hi):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            dx[part] += rng.uniform(0.0, 0.2) * d
        Xs.append(X)
        Ts.append(T + base)
        Es.append(E)
        dids.append(capidx + base)
        dxs.append(dx[capidx])
        surf.append(surface_vertices(T) + base)
        base += X.shape[0]
        cx_prev, a_prev = cx, a
    X = np.concatenate(Xs)
    T = np.concatenate(Ts).astype(np.int32)
    E = np.concatenate(Es)
    didx = np.concatenate(dids).astype(np.int32)
    dxx = np.concatenate(dxs)
    # binding springs between surface vertices of different meshes
    mesh_of = np.concatenate([np.full(x.shape[0], q) for q, x in enumerate(Xs)])
    pairs = []
    for q in range(n_meshes - 1):
        A = surf[q]
        B = surf[q + 1]
        # cell hashing on the bounding box overlap
        XA, XB = X[A], X[B]
        cell = bind_dist
        keyB = np.floor(XB / cell).astype(np.int64)
        table = {}
        for idx, kk in enumerate(map(tuple, keyB)):
            table.setdefault(kk, []).append(idx)
        for ia, pa in enumerate(XA):
            ka = np.floor(pa / cell).astype(np.int64)
            for dxo in (-1, 0, 1):
                for dyo in (-1, 0, 1):
                    for dzo in (-1, 0, 1):
                        for ib in table.get((ka[0] + dxo, ka[1] + dyo, ka[2] + dzo), ()):
                            if np.linalg.norm(XB[ib] - pa) <= bind_dist:
                                pairs.append((A[ia], B[ib]))
    pairs = np.array(sorted(set(pairs)), dtype=np.int64).reshape(-1, 2)
    dset = set(didx.tolist())
    pairs = np.array([p for p in pairs if p[0] not in dset and p[1] not in dset],
                     dtype=np.int64).reshape(-1, 2)
    keep = rng.random(pairs.shape[0]) < bind_frac
    pairs = pairs[keep]
    nwc = pairs.shape[0]
    wc_ptr = (2 * np.arange(nwc + 1)).astype(np.int32)
    wc_vert = pairs.reshape(-1).astype(np.int32)
    wc_w = np.tile([1.0, -1.0], nwc).astype(np.float64)
    kb = 1e4
    wc_K = np.tile([kb, 0.0, 0.0, kb, 0.0, kb], (nwc, 1)).astype(np.float64)
    ymin = X[:, 1].min()
    planes = np.array([[0.0, 1.0, 0.0, ymin + 0.05, 1e5]])
    del mesh_of
    return Scenario(name="muscles_8_ellipsoids", rest_pos=X, tets=T, model=NEOHOOKEAN,
                    E=E, nu=np.full(T.shape[0], 0.45), dirichlet_idx=didx, dirichlet_x=dxx,
                    x0=X.copy(), wc_ptr=wc_ptr, wc_vert=wc_vert, wc_w=wc_w, wc_K=wc_K,
                    planes=planes,
                    solve=dict(accel="chebyshev", rho=0.95, gamma=1.7, max_sweeps=1000,
                               rel_tol=0.0, safeguard="backtrack", real="f32"))


# ----------------------------------------------------------------------------
# planar (d = 2) triangle meshes
# ----------------------------------------------------------------------------
def square_mesh(nx: int, ny: int, h=1.0, diagonal: str = "uniform"):
    """Vertex grid nx*ny (index i + nx j, x <- i, y <- j) with spacing h,
    every square cell split into two counter-clockwise triangles: along the
    (0,0)-(1,1) diagonal everywhere ("uniform", six triangles at an interior
    vertex) or alternating with the other diagonal in a checkerboard
    ("alternate").  Returns (rest_pos float64 [n, 2], tris int32 [m, 3])."""
    hx, hy = (h, h) if np.isscalar(h) else h
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([i.reshape(-1) * hx, j.reshape(-1) * hy], axis=1).astype(np.float64)
    ci, cj = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    ci, cj = ci.reshape(-1), cj.reshape(-1)
    v00 = ci + nx * cj
    v10, v01, v11 = v00 + 1, v00 + nx, v00 + nx + 1
    main = np.stack([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)], 1)
    if diagonal == "uniform":
        T = main
    elif diagonal == "alternate":
        other = np.stack([np.stack([v00, v10, v01], 1), np.stack([v10, v11, v01], 1)], 1)
        T = np.where(((ci + cj) % 2 == 0)[:, None, None], main, other)
    else:
        raise ValueError(diagonal)
    return X, T.reshape(-1, 3).astype(np.int32)


@dataclass
class Scenario2D:
    """One planar problem (inputs only); positions are [n, 2]."""
    name: str
    rest_pos: np.ndarray                       # float64 [n, 2]
    tris: np.ndarray                           # int32 [m, 3], counter-clockwise
    model: str                                 # "nh" | "corotated"
    E: np.ndarray                              # scalar or [m]
    nu: np.ndarray                             # scalar or [m]
    dirichlet_idx: np.ndarray                  # int32 [nd]
    dirichlet_x: np.ndarray                    # float64 [nd, 2]
    x0: np.ndarray                             # float64 [n, 2] initial iterate
    density: float = 0.0
    gravity: tuple = (0.0, 0.0)
    nodal_force: Optional[np.ndarray] = None   # float64 [n, 2]
    wc_ptr: np.ndarray = field(default_factory=lambda: np.zeros(1, np.int32))
    wc_vert: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    wc_w: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float64))
    wc_K: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.float64))   # (xx, xy, yy)
    planes: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), np.float64))  # (nx, ny, d, k)

    @property
    def n_verts(self) -> int:
        return self.rest_pos.shape[0]

    @property
    def n_tris(self) -> int:
        return self.tris.shape[0]

    def initial_iterate(self) -> np.ndarray:
        x = np.array(self.x0, dtype=np.float64, copy=True)
        x[self.dirichlet_idx] = self.dirichlet_x
        return x


def stretched_square(n: int, model: str = NEOHOOKEAN, stretch: float = 1.5, E: float = 1e4,
                     nu: float = 0.3, diagonal: str = "uniform", density: float = 0.0,
                     gravity=(0.0, 0.0), noise: float = 0.0, seed: int = 0) -> Scenario2D:
    """The planar experiment of Sec. "PBNG vs. PBD and Limited Newton": a
    unit square block (n x n vertices) whose left and right sides are pulled
    apart to a total width `stretch` and clamped there (Dirichlet), while the
    interior starts at its rest position (optionally jittered by `noise`
    times the spacing, seeded), so the deformation has to propagate inward.
    The figure shows large, medium and small stretches; the paper gives no
    sizes or material values, so n, stretch, E and nu are free."""
    X, T = square_mesh(n, n, 1.0 / (n - 1), diagonal)
    col = np.arange(n * n) % n
    left, right = np.nonzero(col == 0)[0], np.nonzero(col == n - 1)[0]
    idx = np.concatenate([left, right]).astype(np.int32)
    xd = X[idx].copy()
    half = 0.5 * (stretch - 1.0)
    xd[: left.size, 0] -= half
    xd[left.size:, 0] += half
    x0 = X.copy()
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        x0 += noise / (n - 1) * rng.uniform(-1.0, 1.0, size=x0.shape)
    return Scenario2D(name="stretched_square_%d_%s" % (n, model), rest_pos=X, tris=T, model=model,
                      E=np.asarray(E, np.float64), nu=np.asarray(nu, np.float64), dirichlet_idx=idx,
                      dirichlet_x=xd, x0=x0, density=density, gravity=tuple(gravity))


def planar_terms(n: int = 17, model: str = NEOHOOKEAN, seed: int = 21, k_ground: float = 1e6,
                 n_springs: int = 12) -> Scenario2D:
    """A planar problem with every extra term: an n x n-vertex unit block
    (E = 1e4, nu = 0.3, R0 = 100, gravity -9.8 * 40 along y) hanging from
    its top row, seeded weak constraints (two-vertex springs K = 1e3 I
    between random free vertices, plus three-vertex constraints with random
    weights and a coupled K), and a ground half-plane y >= -0.02 (n = +y,
    k = k_ground) that the bottom row, started 0.01 above it and jittered,
    is pressed into."""
    rng = np.random.default_rng(seed)
    X, T = square_mesh(n, n, 1.0 / (n - 1))
    top = np.nonzero(X[:, 1] > 1.0 - 1e-12)[0].astype(np.int32)
    free = np.setdiff1d(np.arange(n * n), top)
    ptr, vert, w, K = [0], [], [], []
    for _ in range(n_springs):
        a, b = rng.choice(free, 2, replace=False)
        vert += [int(a), int(b)]
        w += [1.0, -1.0]
        ptr.append(len(vert))
        K.append([1e3, 0.0, 1e3])
    for _ in range(n_springs // 3):
        m = rng.choice(free, 3, replace=False)
        vert += [int(v) for v in m]
        w += list(rng.uniform(-1.0, 1.0, 3))
        ptr.append(len(vert))
        K.append([800.0, 150.0, 500.0])
    x0 = X.copy()
    x0[:, 1] -= 0.03 * (1.0 - X[:, 1])           # sag toward the ground: bottom row at -0.03 + 0.01
    x0[:, 1] += 0.01
    x0 += 0.002 * rng.uniform(-1.0, 1.0, x0.shape)
    x0[top] = X[top]
    return Scenario2D(name="planar_terms_%d_%s" % (n, model), rest_pos=X, tris=T, model=model,
                      E=np.asarray(1e4), nu=np.asarray(0.3), dirichlet_idx=top, dirichlet_x=X[top].copy(),
                      x0=x0, density=100.0, gravity=(0.0, -9.8 * 40.0), wc_ptr=np.array(ptr, np.int32),
                      wc_vert=np.array(vert, np.int32), wc_w=np.array(w), wc_K=np.array(K),
                      planes=np.array([[0.0, 1.0, -0.02, k_ground]]))
