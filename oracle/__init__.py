"""FP64 oracle for Position-Based Nonlinear Gauss-Seidel (arXiv 2306.09021).

TEST INFRASTRUCTURE ONLY.  Only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of bench.py may import this package.  It shares no code
with the HIP library (``paper_2306_09021_amd``) and never imports it; both are
fed from the seeded input generators in ``paper_2306_09021_amd.scenarios``,
which hold no solver arithmetic.

The numerical core is plain serial C in ``pbng_oracle.c`` (built with gcc into
``liboracle.so``); this module marshals numpy arrays into it.  ``dense.py``
adds dense-matrix tools for tiny meshes (Newton, adjoint by direct solve).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pbng_oracle.c")
_SRCS = (_SRC, os.path.join(_HERE, "pbng_oracle2d.c"))
_LIB = os.path.join(_HERE, "liboracle.so")

NEOHOOKEAN, COROTATED, STABLE_NEOHOOKEAN = 0, 1, 2
MODEL = {"nh": NEOHOOKEAN, "corotated": COROTATED, "snh": STABLE_NEOHOOKEAN}
ACCEL = {"none": 0, "chebyshev": 1, "sor": 2}
SAFEGUARD = {"none": 0, "backtrack": 1}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint8)


class _Problem(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nt", C.c_int32), ("model", C.c_int32),
                ("X", _dp), ("tets", _ip), ("mu", _dp), ("lam", _dp), ("fext", _dp),
                ("is_dir", _up), ("n_wc", C.c_int32), ("wc_ptr", _ip), ("wc_vert", _ip),
                ("wc_w", _dp), ("wc_K", _dp), ("n_planes", C.c_int32), ("planes", _dp),
                ("minert", _dp), ("xhat", _dp)]


class _Opts(C.Structure):
    _fields_ = [("max_sweeps", C.c_int32), ("check_every", C.c_int32), ("rel_tol", C.c_double),
                ("accel", C.c_int32), ("rho", C.c_double), ("gamma", C.c_double),
                ("omega", C.c_double), ("safeguard", C.c_int32), ("max_halvings", C.c_int32),
                ("skip_tol", C.c_double), ("emulate_f32", C.c_int32), ("n_threads", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("converged", C.c_int32), ("rejected", C.c_int64),
                ("halvings", C.c_int64), ("res0", C.c_double), ("res", C.c_double),
                ("rel", C.c_double), ("energy", C.c_double)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (IEEE double, no fast-math, no FMA)."""
    if (force or not os.path.exists(_LIB)
            or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS)):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.or_lame.argtypes = [C.c_double, C.c_double, _dp, _dp]
        L.or_psi.argtypes = [C.c_int, C.c_double, C.c_double, _dp]
        L.or_psi.restype = C.c_double
        L.or_pk1.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp]
        L.or_nh_dpk1.argtypes = [C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_dpk1.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_mod_hess_density.argtypes = [C.c_double, C.c_double, _dp, _dp]
        L.or_svd3.argtypes = [_dp, _dp, _dp, _dp]
        L.or_prep.argtypes = [C.c_int32, C.c_int32, _dp, _ip, _dp, _dp]
        L.or_prep.restype = C.c_int
        L.or_body_force.argtypes = [C.c_int32, C.c_int32, _ip, _dp, C.c_double, _dp, _dp]
        L.or_lumped_mass.argtypes = [C.c_int32, C.c_int32, _ip, _dp, C.c_double, _dp]
        L.or_color.argtypes = [C.POINTER(_Problem), _ip]
        L.or_color.restype = C.c_int32
        L.or_recolor.argtypes = [C.POINTER(_Problem), C.c_int32, _ip, _ip]
        L.or_recolor.restype = C.c_int32
        L.or_residual.argtypes = [C.POINTER(_Problem), _dp, _dp, _dp]
        L.or_residual.restype = C.c_double
        L.or_chebyshev_weights.argtypes = [C.c_double, C.c_int32, _dp]
        L.or_solve.argtypes = [C.POINTER(_Problem), _ip, _dp, C.POINTER(_Opts),
                               C.POINTER(_Stats), _dp]
        L.or_solve.restype = C.c_int32
        L.or_sweep_energy_trace.argtypes = [C.POINTER(_Problem), _ip, _dp, C.POINTER(_Opts), _dp]
        L.or_sweep_energy_trace.restype = C.c_int32
        L.or_update_vertices.argtypes = [C.POINTER(_Problem), _dp, C.c_int32, _ip,
                                         C.POINTER(_Opts), _dp]
        L.or_update_vertices.restype = C.c_int32
        L.or_hvp.argtypes = [C.POINTER(_Problem), _dp, _dp, _dp]
        L.or_hvp.restype = C.c_int32
        L.or_adjoint_gradients.argtypes = [C.POINTER(_Problem), _dp, _dp, _dp, _dp, _dp]
        L.or_adjoint_gradients.restype = C.c_int32
        L.or_energy_gradient.argtypes = [C.POINTER(_Problem), _dp, _dp]
        L.or_energy_gradient.restype = C.c_int32
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


# ----------------------------------------------------------------------------
# scalar constitutive functions
# ----------------------------------------------------------------------------
def lame(E, nu):
    """Eq. (lame): mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu))."""
    E = np.asarray(E, np.float64)
    nu = np.asarray(nu, np.float64)
    Eb, nb = np.broadcast_arrays(E, nu)
    mu = np.empty(Eb.shape)
    la = np.empty(Eb.shape)
    L = lib()
    m = C.c_double()
    l_ = C.c_double()
    for idx in np.ndindex(Eb.shape):
        L.or_lame(float(Eb[idx]), float(nb[idx]), C.byref(m), C.byref(l_))
        mu[idx] = m.value
        la[idx] = l_.value
    return mu, la


def psi(model, mu, lam, F):
    F = _f64(F, (3, 3))
    return lib().or_psi(model, mu, lam, _d(F))


def pk1(model, mu, lam, F):
    F = _f64(F, (3, 3))
    P = np.zeros((3, 3))
    lib().or_pk1(model, mu, lam, _d(F), _d(P))
    return P


def nh_dpk1(mu, lam, F, dF):
    F = _f64(F, (3, 3))
    dF = _f64(dF, (3, 3))
    out = np.zeros((3, 3))
    lib().or_nh_dpk1(mu, lam, _d(F), _d(dF), _d(out))
    return out


def dpk1(model, mu, lam, F, dF):
    """dP[dF] for any model (the true Hessian density applied to dF)."""
    F = _f64(F, (3, 3))
    dF = _f64(dF, (3, 3))
    out = np.zeros((3, 3))
    lib().or_dpk1(model, mu, lam, _d(F), _d(dF), _d(out))
    return out


def mod_hess_density(mu, lam, F):
    """Fourth-order tensor Ct[alpha, gamma, beta, delta] of Eq. (mod_hess_dens)."""
    F = _f64(F, (3, 3))
    out = np.zeros(81)
    lib().or_mod_hess_density(mu, lam, _d(F), _d(out))
    return out.reshape(3, 3, 3, 3)


def svd3(F):
    F = _f64(F, (3, 3))
    U = np.zeros((3, 3))
    s = np.zeros(3)
    V = np.zeros((3, 3))
    lib().or_svd3(_d(F), _d(U), _d(s), _d(V))
    return U, s, V


def chebyshev_weights(rho, n):
    w = np.zeros(n)
    lib().or_chebyshev_weights(rho, n, _d(w))
    return w


# ----------------------------------------------------------------------------
# problems
# ----------------------------------------------------------------------------
@dataclass
class OracleProblem:
    """A scenario marshalled for the C oracle (keeps the numpy buffers alive)."""
    nv: int
    nt: int
    model: int
    X: np.ndarray
    tets: np.ndarray
    mu: np.ndarray
    lam: np.ndarray
    fext: np.ndarray
    is_dir: np.ndarray
    wc_ptr: np.ndarray
    wc_vert: np.ndarray
    wc_w: np.ndarray
    wc_K: np.ndarray
    planes: np.ndarray
    V0: np.ndarray
    dN: np.ndarray
    dirichlet_idx: np.ndarray
    dirichlet_x: np.ndarray
    mass: np.ndarray = None          # lumped m_ii (Eq. fem_be)
    minert: np.ndarray = None        # m_ii / dt^2 on free vertices, or None
    xhat: np.ndarray = None          # 2 x^n - x^{n-1}

    def set_inertia(self, dt, x_n=None, x_prev=None):
        """Backward-Euler inertia with time step dt and xhat = 2 x^n - x^{n-1};
        dt <= 0 removes it."""
        if dt is None or dt <= 0:
            self.minert = self.xhat = None
            return
        m = self.mass / (dt * dt)
        m[self.is_dir != 0] = 0.0
        self.minert = np.ascontiguousarray(m)
        self.xhat = np.ascontiguousarray(2.0 * _f64(x_n, (-1, 3)) - _f64(x_prev, (-1, 3)))

    def struct(self) -> _Problem:
        s = _Problem()
        s.nv, s.nt, s.model = self.nv, self.nt, self.model
        s.X, s.tets, s.mu, s.lam, s.fext = (_d(self.X), _i(self.tets), _d(self.mu),
                                            _d(self.lam), _d(self.fext))
        s.is_dir = self.is_dir.ctypes.data_as(_up)
        s.n_wc = self.wc_ptr.size - 1
        s.wc_ptr, s.wc_vert, s.wc_w, s.wc_K = (_i(self.wc_ptr), _i(self.wc_vert),
                                                _d(self.wc_w), _d(self.wc_K))
        s.n_planes = self.planes.shape[0]
        s.planes = _d(self.planes)
        if self.minert is not None:
            s.minert, s.xhat = _d(self.minert), _d(self.xhat)
        return s


def make_problem(sc, mu=None, lam=None) -> OracleProblem:
    """Build the oracle's view of a Scenario.  mu / lam override the Lame
    parameters (scalar or per tet) instead of converting sc.E, sc.nu."""
    L = lib()
    X = _f64(sc.rest_pos, (-1, 3))
    T = np.ascontiguousarray(sc.tets, dtype=np.int32).reshape(-1, 4)
    nv, nt = X.shape[0], T.shape[0]
    if mu is None or lam is None:
        m, l_ = lame(sc.E, sc.nu)
        mu = m if mu is None else mu
        lam = l_ if lam is None else lam
    mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, np.float64), (nt,)))
    lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, np.float64), (nt,)))
    dN = np.zeros((max(nt, 1), 4, 3))
    V0 = np.zeros(max(nt, 1))
    rc = L.or_prep(nv, nt, _d(X), _i(T), _d(dN), _d(V0))
    if rc != 0:
        raise ValueError("oracle: invalid mesh (rc=%d)" % rc)
    fext = np.zeros((nv, 3))
    g = np.ascontiguousarray(sc.gravity, dtype=np.float64)
    if sc.density != 0.0 and nt > 0:
        L.or_body_force(nv, nt, _i(T), _d(V0), float(sc.density), _d(g), _d(fext))
    if sc.nodal_force is not None:
        fext += np.asarray(sc.nodal_force, np.float64).reshape(nv, 3)
    is_dir = np.zeros(nv, np.uint8)
    is_dir[np.asarray(sc.dirichlet_idx, np.int64)] = 1
    mass = np.zeros(nv)
    if nt > 0:
        L.or_lumped_mass(nv, nt, _i(T), _d(V0), float(sc.density), _d(mass))
    return OracleProblem(nv=nv, nt=nt, model=MODEL[sc.model],
                         X=X, tets=T, mu=mu, lam=lam, fext=np.ascontiguousarray(fext),
                         is_dir=is_dir,
                         wc_ptr=np.ascontiguousarray(sc.wc_ptr, np.int32),
                         wc_vert=np.ascontiguousarray(sc.wc_vert, np.int32),
                         wc_w=np.ascontiguousarray(sc.wc_w, np.float64),
                         wc_K=np.ascontiguousarray(np.asarray(sc.wc_K, np.float64).reshape(-1, 6)),
                         planes=np.ascontiguousarray(np.asarray(sc.planes, np.float64).reshape(-1, 5)),
                         V0=V0[:nt], dN=dN[:nt],
                         dirichlet_idx=np.asarray(sc.dirichlet_idx, np.int32),
                         dirichlet_x=np.asarray(sc.dirichlet_x, np.float64), mass=mass)


def recolor(op: OracleProblem, colors, nodes):
    """Incremental recolouring after new weak constraints (the problem
    already holds them): returns (colours, number of colours)."""
    s = op.struct()
    out = np.ascontiguousarray(np.array(colors, dtype=np.int32))
    nodes = np.ascontiguousarray(nodes, np.int32)
    nc = lib().or_recolor(C.byref(s), nodes.size, _i(nodes), _i(out))
    if nc < 0:
        raise ValueError("oracle recolouring failed (%d)" % nc)
    return out, int(nc)


def color(op: OracleProblem):
    """Greedy node colouring (Sec. "Coloring and Parallelism").  Returns
    (colors int32 [nv] with -1 on Dirichlet vertices, n_colors)."""
    s = op.struct()
    out = np.zeros(op.nv, np.int32)
    n = lib().or_color(C.byref(s), _i(out))
    if n < 0:
        raise ValueError("oracle colour failed (%d)" % n)
    return out, int(n)


def residual(op: OracleProblem, x):
    """(||r||_2 over free vertices, energy, r [nv, 3])."""
    s = op.struct()
    x = _f64(x, (-1, 3))
    r = np.zeros((op.nv, 3))
    E = C.c_double()
    n = lib().or_residual(C.byref(s), _d(x), _d(r), C.byref(E))
    return float(n), float(E.value), r


def energy_gradient(op: OracleProblem, x):
    s = op.struct()
    x = _f64(x, (-1, 3))
    g = np.zeros((op.nv, 3))
    lib().or_energy_gradient(C.byref(s), _d(x), _d(g))
    return g


def hvp(op: OracleProblem, x, v):
    s = op.struct()
    x = _f64(x, (-1, 3))
    v = _f64(v, (-1, 3))
    out = np.zeros((op.nv, 3))
    rc = lib().or_hvp(C.byref(s), _d(x), _d(v), _d(out))
    if rc:
        raise ValueError("oracle hvp: unsupported (rc=%d)" % rc)
    return out


def adjoint_gradients(op: OracleProblem, x, lam_vec):
    s = op.struct()
    x = _f64(x, (-1, 3))
    lv = _f64(lam_vec, (-1, 3))
    dmu = np.zeros(op.nt)
    dla = np.zeros(op.nt)
    dxd = np.zeros((op.nv, 3))
    rc = lib().or_adjoint_gradients(C.byref(s), _d(x), _d(lv), _d(dmu), _d(dla), _d(dxd))
    if rc:
        raise ValueError("oracle adjoint: unsupported (rc=%d)" % rc)
    return dmu, dla, dxd


def solve(op: OracleProblem, colors, x, max_sweeps=100, accel="none", rho=0.95, gamma=1.7,
          omega=1.7, safeguard="backtrack", max_halvings=8, rel_tol=0.0, check_every=1,
          skip_tol=0.0, emulate_f32=False, n_threads=1, history=False):
    """Run the PBNG iteration in place on a copy of x; returns (x, stats dict
    [, relative-residual history])."""
    s = op.struct()
    x = np.array(x, dtype=np.float64).reshape(-1, 3)
    colors = np.ascontiguousarray(colors, np.int32)
    o = _Opts(max_sweeps=max_sweeps, check_every=check_every, rel_tol=rel_tol,
              accel=ACCEL[accel], rho=rho, gamma=gamma, omega=omega,
              safeguard=SAFEGUARD[safeguard], max_halvings=max_halvings, skip_tol=skip_tol,
              emulate_f32=int(emulate_f32), n_threads=n_threads)
    st = _Stats()
    hist = np.zeros(max(1, max_sweeps // max(1, check_every)))
    rc = lib().or_solve(C.byref(s), _i(colors), _d(x), C.byref(o), C.byref(st), _d(hist))
    if rc:
        raise ValueError("oracle solve failed (%d)" % rc)
    stats = dict(sweeps=st.sweeps, converged=bool(st.converged), rejected=int(st.rejected),
                 halvings=int(st.halvings), res0=st.res0, res=st.res, rel=st.rel,
                 energy=st.energy)
    if history:
        return x, stats, hist[: max(0, st.sweeps // max(1, check_every))]
    return x, stats


def update_vertices(op: OracleProblem, x, verts, safeguard="backtrack", max_halvings=8,
                    emulate_f32=False):
    """New positions of `verts` after one update each from positions x."""
    s = op.struct()
    x = _f64(x, (-1, 3))
    verts = np.ascontiguousarray(verts, np.int32)
    o = _Opts(max_sweeps=1, check_every=1, rel_tol=0.0, accel=0, rho=0, gamma=1, omega=1,
              safeguard=SAFEGUARD[safeguard], max_halvings=max_halvings, skip_tol=0.0,
              emulate_f32=int(emulate_f32), n_threads=1)
    out = np.zeros((verts.size, 3))
    rc = lib().or_update_vertices(C.byref(s), _d(x), verts.size, _i(verts), C.byref(o), _d(out))
    if rc:
        raise ValueError("oracle update failed (%d)" % rc)
    return out


def sweep_energy_trace(op: OracleProblem, colors, x, safeguard="backtrack", max_halvings=8):
    s = op.struct()
    x = np.array(x, dtype=np.float64).reshape(-1, 3)
    colors = np.ascontiguousarray(colors, np.int32)
    o = _Opts(max_sweeps=1, check_every=1, rel_tol=0.0, accel=0, rho=0, gamma=1, omega=1,
              safeguard=SAFEGUARD[safeguard], max_halvings=max_halvings, skip_tol=0.0,
              emulate_f32=0, n_threads=1)
    dE = np.zeros(op.nv)
    n = lib().or_sweep_energy_trace(C.byref(s), _i(colors), _d(x), C.byref(o), _d(dE))
    return dE[:n], x
