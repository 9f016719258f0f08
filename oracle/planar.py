"""FP64 oracle for PBNG on triangle meshes (d = 2) -- TEST INFRASTRUCTURE ONLY.

Marshals numpy arrays into the plain C of ``pbng_oracle2d.c`` (built into
the same ``liboracle.so`` as the 3-D oracle).  Same rules as the package:
only tests/, ``__graft_entry__.smoke()`` and bench.py's ``cpu_baseline`` leg
may use it.  Positions are [n, 2] arrays; matrices are 2x2.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import ACCEL, SAFEGUARD, _Opts, _Stats, _d, _f64, _i, lame, lib as _lib3

NEOHOOKEAN, COROTATED = 0, 1
MODEL = {"nh": NEOHOOKEAN, "corotated": COROTATED}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint8)


class _Problem2(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nt", C.c_int32), ("model", C.c_int32), ("X", _dp),
                ("tris", _ip), ("mu", _dp), ("lam", _dp), ("fext", _dp), ("is_dir", _up),
                ("n_wc", C.c_int32), ("wc_ptr", _ip), ("wc_vert", _ip), ("wc_w", _dp), ("wc_K", _dp),
                ("n_planes", C.c_int32), ("planes", _dp), ("minert", _dp), ("xhat", _dp)]


_ready = False


def lib():
    global _ready
    L = _lib3()
    if not _ready:
        L.or2_rotation.argtypes = [_dp, _dp]
        L.or2_psi.argtypes = [C.c_int, C.c_double, C.c_double, _dp]
        L.or2_psi.restype = C.c_double
        L.or2_pk1.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp]
        L.or2_mod_hess_density.argtypes = [C.c_double, C.c_double, _dp, _dp]
        L.or2_prep.argtypes = [C.c_int32, C.c_int32, _dp, _ip, _dp, _dp]
        L.or2_prep.restype = C.c_int
        L.or2_body_force.argtypes = [C.c_int32, C.c_int32, _ip, _dp, C.c_double, _dp, _dp]
        L.or2_lumped_mass.argtypes = [C.c_int32, C.c_int32, _ip, _dp, C.c_double, _dp]
        L.or2_color.argtypes = [C.POINTER(_Problem2), _ip]
        L.or2_color.restype = C.c_int32
        L.or2_residual.argtypes = [C.POINTER(_Problem2), _dp, _dp, _dp]
        L.or2_residual.restype = C.c_double
        L.or2_solve.argtypes = [C.POINTER(_Problem2), _ip, _dp, C.POINTER(_Opts), C.POINTER(_Stats), _dp]
        L.or2_solve.restype = C.c_int32
        L.or2_sweep_energy_trace.argtypes = [C.POINTER(_Problem2), _ip, _dp, C.POINTER(_Opts), _dp]
        L.or2_sweep_energy_trace.restype = C.c_int32
        L.or2_stress_diff.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, _dp]
        L.or2_hessian_apply.argtypes = [C.POINTER(_Problem2), _dp, _dp, _dp]
        L.or2_hessian_apply.restype = C.c_int32
        L.or2_adjoint_gradients.argtypes = [C.POINTER(_Problem2), _dp, _dp, _dp, _dp]
        L.or2_adjoint_gradients.restype = C.c_int32
        _ready = True
    return L


def rotation(F):
    """Closest proper rotation to a 2x2 F (tr(R^T F) maximal)."""
    F = _f64(F, (2, 2))
    R = np.zeros((2, 2))
    lib().or2_rotation(_d(F), _d(R))
    return R


def psi(model, mu, lam, F):
    return lib().or2_psi(model, mu, lam, _d(_f64(F, (2, 2))))


def pk1(model, mu, lam, F):
    P = np.zeros((2, 2))
    lib().or2_pk1(model, mu, lam, _d(_f64(F, (2, 2))), _d(P))
    return P


def mod_hess_density(mu, lam, F):
    """Ct[alpha, gamma, beta, delta] of Eq. (mod_hess_dens) with d = 2."""
    out = np.zeros(16)
    lib().or2_mod_hess_density(mu, lam, _d(_f64(F, (2, 2))), _d(out))
    return out.reshape(2, 2, 2, 2)


@dataclass
class PlanarProblem:
    nv: int
    nt: int
    model: int
    X: np.ndarray
    tris: np.ndarray
    mu: np.ndarray
    lam: np.ndarray
    fext: np.ndarray
    is_dir: np.ndarray
    A0: np.ndarray
    dN: np.ndarray
    dirichlet_idx: np.ndarray
    dirichlet_x: np.ndarray
    wc_ptr: np.ndarray = None
    wc_vert: np.ndarray = None
    wc_w: np.ndarray = None
    wc_K: np.ndarray = None          # [n_wc, 3] (xx, xy, yy)
    planes: np.ndarray = None        # [n_planes, 4] (nx, ny, d, k)
    mass: np.ndarray = None          # lumped m_ii = R0 sum A0 / 3 (Eq. fem_be, d = 2)
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
        self.xhat = np.ascontiguousarray(2.0 * _f64(x_n, (-1, 2)) - _f64(x_prev, (-1, 2)))

    def struct(self) -> _Problem2:
        s = _Problem2()
        s.nv, s.nt, s.model = self.nv, self.nt, self.model
        s.X, s.tris, s.mu, s.lam, s.fext = (_d(self.X), _i(self.tris), _d(self.mu), _d(self.lam),
                                            _d(self.fext))
        s.is_dir = self.is_dir.ctypes.data_as(_up)
        s.n_wc = self.wc_ptr.size - 1
        s.wc_ptr, s.wc_vert, s.wc_w, s.wc_K = (_i(self.wc_ptr), _i(self.wc_vert), _d(self.wc_w),
                                                _d(self.wc_K))
        s.n_planes = self.planes.shape[0]
        s.planes = _d(self.planes)
        if self.minert is not None:
            s.minert, s.xhat = _d(self.minert), _d(self.xhat)
        return s


def make_problem(sc, mu=None, lam=None) -> PlanarProblem:
    """The oracle's view of a Scenario2D (Lame parameters from sc.E, sc.nu
    unless mu / lam are given, scalar or per triangle)."""
    L = lib()
    X = _f64(sc.rest_pos, (-1, 2))
    T = np.ascontiguousarray(sc.tris, dtype=np.int32).reshape(-1, 3)
    nv, nt = X.shape[0], T.shape[0]
    if mu is None or lam is None:
        m, l_ = lame(sc.E, sc.nu)
        mu = m if mu is None else mu
        lam = l_ if lam is None else lam
    mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, np.float64), (nt,)))
    lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, np.float64), (nt,)))
    dN = np.zeros((max(nt, 1), 3, 2))
    A0 = np.zeros(max(nt, 1))
    rc = L.or2_prep(nv, nt, _d(X), _i(T), _d(dN), _d(A0))
    if rc != 0:
        raise ValueError("planar oracle: invalid mesh (rc=%d)" % rc)
    fext = np.zeros((nv, 2))
    g = np.ascontiguousarray(sc.gravity, dtype=np.float64)
    if sc.density != 0.0 and nt > 0:
        L.or2_body_force(nv, nt, _i(T), _d(A0), float(sc.density), _d(g), _d(fext))
    if sc.nodal_force is not None:
        fext += np.asarray(sc.nodal_force, np.float64).reshape(nv, 2)
    is_dir = np.zeros(nv, np.uint8)
    is_dir[np.asarray(sc.dirichlet_idx, np.int64)] = 1
    mass = np.zeros(nv)
    if nt > 0:
        L.or2_lumped_mass(nv, nt, _i(T), _d(A0), float(sc.density), _d(mass))
    return PlanarProblem(nv=nv, nt=nt, model=MODEL[sc.model], X=X, tris=T, mu=mu, lam=lam,
                         fext=np.ascontiguousarray(fext), is_dir=is_dir, A0=A0[:nt], dN=dN[:nt],
                         dirichlet_idx=np.asarray(sc.dirichlet_idx, np.int32),
                         dirichlet_x=np.asarray(sc.dirichlet_x, np.float64),
                         wc_ptr=np.ascontiguousarray(sc.wc_ptr, np.int32),
                         wc_vert=np.ascontiguousarray(sc.wc_vert, np.int32),
                         wc_w=np.ascontiguousarray(sc.wc_w, np.float64),
                         wc_K=np.ascontiguousarray(np.asarray(sc.wc_K, np.float64).reshape(-1, 3)),
                         planes=np.ascontiguousarray(np.asarray(sc.planes, np.float64).reshape(-1, 4)),
                         mass=mass)


def color(op: PlanarProblem):
    out = np.zeros(op.nv, np.int32)
    n = lib().or2_color(C.byref(op.struct()), _i(out))
    if n < 0:
        raise ValueError("planar oracle colour failed (%d)" % n)
    return out, int(n)


def residual(op: PlanarProblem, x):
    """(||r||_2 over free vertices, energy, r [nv, 2])."""
    x = _f64(x, (-1, 2))
    r = np.zeros((op.nv, 2))
    E = C.c_double()
    n = lib().or2_residual(C.byref(op.struct()), _d(x), _d(r), C.byref(E))
    return float(n), float(E.value), r


def solve(op: PlanarProblem, colors, x, max_sweeps=100, accel="none", rho=0.95, gamma=1.7, omega=1.7,
          safeguard="backtrack", max_halvings=8, rel_tol=0.0, check_every=1, emulate_f32=False,
          history=False):
    x = np.array(x, dtype=np.float64).reshape(-1, 2)
    colors = np.ascontiguousarray(colors, np.int32)
    o = _Opts(max_sweeps=max_sweeps, check_every=check_every, rel_tol=rel_tol, accel=ACCEL[accel],
              rho=rho, gamma=gamma, omega=omega, safeguard=SAFEGUARD[safeguard],
              max_halvings=max_halvings, skip_tol=0.0, emulate_f32=int(emulate_f32), n_threads=1)
    st = _Stats()
    hist = np.zeros(max(1, max_sweeps // max(1, check_every)))
    rc = lib().or2_solve(C.byref(op.struct()), _i(colors), _d(x), C.byref(o), C.byref(st), _d(hist))
    if rc:
        raise ValueError("planar oracle solve failed (%d)" % rc)
    stats = dict(sweeps=st.sweeps, converged=bool(st.converged), rejected=int(st.rejected),
                 halvings=int(st.halvings), res0=st.res0, res=st.res, rel=st.rel, energy=st.energy)
    if history:
        return x, stats, hist[: max(0, st.sweeps // max(1, check_every))]
    return x, stats


def sweep_energy_trace(op: PlanarProblem, colors, x, safeguard="backtrack", max_halvings=8):
    x = np.array(x, dtype=np.float64).reshape(-1, 2)
    colors = np.ascontiguousarray(colors, np.int32)
    o = _Opts(max_sweeps=1, check_every=1, rel_tol=0.0, accel=0, rho=0, gamma=1, omega=1,
              safeguard=SAFEGUARD[safeguard], max_halvings=max_halvings, skip_tol=0.0, emulate_f32=0,
              n_threads=1)
    dE = np.zeros(op.nv)
    n = lib().or2_sweep_energy_trace(C.byref(op.struct()), _i(colors), _d(x), C.byref(o), _d(dE))
    return dE[:n], x


# ---------------------------------------------------------------------------
# adjoint (true Hessian, parameter gradients)
# ---------------------------------------------------------------------------
def stress_diff(model, mu, lam, F, L):
    """dP[L] of the 2x2 first Piola-Kirchhoff stress."""
    out = np.zeros((2, 2))
    lib().or2_stress_diff(model, mu, lam, _d(_f64(F, (2, 2))), _d(_f64(L, (2, 2))), _d(out))
    return out


def hessian_apply(op: PlanarProblem, x, v):
    """H v for every vertex row (v taken as zero on Dirichlet rows)."""
    x = _f64(x, (-1, 2))
    v = _f64(v, (-1, 2))
    out = np.zeros((op.nv, 2))
    rc = lib().or2_hessian_apply(C.byref(op.struct()), _d(x), _d(v), _d(out))
    if rc:
        raise ValueError("planar oracle hessian failed (%d)" % rc)
    return out


def adjoint_gradients(op: PlanarProblem, x, lam):
    """(dL/dmu, dL/dlambda) per triangle from the adjoint lam."""
    x = _f64(x, (-1, 2))
    lam = _f64(lam, (-1, 2))
    dmu, dlam = np.zeros(op.nt), np.zeros(op.nt)
    rc = lib().or2_adjoint_gradients(C.byref(op.struct()), _d(x), _d(lam), _d(dmu), _d(dlam))
    if rc:
        raise ValueError("planar oracle adjoint gradients failed (%d)" % rc)
    return dmu, dlam


def free_dofs(op: PlanarProblem):
    free = np.nonzero(op.is_dir == 0)[0]
    return np.stack([2 * free, 2 * free + 1], axis=1).reshape(-1)


def dense_hessian(op: PlanarProblem, x):
    """The true Hessian restricted to the free degrees of freedom, one
    column per unit vector (small problems only)."""
    dofs = free_dofs(op)
    H = np.zeros((dofs.size, dofs.size))
    for c, d in enumerate(dofs):
        v = np.zeros(2 * op.nv)
        v[d] = 1.0
        H[:, c] = hessian_apply(op, x, v).reshape(-1)[dofs]
    return H


def adjoint(op: PlanarProblem, x, dL_dx):
    """The adjoint of the equilibrium x by its definition: lam = H^{-1} dL/dx
    on the free degrees of freedom (dense solve), dL/dx_D = (dL/dx)_D -
    (H lam)_D, and the parameter gradients.  Returns (lam [nv, 2],
    dL/dx_D [n_dirichlet, 2] in dirichlet_idx order, dL/dmu, dL/dlambda)."""
    b = _f64(dL_dx, (-1, 2)).reshape(-1)
    dofs = free_dofs(op)
    lam = np.zeros(2 * op.nv)
    lam[dofs] = np.linalg.solve(dense_hessian(op, x), b[dofs])
    lam = lam.reshape(-1, 2)
    Hl = hessian_apply(op, x, lam)
    dxd = b.reshape(-1, 2)[op.dirichlet_idx] - Hl[op.dirichlet_idx]
    dmu, dlam = adjoint_gradients(op, x, lam)
    return lam, dxd, dmu, dlam


def newton_equilibrium(op: PlanarProblem, x0, tol=1e-13, max_iter=60):
    """Equilibrium by Newton's method with the dense true Hessian and a
    backtracking line search on the energy (small problems only)."""
    x = np.array(x0, dtype=np.float64).reshape(-1, 2)
    x[op.dirichlet_idx] = op.dirichlet_x
    dofs = free_dofs(op)
    r0 = residual(op, x)[0]
    for _ in range(max_iter):
        rn, E, r = residual(op, x)
        if rn <= tol * max(r0, 1.0):
            break
        step = np.linalg.solve(dense_hessian(op, x), r.reshape(-1)[dofs])
        t = 1.0
        while True:
            xt = x.copy().reshape(-1)
            xt[dofs] += t * step
            xt = xt.reshape(-1, 2)
            if residual(op, xt)[1] <= E + 1e-12 * abs(E) or t < 1e-8:
                break
            t *= 0.5
        x = xt
    return x
