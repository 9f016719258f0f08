"""ctypes binding of the planar family of libpbng (include/pbng2d.h):
argument marshalling only, same library and conventions as ``pbng``.
Positions are [n, 2] torch cuda tensors of the workspace dtype."""
from __future__ import annotations

import ctypes as C
from typing import List, Optional

import numpy as np

from . import pbng as _b
from .pbng import (MODEL, REAL, AdjointOpts, SolveOpts, Stats, _check, _d, _i, _ptr, _stream, adjoint_opts,
                   lame, solve_opts)

_ip = C.POINTER(C.c_int32)
_dp = C.POINTER(C.c_double)


class Problem2D(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tris", C.c_int32), ("rest_pos", _dp), ("tris", _ip),
                ("model", C.c_int32), ("mu", C.c_double), ("lambda_", C.c_double), ("mu_tri", _dp),
                ("lambda_tri", _dp), ("density", C.c_double), ("gravity", C.c_double * 2),
                ("nodal_force", _dp), ("n_dirichlet", C.c_int32), ("dirichlet_idx", _ip),
                ("dirichlet_x", _dp), ("n_wc", C.c_int32), ("wc_ptr", _ip), ("wc_vert", _ip),
                ("wc_w", _dp), ("wc_K", _dp), ("n_planes", C.c_int32), ("planes", _dp)]


_ready = False


def lib():
    global _ready
    L = _b.lib()
    if not _ready:
        vp = C.c_void_p
        i64 = C.POINTER(C.c_int64)
        sigs = {
            "pbng2d_color": ([C.POINTER(Problem2D), _ip, _ip], C.c_int32),
            "pbng2d_workspace_create": ([C.POINTER(Problem2D), _ip, C.c_int32, C.POINTER(vp)], C.c_int32),
            "pbng2d_workspace_destroy": ([vp], C.c_int32),
            "pbng2d_workspace_info": ([vp, i64, i64, i64, _ip, i64], C.c_int32),
            "pbng2d_workspace_colors": ([vp, _ip], C.c_int32),
            "pbng2d_solve": ([vp, vp, C.POINTER(SolveOpts), C.POINTER(Stats), vp], C.c_int32),
            "pbng2d_residual": ([vp, vp, _dp, _dp, vp, vp], C.c_int32),
            "pbng2d_load": ([vp, vp, vp], C.c_int32),
            "pbng2d_store": ([vp, vp, vp], C.c_int32),
            "pbng2d_sweeps": ([vp, C.c_int32, C.POINTER(SolveOpts), vp], C.c_int32),
            "pbng2d_phase_bytes": ([vp, C.c_int32, i64, i64, i64], C.c_int32),
            "pbng2d_workspace_set_inertia": ([vp, C.c_double, vp, vp, vp], C.c_int32),
            "pbng2d_adjoint": ([vp, vp, vp, vp, vp, vp, vp, C.POINTER(AdjointOpts), C.POINTER(Stats), vp],
                               C.c_int32),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _ready = True
    return L


def exported_symbols() -> List[str]:
    return ["pbng2d_color", "pbng2d_workspace_create", "pbng2d_workspace_destroy",
            "pbng2d_workspace_info", "pbng2d_workspace_colors", "pbng2d_solve", "pbng2d_residual",
            "pbng2d_load", "pbng2d_store", "pbng2d_sweeps", "pbng2d_phase_bytes",
            "pbng2d_workspace_set_inertia", "pbng2d_adjoint"]


class HostProblem2D:
    """A planar problem in host memory; keeps the numpy buffers alive."""

    def __init__(self, rest_pos, tris, model, mu, lam, dirichlet_idx, dirichlet_x, density=0.0,
                 gravity=(0.0, 0.0), nodal_force=None, wc_ptr=None, wc_vert=None, wc_w=None, wc_K=None,
                 planes=None):
        self.rest_pos = np.ascontiguousarray(rest_pos, np.float64).reshape(-1, 2)
        self.tris = np.ascontiguousarray(tris, np.int32).reshape(-1, 3)
        nt = self.tris.shape[0]
        mu = np.asarray(mu, np.float64)
        lam = np.asarray(lam, np.float64)
        per = mu.size > 1 or lam.size > 1
        self.mu_tri = np.ascontiguousarray(np.broadcast_to(mu, (nt,))) if per else None
        self.lam_tri = np.ascontiguousarray(np.broadcast_to(lam, (nt,))) if per else None
        self.mu = float(mu.reshape(-1)[0])
        self.lam = float(lam.reshape(-1)[0])
        self.model = MODEL[model] if isinstance(model, str) else int(model)
        self.dirichlet_idx = np.ascontiguousarray(dirichlet_idx, np.int32).reshape(-1)
        self.dirichlet_x = np.ascontiguousarray(dirichlet_x, np.float64).reshape(-1, 2)
        self.density = float(density)
        self.gravity = tuple(float(g) for g in gravity)
        self.nodal_force = (None if nodal_force is None
                            else np.ascontiguousarray(nodal_force, np.float64).reshape(-1, 2))
        self.wc_ptr = np.ascontiguousarray(np.zeros(1) if wc_ptr is None else wc_ptr, np.int32).reshape(-1)
        self.wc_vert = np.ascontiguousarray(np.zeros(0) if wc_vert is None else wc_vert, np.int32).reshape(-1)
        self.wc_w = np.ascontiguousarray(np.zeros(0) if wc_w is None else wc_w, np.float64).reshape(-1)
        self.wc_K = np.ascontiguousarray(np.zeros((0, 3)) if wc_K is None else wc_K, np.float64).reshape(-1, 3)
        self.planes = np.ascontiguousarray(np.zeros((0, 4)) if planes is None else planes,
                                           np.float64).reshape(-1, 4)

    @property
    def n_verts(self):
        return self.rest_pos.shape[0]

    def struct(self) -> Problem2D:
        s = Problem2D()
        s.n_verts, s.n_tris = self.rest_pos.shape[0], self.tris.shape[0]
        s.rest_pos, s.tris = _d(self.rest_pos), _i(self.tris)
        s.model, s.mu, s.lambda_ = self.model, self.mu, self.lam
        s.mu_tri, s.lambda_tri = _d(self.mu_tri), _d(self.lam_tri)
        s.density = self.density
        s.gravity = (C.c_double * 2)(*self.gravity)
        s.nodal_force = _d(self.nodal_force)
        s.n_dirichlet = self.dirichlet_idx.size
        s.dirichlet_idx, s.dirichlet_x = _i(self.dirichlet_idx), _d(self.dirichlet_x)
        s.n_wc = self.wc_ptr.size - 1
        if s.n_wc > 0:
            s.wc_ptr, s.wc_vert = _i(self.wc_ptr), _i(self.wc_vert)
            s.wc_w, s.wc_K = _d(self.wc_w), _d(self.wc_K)
        s.n_planes = self.planes.shape[0]
        if s.n_planes > 0:
            s.planes = _d(self.planes)
        return s


def problem_from_scenario(sc) -> HostProblem2D:
    """Marshal a ``scenarios.Scenario2D``; (E, nu) through the library's
    Lame conversion."""
    mu, lam = lame(sc.E, sc.nu)
    return HostProblem2D(sc.rest_pos, sc.tris, sc.model, mu, lam, sc.dirichlet_idx, sc.dirichlet_x,
                         density=sc.density, gravity=sc.gravity, nodal_force=sc.nodal_force,
                         wc_ptr=sc.wc_ptr, wc_vert=sc.wc_vert, wc_w=sc.wc_w, wc_K=sc.wc_K,
                         planes=sc.planes)


def color(problem: HostProblem2D):
    s = problem.struct()
    out = np.zeros(problem.n_verts, np.int32)
    n = C.c_int32()
    _check(lib().pbng2d_color(C.byref(s), _i(out), C.byref(n)))
    return out, n.value


class Workspace2D:
    """pbng2d_workspace: packed device copy of one planar problem."""

    def __init__(self, problem: HostProblem2D, colors: Optional[np.ndarray] = None, real: str = "f32"):
        if real not in ("f32", "f64"):
            raise ValueError("planar workspaces are f32 or f64")
        self.problem = problem
        self._struct = problem.struct()
        cols = None if colors is None else np.ascontiguousarray(colors, np.int32)
        h = C.c_void_p()
        _check(lib().pbng2d_workspace_create(C.byref(self._struct), _i(cols), REAL[real], C.byref(h)))
        self.handle = h
        self.real = real
        nv, nt, nf, nvis = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        nc = C.c_int32()
        _check(lib().pbng2d_workspace_info(h, C.byref(nv), C.byref(nt), C.byref(nf), C.byref(nc),
                                           C.byref(nvis)))
        self.n_verts, self.n_tris, self.n_free = nv.value, nt.value, nf.value
        self.n_colors, self.n_visits = nc.value, nvis.value

    def close(self):
        if getattr(self, "handle", None):
            lib().pbng2d_workspace_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dtype(self):
        import torch
        return torch.float32 if self.real == "f32" else torch.float64

    def _check_x(self, x):
        import torch
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError("positions must be a torch cuda tensor")
        if x.dtype != self.dtype or tuple(x.shape) != (self.n_verts, 2) or not x.is_contiguous():
            raise ValueError("positions must be a contiguous [%d, 2] %s tensor" % (self.n_verts, self.dtype))

    def solve(self, x, opts: Optional[SolveOpts] = None, stream=None, **kw):
        self._check_x(x)
        o = opts if opts is not None else solve_opts(**kw)
        st = Stats()
        rc = _check(lib().pbng2d_solve(self.handle, _ptr(x), C.byref(o), C.byref(st), _stream(stream)))
        return rc, st.to_dict()

    def residual(self, x, want_r: bool = False, stream=None):
        import torch
        self._check_x(x)
        res, en = C.c_double(), C.c_double()
        r = torch.zeros((self.n_verts, 2), dtype=torch.float64, device=x.device) if want_r else None
        _check(lib().pbng2d_residual(self.handle, _ptr(x), C.byref(res), C.byref(en), _ptr(r), _stream(stream)))
        return (res.value, en.value, r) if want_r else (res.value, en.value)

    def colors(self):
        out = np.zeros(self.n_verts, np.int32)
        _check(lib().pbng2d_workspace_colors(self.handle, _i(out)))
        return out

    def adjoint(self, x_eq, dL_dx, opts: Optional[AdjointOpts] = None, stream=None, **kw):
        """pbng2d_adjoint; returns (status, dict of float64 cuda tensors
        xd [n_dirichlet, 2] (dL/dx_D), mu and lam [n_tris] (dL/dmu,
        dL/dlambda), lam_vec [n_verts, 2] (the adjoint), stats)."""
        import torch
        self._check_x(x_eq)
        self._check_x(dL_dx)
        o = opts if opts is not None else adjoint_opts(**kw)
        dev = x_eq.device
        nd = self.problem.dirichlet_idx.size
        out = {"xd": torch.zeros((max(nd, 1), 2), dtype=torch.float64, device=dev),
               "mu": torch.zeros(max(self.n_tris, 1), dtype=torch.float64, device=dev),
               "lam": torch.zeros(max(self.n_tris, 1), dtype=torch.float64, device=dev),
               "lam_vec": torch.zeros((self.n_verts, 2), dtype=torch.float64, device=dev)}
        st = Stats()
        rc = _check(lib().pbng2d_adjoint(self.handle, _ptr(x_eq), _ptr(dL_dx), _ptr(out["xd"]), _ptr(out["mu"]),
                                         _ptr(out["lam"]), _ptr(out["lam_vec"]), C.byref(o), C.byref(st),
                                         _stream(stream)))
        out["xd"] = out["xd"][:nd]
        out["mu"], out["lam"] = out["mu"][:self.n_tris], out["lam"][:self.n_tris]
        return rc, out, st.to_dict()

    def set_inertia(self, dt, x_n=None, x_prev=None, stream=None):
        """Backward-Euler inertia with time step dt and xhat = 2 x^n - x^{n-1}
        (float64 cuda tensors [n_verts, 2], caller order); dt <= 0 turns it
        off."""
        import torch
        if dt > 0:
            for t in (x_n, x_prev):
                if t is None or t.dtype != torch.float64 or not t.is_cuda or t.numel() != 2 * self.n_verts:
                    raise ValueError("x^n and x^{n-1} must be float64 cuda tensors [%d, 2]" % self.n_verts)
            x_n, x_prev = x_n.contiguous(), x_prev.contiguous()
            _check(lib().pbng2d_workspace_set_inertia(self.handle, float(dt), _ptr(x_n), _ptr(x_prev),
                                                      _stream(stream)))
        else:
            _check(lib().pbng2d_workspace_set_inertia(self.handle, float(dt), None, None, _stream(stream)))

    def load(self, x, stream=None):
        self._check_x(x)
        _check(lib().pbng2d_load(self.handle, _ptr(x), _stream(stream)))

    def store(self, x, stream=None):
        self._check_x(x)
        _check(lib().pbng2d_store(self.handle, _ptr(x), _stream(stream)))

    def sweeps(self, n, opts: Optional[SolveOpts] = None, stream=None, **kw):
        o = opts if opts is not None else solve_opts(**kw)
        _check(lib().pbng2d_sweeps(self.handle, n, C.byref(o), _stream(stream)))

    def phase_bytes(self, color_idx):
        b, v, k = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().pbng2d_phase_bytes(self.handle, color_idx, C.byref(b), C.byref(v), C.byref(k)))
        return b.value, v.value, k.value
