"""ctypes binding of libpbng (include/pbng.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module converts numpy
arrays and torch device tensors into the C structures and pointers of the
ABI, maps negative status codes to exceptions, and raises immediately when
the built library is missing.  Names follow the C functions: ``color``,
``Workspace.solve``, ``Workspace.residual``, ``Workspace.adjoint``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PBNG_LIBRARY") or os.path.join(_HERE, "libpbng.so")

OK, NOT_CONVERGED = 0, 1
ERRORS = {-1: "EINVAL", -2: "EMESH", -3: "EMATERIAL", -4: "ECOLOR", -5: "ENAN", -6: "EHIP",
          -7: "ENOMEM", -8: "EUNSUPPORTED"}
MODEL = {"nh": 0, "corotated": 1, "snh": 2}
REAL = {"f32": 0, "f64": 1, "mixed": 2}
ACCEL = {"none": 0, "chebyshev": 1, "sor": 2}
SAFEGUARD = {"none": 0, "backtrack": 1}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class PBNGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "ERROR"), code, msg))
        self.code = code


class Problem(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32), ("rest_pos", _dp), ("tets", _ip),
                ("model", C.c_int32), ("mu", C.c_double), ("lambda_", C.c_double),
                ("mu_tet", _dp), ("lambda_tet", _dp), ("density", C.c_double),
                ("gravity", C.c_double * 3), ("nodal_force", _dp), ("n_dirichlet", C.c_int32),
                ("dirichlet_idx", _ip), ("dirichlet_x", _dp), ("n_wc", C.c_int32),
                ("wc_ptr", _ip), ("wc_vert", _ip), ("wc_w", _dp), ("wc_K", _dp),
                ("n_planes", C.c_int32), ("planes", _dp)]


class SolveOpts(C.Structure):
    _fields_ = [("max_sweeps", C.c_int32), ("rel_tol", C.c_double), ("check_every", C.c_int32),
                ("accel", C.c_int32), ("rho", C.c_double), ("gamma", C.c_double),
                ("omega", C.c_double), ("safeguard", C.c_int32), ("max_halvings", C.c_int32),
                ("lanes", C.c_int32), ("sweeps_per_graph", C.c_int32), ("resume", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("converged", C.c_int32), ("n_colors", C.c_int32),
                ("rejected", C.c_int32), ("residual0", C.c_double), ("residual", C.c_double),
                ("rel_residual", C.c_double), ("energy", C.c_double), ("time_ms", C.c_double),
                ("time_to_tol_ms", C.c_double), ("vertex_updates", C.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AdjointOpts(C.Structure):
    _fields_ = [("max_sweeps", C.c_int32), ("rel_tol", C.c_double), ("check_every", C.c_int32),
                ("accel", C.c_int32), ("rho", C.c_double), ("gamma", C.c_double),
                ("lanes", C.c_int32)]


_lib = None


def lib():
    """Load libpbng.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpbng.so is not built (%s); run "
                               "`python -m paper_2306_09021_amd.build`" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        sigs = {
            "pbng_version": ([], C.c_int32),
            "pbng_last_error": ([], C.c_char_p),
            "pbng_lame": ([C.c_int64, _dp, _dp, _dp, _dp], C.c_int32),
            "pbng_default_solve_opts": ([C.POINTER(SolveOpts)], C.c_int32),
            "pbng_default_adjoint_opts": ([C.POINTER(AdjointOpts)], C.c_int32),
            "pbng_color": ([C.POINTER(Problem), _ip, _ip], C.c_int32),
            "pbng_workspace_create": ([C.POINTER(Problem), C.c_int32, _ip, C.c_int32,
                                       C.POINTER(vp)], C.c_int32),
            "pbng_workspace_destroy": ([vp], C.c_int32),
            "pbng_workspace_info": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int32)], C.c_int32),
            "pbng_workspace_set_materials": ([vp, vp, vp, vp], C.c_int32),
            "pbng_workspace_set_dirichlet": ([vp, vp, vp], C.c_int32),
            "pbng_workspace_set_inertia": ([vp, C.c_double, vp, vp, vp], C.c_int32),
            "pbng_workspace_set_contacts": ([vp, C.c_int32, vp, vp, C.c_double, vp], C.c_int32),
            "pbng_workspace_colors": ([vp, _ip], C.c_int32),
            "pbng_detect_contacts": ([vp, vp, C.c_double, C.c_int32, vp, vp, _ip, vp], C.c_int32),
            "pbng_solve": ([vp, vp, C.POINTER(SolveOpts), C.POINTER(Stats), vp], C.c_int32),
            "pbng_residual": ([vp, vp, _dp, _dp, vp, vp], C.c_int32),
            "pbng_adjoint": ([vp, vp, vp, vp, vp, vp, vp, C.POINTER(AdjointOpts),
                              C.POINTER(Stats), vp], C.c_int32),
            "pbng_load": ([vp, vp, vp], C.c_int32),
            "pbng_store": ([vp, vp, vp], C.c_int32),
            "pbng_sweeps": ([vp, C.c_int32, C.POINTER(SolveOpts), vp], C.c_int32),
            "pbng_phase": ([vp, C.c_int32, C.POINTER(SolveOpts), vp], C.c_int32),
            "pbng_phase_bytes": ([vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64)], C.c_int32),
            "pbng_autotune": ([vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveOpts), _ip, vp],
                              C.c_int32),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols() -> List[str]:
    return ["pbng_version", "pbng_last_error", "pbng_lame", "pbng_default_solve_opts",
            "pbng_default_adjoint_opts", "pbng_color", "pbng_workspace_create",
            "pbng_workspace_destroy", "pbng_workspace_info", "pbng_workspace_set_materials",
            "pbng_workspace_set_dirichlet", "pbng_workspace_set_inertia",
            "pbng_workspace_set_contacts", "pbng_workspace_colors", "pbng_detect_contacts",
            "pbng_solve",
            "pbng_residual", "pbng_adjoint",
            "pbng_load", "pbng_store", "pbng_sweeps", "pbng_phase", "pbng_phase_bytes",
            "pbng_autotune"]


def _check(rc: int) -> int:
    if rc < 0:
        raise PBNGError(rc, lib().pbng_last_error().decode())
    return rc


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_ip) if a is not None else None


def lame(E, nu):
    """Lame parameters (Eq. lame) from Young's modulus and Poisson's ratio,
    computed by the library (element-wise over arrays)."""
    Eb, nb = np.broadcast_arrays(np.asarray(E, np.float64), np.asarray(nu, np.float64))
    Ef = np.ascontiguousarray(Eb.reshape(-1))
    nf = np.ascontiguousarray(nb.reshape(-1))
    mu = np.empty_like(Ef)
    la = np.empty_like(Ef)
    _check(lib().pbng_lame(Ef.size, _d(Ef), _d(nf), _d(mu), _d(la)))
    return mu.reshape(Eb.shape), la.reshape(Eb.shape)


class HostProblem:
    """A problem statement in host memory; keeps the numpy buffers alive."""

    def __init__(self, rest_pos, tets, model, mu, lam, dirichlet_idx, dirichlet_x, density=0.0,
                 gravity=(0.0, 0.0, 0.0), nodal_force=None, wc_ptr=None, wc_vert=None, wc_w=None,
                 wc_K=None, planes=None):
        self.rest_pos = np.ascontiguousarray(rest_pos, np.float64).reshape(-1, 3)
        self.tets = np.ascontiguousarray(tets, np.int32).reshape(-1, 4)
        nt = self.tets.shape[0]
        mu = np.asarray(mu, np.float64)
        lam = np.asarray(lam, np.float64)
        self.per_tet = mu.ndim > 0 and mu.size > 1 or lam.ndim > 0 and lam.size > 1
        if self.per_tet:
            self.mu_tet = np.ascontiguousarray(np.broadcast_to(mu, (nt,)))
            self.lam_tet = np.ascontiguousarray(np.broadcast_to(lam, (nt,)))
        else:
            self.mu_tet = self.lam_tet = None
        self.mu = float(mu.reshape(-1)[0]) if mu.size else 0.0
        self.lam = float(lam.reshape(-1)[0]) if lam.size else 0.0
        self.model = MODEL[model] if isinstance(model, str) else int(model)
        self.dirichlet_idx = np.ascontiguousarray(dirichlet_idx, np.int32).reshape(-1)
        self.dirichlet_x = np.ascontiguousarray(dirichlet_x, np.float64).reshape(-1, 3)
        self.density = float(density)
        self.gravity = tuple(float(g) for g in gravity)
        self.nodal_force = (None if nodal_force is None
                            else np.ascontiguousarray(nodal_force, np.float64).reshape(-1, 3))
        self.wc_ptr = None if wc_ptr is None or len(wc_ptr) <= 1 else np.ascontiguousarray(wc_ptr, np.int32)
        self.wc_vert = None if self.wc_ptr is None else np.ascontiguousarray(wc_vert, np.int32)
        self.wc_w = None if self.wc_ptr is None else np.ascontiguousarray(wc_w, np.float64)
        self.wc_K = None if self.wc_ptr is None else np.ascontiguousarray(wc_K, np.float64).reshape(-1, 6)
        pl = None if planes is None else np.ascontiguousarray(planes, np.float64).reshape(-1, 5)
        self.planes = pl if pl is not None and pl.shape[0] > 0 else None

    @property
    def n_verts(self):
        return self.rest_pos.shape[0]

    @property
    def n_tets(self):
        return self.tets.shape[0]

    def struct(self) -> Problem:
        s = Problem()
        s.n_verts = self.rest_pos.shape[0]
        s.n_tets = self.tets.shape[0]
        s.rest_pos = _d(self.rest_pos)
        s.tets = _i(self.tets)
        s.model = self.model
        s.mu = self.mu
        s.lambda_ = self.lam
        s.mu_tet = _d(self.mu_tet)
        s.lambda_tet = _d(self.lam_tet)
        s.density = self.density
        s.gravity = (C.c_double * 3)(*self.gravity)
        s.nodal_force = _d(self.nodal_force)
        s.n_dirichlet = self.dirichlet_idx.size
        s.dirichlet_idx = _i(self.dirichlet_idx)
        s.dirichlet_x = _d(self.dirichlet_x)
        s.n_wc = 0 if self.wc_ptr is None else self.wc_ptr.size - 1
        s.wc_ptr = _i(self.wc_ptr)
        s.wc_vert = _i(self.wc_vert)
        s.wc_w = _d(self.wc_w)
        s.wc_K = _d(self.wc_K)
        s.n_planes = 0 if self.planes is None else self.planes.shape[0]
        s.planes = _d(self.planes)
        return s


def problem_from_scenario(sc) -> HostProblem:
    """Marshal a ``scenarios.Scenario``; (E, nu) go through the library's
    Lame conversion."""
    mu, lam = lame(sc.E, sc.nu)
    return HostProblem(sc.rest_pos, sc.tets, sc.model, mu, lam, sc.dirichlet_idx, sc.dirichlet_x,
                       density=sc.density, gravity=sc.gravity, nodal_force=sc.nodal_force,
                       wc_ptr=sc.wc_ptr, wc_vert=sc.wc_vert, wc_w=sc.wc_w, wc_K=sc.wc_K,
                       planes=sc.planes)


def color(problem: HostProblem):
    """pbng_color: (colors int32 [n_verts], n_colors)."""
    s = problem.struct()
    out = np.zeros(problem.n_verts, np.int32)
    n = C.c_int32()
    _check(lib().pbng_color(C.byref(s), _i(out), C.byref(n)))
    return out, n.value


def solve_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    _check(lib().pbng_default_solve_opts(C.byref(o)))
    for k, v in kw.items():
        if k == "accel":
            v = ACCEL[v] if isinstance(v, str) else v
        if k == "safeguard":
            v = SAFEGUARD[v] if isinstance(v, str) else v
        setattr(o, k, v)
    return o


def adjoint_opts(**kw) -> AdjointOpts:
    o = AdjointOpts()
    _check(lib().pbng_default_adjoint_opts(C.byref(o)))
    for k, v in kw.items():
        if k == "accel":
            v = ACCEL[v] if isinstance(v, str) else v
        setattr(o, k, v)
    return o


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Workspace:
    """pbng_workspace: packed device copy of one or more problems."""

    def __init__(self, problems: Sequence[HostProblem], colors: Optional[np.ndarray] = None,
                 real: str = "f32"):
        self.problems = list(problems)
        n = len(self.problems)
        arr = (Problem * n)(*[p.struct() for p in self.problems])
        self._structs = arr
        cols = None if colors is None else np.ascontiguousarray(colors, np.int32)
        h = C.c_void_p()
        _check(lib().pbng_workspace_create(arr, n, _i(cols), REAL[real], C.byref(h)))
        self.handle = h
        self.real = real
        nv, nt, nf, nvis = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        nc, ni = C.c_int32(), C.c_int32()
        _check(lib().pbng_workspace_info(h, C.byref(nv), C.byref(nt), C.byref(nf), C.byref(nc),
                                         C.byref(nvis), C.byref(ni)))
        self.n_verts, self.n_tets, self.n_free = nv.value, nt.value, nf.value
        self.n_colors, self.n_visits, self.n_instances = nc.value, nvis.value, ni.value

    def close(self):
        if getattr(self, "handle", None):
            lib().pbng_workspace_destroy(self.handle)
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
        if x.dtype != self.dtype or tuple(x.shape) != (self.n_verts, 3) or not x.is_contiguous():
            raise ValueError("positions must be a contiguous [%d, 3] %s tensor"
                             % (self.n_verts, self.dtype))

    def solve(self, x, opts: Optional[SolveOpts] = None, stream=None, **kw):
        """In-place solve of x ([n_verts, 3] cuda tensor of the workspace
        dtype).  Returns (status, [per-instance stats dict])."""
        self._check_x(x)
        o = opts if opts is not None else solve_opts(**kw)
        st = (Stats * self.n_instances)()
        rc = _check(lib().pbng_solve(self.handle, _ptr(x), C.byref(o), st, _stream(stream)))
        return rc, [s.to_dict() for s in st]

    def residual(self, x, want_r: bool = False, stream=None):
        """FP64 (||r|| per instance, energy per instance[, r tensor])."""
        import torch
        self._check_x(x)
        res = np.zeros(self.n_instances)
        en = np.zeros(self.n_instances)
        r = torch.zeros((self.n_verts, 3), dtype=torch.float64, device=x.device) if want_r else None
        _check(lib().pbng_residual(self.handle, _ptr(x), _d(res), _d(en), _ptr(r), _stream(stream)))
        return (res, en, r) if want_r else (res, en)

    def adjoint(self, x_eq, dL_dx, opts: Optional[AdjointOpts] = None, stream=None,
                want=("xd", "mu", "lam", "lam_vec"), **kw):
        """pbng_adjoint; returns (status, outputs dict, [stats])."""
        import torch
        self._check_x(x_eq)
        self._check_x(dL_dx)
        dev = x_eq.device
        nd = sum(p.dirichlet_idx.size for p in self.problems)
        out = {}
        if "xd" in want:
            out["xd"] = torch.zeros((nd, 3), dtype=torch.float64, device=dev)
        if "mu" in want:
            out["mu"] = torch.zeros(self.n_tets, dtype=torch.float64, device=dev)
        if "lam" in want:
            out["lam"] = torch.zeros(self.n_tets, dtype=torch.float64, device=dev)
        if "lam_vec" in want:
            out["lam_vec"] = torch.zeros((self.n_verts, 3), dtype=torch.float64, device=dev)
        o = opts if opts is not None else adjoint_opts(**kw)
        st = (Stats * self.n_instances)()
        rc = _check(lib().pbng_adjoint(self.handle, _ptr(x_eq), _ptr(dL_dx), _ptr(out.get("xd")),
                                       _ptr(out.get("mu")), _ptr(out.get("lam")),
                                       _ptr(out.get("lam_vec")), C.byref(o), st, _stream(stream)))
        return rc, out, [s.to_dict() for s in st]

    def set_materials(self, mu, lam, stream=None):
        import torch
        for t in (mu, lam):
            if t.dtype != torch.float64 or not t.is_cuda or t.numel() != self.n_tets:
                raise ValueError("materials must be float64 cuda tensors of %d tets" % self.n_tets)
        _check(lib().pbng_workspace_set_materials(self.handle, _ptr(mu.contiguous()),
                                                  _ptr(lam.contiguous()), _stream(stream)))

    def set_dirichlet(self, xd, stream=None):
        import torch
        if xd.dtype != torch.float64 or not xd.is_cuda:
            raise ValueError("Dirichlet targets must be a float64 cuda tensor")
        _check(lib().pbng_workspace_set_dirichlet(self.handle, _ptr(xd.contiguous()),
                                                  _stream(stream)))

    def set_inertia(self, dt, x_n=None, x_prev=None, stream=None):
        """Backward-Euler inertia with time step dt and xhat = 2 x^n - x^{n-1}
        (float64 cuda tensors [n_verts, 3], caller order); dt <= 0 turns it
        off."""
        import torch
        if dt > 0:
            for t in (x_n, x_prev):
                if t is None or t.dtype != torch.float64 or not t.is_cuda or \
                        t.numel() != 3 * self.n_verts:
                    raise ValueError("x^n and x^{n-1} must be float64 cuda tensors [%d, 3]"
                                     % self.n_verts)
            x_n, x_prev = x_n.contiguous(), x_prev.contiguous()
            _check(lib().pbng_workspace_set_inertia(self.handle, float(dt), _ptr(x_n),
                                                    _ptr(x_prev), _stream(stream)))
        else:
            _check(lib().pbng_workspace_set_inertia(self.handle, float(dt), None, None,
                                                    _stream(stream)))

    def set_contacts(self, pairs, normals, k_n, stream=None):
        """Vertex-vertex contacts: pairs int32 cuda [n, 2] (caller indices),
        normals float64 cuda [n, 3], stiffness k_n; n = 0 removes them."""
        import torch
        n = int(pairs.shape[0]) if pairs is not None else 0
        if n > 0:
            if pairs.dtype != torch.int32 or not pairs.is_cuda or tuple(pairs.shape) != (n, 2):
                raise ValueError("pairs must be an int32 cuda tensor [n, 2]")
            if normals.dtype != torch.float64 or not normals.is_cuda or \
                    tuple(normals.shape) != (n, 3):
                raise ValueError("normals must be a float64 cuda tensor [n, 3]")
            pairs, normals = pairs.contiguous(), normals.contiguous()
            _check(lib().pbng_workspace_set_contacts(self.handle, n, _ptr(pairs), _ptr(normals),
                                                     float(k_n), _stream(stream)))
        else:
            _check(lib().pbng_workspace_set_contacts(self.handle, 0, None, None, float(k_n),
                                                     _stream(stream)))

    def detect_contacts(self, x, radius, max_pairs=1 << 20, stream=None):
        """Proximity pairs at positions x: (pairs int32 cuda [n, 2], normals
        float64 cuda [n, 3])."""
        import torch
        self._check_x(x)
        pairs = torch.empty((max_pairs, 2), dtype=torch.int32, device=x.device)
        normals = torch.empty((max_pairs, 3), dtype=torch.float64, device=x.device)
        n = C.c_int32(0)
        _check(lib().pbng_detect_contacts(self.handle, _ptr(x), float(radius), int(max_pairs),
                                          _ptr(pairs), _ptr(normals), C.byref(n), _stream(stream)))
        return pairs[:n.value], normals[:n.value]

    def colors(self):
        """Current colour of every vertex (caller order, -1 on Dirichlet)."""
        out = np.zeros(self.n_verts, np.int32)
        _check(lib().pbng_workspace_colors(self.handle, out.ctypes.data_as(_ip)))
        return out

    # measurement access ---------------------------------------------------
    def load(self, x, stream=None):
        self._check_x(x)
        _check(lib().pbng_load(self.handle, _ptr(x), _stream(stream)))

    def store(self, x, stream=None):
        self._check_x(x)
        _check(lib().pbng_store(self.handle, _ptr(x), _stream(stream)))

    def sweeps(self, n, opts: Optional[SolveOpts] = None, stream=None, **kw):
        o = opts if opts is not None else solve_opts(**kw)
        _check(lib().pbng_sweeps(self.handle, n, C.byref(o), _stream(stream)))

    def phase(self, color_idx, opts: Optional[SolveOpts] = None, stream=None, **kw):
        o = opts if opts is not None else solve_opts(**kw)
        _check(lib().pbng_phase(self.handle, color_idx, C.byref(o), _stream(stream)))

    def autotune(self, x, opts: Optional[SolveOpts] = None, stream=None, **kw):
        """pbng_autotune: returns (tuned SolveOpts, lanes per colour)."""
        self._check_x(x)
        o = opts if opts is not None else solve_opts(**kw)
        tuned = SolveOpts()
        lanes = np.zeros(self.n_colors, np.int32)
        _check(lib().pbng_autotune(self.handle, _ptr(x), C.byref(o), C.byref(tuned), _i(lanes),
                                   _stream(stream)))
        return tuned, lanes

    def phase_bytes(self, color_idx):
        b, v, k = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().pbng_phase_bytes(self.handle, color_idx, C.byref(b), C.byref(v), C.byref(k)))
        return b.value, v.value, k.value


def concat_positions(xs: Sequence[np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(x, np.float64).reshape(-1, 3) for x in xs])
