"""Helpers shared by the GPU tests: build workspaces from scenarios, move
positions between numpy and torch, and name every case before it runs."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2306_09021_amd import pbng

torch = pytest.importorskip("torch")


def announce(msg):
    print("[gpu-case] %s" % msg, flush=True)
    sys.stdout.flush()


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pbng.lib()  # raises if the HIP library is missing: no silent fallback


def dev_x(x, real):
    dt = torch.float32 if real == "f32" else torch.float64
    return torch.tensor(np.asarray(x, np.float64).reshape(-1, 3), dtype=dt, device="cuda").contiguous()


def host(t):
    return t.detach().double().cpu().numpy()


def workspace(scs, real, colors=None):
    hps = [pbng.problem_from_scenario(s) for s in scs]
    return pbng.Workspace(hps, colors=colors, real=real)


def oracle_solve(sc, sweeps, **kw):
    op = O.make_problem(sc)
    col, _ = O.color(op)
    x, st = O.solve(op, col, sc.initial_iterate(), max_sweeps=sweeps, **kw)
    return x, st, op


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def disp_err(a, b, X):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b - X), 1e-300))
