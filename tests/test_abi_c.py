"""The C ABI from C: a C99 program including include/pbng.h and
include/pbng2d.h compiles with -Wall -Werror, links libpbng.so and runs its
host-only entry points (no GPU)."""
import os
import shutil
import subprocess

import pytest

from paper_2306_09021_amd import pbng

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_caller_compiles_links_and_runs(tmp_path):
    lib = pbng.LIB_PATH
    if not os.path.exists(lib):
        pytest.skip("libpbng.so is not built")
    exe = str(tmp_path / "abi_host")
    libdir = os.path.dirname(lib)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-o", exe,
                           os.path.join(ROOT, "tests", "c", "abi_host.c"), "-I" + os.path.join(ROOT, "include"),
                           "-L" + libdir, "-l:libpbng.so", "-Wl,-rpath," + libdir, "-lm"])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "FAIL" not in out.stdout


@pytest.mark.gpu
@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_caller_solves_on_the_gpu(tmp_path):
    """A C99 program with device memory from the HIP runtime and no Python
    binding solves a twisted box through libpbng (FP64, 30 sweeps with the
    safeguard); its positions and residual match the oracle's."""
    import numpy as np

    import oracle as O
    from paper_2306_09021_amd import scenarios as S
    from tests.gpu_util import require_gpu
    require_gpu()
    lib = pbng.LIB_PATH
    exe = str(tmp_path / "abi_gpu")
    libdir = os.path.dirname(lib)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__", "-o", exe,
                           os.path.join(ROOT, "tests", "c", "abi_gpu.c"), "-I" + os.path.join(ROOT, "include"),
                           "-I/opt/rocm/include", "-L" + libdir, "-l:libpbng.so", "-Wl,-rpath," + libdir,
                           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    sc = S.twist_box(6, "corotated", 1e4, 0.3, 60.0, 1.2, 0.01, seed=2)
    mu, lam = O.lame(float(sc.E), float(sc.nu))
    inp, outp = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(inp, "wb") as f:
        f.write(np.array([sc.n_verts, sc.n_tets, sc.dirichlet_idx.size, 1], np.int32).tobytes())
        f.write(np.array([mu, lam], np.float64).tobytes())
        f.write(np.ascontiguousarray(sc.rest_pos, np.float64).tobytes())
        f.write(np.ascontiguousarray(sc.tets, np.int32).tobytes())
        f.write(np.ascontiguousarray(sc.dirichlet_idx, np.int32).tobytes())
        f.write(np.ascontiguousarray(sc.dirichlet_x, np.float64).tobytes())
        f.write(np.ascontiguousarray(sc.initial_iterate(), np.float64).tobytes())
    print("[gpu-case] C caller twist6 corotated f64", flush=True)
    out = subprocess.run([exe, inp, outp, "30"], capture_output=True, text=True, timeout=120)
    print(out.stdout, out.stderr)
    assert out.returncode == 0
    res = np.fromfile(outp, np.float64)
    xg = res[:3 * sc.n_verts].reshape(-1, 3)
    op = O.make_problem(sc)
    col, ncol = O.color(op)
    xo, _ = O.solve(op, col, sc.initial_iterate(), max_sweeps=30, safeguard="backtrack")
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)
    ro = O.residual(op, xo)[0]
    assert abs(res[-2] - ro) <= 1e-8 * ro and int(res[-1]) == ncol
