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
