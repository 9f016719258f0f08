"""Build libpbng.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2306_09021_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpbng.so")
# (source, extra defines, object name): the kernel file is compiled once per
# instantiation set, in parallel
UNITS = [("pbng_kernels.hip", ["-DPBNG_KERNEL_SET=0"], "kernels_f32.o"),
         ("pbng_kernels.hip", ["-DPBNG_KERNEL_SET=1"], "kernels_f64.o"),
         ("pbng_kernels.hip", ["-DPBNG_KERNEL_SET=2"], "kernels_mixed.o"),
         ("pbng_contacts.hip", [], "contacts.o"),
         ("pbng_upload.hip", [], "upload.o"),
         ("pbng2d_kernels.hip", [], "planar_kernels.o"),
         ("pbng_host.cpp", [], "host.o"),
         ("pbng2d_host.cpp", [], "planar_host.o")]
ARCH = os.environ.get("PBNG_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# keep the compiler from forming packed FP32 instructions
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (p.stdout + p.stderr).splitlines()
                    if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if p.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(verbose: bool = False, out: str = LIB, extra=()) -> str:
    """Compile every source and link libpbng.so (or `out`); always
    recompiles.  `extra` adds compiler flags (e.g. -D switches)."""
    from concurrent.futures import ThreadPoolExecutor
    objs = []
    cmds = []
    bdir = os.path.join(HERE, "_build", os.path.basename(out))
    os.makedirs(bdir, exist_ok=True)
    for src, defs, oname in UNITS:
        obj = os.path.join(bdir, oname)
        cmd = ["hipcc", "-c"] + (["-x", "hip"] if src.endswith(".hip") else [])
        cmd += [os.path.join(CSRC, src), "-o", obj] + COMMON + defs + list(extra)
        cmd += DEVICE if src.endswith(".hip") else ["-D__HIP_PLATFORM_AMD__"]
        cmds.append(cmd)
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(7, os.cpu_count() or 1)) as ex:
        for log in ex.map(_run, cmds):
            if verbose and log.strip():
                print(log)
    tmp = out + ".tmp%d" % os.getpid()
    _run(["hipcc", "-shared", "-o", tmp] + objs + DEVICE + ["-lamdhip64"])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "-v"]
    out = LIB
    extra = []
    for a in args:
        if a.startswith("--out="):
            out = os.path.abspath(a[len("--out="):])
        else:
            extra.append(a)
    print(build(verbose="-v" in sys.argv, out=out, extra=extra))
