"""Host-only contracts (no GPU): the product path refuses to run without the
HIP library instead of falling back to anything on the CPU, and bench.py
measures one GPU only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(code, env):
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=300)


def test_missing_library_fails_loudly(tmp_path):
    env = dict(os.environ, PBNG_LIBRARY=str(tmp_path / "absent" / "libpbng.so"))
    code = ("import sys\n"
            "from paper_2306_09021_amd import pbng, pbng2d, scenarios as S\n"
            "fails = 0\n"
            "for f in (pbng.lib, pbng2d.lib, lambda: pbng.color(pbng.problem_from_scenario(S.twist_box(3, 'nh', 1e4, 0.3, 0.0, 1.0, 0.0))),\n"
            "          lambda: pbng2d.color(pbng2d.problem_from_scenario(S.stretched_square(5, 'nh', 1.2)))):\n"
            "    try:\n"
            "        f()\n"
            "    except RuntimeError as e:\n"
            "        fails += 'not built' in str(e)\n"
            "print(fails)\n"
            "sys.exit(0 if fails == 4 else 1)\n")
    out = _run(code, env)
    assert out.returncode == 0, out.stdout + out.stderr


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 2
    assert "one GPU" in out.stderr and out.stdout == ""
