"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2306_09021_amd.profsum counters --fetch DIR --write DIR \\
      --copy-mib 512 --last 100 --json OUT.json --md OUT.md --cmd-fetch "..." --cmd-write "..."
  python -m paper_2306_09021_amd.profsum stats --stats DIR --md OUT.md --cmd "..." [--top 12]

`counters` scales the per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the
colour-phase kernel by what the same counters read for a device-to-device
copy of known size (the copies that `bench.py --copy-calibration` issues
first), averages the last `--last` dispatches (the roofline sweeps that end
a `bench.py` run) and records the SHA-256 of the kernel sources, so that
`bench.py` reports the traffic only while the kernel is unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# sources that define each profiled kernel (a change to any of them makes the
# counter profile stale)
KERNEL_SOURCES = {
    "k_phase": ["pbng_kernels.hip", "pbng_math.hpp", "pbng_internal.hpp", "pbng_device.hpp"],
    "k2_phase": ["pbng2d_kernels.hip", "pbng2d.hpp", "pbng_math.hpp", "pbng_internal.hpp",
                 "pbng_device.hpp"],
}


def kernel_sources_sha256(kernel: str = "k_phase") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _rows(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _dispatches(d: str, counter: str):
    """(dispatch id, kernel name, grid, value) in dispatch order."""
    out = {}
    for r in _rows(d, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        k = int(r["Dispatch_Id"])
        v = float(r["Counter_Value"])
        if k in out:
            out[k] = (out[k][0], out[k][1], out[k][2] + v)   # summed over dimensions
        else:
            out[k] = (r["Kernel_Name"], int(r["Grid_Size"]), v)
    return [(k,) + out[k] for k in sorted(out)]


def _copy_scale(disp, copy_kib: float, counter: str) -> float:
    vals = [v for _, name, _, v in disp if "copyBuffer" in name and v > 0.25 * copy_kib]
    if not vals:
        raise RuntimeError("no calibration copy found for %s" % counter)
    return copy_kib / (sum(vals) / len(vals)), vals


def counters(a):
    copy_kib = a.copy_mib * 1024.0
    fetch = _dispatches(a.fetch, "FETCH_SIZE")
    write = _dispatches(a.write, "WRITE_SIZE")
    fs, fvals = _copy_scale(fetch, copy_kib, "FETCH_SIZE")
    ws, wvals = _copy_scale(write, copy_kib, "WRITE_SIZE")
    fk = [d for d in fetch if (a.kernel + "<") in d[1]][-a.last:]
    wk = [d for d in write if (a.kernel + "<") in d[1]][-a.last:]
    if len(fk) < a.last or len(wk) < a.last:
        raise RuntimeError("fewer than %d %s dispatches" % (a.last, a.kernel))
    f_mean = sum(d[3] for d in fk) / len(fk) * 1024.0 * fs
    w_mean = sum(d[3] for d in wk) / len(wk) * 1024.0 * ws
    res = {"kernel": a.kernel + " " + a.workload, "sources": KERNEL_SOURCES[a.kernel],
           "sources_sha256": kernel_sources_sha256(a.kernel), "fetch_scale": fs, "write_scale": ws,
           "fetch_bytes_per_launch": f_mean, "write_bytes_per_launch": w_mean,
           "traffic_bytes_per_launch": f_mean + w_mean, "launches": a.last}
    with open(a.json, "w") as f:
        json.dump(res, f, indent=1)

    def table(rows, scale, title):
        agg = {}
        for _, name, grid, v in rows:
            key = (name, grid)
            n, s = agg.get(key, (0, 0.0))
            agg[key] = (n + 1, s + v)
        out = ["| %s: kernel | grid | dispatches | raw KiB per launch | scaled MB per launch |" % title,
               "|---|---|---|---|---|"]
        for (name, grid), (n, s) in agg.items():
            out.append("| `%s` | %d | %d | %.0f | %.2f |" % (short_name(name), grid, n, s / n,
                                                            s / n * 1024 * scale / 1e6))
        return out

    lines = ["# HBM counters: %s on the %s" % (a.kernel, a.workload), "",
             "Commands (one counter per pass, from the repository root):", "",
             "    " + a.cmd_fetch, "    " + a.cmd_write, "",
             "Calibration: each %d MiB device-to-device copy (`copyBuffer`) reads FETCH_SIZE = %s KiB "
             "and WRITE_SIZE = %s KiB for %d KiB read and written: read scale %.3f, write scale %.3f."
             % (a.copy_mib, ", ".join("%.0f" % v for v in fvals), ", ".join("%.0f" % v for v in wvals),
                copy_kib, fs, ws), "",
             "The last %d `%s` dispatches of each pass (the roofline sweeps of `bench.py`):" % (a.last, a.kernel),
             ""]
    lines += table(fk, fs, "FETCH_SIZE") + [""] + table(wk, ws, "WRITE_SIZE") + [""]
    lines.append("Average scaled traffic per launch: %.2f MB read + %.2f MB written = %.2f MB; "
                 "sources SHA-256 %s." % (f_mean / 1e6, w_mean / 1e6, (f_mean + w_mean) / 1e6,
                                         res["sources_sha256"][:16]))
    with open(a.md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(res))


def short_name(name: str) -> str:
    """Kernel name without return type, anonymous namespace and arguments."""
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0]


def stats(a):
    rows = _rows(a.stats, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["Percentage"]))
    lines = ["# %s" % a.title, "", "Command (from the repository root, one MI355X):", "", "    " + a.cmd, "",
             "Kernel statistics (`kernel_stats.csv`), top %d by total time:" % a.top, "",
             "| kernel | calls | avg ns | % time |", "|---|---|---|---|"]
    for r in rows[:a.top]:
        lines.append("| `%s` | %s | %.0f | %.2f |" % (short_name(r["Name"]), r["Calls"],
                                                     float(r["AverageNs"]), float(r["Percentage"])))
    if a.match:
        sel = [r for r in rows if a.match in r["Name"]]
        calls = sum(int(r["Calls"]) for r in sel)
        tot = sum(float(r["TotalDurationNs"]) for r in sel)
        lines += ["", "All `%s` variants: %d calls, average %.0f ns." % (a.match, calls,
                                                                        tot / max(calls, 1))]
        lines += ["", "| variant | calls | avg ns |", "|---|---|---|"]
        for r in sel:
            lines.append("| `%s` | %s | %.0f |" % (short_name(r["Name"]), r["Calls"],
                                                  float(r["AverageNs"])))
    with open(a.md, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--copy-mib", type=int, default=512)
    c.add_argument("--last", type=int, default=100)
    c.add_argument("--kernel", default="k_phase")
    c.add_argument("--workload", default="128x32x32 beam, FP32")
    c.add_argument("--json", required=True)
    c.add_argument("--md", required=True)
    c.add_argument("--cmd-fetch", default="")
    c.add_argument("--cmd-write", default="")
    s = sub.add_parser("stats")
    s.add_argument("--stats", required=True)
    s.add_argument("--md", required=True)
    s.add_argument("--cmd", default="")
    s.add_argument("--title", default="Kernel statistics")
    s.add_argument("--top", type=int, default=12)
    s.add_argument("--match", default="")
    a = ap.parse_args()
    counters(a) if a.mode == "counters" else stats(a)


if __name__ == "__main__":
    main()
