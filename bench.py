"""Benchmark of the PBNG hot path on one MI355X.

Headline workload: the 128x32x32-vertex cantilever beam (131,072 vertices,
610,235 tets, Neo-Hookean E = 1e5, nu = 0.45, gravity at density 1000, x = 0
face pinned), FP32 sweeps with FP64 residuals, SOR omega = 1.6 across
sweeps, safeguarded local steps, run to 1e-5 relative residual or 2000
sweeps.  One step = one whole solve from the initial iterate (sweeps with
the fused blend, FP64 residual checks), with the packed problem resident in
HBM.  Lanes per colour and sweeps per graph come from the library's
autotuner, run before the timed region.

Prints one JSON line: vertex updates per second over the timed steps, the
roofline of the dominant kernel (the colour-phase vertex update) measured
live with HIP events on the launch stream, the FP64 oracle timed on the host
cores on a bounded sample, and sub-reports: the beam's time to 1e-5 with FP64
master positions, batched cubes (one batched
solve against per-instance solves, time to 1e-5), the differentiable cubes
(forward and adjoint sweeps), the muscles, the paper's blocks, backward
Euler, collisions and the planar (triangle-mesh) square.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "k_phase_beam_128x32x32_f32_counters.json")
PLANAR_COUNTERS = os.path.join(ROOT, "profiles", "k2_phase_square_1025x1025_f32_counters.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--check-every", type=int, default=50)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and differentiable sub-reports")
    ap.add_argument("--cpu-sweeps", type=int, default=300)
    ap.add_argument("--roofline-sweeps", type=int, default=20)
    ap.add_argument("--max-sweeps", type=int, default=0,
                    help="override the sweep cap (short profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB: run device-to-device copies of this size first, so that a "
                         "counter profile holds a plain copy kernel of known traffic")
    ap.add_argument("--batched-subset", type=int, default=32,
                    help="instances solved one by one for the per-instance comparison")
    ap.add_argument("--diff-instances", type=int, default=64)
    ap.add_argument("--planar-only", action="store_true",
                    help="run only the planar (triangle-mesh) report and print it (profiling)")
    ap.add_argument("--planar-sweeps", type=int, default=200)
    ap.add_argument("--only", default="",
                    help="run only these sub-reports (comma-separated: batched, backward_euler, ...) "
                         "and print them (profiling)")
    return ap.parse_args()


def progress(msg):
    """One line per finished part of the run, on stderr (the JSON line is the
    only stdout output)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def traffic_per_launch(path=COUNTERS, kernel="k_phase"):
    """(HBM bytes per launch of `kernel`, note) from its committed counter
    profile; bytes are None when the kernel sources changed since it was
    taken (or there is no profile)."""
    try:
        with open(path) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None, "no counter profile"
    from paper_2306_09021_amd.profsum import kernel_sources_sha256
    if c.get("sources_sha256") != kernel_sources_sha256(kernel):
        return None, "kernel changed since the counter profile was taken"
    note = ("bytes per launch from rocprofv3 FETCH_SIZE x%.3f + WRITE_SIZE x%.3f (scales from a copy "
            "of known size)" % (c["fetch_scale"], c["write_scale"]))
    return c.get("traffic_bytes_per_launch"), note


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver's multi-GPU path is not part of this "
              "build (independent instances would shard without communication). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2306_09021_amd import pbng
    from paper_2306_09021_amd import scenarios as S

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()          # default priority; non-null so graphs can be captured
    torch.cuda.set_stream(stream)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.planar_only:
        print(json.dumps({"planar": planar_report(torch, stream, sweeps=args.planar_sweeps)}))
        return
    if args.only:
        from paper_2306_09021_amd import pbng
        from paper_2306_09021_amd import scenarios as S
        reports = sub_reports(args, pbng, S, torch, stream)
        names = args.only.split(",")
        unknown = [n for n in names if n not in reports]
        if unknown:
            print("unknown sub-report(s) %r" % unknown, file=sys.stderr)
            sys.exit(2)
        print(json.dumps({n: reports[n]() for n in names}))
        return

    sc = S.config_beam_f32()
    # SOR omega = 1.6: the Chebyshev rho = 0.995 / relaxation 1.6 reading
    # diverges on this beam in exact arithmetic (oracle and GPU agree)
    sopts = dict(max_sweeps=2000, rel_tol=1e-5, accel="sor", omega=1.6, safeguard="backtrack")
    if args.max_sweeps > 0:
        sopts["max_sweeps"] = args.max_sweeps
    cfg = {"workload": "beam_128x32x32_neohookean_gravity", "vertices": sc.n_verts,
           "tets": sc.n_tets, "free_vertices": sc.n_free, "constitutive_model": "neo-hookean",
           "E": 1e5, "nu": 0.45, "density": 1000.0, "accel": "sor omega=1.6",
           "safeguard": "backtrack", "rel_tol": 1e-5, "max_sweeps": sopts["max_sweeps"],
           "positions": "f32", "sweep_arithmetic": "f32", "residual": "f64"}
    ws = pbng.Workspace([pbng.problem_from_scenario(sc)], real="f32")
    x0 = torch.tensor(sc.initial_iterate(), dtype=torch.float32, device="cuda")
    x = x0.clone()
    opts = pbng.solve_opts(check_every=args.check_every, **sopts)
    if not args.no_autotune:
        opts, lanes = ws.autotune(x0, opts, stream=stream)
        cfg["lanes_per_colour"] = [int(v) for v in lanes]
        cfg["sweeps_per_graph"] = int(opts.sweeps_per_graph)

    def step():
        x.copy_(x0)
        return ws.solve(x, opts, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        rc, st = step()
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    updates = sum(sum(s["vertex_updates"] for s in st) for st in stats)
    last = stats[-1]
    value = updates / elapsed

    # roofline of the dominant kernel (the colour-phase vertex update, same
    # variant as the solve): HIP events on the launch stream bracket
    # back-to-back sweeps of launches, so the average launch duration is the
    # kernel time plus the (sub-microsecond) gaps between dependent launches
    ws.load(x0, stream=stream)
    n_col = ws.n_colors
    ws.sweeps(3, opts, stream=stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.roofline_sweeps):
        for c in range(n_col):
            ws.phase(c, opts, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    n_launch = args.roofline_sweeps * n_col
    avg_dur = ev0.elapsed_time(ev1) * 1e-3 / n_launch
    total_bytes = 0
    for c in range(n_col):
        b, v, k = ws.phase_bytes(c)
        total_bytes += args.roofline_sweeps * (b + 48 * v)
    avg_bytes = total_bytes / n_launch
    achieved = avg_bytes / avg_dur / 1e9
    tr, tr_note = traffic_per_launch()
    copy_big = copy_bandwidth(torch, stream, 1 << 30, 10)
    copy_same = copy_bandwidth(torch, stream, int(avg_bytes), n_launch)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (int(tr) if tr is not None else None),
                "traffic_note": tr_note,
                "kernel": "k_phase (colour-phase vertex update)",
                "avg_launch_us": round(avg_dur * 1e6, 2),
                "avg_algorithmic_bytes": int(avg_bytes), "launches_timed": n_launch,
                "copy_GBs_1GiB": round(copy_big, 1),
                "frac_of_copy_1GiB": round(achieved / copy_big, 4),
                "copy_GBs_same_bytes_per_launch": round(copy_same, 1),
                "frac_of_copy_same_bytes": round(achieved / copy_same, 4)}

    progress("beam: %.3e vertex updates/s, k_phase %.2f us per launch" % (value, avg_dur * 1e6))
    cpu = None if args.no_cpu_baseline else cpu_baseline(sc, args.cpu_sweeps)
    if cpu:
        progress("cpu baseline: %.3e vertex updates/s" % cpu["value"])
    extras = {}
    if not args.no_extras:
        for name, fn in sub_reports(args, pbng, S, torch, stream).items():
            # a failing sub-report is recorded, not fatal to the headline line
            try:
                extras[name] = fn()
            except Exception as e:  # noqa: BLE001
                extras[name] = {"error": "%s: %s" % (type(e).__name__, e)}
            torch.cuda.synchronize()
            progress("%s report done" % name)

    sweeps = max(s["sweeps"] for s in last)
    line = {
        "metric": "vertex-updates/s & time to 1e-5 rel residual; batched+adjoint vs plain",
        "value": round(value, 1),
        "unit": "vertex updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator; no dataset)",
        "config": cfg,
        "sweeps_per_step": sweeps,
        "converged": bool(all(s["converged"] for s in last)),
        "rel_residual_fp64": max(s["rel_residual"] for s in last),
        "time_to_tol_ms": (max(s["time_to_tol_ms"] for s in last)
                           if all(s["converged"] for s in last) else None),
        "energy_fp64": sum(s["energy"] for s in last),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extras)
    print(json.dumps(line))


def beam_to_tol_report(pbng, S, torch, stream, max_sweeps=40000):
    """Time to 1e-5 relative residual on the headline beam.  With FP32
    positions the FP64 residual of the beam stalls near 0.8 (position
    rounding makes force noise above its small gravity load), so the same
    configuration (SOR omega = 1.6, safeguard) runs in PBNG_MIXED: an FP64
    master copy of the positions with FP32 sweep arithmetic."""
    sc = S.config_beam_f32()
    ws = pbng.Workspace([pbng.problem_from_scenario(sc)], real="mixed")
    x0 = torch.tensor(sc.initial_iterate(), dtype=torch.float64, device="cuda")
    opts = pbng.solve_opts(max_sweeps=max_sweeps, rel_tol=1e-5, check_every=100, accel="sor", omega=1.6,
                           safeguard="backtrack")
    opts, lanes = ws.autotune(x0, opts, stream=stream)
    x = x0.clone()
    ws.solve(x, pbng.solve_opts(max_sweeps=200, rel_tol=0.0, check_every=200, accel="sor", omega=1.6,
                                safeguard="backtrack"), stream=stream)          # warm-up
    x.copy_(x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ws.solve(x, opts, stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s0 = st[0]
    return {"workload": "beam_128x32x32_neohookean_gravity", "real": "mixed", "accel": "sor omega=1.6",
            "rel_tol": 1e-5, "max_sweeps": max_sweeps, "converged": bool(s0["converged"]),
            "sweeps": s0["sweeps"], "rel_residual_fp64": s0["rel_residual"],
            "time_to_tol_ms": (round(s0["time_to_tol_ms"], 2) if s0["converged"] else None),
            "wall_s": round(el, 4), "vertex_updates_per_s": round(s0["vertex_updates"] / el, 1),
            "lanes_per_colour": [int(v) for v in lanes], "sweeps_per_graph": int(opts.sweeps_per_graph)}


def sub_reports(args, pbng, S, torch, stream):
    """The sub-reports of the bench line, in order, by name."""
    return {"beam_to_tol": lambda: beam_to_tol_report(pbng, S, torch, stream),
            "batched": lambda: batched_report(pbng, S, torch, stream, args.batched_subset),
            "differentiable": lambda: differentiable_report(pbng, S, torch, stream, args.diff_instances),
            "muscles": lambda: muscles_report(pbng, S, torch, stream),
            "paper_blocks": lambda: paper_boxes_report(pbng, S, torch, stream),
            "backward_euler": lambda: dynamics_report(pbng, S, torch, stream),
            "collisions": lambda: collision_report(pbng, S, torch, stream),
            "planar": lambda: planar_report(torch, stream, sweeps=args.planar_sweeps),
            "planar_terms": lambda: planar_terms_report(torch, stream)}


def batched_report(pbng, S, torch, stream, subset):
    """Batched cubes (256, n ~ U{4..32}, corotated, MIXED: FP32 sweeps on
    FP64 positions): one batched solve to 1e-5; then a seeded subset solved
    once batched and once instance by instance."""
    scs = S.config_batched()
    so = dict(max_sweeps=20000, rel_tol=1e-5, check_every=100, accel="chebyshev", rho=0.95,
              gamma=1.7, safeguard="backtrack")
    out = {"instances": len(scs), "vertices": int(sum(s.n_verts for s in scs)),
           "tets": int(sum(s.n_tets for s in scs)), "real": "mixed",
           "accel": "chebyshev rho=0.95 gamma=1.7", "rel_tol": 1e-5, "max_sweeps": 20000}
    ws = pbng.Workspace([pbng.problem_from_scenario(s) for s in scs], real="mixed")
    x0 = torch.tensor(pbng.concat_positions([s.initial_iterate() for s in scs]),
                      dtype=torch.float64, device="cuda")
    opts = pbng.solve_opts(**so)
    opts, _ = ws.autotune(x0, opts, stream=stream)
    x = x0.clone()
    ws.solve(x, opts, stream=stream)   # warm
    x.copy_(x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ws.solve(x, opts, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    conv = [s for s in st if s["converged"]]
    out.update({"wall_s": round(t, 3), "converged": len(conv),
                "time_to_tol_all_converged_ms": round(max(s["time_to_tol_ms"] for s in conv), 1)
                if conv else None,
                "vertex_updates_per_s": round(sum(s["vertex_updates"] for s in st) / t, 1),
                "not_converged_rel_residual": [round(s["rel_residual"], 8) for s in st
                                               if not s["converged"]]})
    # the batched sweep's roofline: back-to-back sweeps (all instances in
    # every colour phase) timed with HIP events on the launch stream, over
    # the algorithmic bytes of the phases plus the blend
    ws.load(x0, stream=stream)
    ws.sweeps(3, opts, stream=stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    n_sw = 10
    ev0.record(stream)
    ws.sweeps(n_sw, opts, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    sweep_s = ev0.elapsed_time(ev1) * 1e-3 / n_sw
    per_sweep = sum(ws.phase_bytes(c)[0] + 48 * ws.phase_bytes(c)[1] for c in range(ws.n_colors))
    out["sweep"] = {"ms": round(sweep_s * 1e3, 4), "colours": ws.n_colors,
                    "algorithmic_bytes": int(per_sweep),
                    "achieved_GBs": round(per_sweep / sweep_s / 1e9, 1),
                    "frac_of_hbm_peak": round(per_sweep / sweep_s / 1e9 / HBM_PEAK_GBS, 4),
                    "bound": "valu (corotated polar decomposition per visit)"}
    # subset: batched vs one instance at a time
    rng = np.random.default_rng(44)
    idx = sorted(rng.choice(len(scs), size=min(subset, len(scs)), replace=False).tolist())
    sub = [scs[i] for i in idx]
    wsb = pbng.Workspace([pbng.problem_from_scenario(s) for s in sub], real="mixed")
    xb0 = torch.tensor(pbng.concat_positions([s.initial_iterate() for s in sub]),
                       dtype=torch.float64, device="cuda")
    xb = xb0.clone()
    wsb.solve(xb, opts, stream=stream)
    xb.copy_(xb0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rcb, stb = wsb.solve(xb, opts, stream=stream)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    singles = [pbng.Workspace([pbng.problem_from_scenario(s)], real="mixed") for s in sub]
    xs0 = [torch.tensor(s.initial_iterate(), dtype=torch.float64, device="cuda") for s in sub]
    plain = pbng.solve_opts(**so)
    xs = [v.clone() for v in xs0]
    for w, v in zip(singles, xs):
        w.solve(v, plain, stream=stream)
    for v, v0 in zip(xs, xs0):
        v.copy_(v0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts, walls = [], []
    for w, v in zip(singles, xs):
        t1 = time.perf_counter()
        rcs, s1 = w.solve(v, plain, stream=stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t1)
        sts.append(s1[0])
    ts = time.perf_counter() - t0
    # instances that reach the tolerance in both runs (an instance stuck at
    # its FP32-arithmetic floor runs to the sweep cap in both and would
    # dominate both times)
    both = [i for i in range(len(sub)) if stb[i]["converged"] and sts[i]["converged"]]
    t_batched = max(stb[i]["time_to_tol_ms"] for i in both) / 1e3 if both else None
    t_single = sum(walls[i] for i in both) if both else None
    out["subset"] = {"instances": len(sub), "seed": 44,
                     "converged_in_both": len(both),
                     "batched_time_to_tol_s": round(t_batched, 4) if both else None,
                     "per_instance_time_to_tol_s": round(t_single, 4) if both else None,
                     "speedup_time_to_tol": round(t_single / t_batched, 2) if both else None,
                     "batched_wall_s_incl_capped": round(tb, 4),
                     "per_instance_wall_s_incl_capped": round(ts, 4)}
    return out


def differentiable_report(pbng, S, torch, stream, n_inst):
    """Differentiable cubes (32^3, Neo-Hookean, per-tet Lame, MIXED): forward
    solve and adjoint solve to 1e-5 (above their FP32-arithmetic floors) for
    all instances at once."""
    scs = S.config_differentiable(n_inst)
    ws = pbng.Workspace([pbng.problem_from_scenario(s) for s in scs], real="mixed")
    x0 = torch.tensor(pbng.concat_positions([s.initial_iterate() for s in scs]),
                      dtype=torch.float64, device="cuda")
    T = torch.tensor(pbng.concat_positions([s.loss_target for s in scs]), dtype=torch.float64,
                     device="cuda")
    free = np.ones((x0.shape[0], 1))
    off = 0
    for s in scs:
        free[off + s.dirichlet_idx] = 0.0
        off += s.n_verts
    freet = torch.tensor(free, dtype=torch.float64, device="cuda")
    so = pbng.solve_opts(max_sweeps=20000, rel_tol=1e-5, check_every=100, accel="chebyshev",
                         rho=0.98, gamma=1.0, safeguard="backtrack")
    so, _ = ws.autotune(x0, so, stream=stream)
    ao = pbng.adjoint_opts(max_sweeps=20000, rel_tol=1e-5, check_every=100, accel="chebyshev",
                           rho=0.98, gamma=1.0)
    x = x0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ws.solve(x, so, stream=stream)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    g = (2.0 * (x - T) * freet).contiguous()
    t0 = time.perf_counter()
    rca, out, sta = ws.adjoint(x, g, ao, stream=stream, want=("xd", "mu", "lam"))
    torch.cuda.synchronize()
    ta = time.perf_counter() - t0
    fw_upd = sum(s["vertex_updates"] for s in st)
    ad_upd = sum(s["vertex_updates"] for s in sta)
    # roofline of the forward sweep (algorithmic bytes in the FP32 form of
    # the definition: 60 B per visit without the 8 B of per-tet Lame)
    roof = sweep_roofline(ws, x0, so, torch, stream)
    others = {m: _adjoint_model(pbng, S, torch, stream, m, so, ao) for m in ("corotated", "snh")}
    return {"instances": len(scs), "vertices": int(x0.shape[0]), "real": "mixed",
            "forward_sweep_roofline": roof,
            "other_models_8_instances": others,
            "forward": {"rel_tol": 1e-5, "wall_s": round(tf, 3),
                        "converged": int(sum(s["converged"] for s in st)),
                        "max_sweeps_used": int(max(s["sweeps"] for s in st)),
                        "max_rel_residual": max(s["rel_residual"] for s in st),
                        "vertex_updates_per_s": round(fw_upd / tf, 1)},
            "adjoint": {"rel_tol": 1e-5, "wall_s": round(ta, 3),
                        "converged": int(sum(s["converged"] for s in sta)),
                        "max_sweeps_used": int(max(s["sweeps"] for s in sta)),
                        "max_rel_residual": max(s["rel_residual"] for s in sta),
                        "vertex_updates_per_s": round(ad_upd / ta, 1)}}


def _adjoint_model(pbng, S, torch, stream, model, so, ao, n_inst=8):
    """Forward and adjoint solves to 1e-5 for the first n_inst differentiable
    cubes with another model (the adjoint's diagonal blocks are then the
    modified matrices A_ii)."""
    scs = S.config_differentiable(n_inst)
    for sc in scs:
        sc.model = model
    ws = pbng.Workspace([pbng.problem_from_scenario(s) for s in scs], real="mixed")
    x = torch.tensor(pbng.concat_positions([s.initial_iterate() for s in scs]), dtype=torch.float64,
                     device="cuda")
    T = torch.tensor(pbng.concat_positions([s.loss_target for s in scs]), dtype=torch.float64, device="cuda")
    free = np.ones((x.shape[0], 1))
    off = 0
    for s in scs:
        free[off + s.dirichlet_idx] = 0.0
        off += s.n_verts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = ws.solve(x, so, stream=stream)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    g = (2.0 * (x - T) * torch.tensor(free, dtype=torch.float64, device="cuda")).contiguous()
    t0 = time.perf_counter()
    _, _, sta = ws.adjoint(x, g, ao, stream=stream, want=("xd", "mu", "lam"))
    torch.cuda.synchronize()
    ta = time.perf_counter() - t0
    return {"forward_wall_s": round(tf, 3), "forward_converged": int(sum(s["converged"] for s in st)),
            "forward_max_sweeps": int(max(s["sweeps"] for s in st)),
            "adjoint_wall_s": round(ta, 3), "adjoint_converged": int(sum(s["converged"] for s in sta)),
            "adjoint_max_sweeps": int(max(s["sweeps"] for s in sta)),
            "adjoint_max_rel_residual": max(s["rel_residual"] for s in sta)}


def copy_bandwidth(torch, stream, moved_bytes, reps):
    """Device-to-device copy bandwidth (bytes read + bytes written per second)
    of back-to-back copies that each move moved_bytes in total, timed with
    HIP events on the launch stream: the measured ceiling that the phase
    kernels are compared with, once at 1 GiB and once at their own bytes
    per launch."""
    n = max(1, moved_bytes // 8)
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    ev1.record(stream)
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) * 1e-3 / reps
    return 8.0 * n / t / 1e9


def sweep_roofline(ws, x, opts, torch, stream, n_sweeps=10):
    """HBM roofline of a workspace's colour-phase sweeps in its current state
    (inertia, contacts and recolouring included): back-to-back sweeps from x
    timed with HIP events on the launch stream, against the algorithmic
    bytes of the phases (pbng_phase_bytes) plus the blend's 48 bytes per
    vertex.  Leaves the workspace's internal iterate changed."""
    ws.load(x, stream=stream)
    ws.sweeps(2, opts, stream=stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    ws.sweeps(n_sweeps, opts, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) * 1e-3 / n_sweeps
    blend = 48 if opts.accel != 0 else 0
    b = sum(ws.phase_bytes(c)[0] + blend * ws.phase_bytes(c)[1] for c in range(ws.n_colors))
    return {"sweep_us": round(t * 1e6, 2), "algorithmic_bytes_per_sweep": int(b),
            "achieved_GBs": round(b / t / 1e9, 1), "frac_of_hbm_peak": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}


def muscles_report(pbng, S, torch, stream):
    """Muscle stand-in (8 ellipsoids, 320k vertices, per-tet E, binding
    springs, ground contact): 1000 Chebyshev sweeps in FP32 and MIXED."""
    sc = S.config_muscles()
    out = {"vertices": sc.n_verts, "tets": sc.n_tets, "springs": int(sc.wc_ptr.size - 1),
           "accel": "chebyshev rho=0.95 gamma=1.7", "sweeps": 1000}
    for real in ("f32", "mixed"):
        ws = pbng.Workspace([pbng.problem_from_scenario(sc)], real=real)
        dt = torch.float32 if real == "f32" else torch.float64
        x0 = torch.tensor(sc.initial_iterate(), dtype=dt, device="cuda")
        so = pbng.solve_opts(max_sweeps=1000, rel_tol=0.0, check_every=100, accel="chebyshev",
                             rho=0.95, gamma=1.7, safeguard="backtrack")
        so, _ = ws.autotune(x0, so, stream=stream)
        x = x0.clone()
        ws.solve(x, so, stream=stream)
        x.copy_(x0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = ws.solve(x, so, stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[real] = {"colors": st[0]["n_colors"], "wall_s": round(t, 4),
                     "vertex_updates_per_s": round(st[0]["vertex_updates"] / t, 1),
                     "rel_residual_fp64": st[0]["rel_residual"],
                     "safeguard_rejections": st[0]["rejected"],
                     "sweep_roofline": sweep_roofline(ws, x0, so, torch, stream)}
    return out


def paper_boxes_report(pbng, S, torch, stream):
    """The paper's quasistatic stretching blocks (Table 3 rows with 1
    substep): 32^3 corotated, Neo-Hookean and stable Neo-Hookean at 40
    iterations per frame, 64^3
    at 20, 128^3 at 40.  A frame sets that frame's Dirichlet targets and runs
    the iterations from the previous frame's positions (Chebyshev rho = 0.95,
    relaxation 1.7, FP32, lanes and graph replay from the autotuner), with
    one FP64 residual at the end.  The paper's
    per-frame times were measured on a 64-core CPU; they are context."""
    rows = [(32, "corotated", 40, 1300.0), (32, "nh", 40, 825.0), (32, "snh", 40, 1300.0),
            (64, "corotated", 20, 1300.0), (128, "corotated", 40, 61000.0)]
    out = []
    for n, model, iters, paper_ms in rows:
        # the motion spans 60 frames; frame 1 warms up, frames 2-4 are timed
        sc, frames = S.paper_box_frames(n, model, n_frames=60)
        frames = frames[:4]
        ws = pbng.Workspace([pbng.problem_from_scenario(sc)], real="f32")
        so = pbng.solve_opts(max_sweeps=iters, rel_tol=0.0, check_every=iters, accel="chebyshev",
                             rho=0.95, gamma=1.7, safeguard="backtrack")
        x = torch.tensor(sc.initial_iterate(), dtype=torch.float32, device="cuda")
        xds = [torch.tensor(f, dtype=torch.float64, device="cuda") for f in frames]
        ws.set_dirichlet(xds[0], stream=stream)
        so, lanes = ws.autotune(x, so, stream=stream)
        ws.solve(x, so, stream=stream)          # frame 1 (warm-up)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = []
        for xd in xds[1:]:
            ws.set_dirichlet(xd, stream=stream)
            rc, st = ws.solve(x, so, stream=stream)
            sts.append(st[0])
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / len(xds[1:])
        roof = sweep_roofline(ws, x, so, torch, stream)
        out.append({"block": "%d^3" % n, "vertices": sc.n_verts, "tets": sc.n_tets, "sweep_roofline": roof,
                    "lanes_per_colour": [int(v) for v in lanes], "sweeps_per_graph": int(so.sweeps_per_graph),
                    "model": model, "iterations_per_frame": iters,
                    "ms_per_frame": round(t * 1e3, 3),
                    "vertex_updates_per_s": round(sc.n_free * iters / t, 1),
                    "frame_rel_residual_fp64": [round(s["rel_residual"], 6) for s in sts],
                    "paper_ms_per_frame_cpu": paper_ms})
        del ws, x, xds
        torch.cuda.empty_cache()
    return out


def dynamics_report(pbng, S, torch, stream, frames=8):
    """Backward Euler (inertia term of Eq. fem_be): the 128x32x32 Neo-Hookean
    beam released from rest under gravity, one step of dt = 1/30 s per
    frame, 40 Chebyshev iterations per frame, FP32."""
    sc = S.config_beam_f32()
    dt, iters = 1.0 / 30.0, 40
    ws = pbng.Workspace([pbng.problem_from_scenario(sc)], real="f32")
    so = pbng.solve_opts(max_sweeps=iters, rel_tol=0.0, check_every=iters, accel="chebyshev",
                         rho=0.95, gamma=1.7, safeguard="backtrack")
    x_prev = torch.tensor(sc.initial_iterate(), dtype=torch.float64, device="cuda")
    x_n = x_prev.clone()
    x = x_n.float()
    times, rels = [], []
    for f in range(frames):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ws.set_inertia(dt, x_n, x_prev, stream=stream)
        rc, st = ws.solve(x, so, stream=stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        rels.append(st[0]["rel_residual"])
        x_prev, x_n = x_n, x.double()
    tip = float(x_n[:, 1].min() - x_prev.new_tensor(sc.initial_iterate())[:, 1].min())
    t = sum(times[1:]) / (frames - 1)
    roof = sweep_roofline(ws, x, so, torch, stream)
    return {"workload": "beam 128x32x32 Neo-Hookean, gravity, dt = 1/30 s", "frames": frames,
            "iterations_per_frame": iters, "ms_per_frame": round(t * 1e3, 3),
            "vertex_updates_per_s": round(sc.n_free * iters / t, 1),
            "frame_rel_residual_fp64": [round(r, 6) for r in rels],
            "lowest_point_drop_m": round(-tip, 6), "sweep_roofline_with_inertia": roof}


def collision_report(pbng, S, torch, stream, frames=8):
    """The paper's two colliding blocks (Sec. "Collisions"; Table 3 row "Two
    moving blocks colliding": 8.2K vertices, 33K tets, corotated, 17
    substeps and 136 iterations per frame): two 16^3-vertex blocks, R0 = 10,
    E = 1000, the right block's clamped face driven toward the left one at
    0.3 m/s.  Every substep (dt = 1/30/17) detects contacts within 0.03,
    installs them (k_n = 1e8, recolouring), sets the backward-Euler inertia
    and runs 8 Chebyshev iterations (MIXED).  Timed: frames 2..8."""
    sc = S.two_blocks(16, gap=0.02, model="corotated", drive=0.0)
    ws = pbng.Workspace([pbng.problem_from_scenario(sc)], real="mixed")
    sub, iters, kn, radius, vel = 17, 8, 1e8, 0.03, 0.3
    dt = 1.0 / 30.0 / sub
    so = pbng.solve_opts(max_sweeps=iters, rel_tol=0.0, check_every=iters, accel="chebyshev",
                         rho=0.95, gamma=1.2, safeguard="backtrack")
    half = sc.n_verts // 2
    right = torch.tensor(np.nonzero(sc.dirichlet_idx >= half)[0], device="cuda")
    xd0 = torch.tensor(sc.dirichlet_x, dtype=torch.float64, device="cuda")
    x_prev = torch.tensor(sc.initial_iterate(), dtype=torch.float64, device="cuda")
    x_n = x_prev.clone()
    x = x_n.clone()
    t, times, n_contacts, n_colors = 0.0, [], [], []
    for f in range(frames):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(sub):
            t += dt
            xd = xd0.clone()
            xd[right, 0] -= vel * t
            ws.set_dirichlet(xd, stream=stream)
            pairs, normals = ws.detect_contacts(x, radius, max_pairs=1 << 16, stream=stream)
            ws.set_contacts(pairs, normals, kn, stream=stream)
            ws.set_inertia(dt, x_n, x_prev, stream=stream)
            rc, st = ws.solve(x, so, stream=stream)
            x_prev, x_n = x_n, x.clone()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        n_contacts.append(int(pairs.shape[0]))
        n_colors.append(int(st[0]["n_colors"]))
    tm = sum(times[1:]) / (frames - 1)
    roof = sweep_roofline(ws, x, so, torch, stream)
    return {"workload": "two blocks 2 x 16^3 vertices, corotated, backward Euler with contacts",
            "sweep_roofline_with_contacts": roof,
            "vertices": sc.n_verts, "tets": sc.n_tets, "substeps_per_frame": sub,
            "iterations_per_frame": sub * iters, "ms_per_frame": round(tm * 1e3, 3),
            "contacts_per_frame_end": n_contacts, "colours": n_colors,
            "paper_ms_per_frame_cpu": 1630.0}


def planar_terms_report(torch, stream, n=1025, frames=5, iters=40, roof_sweeps=20):
    """The planar path with every extra term at full size: an n x n block
    hanging from its top row under strong gravity, 2000 seeded springs and
    666 three-vertex weak constraints, a stiff ground half-plane it is
    pressed into, and backward-Euler frames (dt = 1/100, FP32, 40 plain
    iterations per frame, safeguard on; the Chebyshev blend with rho = 0.9
    diverges on this problem, in the oracle too, from 129^2 vertices on).
    Timed: frames 2..frames.  The sweep roofline counts the elastic visit
    records of pbng2d_phase_bytes, not the constraint, half-plane and
    inertia data."""
    from paper_2306_09021_amd import pbng2d
    from paper_2306_09021_amd import scenarios as S
    sc = S.planar_terms(n, "nh", n_springs=2000)
    ws = pbng2d.Workspace2D(pbng2d.problem_from_scenario(sc), real="f32")
    dt = 0.01
    opts = pbng2d.solve_opts(accel="none", safeguard="backtrack", rel_tol=0.0, max_sweeps=iters,
                             check_every=iters)
    x = torch.tensor(sc.initial_iterate(), dtype=torch.float32, device="cuda")
    x_prev = x.double().clone()
    x_n = x_prev.clone()
    times, rel = [], []
    for f in range(frames):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ws.set_inertia(dt, x_n, x_prev, stream=stream)
        _, st = ws.solve(x, opts, stream=stream)
        x_prev, x_n = x_n, x.double().clone()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        rel.append(round(st["rel_residual"], 6))
    tm = sum(times[1:]) / (frames - 1)
    ws.load(x, stream=stream)
    ws.sweeps(3, opts, stream=stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    ws.sweeps(roof_sweeps, opts, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) * 1e-3 / roof_sweeps
    b = sum(ws.phase_bytes(c)[0] for c in range(ws.n_colors))
    return {"workload": "hanging_block_%dx%d_neohookean_springs_ground_backward_euler" % (n, n),
            "vertices": ws.n_verts, "triangles": ws.n_tris, "weak_constraints": int(sc.wc_ptr.size - 1),
            "colours": ws.n_colors, "iterations_per_frame": iters, "ms_per_frame": round(tm * 1e3, 3),
            "vertex_updates_per_s": round(iters * ws.n_free / tm, 1), "frame_rel_residual_fp64": rel,
            "sweep_roofline": {"sweep_us": round(t * 1e6, 2), "algorithmic_bytes_per_sweep": int(b),
                               "achieved_GBs": round(b / t / 1e9, 1),
                               "frac_of_hbm_peak": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}}


def planar_report(torch, stream, n=1025, sweeps=200, roof_sweeps=20):
    """The planar experiment of Sec. "PBNG vs. PBD and Limited Newton" on a
    triangle mesh: an n x n-vertex unit square whose left and right sides
    are pulled to 1.5 times its width and clamped, interior starting at rest
    (Neo-Hookean, E = 1e4, nu = 0.3, uniform diagonals).  Plain FP32 sweeps
    with the safeguard, FP64 residuals: the experiment compares plain PBNG
    iterations, and with the initial stretch concentrated in the first
    column of triangles (F about 250 at this size) the Chebyshev and SOR
    blends diverge from 257^2 and 129^2 vertices on (oracle and GPU alike).
    Reports vertex
    updates per second over `sweeps` sweeps, the FP64 relative residual after
    50 and after `sweeps` sweeps, the HBM roofline of the planar
    colour-phase kernel from HIP events on the launch stream, the corotated
    square's rate, and `sweeps` adjoint sweeps at the rest state."""
    from paper_2306_09021_amd import pbng2d
    from paper_2306_09021_amd import scenarios as S
    sc = S.stretched_square(n, "nh", 1.5)
    ws = pbng2d.Workspace2D(pbng2d.problem_from_scenario(sc), real="f32")
    x0 = torch.tensor(sc.initial_iterate(), dtype=torch.float32, device="cuda")
    kw = dict(accel="none", safeguard="backtrack", rel_tol=0.0)
    x = x0.clone()
    _, st50 = ws.solve(x, max_sweeps=50, check_every=50, stream=stream, **kw)
    x.copy_(x0)
    ws.solve(x, max_sweeps=sweeps, check_every=sweeps, stream=stream, **kw)   # warm-up
    x.copy_(x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = ws.solve(x, max_sweeps=sweeps, check_every=sweeps, stream=stream, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def launch_time(opts, n_sweeps):
        """Average colour-phase launch duration over n_sweeps back-to-back
        sweeps, HIP events on the launch stream."""
        ws.load(x0, stream=stream)
        ws.sweeps(3, opts, stream=stream)
        ev0.record(stream)
        ws.sweeps(n_sweeps, opts, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) * 1e-3 / (n_sweeps * ws.n_colors)

    lanes_us = {l: round(1e6 * launch_time(pbng2d.solve_opts(lanes=l, **kw), 10), 2) for l in (2, 4, 8)}
    opts = pbng2d.solve_opts(**kw)           # the library's default: 4 lanes per vertex
    avg = launch_time(opts, roof_sweeps)
    n_launch = roof_sweeps * ws.n_colors
    per_sweep = sum(ws.phase_bytes(c)[0] for c in range(ws.n_colors))
    gbs = per_sweep / ws.n_colors / avg / 1e9
    tr, tr_note = traffic_per_launch(PLANAR_COUNTERS, "k2_phase")
    # the corotated model on the same square (rotation of each 2x2 F per visit)
    scc = S.stretched_square(n, "corotated", 1.5)
    wsc = pbng2d.Workspace2D(pbng2d.problem_from_scenario(scc), real="f32")
    xc = x0.clone()
    wsc.solve(xc, max_sweeps=20, check_every=20, stream=stream, **kw)                 # warm-up
    xc.copy_(x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stc = wsc.solve(xc, max_sweeps=sweeps, check_every=sweeps, stream=stream, **kw)
    torch.cuda.synchronize()
    elc = time.perf_counter() - t0
    # adjoint sweeps of the same square at its rest state, where H is the
    # (positive definite) linear-elastic stiffness: block Gauss-Seidel for
    # the right-hand side x - X of the iterate reached above
    xr = torch.tensor(sc.rest_pos, dtype=x.dtype, device="cuda").contiguous()
    b = (x.double() - xr.double()).to(x.dtype).contiguous()
    ao = pbng2d.adjoint_opts(max_sweeps=sweeps, rel_tol=0.0, check_every=sweeps)
    ws.adjoint(xr, b, ao, stream=stream)                                                # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, sta = ws.adjoint(xr, b, ao, stream=stream)
    torch.cuda.synchronize()
    ela = time.perf_counter() - t0
    return {"workload": "stretched_square_%dx%d_neohookean" % (n, n), "vertices": ws.n_verts,
            "adjoint": {"ms_per_sweep": round(1e3 * ela / sweeps, 4),
                        "vertex_updates_per_s": round(sta["vertex_updates"] / ela, 1),
                        "rel_residual_after": sta["rel_residual"]},
            "corotated": {"ms_per_sweep": round(1e3 * elc / sweeps, 4),
                          "vertex_updates_per_s": round(stc["vertex_updates"] / elc, 1),
                          "rel_residual_after": stc["rel_residual"]},
            "triangles": ws.n_tris, "free_vertices": ws.n_free, "colours": ws.n_colors,
            "sweeps": st["sweeps"], "ms_per_sweep": round(1e3 * el / sweeps, 4),
            "vertex_updates_per_s": round(st["vertex_updates"] / el, 1),
            "rel_residual_after_50": st50["rel_residual"], "rel_residual_after": st["rel_residual"],
            "roofline": {"bound": "hbm", "kernel": "k2_phase (planar colour-phase vertex update)",
                         "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": (int(tr) if tr is not None else None),
                         "traffic_note": tr_note,
                         "avg_launch_us": round(avg * 1e6, 2),
                         "avg_algorithmic_bytes": int(per_sweep / ws.n_colors), "launches_timed": n_launch},
            "launch_us_by_lanes": lanes_us}


def cpu_baseline(sc, sweeps):
    """The FP64 oracle as it stands, on the host cores, over the first
    `sweeps` sweeps of the same workload (bounded sample)."""
    import oracle as O
    op = O.make_problem(sc)
    col, _ = O.color(op)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    t0 = time.perf_counter()
    _, st = O.solve(op, col, sc.initial_iterate(), max_sweeps=sweeps, accel="sor", omega=1.6,
                    safeguard="backtrack", check_every=sweeps, n_threads=threads)
    t = time.perf_counter() - t0
    # the serial definition as well: one thread over a shorter sample
    s1 = max(1, sweeps // 15)
    t1 = time.perf_counter()
    _, st1 = O.solve(op, col, sc.initial_iterate(), max_sweeps=s1, accel="sor", omega=1.6,
                     safeguard="backtrack", check_every=s1, n_threads=1)
    t1 = time.perf_counter() - t1
    return {"value": round(sc.n_free * st["sweeps"] / t, 1), "unit": "vertex updates/s",
            "cores": threads, "kind": "oracle",
            "sample": "first %d sweeps of the same beam (FP64 C oracle, OpenMP within a colour, "
                      "residual at start and end), %.1f s" % (st["sweeps"], t),
            "single_thread": {"value": round(sc.n_free * st1["sweeps"] / t1, 1), "cores": 1,
                              "sample": "first %d sweeps, residual at start and end, %.1f s" % (st1["sweeps"], t1)}}


if __name__ == "__main__":
    main()
