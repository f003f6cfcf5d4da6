"""Throughput of the fused collide-limit-stream step on one MI355X.

Workload: the blast problem on an 8192 x 8192 periodic grid (rho = 1 + 0.01 xi,
v = 0, p = 1e3 inside radius 0.1 about the centre, 1e-2 outside), gamma = 1.4,
alpha = 1/2, a^n = 4 lambda^n, PP density + pressure limiters.  The headline
`value` is the FP32-state form (float32 distributions and collide/stream
arithmetic, theta solve and wavespeed reduction in float64); the float64 form
is measured on the same workload and reported beside it.

A step is one kernel launch over all cells.  Inputs are resident in HBM
before the timed region; the timed region holds exactly `steps` launches,
bracketed by device synchronisations and timed with HIP events on the stream
the kernels run on.

Roofline: the state is 20 scalars per cell read once and written once,
so the algorithmic traffic is 160 B per cell-update (FP32 state) and 320 B
(FP64); achieved = bytes x cells / average launch time, against the 8 TB/s
HBM3E peak.  `traffic` comes from the rocprofv3 FETCH_SIZE / WRITE_SIZE
counters recorded under profiles/ (null if absent for this kernel build).

cpu_baseline: the FP64 CPU oracle (OpenMP over rows, all host cores) timed on
a bounded sample of the same workload: the blast on a 2048 x 2048 grid for
80 steps (about 10-20 s of host time).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s (GLUPS) + % HBM roofline, FP64 vs FP32 form, 1 MI355X"
HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = {"fp32": 160.0, "fp64": 320.0}
PMC_FILE = os.path.join(ROOT, "profiles", "traffic_step_blast8192.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--forms", default="fp32,fp64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=2048)
    ap.add_argument("--cpu-steps", type=int, default=80)
    ap.add_argument("--calib-gib", type=float, default=0.0,
                    help="also run a plain device copy of this many GiB (counter calibration)")
    return ap.parse_args()


def calibration_copy(gib):
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings give the
    scale between those counters and bytes moved."""
    import torch

    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 3}


def time_form(form, u0t, n, steps, warmup, autotune):
    import torch

    from paper_2411_15001_amd import binding as B
    from paper_2411_15001_amd.solver import Solver

    prec = B.LBM_FP32_STATE if form == "fp32" else B.LBM_FP64
    s = Solver(u0t, precision=prec, limiters=B.LBM_RHO_PP | B.LBM_PRESSURE)
    if autotune:
        rows, waves = s.autotune(os.path.join(ROOT, "paper_2411_15001_amd", "autotune_cache.json"))
    else:
        rows, waves = B.lbm_get_launch(s.ctx)
    s.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    st = s.moments(check=False)[1]
    d = s.diagnostics()
    s.close()
    del s
    torch.cuda.empty_cache()
    cells = n * n
    avg_ms = ms / steps
    glups = cells * steps / (ms * 1e-3) / 1e9
    achieved = BYTES_PER_CELL[form] * cells / (avg_ms * 1e-3) / 1e9
    return {
        "value": glups, "ms_per_step": avg_ms, "wall_s": wall, "status": int(st),
        "launch": {"strip_rows": rows, "waves_per_group": waves},
        "diag": {"t": d["t"], "lambda": d["lam"], "n_bad": d["n_bad"], "n_guard": d["n_guard"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
    }


def traffic_for(form):
    """Measured HBM bytes per launch (rocprofv3 counters), if recorded for the
    current library build."""
    try:
        with open(PMC_FILE) as f:
            rec = json.load(f)
    except OSError:
        return None
    lib = os.path.join(ROOT, "paper_2411_15001_amd", "libvlbm.so")
    import hashlib

    h = hashlib.sha256()
    for name in ("step.hip", "vlbm_internal.h"):
        with open(os.path.join(ROOT, "paper_2411_15001_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    entry = rec.get(form)
    if not entry or entry.get("source_sha256") != h.hexdigest() or not os.path.exists(lib):
        return None
    return entry.get("bytes_per_launch")


def cpu_baseline(n, steps):
    import oracle
    from paper_2411_15001_amd import cases

    oracle.lib()
    u0 = cases.blast(n, seed=0)
    cfg = oracle.Config(nx=n, ny=n, limiters=oracle.RHO_PP | oracle.PRESSURE)
    S, _ = oracle.init(cfg, u0)
    t0 = time.perf_counter()
    oracle.run(cfg, S, steps)
    dt = time.perf_counter() - t0
    return {"value": n * n * steps / dt / 1e9, "unit": "GLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "FP64 oracle on the blast workload at %dx%d for %d steps (%.1f s), "
                      "OpenMP over rows" % (n, n, steps, dt)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2411_15001_amd import cases

    torch.cuda.set_device(0)
    u0 = cases.blast(a.n, seed=0)
    u0t = torch.from_numpy(u0).cuda()
    del u0
    forms = {}
    for form in a.forms.split(","):
        forms[form] = time_form(form, u0t, a.n, a.steps, a.warmup, not a.no_autotune)
        forms[form]["roofline"]["traffic"] = traffic_for(form)
        print("# %s: %.3f GLUPS, %.4f ms/step, %.1f%% of HBM peak" % (
            form, forms[form]["value"], forms[form]["ms_per_step"],
            100 * forms[form]["roofline"]["frac"]), file=sys.stderr, flush=True)
    del u0t
    head = "fp32" if "fp32" in forms else next(iter(forms))
    H = forms[head]
    out = {
        "metric": METRIC,
        "value": H["value"],
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": H["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (theta solve and CFL reduce f64)" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "blast %dx%d periodic, gamma 1.4, alpha 1/2, a = 4 lambda, "
                               "PP + pressure limiters, %s form" % (a.n, a.n, head),
                   "grid": [a.n, a.n], "steps": a.steps},
        "roofline": H["roofline"],
        "forms": {k: {kk: vv for kk, vv in v.items()} for k, v in forms.items()},
    }
    if "fp32" in forms and "fp64" in forms:
        out["fp32_speedup_over_fp64"] = forms["fp32"]["value"] / forms["fp64"]["value"]
    if a.calib_gib > 0:
        out["calibration_copy"] = calibration_copy(a.calib_gib)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.cpu_n, a.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
