"""Benchmark of the complex-plane scan on one MI355X.

A step is one full scan of the benchmark workload -- 1024 x 1024 cell-centred
points over Re x in [-16, 8], Im x in [-8, 8], m1 = m2 = 1, mu^2 = 1,
Lambda^2 = 1e6, 256 radial x 128 angular (+16 arc) nodes, FP64 -- through
the C ABI (gf_scan_plan) with the plan and the output buffer already resident
on the device.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector (packed issue)
FLOPS_PER_EVAL = 13        # one term w/(U - V z): 5 FMA (x2) + 2 MUL + 1 RCP


def evals_per_scan(cls, quad) -> int:
    """Integrand evaluations (angular terms) one scan performs, from its class
    map: R points n_r nodes, Y points n_r + n_arc, YRES and MIRROR points
    (whose conjugate is a YRES point) n_r + n_arc + 1; times n_angular."""
    import numpy as np
    c = np.asarray(cls).ravel()
    nr, na, nc = quad.n_radial, quad.n_angular, quad.n_arc
    n_r = int((c == 0).sum())
    n_y = int((c == 1).sum())
    n_res = int(((c == 2) | (c == 3)).sum())
    return na * (n_r * nr + n_y * (nr + nc) + n_res * (nr + nc + 1))


def cpu_baseline(params, quad, grid, seconds: float):
    """The CPU oracle timed on a bounded random sample of the same grid."""
    import numpy as np
    import oracle
    from paper_1205_0752_amd.workloads import sample_points
    oracle.build()
    idx = sample_points(grid, 64, seed=7)
    x = oracle.grid_points_at(grid, idx)
    t = time.perf_counter()
    _, c = oracle.eval_points(params, quad, x)
    dt = time.perf_counter() - t
    n = int(min(grid.n_points, max(64, len(idx) * seconds / max(dt, 1e-3))))
    idx = sample_points(grid, n, seed=8)
    x = oracle.grid_points_at(grid, idx)
    t = time.perf_counter()
    _, c = oracle.eval_points(params, quad, x)
    dt = time.perf_counter() - t
    ev = evals_per_scan(c, quad)
    return {"value": ev / dt, "unit": "evals/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{len(idx)} random points of the same grid ({ev:.3e} evals, {dt:.1f} s)",
            "points_per_s": len(idx) / dt}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c1_fp64_1024sq")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per point (0 = automatic)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the scan "
              "shards by grid tiles with no communication, but only one GPU is used here)",
              file=sys.stderr)
        return 2

    import torch
    import paper_1205_0752_amd as gf
    from paper_1205_0752_amd.workloads import CONFIGS

    params, grid, quad = CONFIGS[args.config]
    torch.cuda.set_device(0)
    plan = gf.Plan(params, quad)
    out = gf.empty_result(grid)
    cls = torch.empty((grid.n_im, grid.n_re), dtype=torch.int8, device="cuda")
    gf.scan_plan(plan, grid, out, cls, lanes=args.lanes)
    torch.cuda.synchronize()
    evals = evals_per_scan(cls.cpu().numpy(), quad)
    lanes = args.lanes or plan.auto_lanes(grid)

    for _ in range(args.warmup):
        gf.scan_plan(plan, grid, out, lanes=args.lanes)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        gf.scan_plan(plan, grid, out, lanes=args.lanes, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    sec = ms / 1e3
    flops = evals * FLOPS_PER_EVAL
    achieved = flops / sec / 1e12
    result = {
        "metric": "complex grid points/s & integrand evals/s (FP64 vs FP32+compensated); "
                  "p99 scan latency",
        "value": evals / sec,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {grid.n_re}x{grid.n_im} grid, "
                               f"{quad.n_radial}x{quad.n_angular}(+{quad.n_arc} arc) nodes, "
                               f"m1^2={params.m1sq}, m2^2={params.m2sq}, mu^2={params.mu2}, "
                               f"Lambda^2={params.lambda2:g}",
                   "grid_points": grid.n_points, "evals_per_step": evals,
                   "lanes_per_point": lanes, "parallelism": "single GPU"},
        "points_per_s": grid.n_points / sec,
        "wall_s_timed": wall,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "scan_fp64_kernel", "flops_per_eval": FLOPS_PER_EVAL},
    }
    plan.close()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(params, quad, grid, args.cpu_seconds)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
