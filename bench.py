"""Benchmark of the complex-plane scan on one MI355X.

A step is one full scan of the benchmark workload -- 1024 x 1024 cell-centred
points over Re x in [-16, 8], Im x in [-8, 8], m1 = m2 = 1, mu^2 = 1,
Lambda^2 = 1e6, 256 radial x 128 angular (+16 arc) nodes, FP64 -- through
the C ABI (gf_scan_plan) with the plan and the output buffer already resident
on the device.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Besides the headline line's timed scans it reports, on the same box: the
scan-latency percentiles of 200 individually timed scans, the FP32C leg, the
diagnostics and extensions, serving (capacity, then 10,000-request Poisson
traces offered at 50 % and 80 % of it), and the CPU oracle leg (timing, and
the FP32C and FP64 scans' errors against the oracle per band).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector (packed issue)
# Algorithmic flops per integrand evaluation of the folded angular sum: one
# symmetric node pair (two evaluations) costs D = U^2 - V^2 z^2 (2 FMA), |D|^2
# (1 MUL + 1 FMA), 1/|D|^2 (1 RCP), 2w/|D|^2 (1 MUL), acc += t conj(D) (2 FMA)
# = 13 flops with FMA = 2, MUL = RCP = 1; Newton steps, the shared-reciprocal
# multiplies and compensation are not counted.
FLOPS_PER_EVAL = 6.5


# The count for one unfolded angular term D = U - V z, |D|^2, w/|D|^2,
# acc += t conj(D): 13 flops.  The kernel folds each symmetric pair into one
# denominator, so that count prices twice the work the kernel does per
# evaluation; it is reported beside the folded count, as a fraction of peak
# that can exceed 1.
FLOPS_PER_EVAL_UNFOLDED = 13.0

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "scan_kernel_fp64_bench_workload_traffic.json")
FLOPS_FILE = os.path.join(ROOT, "profiles", "scan_kernel_fp64_bench_workload_flops.json")
# the sources that define the scan kernels' machine code
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1205_0752_amd", "csrc", name)
                  for name in ("gf_internal.h", "gf_device.h", "gf_kernels.hip")]


def kernel_source_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by a plain copy's reading), or None
    when there is none for this kernel or the kernel sources have changed since
    the counters were taken (the summary records their sha256)."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        sha = kernel_source_sha256()
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("kernels_source_sha256") != sha:
        return None
    return float(rec["traffic_bytes_per_launch"])


def measured_flops(kernel: str):
    """Hardware FP64 flops per launch of `kernel` (SQ_INSTS_VALU_FLOPS_FP64 x 64
    lanes, one rocprofv3 --pmc run) from the committed summary, or None when
    there is none for this kernel or its sources have changed since."""
    try:
        with open(FLOPS_FILE) as f:
            rec = json.load(f)
        sha = kernel_source_sha256()
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("kernels_source_sha256") != sha:
        return None
    return float(rec["fp64_flops_per_launch"])


def roofline_conventions(evals: int, sec: float, peak: float, kernel: str):
    """The dominant kernel's FLOP rate and fraction of the FP64 vector peak
    under three counts: the folded pair (6.5 flops per evaluation, the
    `roofline` figure), one unfolded term (13), and the hardware's
    own FP64 flop counter from the committed profile."""
    out = {}
    for name, fpe in (("folded_pair", FLOPS_PER_EVAL), ("unfolded_term", FLOPS_PER_EVAL_UNFOLDED)):
        tf = evals * fpe / sec / 1e12
        out[name] = {"flops_per_eval": fpe, "achieved_tflops": tf, "frac": tf / peak}
    hw = measured_flops(kernel)
    if hw is not None:
        tf = hw / sec / 1e12
        out["hardware_counter"] = {"flops_per_eval": hw / evals, "achieved_tflops": tf,
                                   "frac": tf / peak, "source": os.path.relpath(FLOPS_FILE, ROOT)}
    else:
        out["hardware_counter"] = None
    return out


def evals_per_scan(cls, quad) -> int:
    """Integrand evaluations (angular terms) one scan performs, from its class
    map: R points n_r nodes, Y points n_r + n_arc, YRES and MIRROR points
    (whose conjugate is a YRES point) n_r + n_arc + 1; LONG points (each pole
    term on the ray, on one closing arc and, for the pole-sum benchmark's
    conjugate pair with two real k-leg poles, two residues of the blocked
    term: n_r + n_arc + 1 per pole on average) n_r + n_arc + 1; times
    n_angular."""
    import numpy as np
    c = np.asarray(cls).ravel()
    nr, na, nc = quad.n_radial, quad.n_angular, quad.n_arc
    n_r = int((c == 0).sum())
    n_y = int((c == 1).sum())
    n_res = int(((c == 2) | (c == 3) | (c == 5)).sum())
    return na * (n_r * nr + n_y * (nr + nc) + n_res * (nr + nc + 1))


def cpu_baseline(params, quad, grid, seconds: float):
    """The CPU oracle timed on a bounded random sample of the same grid: a
    calibration sample sets the size of a second sample meant to take about
    `seconds`, which is the one reported."""
    import oracle
    from paper_1205_0752_amd.workloads import sample_points
    oracle.build()
    n = 4096
    for attempt in range(3):
        idx = sample_points(grid, min(n, grid.n_points), seed=7 + attempt)
        x = oracle.grid_points_at(grid, idx)
        t = time.perf_counter()
        _, c = oracle.eval_points(params, quad, x)
        dt = time.perf_counter() - t
        if dt >= 0.5 * seconds or len(idx) == grid.n_points or attempt == 2:
            break
        n = int(min(grid.n_points, len(idx) * seconds / max(dt, 1e-3)))
    ev = evals_per_scan(c, quad)
    out = {"value": ev / dt, "unit": "evals/s", "cores": oracle.threads(), "kind": "oracle",
           "sample": f"{len(idx)} random points of the same grid ({ev:.3e} evals, {dt:.1f} s)",
           "points_per_s": len(idx) / dt}
    # the same oracle on one core: a child process with OMP_NUM_THREADS=1 (it
    # loads only the oracle and numpy), on a sample sized for about 3 s
    m = max(64, int(len(idx) * 3.0 / max(dt * oracle.threads(), 1e-3)))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(m)],
                           env=env, capture_output=True, text=True, timeout=120)
        out["single_core"] = json.loads(r.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        out["single_core"] = {"error": str(e)}
    return out


def errors_vs_oracle(params, grid, quad, g32, g64, n_other=4000, seed=13):
    """The FP32C and FP64 scans of the mixed-precision workload (same grid and
    nodes) against the FP64 oracle, max and mean abs/rel error, separately at
    every point within 0.05 of the cut x < -(m1 + m2)^2 and at n_other random
    points elsewhere (part of the CPU leg: the oracle runs on the host)."""
    import numpy as np
    import oracle
    oracle.build()
    d_re = (grid.re_hi - grid.re_lo) / grid.n_re
    d_im = (grid.im_hi - grid.im_lo) / grid.n_im
    a = np.arange(grid.n_re)
    b = np.arange(grid.n_im)
    xr = np.broadcast_to(grid.re_lo + (a[None, :] + 0.5) * d_re, (grid.n_im, grid.n_re)).ravel()
    xi = np.broadcast_to(grid.im_lo + (b[:, None] + 0.5) * d_im, (grid.n_im, grid.n_re)).ravel()
    thr = (abs(complex(params.m1sq)) ** 0.5 + abs(complex(params.m2sq)) ** 0.5) ** 2
    band = np.nonzero((np.abs(xi) < 0.05) & (xr < -thr))[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    other = np.setdiff1d(rng.choice(grid.n_points, n_other + band.size, replace=False), band)[:n_other]
    t = time.perf_counter()
    rep = {}
    for name, idx in (("cut_band", band), ("elsewhere", np.sort(other))):
        x = oracle.grid_points_at(grid, idx)
        go, _ = oracle.eval_points(params, quad, x)
        ok = np.isfinite(go)
        for prec, g in (("fp32c", g32), ("fp64", g64)):
            err = np.abs(g[idx][ok] - go[ok])
            rel = err / np.abs(go[ok])
            rep.setdefault(prec, {})[name] = {
                "points": int(ok.sum()), "max_abs": float(err.max()), "mean_abs": float(err.mean()),
                "max_rel": float(rel.max()), "mean_rel": float(rel.mean()),
                "max_over_fp32_bar": float(np.max(err / (1e-6 * np.maximum(np.abs(go[ok]), 1.0))))}
    rep["oracle_seconds"] = time.perf_counter() - t
    rep["sample"] = (f"all {band.size} points of the cut band and {other.size} random points "
                     f"elsewhere of {grid.n_re}x{grid.n_im}")
    return rep


def cpu_worker(n_points: int) -> int:
    """Child of cpu_baseline: times the oracle on `n_points` random points of the
    bench grid and prints one JSON object (never touches the GPU)."""
    import oracle
    from paper_1205_0752_amd.workloads import CONFIGS, sample_points
    params, grid, quad = CONFIGS["c1_fp64_1024sq"]
    oracle.build()
    idx = sample_points(grid, min(n_points, grid.n_points), seed=11)
    x = oracle.grid_points_at(grid, idx)
    t = time.perf_counter()
    _, c = oracle.eval_points(params, quad, x)
    dt = time.perf_counter() - t
    ev = evals_per_scan(c, quad)
    print(json.dumps({"value": ev / dt, "unit": "evals/s", "cores": oracle.threads(),
                      "sample": f"{len(idx)} random points ({ev:.3e} evals, {dt:.2f} s)"}))
    return 0


def scan_kernel_name(params, quad, lanes, props=None):
    """The kernel instance a scan launches: scan_kernel_<prec><L, TAYLOR, SPLIT,
    POLES> (pole sums always run the instance with the t^n epilogue)."""
    poles = props is not None
    taylor = poles or getattr(params, "taylor_order", 0) > 0
    split = bool(getattr(quad, "radial_split", 0)) and not poles
    b = lambda v: "true" if v else "false"  # noqa: E731
    return (f"scan_kernel_{'fp64' if quad.precision == 0 else 'fp32c'}<{lanes}, {b(taylor)}, "
            f"{b(split)}, {b(poles)}>")


def time_scan(gf, torch, params, grid, quad, steps, warmup, lanes, props=None, latency_scans=0):
    """Times `steps` scans with HIP events on the launch stream (one event
    between consecutive scans, so each scan's duration is known as well as the
    mean); the plan and the output buffer are resident before timing starts.
    Evaluations count one angular term per (p-k)-leg pole."""
    plan = gf.Plan(params, quad, props=props)
    out = gf.empty_result(grid)
    cls = torch.empty((grid.n_im, grid.n_re), dtype=torch.int8, device="cuda")
    gf.scan_plan(plan, grid, out, cls, lanes=lanes)
    torch.cuda.synchronize()
    evals = evals_per_scan(cls.cpu().numpy(), quad) * (len(props.poles1) if props else 1)
    used_lanes = lanes or plan.auto_lanes(grid)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        gf.scan_plan(plan, grid, out, lanes=lanes, stream=stream)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(steps):
        gf.scan_plan(plan, grid, out, lanes=lanes, stream=stream)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = evs[0].elapsed_time(evs[-1]) / steps
    # scan latency: a separate sample of back-to-back scans, each between its
    # own pair of events (after the timed region)
    n_lat = max(latency_scans, 0)
    lat = []
    if n_lat:
        ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat + 1)]
        ev2[0].record(stream)
        for i in range(n_lat):
            gf.scan_plan(plan, grid, out, lanes=lanes, stream=stream)
            ev2[i + 1].record(stream)
        torch.cuda.synchronize()
        lat = sorted(ev2[i].elapsed_time(ev2[i + 1]) for i in range(n_lat))
    plan.close()
    sec = ms / 1e3
    res = {"ms": ms, "evals": evals, "evals_per_s": evals / sec,
           "points_per_s": grid.n_points / sec, "tflops": evals * FLOPS_PER_EVAL / sec / 1e12,
           "wall": wall, "lanes": used_lanes, "sec": sec,
           "kernel": scan_kernel_name(params, quad, used_lanes, props)}
    if lat:
        res["latency_ms"] = {"scans": n_lat, "p50": lat[(n_lat - 1) // 2],
                             "p99": lat[min(n_lat - 1, math.ceil(0.99 * n_lat) - 1)],
                             "max": lat[-1]}
    return res


def time_launches(torch, fn, reps):
    """Average duration of `fn()` (launches on torch's current stream), by HIP
    events over `reps` back-to-back calls after one warm-up call."""
    fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def extensions(gf, torch):
    """The diagnostics and the alternative angular rule at bench-sized inputs:
    y-plane scan (1024^2 y points at x = 2 + 1.5i, 128 angular nodes, the
    subtracted integrand: two angular sums per point), the obstruction map
    (1024^2 x points of the bench box, 4096 samples per contour part) and the
    bench scan with the tanh-sinh angular rule (129 nodes) and with the Taylor
    subtraction t^2."""
    import dataclasses
    from paper_1205_0752_amd.workloads import CONFIGS, Grid, Quadrature
    p, g, q = CONFIGS["c1_fp64_1024sq"]
    out = {}
    plan = gf.Plan(p, q)
    yg = Grid(1024, 1024, -8.0, 8.0, -8.0, 8.0)
    buf = gf.empty_result(yg)
    ms = time_launches(torch, lambda: gf.yscan_plan(plan, 2.0 + 1.5j, yg, gf.YSCAN_INTEGRAND, buf), 10)
    plan.close()
    ev = yg.n_points * 2 * q.n_angular
    out["yscan"] = {"workload": "1024x1024 y grid over [-8,8]^2, x = 2+1.5i, 128 angular nodes, "
                                "subtracted integrand", "ms": ms, "evals_per_s": ev / (ms / 1e3),
                    "tflops": ev * FLOPS_PER_EVAL / (ms / 1e3) / 1e12,
                    "kernel": "yscan_kernel"}
    ob = torch.empty((g.n_im, g.n_re), dtype=torch.uint8, device="cuda")
    ms = time_launches(torch, lambda: gf.obstruction_map(p, g, 4096, ob), 3)
    out["obstruction_map"] = {"workload": "bench box, 1024x1024 points, 4096 samples per part",
                              "ms": ms, "points_per_s": g.n_points / (ms / 1e3),
                              "kernel": "obstruction_kernel"}
    qt = Quadrature(q.n_radial, 129, q.n_arc, gf.FP64, gf.TANH_SINH)
    t = time_scan(gf, torch, p, g, qt, 5, 1, 0)
    out["tanh_sinh_scan"] = {"workload": "bench box and radial/arc nodes, 129 tanh-sinh angular nodes",
                             "ms": t["ms"], "evals_per_s": t["evals_per_s"], "tflops": t["tflops"],
                             "frac_of_fp64_peak": t["tflops"] / FP64_PEAK_TFLOPS}
    t = time_scan(gf, torch, p, g, dataclasses.replace(q, radial_split=1), 5, 1, 0)
    out["split_radial_scan"] = {"workload": "bench workload with the split radial rule "
                                            "(4 pieces of 64 nodes per point)",
                                "ms": t["ms"], "evals_per_s": t["evals_per_s"],
                                "tflops": t["tflops"],
                                "frac_of_fp64_peak": t["tflops"] / FP64_PEAK_TFLOPS,
                                "kernel": t["kernel"]}
    from paper_1205_0752_amd.workloads import Propagators
    props = Propagators(Propagators.conjugate_pair(1.0 + 0.8j, 0.5), ((1.0, 0.6), (3.0, 0.4)))
    t = time_scan(gf, torch, p, g, q, 5, 1, 0, props=props)
    out["pole_sum_scan"] = {"workload": "bench box and nodes with pole-sum propagators: a "
                                        "complex-conjugate pair (1 +- 0.8i) on the (p-k) leg, "
                                        "two real poles on the k leg",
                            "ms": t["ms"], "evals_per_s": t["evals_per_s"], "tflops": t["tflops"],
                            "frac_of_fp64_peak": t["tflops"] / FP64_PEAK_TFLOPS,
                            "kernel": t["kernel"]}
    # the same with a numerator N(k^2, p.k) of every degree up to 2 in each
    # (one more real pair sum per folded pair, three polynomials per node)
    num = ((0, 0, 0.8 - 0.1j), (1, 0, 0.3 + 0.2j), (2, 0, 0.01 - 0.05j), (0, 1, 0.4),
           (1, 1, -0.2 + 0.1j), (2, 1, 0.02), (0, 2, 0.1 - 0.3j), (1, 2, 0.05), (2, 2, 0.01 + 0.01j))
    t = time_scan(gf, torch, p, g, q, 5, 1, 0,
                  props=Propagators(props.poles1, props.poles2, num))
    out["numerator_scan"] = {"workload": "the pole-sum scan with a complex numerator "
                                         "sum_{i,j<=2} n_ij (k^2)^i (p.k)^j",
                             "ms": t["ms"], "evals_per_s": t["evals_per_s"],
                             "kernel": t["kernel"]}
    t = time_scan(gf, torch, dataclasses.replace(p, taylor_order=2), g, q, 5, 1, 0)
    out["taylor2_scan"] = {"workload": "bench workload with the subtraction t^2 about mu^2",
                           "ms": t["ms"], "evals_per_s": t["evals_per_s"], "tflops": t["tflops"],
                           "frac_of_fp64_peak": t["tflops"] / FP64_PEAK_TFLOPS,
                           "kernel": t["kernel"]}
    return out


def fp32c_errors(gf, torch, params, grid, quad):
    """Error of an FP32C scan against the FP64 path (same grid and nodes; the
    FP64 path matches the CPU oracle to 1e-12), max and mean, absolute and
    relative, within 0.05 of the cut x < -(m1 + m2)^2 and elsewhere."""
    import dataclasses
    import numpy as np
    q64 = dataclasses.replace(quad, precision=gf.FP64)
    outs = []
    for q in (quad, q64):
        plan = gf.Plan(params, q)
        outs.append(gf.scan_plan(plan, grid))
        torch.cuda.synchronize()
        plan.close()
    g32, g64 = (o.cpu().numpy().ravel() for o in outs)
    arrays = (g32, g64)
    a = np.arange(grid.n_re)
    b = np.arange(grid.n_im)
    xr = np.broadcast_to(grid.re_lo + (a[None, :] + 0.5) * (grid.re_hi - grid.re_lo) / grid.n_re,
                         (grid.n_im, grid.n_re)).ravel()
    xi = np.broadcast_to(grid.im_lo + (b[:, None] + 0.5) * (grid.im_hi - grid.im_lo) / grid.n_im,
                         (grid.n_im, grid.n_re)).ravel()
    thr = (abs(complex(params.m1sq)) ** 0.5 + abs(complex(params.m2sq)) ** 0.5) ** 2
    band = (np.abs(xi) < 0.05) & (xr < -thr)
    rep = {}
    for name, m in (("cut_band", band), ("elsewhere", ~band)):
        if not m.any():
            continue
        err = np.abs(g32[m] - g64[m])
        rel = err / np.abs(g64[m])
        rep[name] = {"points": int(m.sum()), "max_abs": float(err.max()),
                     "mean_abs": float(err.mean()), "max_rel": float(rel.max()),
                     "mean_rel": float(rel.mean()),
                     "frac_rel_le_1e-6": float(np.mean(rel <= 1e-6))}
    return rep, arrays


def evals_from_class_maps(gf, reqs) -> int:
    """Integrand evaluations the served requests took, counted from each
    request's class map (evals_per_scan with the request's own node counts).
    The class of a point does not depend on the node counts, so the maps come
    from scans of the same parameters and grids with the smallest quadrature
    (after the trace, outside its timing)."""
    import torch
    from paper_1205_0752_amd.workloads import Quadrature
    n_max = max(r.grid.n_points for r in reqs)
    out = torch.empty(n_max, dtype=torch.complex128, device="cuda")
    cls = torch.empty(n_max, dtype=torch.int8, device="cuda")
    tiny = Quadrature(1, 2, 1)
    total = 0
    for r in reqs:
        n = r.grid.n_points
        plan = gf.Plan(r.params, tiny)
        gf.scan_plan(plan, r.grid, out[:n].view(r.grid.n_im, r.grid.n_re),
                     cls[:n].view(r.grid.n_im, r.grid.n_re))
        total += evals_per_scan(cls[:n].cpu().numpy(), r.quad)
        plan.close()
    return total


def serve_trace(gf, n_requests, rate, budget_bytes, seed=0):
    """Replays a seeded Poisson trace of scan requests in real time against the
    continuous-batching server; results are released as they complete."""
    from paper_1205_0752_amd.workloads import serving_trace
    reqs = serving_trace(n_requests, rate, seed=seed)
    lag = 0.0
    with gf.Server(budget_bytes=budget_bytes, max_inflight=4096) as srv:
        t0 = time.perf_counter()
        outstanding = 0
        i = 0
        while i < len(reqs) or outstanding:
            now = time.perf_counter() - t0
            if i < len(reqs) and reqs[i].arrival_s <= now:
                srv.submit(reqs[i].params, reqs[i].grid, reqs[i].quad)
                lag = max(lag, now - reqs[i].arrival_s)
                i += 1
                outstanding += 1
                continue
            wait_ms = (reqs[i].arrival_s - now) * 1e3 if i < len(reqs) else 1000.0
            t = srv.wait_any(max(wait_ms, 0.0))
            if t is not None:
                srv.release(t)
                outstanding -= 1
        wall = time.perf_counter() - t0
        st = srv.stats()
    span = st["first_submit_to_last_done_s"]
    served_evals = evals_from_class_maps(gf, reqs)
    return {"requests": n_requests, "arrival_rate_per_s": rate, "seed": seed,
            "completed": st["completed"], "wall_s": wall,
            "throughput_req_per_s": st["completed"] / span,
            "points_per_s": st["points_done"] / span,
            "evals_per_s": served_evals / span,
            "evals_served": served_evals,
            "nominal_evals_per_s": st["nominal_evals_done"] / span,
            "latency_ms": {"mean": st["latency_mean_ms"], "p50": st["latency_p50_ms"],
                           "p90": st["latency_p90_ms"], "p99": st["latency_p99_ms"],
                           "max": st["latency_max_ms"]},
            "max_submit_lag_ms": lag * 1e3, "batches": st["batches"],
            "device_budget_bytes": st["bytes_budget"], "peak_bytes": st["bytes_peak"]}


def progress(msg: str) -> None:
    """One line per finished phase on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c1_fp64_1024sq")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per point (0 = automatic)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp32c", action="store_true")
    ap.add_argument("--skip-serving", action="store_true")
    ap.add_argument("--skip-extensions", action="store_true",
                    help="skip the y-plane scan, obstruction map and tanh-sinh measurements")
    ap.add_argument("--latency-scans", type=int, default=200,
                    help="individually timed scans for the scan-latency percentiles")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-loads", default="0.5,0.8",
                    help="offered Poisson rates as fractions of the measured capacity")
    ap.add_argument("--serve-budget", type=int, default=1 << 30, help="device bytes")
    ap.add_argument("--profile-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes three times "
                         "(reference for the HBM traffic counters) and exit")
    ap.add_argument("--cpu-worker", type=int, default=0, metavar="POINTS",
                    help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        return cpu_worker(args.cpu_worker)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the scan "
              "shards by grid tiles with no communication, but only one GPU is used here)",
              file=sys.stderr)
        return 2

    import torch
    import paper_1205_0752_amd as gf
    from paper_1205_0752_amd.workloads import CONFIGS

    if args.profile_copy:
        n = args.profile_copy // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "repeats": 3}), flush=True)
        return 0

    params, grid, quad = CONFIGS[args.config]
    torch.cuda.set_device(0)
    t = time_scan(gf, torch, params, grid, quad, args.steps, args.warmup, args.lanes,
                  latency_scans=args.latency_scans)
    peak = FP64_PEAK_TFLOPS if quad.precision == 0 else FP32_PEAK_TFLOPS
    progress(f"timed scans: {t['ms']:.3f} ms per step")
    result = {
        "metric": "complex grid points/s & integrand evals/s (FP64 vs FP32+compensated); "
                  "p99 scan latency",
        "value": t["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if quad.precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {grid.n_re}x{grid.n_im} grid, "
                               f"{quad.n_radial}x{quad.n_angular}(+{quad.n_arc} arc) nodes, "
                               f"m1^2={params.m1sq}, m2^2={params.m2sq}, mu^2={params.mu2}, "
                               f"Lambda^2={params.lambda2:g}",
                   "grid_points": grid.n_points, "evals_per_step": t["evals"],
                   "lanes_per_point": t["lanes"],
                   "tail": ("the last rows at 16 lanes per point in the same launch (about 16 "
                            "points per resident wave)") if t["lanes"] == 1 else None,
                   "parallelism": "single GPU"},
        "points_per_s": t["points_per_s"],
        "scan_latency_ms": t.get("latency_ms"),
        "wall_s_timed": t["wall"],
        "roofline": {"bound": "alu", "achieved": t["tflops"],
                     "peak": FP64_PEAK_TFLOPS if quad.precision == 0 else FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s",
                     "frac": t["tflops"] / (FP64_PEAK_TFLOPS if quad.precision == 0
                                            else FP32_PEAK_TFLOPS),
                     "traffic": (measured_traffic(t["kernel"])
                                 if args.config == "c1_fp64_1024sq" else None),
                     "kernel": t["kernel"], "flops_per_eval": FLOPS_PER_EVAL,
                     "conventions": (roofline_conventions(t["evals"], t["sec"], peak, t["kernel"])
                                     if quad.precision == 0 else None)},
        # the paper's Table 1 ("Execution time"): total running time of its
        # program for one unstated parameter set -- context, not a target
        "paper_context": {"table1_total_runtime": {
            "Intel Xeon X5650, one core": "252 min 2 s", "NVIDIA GeForce GTX 550 Ti": "6 min 21 s",
            "NVIDIA GeForce GTX 480": "4 min 21 s", "NVIDIA Tesla C2070": "2 min 38 s"},
            "workload": "unstated; grid fill, per-point quadrature and host transfers",
            "precision": "not stated"},
    }
    if not args.skip_fp32c and args.config == "c1_fp64_1024sq":
        p2, g2, q2 = CONFIGS["c2_fp32c_1024sq"]
        t2 = time_scan(gf, torch, p2, g2, q2, max(2, args.steps // 2), 1, 0)
        err_fp64, fp32c_arrays = fp32c_errors(gf, torch, p2, g2, q2)
        progress(f"fp32c leg: {t2['ms']:.3f} ms per step")
        result["fp32c"] = {"workload": f"c2_fp32c_1024sq: {g2.n_re}x{g2.n_im} grid, "
                                       f"{q2.n_radial}x{q2.n_angular}(+{q2.n_arc} arc) nodes",
                           "evals_per_s": t2["evals_per_s"], "points_per_s": t2["points_per_s"],
                           "ms_per_step": t2["ms"],
                           "tflops": t2["tflops"],
                           "frac_of_fp32_peak": t2["tflops"] / FP32_PEAK_TFLOPS,
                           "frac_of_fp32_nonpacked": t2["tflops"] / FP64_PEAK_TFLOPS,
                           "lanes_per_point": t2["lanes"], "kernel": t2["kernel"],
                           "error_vs_fp64": err_fp64}
    if not args.skip_extensions and args.config == "c1_fp64_1024sq":
        result["extensions"] = extensions(gf, torch)
        progress("extensions done")
    if not args.skip_serving and args.config == "c1_fp64_1024sq":
        # capacity: the trace generator offered well above what the device sustains
        cap = serve_trace(gf, 1500, 4000.0, args.serve_budget)
        capacity = cap["throughput_req_per_s"]
        progress(f"serving capacity: {capacity:.0f} requests/s")
        result["serving_capacity"] = {k: cap[k] for k in (
            "requests", "arrival_rate_per_s", "completed", "throughput_req_per_s", "evals_per_s",
            "nominal_evals_per_s", "batches", "latency_ms")}
        result["serving"] = []
        for load in (float(v) for v in args.serve_loads.split(",") if v):
            rec = serve_trace(gf, args.serve_requests, round(load * capacity, 1), args.serve_budget)
            rec["offered_fraction_of_capacity"] = load
            result["serving"].append(rec)
            progress(f"serving at {load:.0%} of capacity: p99 {rec['latency_ms']['p99']:.1f} ms")
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(params, quad, grid, args.cpu_seconds)
        progress("cpu baseline done")
        if "fp32c" in result:
            p2, g2, q2 = CONFIGS["c2_fp32c_1024sq"]
            result["fp32c"]["error_vs_oracle"] = errors_vs_oracle(p2, g2, q2, *fp32c_arrays)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
