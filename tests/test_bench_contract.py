"""The measurement side of bench.py, on the CPU: the one-GPU contract, the
evaluation count from a class map, the kernel names the profiles are keyed
by, and the roofline figures under the three flop counts."""
import json
import os
import subprocess
import sys

import numpy as np

import bench
from paper_1205_0752_amd.workloads import CONFIGS, Params, Quadrature

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_evaluations_follow_the_class_map():
    q = Quadrature(256, 128, 16)
    cls = np.array([0, 1, 2, 3, 4, 5, 1, 0], dtype=np.int8)
    # R: n_r nodes; Y: n_r + n_arc; YRES, MIRROR, LONG: one more; SINGULAR: none
    nodes = 2 * 256 + 2 * (256 + 16) + 3 * (256 + 16 + 1)
    assert bench.evals_per_scan(cls, q) == 128 * nodes
    assert bench.evals_per_scan(np.full(10, 4, dtype=np.int8), q) == 0


def test_kernel_names_match_the_profiled_instances():
    p, g, q = CONFIGS["c1_fp64_1024sq"]
    assert bench.scan_kernel_name(p, q, 1) == "scan_kernel_fp64<1, false, false, false>"
    p2, _, q2 = CONFIGS["c2_fp32c_1024sq"]
    assert bench.scan_kernel_name(p2, q2, 2) == "scan_kernel_fp32c<2, false, false, false>"
    # t^n, the split rule, pole sums (which always carry the t^n epilogue)
    assert bench.scan_kernel_name(Params(taylor_order=2), q, 1) == \
        "scan_kernel_fp64<1, true, false, false>"
    assert bench.scan_kernel_name(p, Quadrature(256, 128, 16, 0, 0, 1), 1) == \
        "scan_kernel_fp64<1, false, true, false>"
    assert bench.scan_kernel_name(p, q, 1, props=object()) == \
        "scan_kernel_fp64<1, true, false, true>"


def test_profiles_are_used_only_for_the_sources_they_were_taken_on():
    """The committed traffic and flop figures are keyed by kernel name and
    by the sha256 of the kernel sources; bench reads them only when both
    match, so a changed kernel reports no stale figure."""
    k = "scan_kernel_fp64<1, false, false, false>"
    with open(bench.TRAFFIC_FILE) as f:
        traffic = json.load(f)
    with open(bench.FLOPS_FILE) as f:
        flops = json.load(f)
    assert traffic["kernel"] == k and flops["kernel"] == k
    current = traffic["kernels_source_sha256"] == bench.kernel_source_sha256()
    assert (bench.measured_traffic(k) is not None) == current
    assert (bench.measured_flops(k) is not None) == current
    if current:
        assert bench.measured_traffic(k) == traffic["traffic_bytes_per_launch"]
        assert bench.measured_flops(k) == flops["fp64_flops_per_launch"]
    assert bench.measured_traffic("scan_kernel_fp64<2, false, false, false>") is None
    assert bench.measured_flops("scan_kernel_fp32c<1, false, false, false>") is None


def test_roofline_conventions():
    evals, sec, peak = 3.6419e10, 4.3e-3, 78.6
    k = "scan_kernel_fp64<1, false, false, false>"
    r = bench.roofline_conventions(evals, sec, peak, k)
    assert abs(r["folded_pair"]["achieved_tflops"] - evals * 6.5 / sec / 1e12) < 1e-9
    assert abs(r["unfolded_term"]["frac"] - 2.0 * r["folded_pair"]["frac"]) < 1e-12
    hw = bench.measured_flops(k)
    if hw is None:
        assert r["hardware_counter"] is None
    else:
        assert abs(r["hardware_counter"]["flops_per_eval"] - hw / evals) < 1e-12
        # the hardware counts about the algorithm's folded flops
        assert 0.9 < r["hardware_counter"]["flops_per_eval"] / 6.5 < 1.1
