"""MI355X (gfx950) complex-plane scans of a BPHZ-subtracted one-loop two-point
function: Python face of the C-ABI library declared in include/gf.h.

    from paper_1205_0752_amd import Params, Grid, Quadrature, Plan, scan_plan
    plan = Plan(Params(1.0, 1.0, 1.0, 1e6), Quadrature(256, 128, 16))
    g = scan_plan(plan, Grid(1024, 1024, -16, 8, -8, 8))   # complex128 on cuda

The library is loaded on first use; importing this package does not touch the
GPU.
"""
from ._binding import (CLASS_MIRROR, CLASS_R, CLASS_SINGULAR, CLASS_Y, CLASS_YRES, EXPORTS,
                       REQ_DONE, REQ_QUEUED, REQ_RUNNING, YSCAN_ANGULAR, YSCAN_INTEGRAND, GFError,
                       LIB_PATH, Plan, Server, cache_clear, cut_curve, yscan_plan, empty_result, load, scan, scan_plan,
                       version)
from .workloads import CONFIGS, FP32C, FP64, Grid, Params, Quadrature

__all__ = ["Params", "Grid", "Quadrature", "Plan", "Server", "scan", "scan_plan", "cache_clear",
           "empty_result", "yscan_plan", "cut_curve", "YSCAN_ANGULAR", "YSCAN_INTEGRAND", "version", "load", "GFError", "EXPORTS", "LIB_PATH", "FP64", "FP32C",
           "CONFIGS", "REQ_QUEUED", "REQ_RUNNING", "REQ_DONE", "CLASS_R", "CLASS_Y", "CLASS_YRES", "CLASS_MIRROR", "CLASS_SINGULAR"]
