"""MI355X (gfx950) complex-plane scans of a BPHZ-subtracted one-loop two-point
function: Python face of the C-ABI library declared in include/gf.h.

    from paper_1205_0752_amd import Params, Grid, Quadrature, Plan, scan_plan
    plan = Plan(Params(1.0, 1.0, 1.0, 1e6), Quadrature(256, 128, 16))
    g = scan_plan(plan, Grid(1024, 1024, -16, 8, -8, 8))   # complex128 on cuda

The library is loaded on first use; importing this package does not touch the
GPU.
"""
from ._binding import (CLASS_LONG, CLASS_MIRROR, CLASS_R, CLASS_SINGULAR, CLASS_Y, CLASS_YRES, EXPORTS,
                       LIB_PATH, NO_CONTOUR, OBSTRUCTED_CONTOUR, OBSTRUCTED_REAL_AXIS, REQ_DONE,
                       REQ_QUEUED, REQ_RUNNING, YSCAN_ANGULAR, YSCAN_INTEGRAND, GFError, Plan,
                       Server, cache_clear, cut_curve, empty_result, fit_poles, load,
                       obstruction_map, scan,
                       scan_noalloc, scan_plan, version, yscan_plan)
from .workloads import (CONFIGS, FP32C, FP64, GC1, GC2, GL, TANH_SINH, Grid, Params, Propagators,
                        Quadrature)

__all__ = ["Params", "Propagators", "Grid", "Quadrature", "Plan", "Server", "scan", "scan_noalloc", "scan_plan", "cache_clear",
           "empty_result", "yscan_plan", "cut_curve", "obstruction_map", "fit_poles", "version", "load", "GFError", "EXPORTS",
           "LIB_PATH", "FP64", "FP32C", "GC2", "GC1", "TANH_SINH", "GL", "CONFIGS",
           "YSCAN_ANGULAR", "YSCAN_INTEGRAND", "OBSTRUCTED_REAL_AXIS", "OBSTRUCTED_CONTOUR",
           "NO_CONTOUR", "REQ_QUEUED", "REQ_RUNNING", "REQ_DONE",
           "CLASS_R", "CLASS_Y", "CLASS_YRES", "CLASS_MIRROR", "CLASS_SINGULAR", "CLASS_LONG"]
