"""ctypes binding of the gf C ABI (include/gf.h).

Argument marshalling only: every step of a scan runs in the HIP library.
PyTorch supplies device memory (result tensors) and the HIP stream.  The
library must have been built (`paper_1205_0752_amd.build.build()`); loading
fails loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

from .workloads import FP32C, FP64, Grid, Params, Quadrature

_HERE = os.path.dirname(os.path.abspath(__file__))
#: the in-tree build; GF_LIBRARY may name another build of the same sources
LIB_PATH = os.environ.get("GF_LIBRARY") or os.path.join(_HERE, "_libgf.so")

GF_OK = 0
GF_EINVAL = -1
GF_EUNSUPPORTED = -2
GF_ENOMEM = -3
GF_EDEVICE = -4
GF_EBUDGET = -5
GF_ENOTFOUND = -6

CLASS_R, CLASS_Y, CLASS_YRES, CLASS_MIRROR, CLASS_SINGULAR, CLASS_LONG = 0, 1, 2, 3, 4, 5

#: every symbol include/gf.h declares
EXPORTS = ("gf_plan", "gf_plan_ex", "gf_scan_plan", "gf_scan_plan_ex", "gf_scan", "gf_scan_noalloc",
           "gf_free", "gf_cache_clear",
           "gf_plan_jmu", "gf_plan_taylor", "gf_plan_auto_lanes", "gf_fit_poles", "gf_last_error",
           "gf_version",
           "gf_yscan_plan", "gf_cut_curve", "gf_obstruction_map",
           "gf_server_create", "gf_server_submit", "gf_server_submit_ex", "gf_server_poll",
           "gf_server_wait",
           "gf_server_wait_any", "gf_server_result", "gf_server_copy_result",
           "gf_server_release", "gf_server_stats_get", "gf_server_destroy")

REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2


class GFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gf error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("m1sq_re", ctypes.c_double), ("m1sq_im", ctypes.c_double),
                ("m2sq_re", ctypes.c_double), ("m2sq_im", ctypes.c_double),
                ("mu2", ctypes.c_double), ("lambda2", ctypes.c_double),
                ("scale", ctypes.c_double), ("taylor_order", ctypes.c_int32),
                ("dimension", ctypes.c_int32)]


class _Quad(ctypes.Structure):
    _fields_ = [("n_radial", ctypes.c_int32), ("n_angular", ctypes.c_int32),
                ("n_arc", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("angular_rule", ctypes.c_int32), ("radial_split", ctypes.c_int32)]


MAX_POLES = 8


class _Props(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32)] + [
        (name, ctypes.c_double * MAX_POLES)
        for name in ("m1sq_re", "m1sq_im", "c1_re", "c1_im", "m2sq_re", "m2sq_im", "c2_re",
                     "c2_im")] + [
        ("numerator", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("num_re", ctypes.c_double * 9), ("num_im", ctypes.c_double * 9)]


def c_props(props):
    """ctypes record of a Propagators object (None -> None)."""
    if props is None:
        return None
    r = _Props()
    r.n1, r.n2 = len(props.poles1), len(props.poles2)
    if not (1 <= r.n1 <= MAX_POLES and 1 <= r.n2 <= MAX_POLES):
        raise ValueError(f"each propagator needs 1..{MAX_POLES} poles")
    for k, (m, c) in enumerate(props.poles1):
        m, c = complex(m), complex(c)
        r.m1sq_re[k], r.m1sq_im[k], r.c1_re[k], r.c1_im[k] = m.real, m.imag, c.real, c.imag
    for k, (m, c) in enumerate(props.poles2):
        m, c = complex(m), complex(c)
        r.m2sq_re[k], r.m2sq_im[k], r.c2_re[k], r.c2_im[k] = m.real, m.imag, c.real, c.imag
    num = getattr(props, "numerator", ())
    if num:
        r.numerator = 1
        for i, j, c in num:
            if not (0 <= i <= 2 and 0 <= j <= 2):
                raise ValueError("numerator powers i, j must lie in 0..2")
            c = complex(c)
            r.num_re[3 * i + j] += c.real
            r.num_im[3 * i + j] += c.imag
    return r


class _Grid(ctypes.Structure):
    _fields_ = [("n_re", ctypes.c_int32), ("n_im", ctypes.c_int32),
                ("re_lo", ctypes.c_double), ("re_hi", ctypes.c_double),
                ("im_lo", ctypes.c_double), ("im_hi", ctypes.c_double)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("device_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("batch_evals", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "completed", "released", "rejected", "queued", "running", "bytes_in_use",
        "bytes_peak", "bytes_budget", "batches", "work_items", "points_done")] + [
        (n, ctypes.c_double) for n in (
            "nominal_evals_done", "latency_mean_ms", "latency_p50_ms", "latency_p90_ms",
            "latency_p99_ms", "latency_max_ms", "first_submit_to_last_done_s")]


_lib = None


def load():
    """Loads the built library (once)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"the gfx950 library is not built ({LIB_PATH} missing); "
                               "run paper_1205_0752_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        lib.gf_plan.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Quad),
                                ctypes.POINTER(vp)]
        lib.gf_plan_ex.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Props),
                                   ctypes.POINTER(_Quad), ctypes.POINTER(vp)]
        lib.gf_scan_plan.argtypes = [vp, ctypes.POINTER(_Grid), vp, vp, vp]
        lib.gf_scan_plan_ex.argtypes = [vp, ctypes.POINTER(_Grid), vp, vp, ctypes.c_int, vp]
        lib.gf_scan.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid),
                                ctypes.POINTER(_Quad), vp, vp]
        lib.gf_scan_noalloc.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid),
                                        ctypes.POINTER(_Quad), vp, vp]
        lib.gf_free.argtypes = [vp]
        lib.gf_free.restype = None
        lib.gf_cache_clear.argtypes = []
        lib.gf_cache_clear.restype = None
        lib.gf_plan_jmu.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        lib.gf_plan_auto_lanes.argtypes = [vp, ctypes.POINTER(_Grid)]
        lib.gf_plan_taylor.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        lib.gf_last_error.restype = ctypes.c_char_p
        lib.gf_version.restype = ctypes.c_char_p
        lib.gf_yscan_plan.argtypes = [vp, ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(_Grid), ctypes.c_int, vp, vp]
        lib.gf_cut_curve.argtypes = [ctypes.POINTER(_Params), ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        dp = ctypes.POINTER(ctypes.c_double)
        lib.gf_fit_poles.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_int), dp, dp, dp, dp, dp]
        lib.gf_obstruction_map.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Grid),
                                           ctypes.c_int, vp, vp]
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.gf_server_create.argtypes = [ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]
        lib.gf_server_submit.argtypes = [vp, ctypes.POINTER(_Params), ctypes.POINTER(_Grid),
                                         ctypes.POINTER(_Quad), u64p]
        lib.gf_server_submit_ex.argtypes = [vp, ctypes.POINTER(_Params), ctypes.POINTER(_Props),
                                            ctypes.POINTER(_Grid), ctypes.POINTER(_Quad), u64p]
        lib.gf_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
        lib.gf_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double]
        lib.gf_server_wait_any.argtypes = [vp, ctypes.c_double, u64p]
        lib.gf_server_result.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp),
                                         ctypes.POINTER(ctypes.c_int64)]
        lib.gf_server_copy_result.argtypes = [vp, ctypes.c_uint64, vp]
        lib.gf_server_release.argtypes = [vp, ctypes.c_uint64]
        lib.gf_server_stats_get.argtypes = [vp, ctypes.POINTER(_ServerStats)]
        lib.gf_server_destroy.argtypes = [vp]
        _lib = lib
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise GFError(rc, load().gf_last_error().decode())
    return rc


def c_params(p: Params) -> _Params:
    m1, m2 = complex(p.m1sq), complex(p.m2sq)
    return _Params(m1.real, m1.imag, m2.real, m2.imag, float(p.mu2), float(p.lambda2),
                   float(p.scale), int(getattr(p, "taylor_order", 0)),
                   int(getattr(p, "dimension", 4)))


def c_quad(q: Quadrature) -> _Quad:
    return _Quad(int(q.n_radial), int(q.n_angular), int(q.n_arc), int(q.precision),
                 int(q.angular_rule), int(getattr(q, "radial_split", 0)))


def c_grid(g: Grid) -> _Grid:
    return _Grid(int(g.n_re), int(g.n_im), float(g.re_lo), float(g.re_hi), float(g.im_lo),
                 float(g.im_hi))


def _stream_handle(stream):
    if isinstance(stream, int):  # a raw hipStream_t (0 = default stream)
        return ctypes.c_void_p(stream)
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """Device-resident node tables and subtraction constant for one
    (params, quadrature), optionally with pole-sum propagators; see gf_plan and
    gf_plan_ex."""

    def __init__(self, params: Params, quad: Quadrature, props=None):
        self.params = params
        self.quad = quad
        self.props = props
        h = ctypes.c_void_p()
        pr = c_props(props)
        _check(load().gf_plan_ex(ctypes.byref(c_params(params)),
                                 ctypes.byref(pr) if pr is not None else None,
                                 ctypes.byref(c_quad(quad)), ctypes.byref(h)))
        self._h = h
        #: the GPU the plan's tables live on (the current device at creation)
        self.device = _current_device()

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise RuntimeError("plan is closed")
        return self._h

    def jmu(self) -> complex:
        re, im = ctypes.c_double(), ctypes.c_double()
        _check(load().gf_plan_jmu(self.handle, ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def taylor(self):
        """K_0..K_n, the Taylor coefficients of the subtraction at mu^2."""
        n = max(int(getattr(self.params, "taylor_order", 0)), 0)
        buf = (ctypes.c_double * (2 * (n + 1)))()
        _check(load().gf_plan_taylor(self.handle, buf))
        return [complex(buf[2 * i], buf[2 * i + 1]) for i in range(n + 1)]

    def auto_lanes(self, grid: Grid) -> int:
        return _check(load().gf_plan_auto_lanes(self.handle, ctypes.byref(c_grid(grid))))

    def close(self):
        """Frees the plan; the caller synchronises the streams that used it."""
        if self._h is not None:
            load().gf_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_out(t, dtype, n: int, device: int, name: str = "out"):
    """Raises ValueError unless `t` is a contiguous tensor of `dtype` with `n`
    elements on GPU `device`: the library writes through its raw address."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements (n_re * n_im), got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{name} must be on GPU {device}, got {t.device}")


def _current_device() -> int:
    import torch
    return torch.cuda.current_device()


def empty_result(grid: Grid, device=None):
    import torch
    return torch.empty((grid.n_im, grid.n_re), dtype=torch.complex128,
                       device=device or torch.device("cuda", torch.cuda.current_device()))


def scan_plan(plan: Plan, grid: Grid, out=None, cls=None, lanes: int = 0, stream=None):
    """Launches gf_scan_plan_ex; returns `out` (complex128 [n_im, n_re]),
    asynchronous on `stream` (default: torch's current stream)."""
    import torch
    if cls is not None:
        _check_out(cls, torch.int8, grid.n_points, plan.device, "cls")
    if out is None:
        out = empty_result(grid, torch.device("cuda", plan.device))
    _check_out(out, torch.complex128, grid.n_points, plan.device)
    _check(load().gf_scan_plan_ex(plan.handle, ctypes.byref(c_grid(grid)),
                                  ctypes.c_void_p(out.data_ptr() if grid.n_points else 0),
                                  ctypes.c_void_p(cls.data_ptr() if cls is not None else 0),
                                  int(lanes), _stream_handle(stream)))
    return out


YSCAN_ANGULAR, YSCAN_INTEGRAND = 0, 1


def yscan_plan(plan: Plan, x: complex, ygrid: Grid, what: int = YSCAN_ANGULAR, out=None,
               stream=None):
    """y-plane diagnostic (gf_yscan_plan): <1/D1>(x, y) or the subtracted
    y-integrand on a grid of complex y; complex128 [n_im, n_re] on the device."""
    import torch
    if out is None:
        out = empty_result(ygrid, torch.device("cuda", plan.device))
    _check_out(out, torch.complex128, ygrid.n_points, plan.device)
    x = complex(x)
    _check(load().gf_yscan_plan(plan.handle, x.real, x.imag, ctypes.byref(c_grid(ygrid)), int(what),
                                ctypes.c_void_p(out.data_ptr() if ygrid.n_points else 0),
                                _stream_handle(stream)))
    return out


def cut_curve(params: Params, x: complex, n: int = 513):
    """Both branches of the y-plane cut of eq. 25 at n angles in [0, pi]
    (gf_cut_curve): returns (y_plus, y_minus) as numpy complex arrays."""
    import numpy as np
    out = np.zeros(4 * n)
    x = complex(x)
    _check(load().gf_cut_curve(ctypes.byref(c_params(params)), x.real, x.imag, int(n),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out[0::4] + 1j * out[1::4], out[2::4] + 1j * out[3::4]


def fit_poles(s, p, max_poles: int = MAX_POLES, tol: float = 1e-12, weight=None):
    """Pole sum fitted to tabulated P(s_i), s_i >= 0 (gf_fit_poles), with
    optional positive weights of the error measure: returns (poles, max_err)
    with poles a tuple of (m^2, c) for Propagators."""
    import numpy as np
    s = np.ascontiguousarray(np.asarray(s, dtype=np.float64).ravel())
    p = np.asarray(p, dtype=np.complex128).ravel()
    if p.size != s.size:
        raise ValueError("s and p must have the same length")
    pr = np.ascontiguousarray(p.real)
    pi = np.ascontiguousarray(p.imag)
    wt = None
    if weight is not None:
        wt = np.ascontiguousarray(np.asarray(weight, dtype=np.float64).ravel())
        if wt.size != s.size:
            raise ValueError("s and weight must have the same length")
    m2r, m2i, cr, ci = (np.zeros(MAX_POLES) for _ in range(4))
    n_poles = ctypes.c_int(0)
    err = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(load().gf_fit_poles(s.ctypes.data_as(dp), pr.ctypes.data_as(dp), pi.ctypes.data_as(dp),
                               wt.ctypes.data_as(dp) if wt is not None else None,
                               int(s.size), int(max_poles), float(tol), ctypes.byref(n_poles),
                               m2r.ctypes.data_as(dp), m2i.ctypes.data_as(dp),
                               cr.ctypes.data_as(dp), ci.ctypes.data_as(dp), ctypes.byref(err)))
    k = n_poles.value
    return tuple((complex(m2r[a], m2i[a]), complex(cr[a], ci[a])) for a in range(k)), err.value


OBSTRUCTED_REAL_AXIS, OBSTRUCTED_CONTOUR, NO_CONTOUR = 1, 2, 4


def obstruction_map(params: Params, grid: Grid, n_samples: int = 4096, out=None, stream=None):
    """Per grid point, bit 0: the angular cut crosses the real segment
    [0, Lambda^2]; bit 1: it crosses the contour the scan uses; bit 2: no
    contour (gf_obstruction_map).  uint8 [n_im, n_re] on the device."""
    import torch
    dev = _current_device()
    if out is None:
        out = torch.empty((grid.n_im, grid.n_re), dtype=torch.uint8, device=torch.device("cuda", dev))
    _check_out(out, torch.uint8, grid.n_points, dev)
    _check(load().gf_obstruction_map(ctypes.byref(c_params(params)), ctypes.byref(c_grid(grid)),
                                     int(n_samples),
                                     ctypes.c_void_p(out.data_ptr() if grid.n_points else 0),
                                     _stream_handle(stream)))
    return out


def scan(params: Params, grid: Grid, quad: Quadrature, out=None, stream=None):
    """One-call scan (gf_scan): plan looked up in the library's cache."""
    import torch
    dev = _current_device()
    if out is None:
        out = empty_result(grid, torch.device("cuda", dev))
    _check_out(out, torch.complex128, grid.n_points, dev)
    _check(load().gf_scan(ctypes.byref(c_params(params)), ctypes.byref(c_grid(grid)),
                          ctypes.byref(c_quad(quad)),
                          ctypes.c_void_p(out.data_ptr() if grid.n_points else 0),
                          _stream_handle(stream)))
    return out


def scan_noalloc(params: Params, grid: Grid, quad: Quadrature, out, stream=None):
    """gf_scan_noalloc: the one-call scan with node tables in the library's
    static device buffer (nothing allocated); `out` is required."""
    import torch
    dev = _current_device()
    _check_out(out, torch.complex128, grid.n_points, dev)
    _check(load().gf_scan_noalloc(ctypes.byref(c_params(params)), ctypes.byref(c_grid(grid)),
                                  ctypes.byref(c_quad(quad)),
                                  ctypes.c_void_p(out.data_ptr() if grid.n_points else 0),
                                  _stream_handle(stream)))
    return out


class Server:
    """Continuous-batching scan server (gf_server_*) on the current device."""

    def __init__(self, budget_bytes: int = 1 << 30, max_inflight: int = 1024,
                 batch_evals: float = 0.0):
        h = ctypes.c_void_p()
        cfg = _ServerConfig(int(budget_bytes), int(max_inflight), float(batch_evals))
        _check(load().gf_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("server is closed")
        return self._h

    def submit(self, params: Params, grid: Grid, quad: Quadrature, props=None) -> int:
        t = ctypes.c_uint64()
        pr = c_props(props)
        _check(load().gf_server_submit_ex(self.handle, ctypes.byref(c_params(params)),
                                          ctypes.byref(pr) if pr is not None else None,
                                          ctypes.byref(c_grid(grid)), ctypes.byref(c_quad(quad)),
                                          ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> int:
        st = ctypes.c_int()
        _check(load().gf_server_poll(self.handle, ticket, ctypes.byref(st)))
        return st.value

    def wait(self, ticket: int, timeout_ms: float = -1.0) -> bool:
        return _check(load().gf_server_wait(self.handle, ticket, float(timeout_ms))) == 1

    def wait_any(self, timeout_ms: float = -1.0):
        """Next completed ticket, or None on timeout."""
        t = ctypes.c_uint64()
        r = _check(load().gf_server_wait_any(self.handle, float(timeout_ms), ctypes.byref(t)))
        return t.value if r == 1 else None

    def result(self, ticket: int):
        """The result as a numpy complex128 array [n_im, n_re] (copied to host)."""
        import numpy as np
        p = ctypes.c_void_p()
        n = ctypes.c_int64()
        _check(load().gf_server_result(self.handle, ticket, ctypes.byref(p), ctypes.byref(n)))
        out = np.empty(n.value, dtype=np.complex128)
        if n.value:
            _check(load().gf_server_copy_result(self.handle, ticket,
                                                ctypes.c_void_p(out.ctypes.data)))
        return out

    def release(self, ticket: int):
        _check(load().gf_server_release(self.handle, ticket))

    def stats(self) -> dict:
        st = _ServerStats()
        _check(load().gf_server_stats_get(self.handle, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in _ServerStats._fields_}

    def close(self):
        if self._h is not None:
            load().gf_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cache_clear():
    load().gf_cache_clear()


def version() -> str:
    return load().gf_version().decode()


__all__ = ["Plan", "Server", "scan", "scan_noalloc", "scan_plan", "yscan_plan", "cut_curve", "obstruction_map",
           "fit_poles",
           "cache_clear",
           "version", "load", "GFError",
           "EXPORTS",
           "FP64", "FP32C", "LIB_PATH", "empty_result"]
