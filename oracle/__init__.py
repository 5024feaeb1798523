"""CPU oracle for the subtracted one-loop two-point integral on a complex x grid.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does,
and the two share no code.

`gf_oracle.c` is the plain FP64 implementation (OpenMP over points),
`gf_oracle_q.c` the same quadrature in __float128, `closed_forms.py` the
analytic references the oracle is pinned against.  `build()` compiles the two
C files with gcc into this directory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB64 = os.path.join(_HERE, "_liborc.so")
_LIBQ = os.path.join(_HERE, "_liborcq.so")

# contour classes (numbering shared by both oracle files)
R, Y, YRES, MIRROR, SINGULAR, LONG = 0, 1, 2, 3, 4, 5
CLASS_NAMES = {R: "R", Y: "Y", YRES: "YRES", MIRROR: "MIRROR", SINGULAR: "SINGULAR", LONG: "LONG"}


class _Problem(ctypes.Structure):
    _fields_ = [("m1sq_re", ctypes.c_double), ("m1sq_im", ctypes.c_double),
                ("m2sq_re", ctypes.c_double), ("m2sq_im", ctypes.c_double),
                ("mu2", ctypes.c_double), ("lambda2", ctypes.c_double),
                ("scale", ctypes.c_double),
                ("n_radial", ctypes.c_int), ("n_angular", ctypes.c_int),
                ("n_arc", ctypes.c_int), ("angular_rule", ctypes.c_int),
                ("taylor_order", ctypes.c_int), ("dimension", ctypes.c_int),
                ("radial_split", ctypes.c_int), ("n1", ctypes.c_int), ("n2", ctypes.c_int),
                ("p1", ctypes.c_double * 32), ("p2", ctypes.c_double * 32),
                ("num_on", ctypes.c_int), ("num", ctypes.c_double * 18)]


def build(verbose: bool = False) -> None:
    """Compile both oracle libraries with gcc (always recompiles)."""
    flags = ["-O2", "-fPIC", "-shared", "-fopenmp", "-std=gnu11"]
    for src, out, libs in (("gf_oracle.c", _LIB64, ["-lm"]),
                           ("gf_oracle_q.c", _LIBQ, ["-lquadmath", "-lm"])):
        cmd = ["gcc", *flags, "-o", out + ".tmp", os.path.join(_HERE, src), *libs]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    global _lib, _libq
    _lib = _libq = None


_lib = None
_libq = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB64):
            build()
        lib = ctypes.CDLL(_LIB64)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        lib.orc_gauss_cheb2.argtypes = [ctypes.c_int, dp, dp]
        lib.orc_angular_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        lib.orc_angular_rule_dim.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        lib.orc_angular_sum.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, dp, dp]
        lib.orc_eval_points.argtypes = [ctypes.POINTER(_Problem), ctypes.c_long, dp, dp,
                                        ctypes.c_int, dp, ctypes.c_char_p, dp]
        lib.orc_scan.argtypes = [ctypes.POINTER(_Problem), ctypes.c_long, ctypes.c_long,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, dp, ctypes.c_char_p, dp]
        lib.orc_grid_point.argtypes = [ctypes.c_long] * 4 + [ctypes.c_double] * 4 + [dp, dp]
        lib.orc_jmu.argtypes = [ctypes.POINTER(_Problem), dp, dp]
        lib.orc_classify_points.argtypes = [ctypes.POINTER(_Problem), ctypes.c_long, dp, dp,
                                            ctypes.c_char_p]
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_obstruction.argtypes = [ctypes.POINTER(_Problem), ctypes.c_long, dp, dp,
                                        ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p]
        lib.orc_taylor.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int, dp,
                                   ctypes.POINTER(ctypes.c_double)]
        lib.orc_radial_nodes_at.argtypes = [ctypes.POINTER(_Problem), ctypes.c_double,
                                            ctypes.c_double, dp, dp]
        lib.orc_yscan.argtypes = [ctypes.POINTER(_Problem), ctypes.c_double, ctypes.c_double,
                                  ctypes.c_long, dp, dp, ctypes.c_int, dp]
        lib.orc_point_contours.argtypes = [ctypes.POINTER(_Problem), ctypes.c_long, dp, dp,
                                           ctypes.POINTER(ctypes.c_int)]
        _lib = lib
    return _lib


def _loadq():
    global _libq
    if _libq is None:
        if not os.path.exists(_LIBQ):
            build()
        lib = ctypes.CDLL(_LIBQ)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orcq_eval_points.argtypes = [ctypes.POINTER(_Problem), ctypes.c_long, dp, dp,
                                         dp, ctypes.c_char_p]
        lib.orcq_eval_points_sets.argtypes = [ctypes.POINTER(_Problem), ctypes.c_long, dp, dp,
                                              ctypes.POINTER(ctypes.c_int), dp]
        _libq = lib
    return _libq


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def problem(params, quad, props=None) -> _Problem:
    """ctypes problem record from workload Params / Quadrature objects and,
    optionally, pole-sum Propagators (poles1, poles2: tuples of (m^2, c))."""
    m1, m2 = complex(params.m1sq), complex(params.m2sq)
    pr = _Problem(m1.real, m1.imag, m2.real, m2.imag, float(params.mu2),
                  float(params.lambda2), float(params.scale),
                  int(quad.n_radial), int(quad.n_angular), int(quad.n_arc),
                  int(getattr(quad, "angular_rule", 0)),
                  int(getattr(params, "taylor_order", 0)),
                  int(getattr(params, "dimension", 4)),
                  int(getattr(quad, "radial_split", 0)))
    if props is not None:
        pr.n1, pr.n2 = len(props.poles1), len(props.poles2)
        for arr, poles in ((pr.p1, props.poles1), (pr.p2, props.poles2)):
            for k, (m, c) in enumerate(poles):
                m, c = complex(m), complex(c)
                arr[4 * k], arr[4 * k + 1], arr[4 * k + 2], arr[4 * k + 3] = m.real, m.imag, c.real, c.imag
        for i, j, c in getattr(props, "numerator", ()):
            c = complex(c)
            pr.num_on = 1
            pr.num[2 * (3 * i + j)] += c.real
            pr.num[2 * (3 * i + j) + 1] += c.imag
    return pr


# ---------------------------------------------------------------- rules

def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    _load().orc_gauss_legendre(n, _dp(x), _dp(w))
    return x, w


def gauss_cheb2(n: int):
    z = np.zeros(n)
    w = np.zeros(n)
    _load().orc_gauss_cheb2(n, _dp(z), _dp(w))
    return z, w


def angular_rule(rule: int, n: int, dim: int = 4):
    """Nodes and weights of angular rule `rule` (0 GC-II, 1 GC-I, 2 tanh-sinh,
    3 Gauss-Legendre) for the normalised D-dimensional angular measure
    (1-z^2)^{(D-3)/2} dz / N_D (D = 4: (2/pi) sqrt(1-z^2) dz)."""
    z = np.zeros(n)
    w = np.zeros(n)
    lib = _load()
    rc = (lib.orc_angular_rule(int(rule), int(n), _dp(z), _dp(w)) if dim == 4 and rule != 3
          else lib.orc_angular_rule_dim(int(rule), int(dim), int(n), _dp(z), _dp(w)))
    if rc != 0:
        raise ValueError(f"angular rule {rule} with {n} nodes in D = {dim} is not defined")
    return z, w


def angular_sum(u: complex, v: complex, n: int) -> complex:
    """sum_j w_j / (u - v z_j) with the oracle's GC-II rule of order n."""
    re = ctypes.c_double()
    im = ctypes.c_double()
    _load().orc_angular_sum(u.real, u.imag, v.real, v.imag, n, ctypes.byref(re),
                            ctypes.byref(im))
    return complex(re.value, im.value)


# ---------------------------------------------------------------- evaluation

def grid_points(grid) -> np.ndarray:
    """Cell-centred x of every grid point (row-major, Re fastest), complex128."""
    lib = _load()
    out = np.empty(grid.n_points, dtype=np.complex128)
    xr = ctypes.c_double()
    xi = ctypes.c_double()
    for b in range(grid.n_im):
        for a in range(grid.n_re):
            lib.orc_grid_point(a, b, grid.n_re, grid.n_im, grid.re_lo, grid.re_hi,
                               grid.im_lo, grid.im_hi, ctypes.byref(xr), ctypes.byref(xi))
            out[b * grid.n_re + a] = complex(xr.value, xi.value)
    return out


def grid_points_at(grid, flat_idx) -> np.ndarray:
    """Cell-centred x at the given flat indices (b * n_re + a)."""
    lib = _load()
    flat_idx = np.asarray(flat_idx, dtype=np.int64)
    out = np.empty(flat_idx.size, dtype=np.complex128)
    xr = ctypes.c_double()
    xi = ctypes.c_double()
    for k, f in enumerate(flat_idx.tolist()):
        b, a = divmod(f, grid.n_re)
        lib.orc_grid_point(a, b, grid.n_re, grid.n_im, grid.re_lo, grid.re_hi,
                           grid.im_lo, grid.im_hi, ctypes.byref(xr), ctypes.byref(xi))
        out[k] = complex(xr.value, xi.value)
    return out


def eval_points(params, quad, x, force_class: int | None = None, want_cond: bool = False,
                props=None):
    """G at arbitrary complex points x.  Returns (g, cls[, cond])."""
    lib = _load()
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).ravel())
    xr = np.ascontiguousarray(x.real)
    xi = np.ascontiguousarray(x.imag)
    g = np.zeros(2 * x.size)
    cls = ctypes.create_string_buffer(max(x.size, 1))
    cond = np.zeros(x.size) if want_cond else None
    pr = problem(params, quad, props)
    rc = lib.orc_eval_points(ctypes.byref(pr), x.size, _dp(xr), _dp(xi),
                             -1 if force_class is None else int(force_class), _dp(g), cls,
                             _dp(cond) if want_cond else None)
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    gc = g[0::2] + 1j * g[1::2]
    c = np.frombuffer(cls.raw[:x.size], dtype=np.int8).copy()
    if want_cond:
        return gc, c, cond
    return gc, c


def scan(params, quad, grid, want_cond: bool = False, props=None):
    """G on the whole grid (row-major, Re fastest)."""
    lib = _load()
    n = grid.n_points
    g = np.zeros(2 * n)
    cls = ctypes.create_string_buffer(max(n, 1))
    cond = np.zeros(n) if want_cond else None
    pr = problem(params, quad, props)
    rc = lib.orc_scan(ctypes.byref(pr), grid.n_re, grid.n_im, grid.re_lo, grid.re_hi,
                      grid.im_lo, grid.im_hi, _dp(g), cls, _dp(cond) if want_cond else None)
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    gc = g[0::2] + 1j * g[1::2]
    c = np.frombuffer(cls.raw[:n], dtype=np.int8).copy()
    if want_cond:
        return gc, c, cond
    return gc, c


def eval_points_q(params, quad, x):
    """Quad-precision brute force of the same quadrature (every angular rule,
    Taylor order and dimension; single poles, unsplit radial rule).  Returns
    (g, cls)."""
    if getattr(quad, "radial_split", 0):
        raise ValueError("the quad-precision twin implements the unsplit radial rule only")
    lib = _loadq()
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).ravel())
    xr = np.ascontiguousarray(x.real)
    xi = np.ascontiguousarray(x.imag)
    g = np.zeros(2 * x.size)
    cls = ctypes.create_string_buffer(max(x.size, 1))
    pr = problem(params, quad)
    if lib.orcq_eval_points(ctypes.byref(pr), x.size, _dp(xr), _dp(xi), _dp(g), cls) != 0:
        raise ValueError("the quad-precision twin rejected the problem")
    return g[0::2] + 1j * g[1::2], np.frombuffer(cls.raw[:x.size], dtype=np.int8).copy()


def eval_points_q_sets(params, quad, x, props=None):
    """Quad-precision run of the same quadrature for pole sums, numerators and
    every contour class (the long way round included), on the contours the
    FP64 oracle chooses (passed as data: the comparison measures rounding
    only).  Returns G (NaN where no contour)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).ravel())
    xr = np.ascontiguousarray(x.real)
    xi = np.ascontiguousarray(x.imag)
    pr = problem(params, quad, props)
    info = np.zeros(7 * max(x.size, 1), dtype=np.int32)
    ip = info.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    _load().orc_point_contours(ctypes.byref(pr), x.size, _dp(xr), _dp(xi), ip)
    g = np.zeros(2 * x.size)
    if _loadq().orcq_eval_points_sets(ctypes.byref(pr), x.size, _dp(xr), _dp(xi), ip, _dp(g)) != 0:
        raise ValueError("the quad-precision twin rejected the problem")
    return g[0::2] + 1j * g[1::2]


def yscan(params, quad, x: complex, y, what: int = 0, props=None) -> np.ndarray:
    """y-plane diagnostic at fixed x: <1/D1>(x, y) (what = 0) or the subtracted
    y-integrand y/(y + m2^2)(<1/D1>(x, y) - <1/D1>(mu^2, y)) (what = 1)."""
    y = np.ascontiguousarray(np.asarray(y, dtype=np.complex128).ravel())
    yr = np.ascontiguousarray(y.real)
    yi = np.ascontiguousarray(y.imag)
    out = np.zeros(2 * y.size)
    pr = problem(params, quad, props)
    _load().orc_yscan(ctypes.byref(pr), complex(x).real, complex(x).imag, y.size, _dp(yr), _dp(yi),
                      int(what), _dp(out))
    return out[0::2] + 1j * out[1::2]


def obstruction(params, x, n_samples: int = 4096):
    """Per point: bit 0 the angular cut crosses the real segment [0, Lambda^2],
    bit 1 it crosses the contour of the class rule, bit 2 no contour; and a
    flag where a decision sits within rounding of its threshold."""
    from types import SimpleNamespace
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).ravel())
    xr = np.ascontiguousarray(x.real)
    xi = np.ascontiguousarray(x.imag)
    out = ctypes.create_string_buffer(max(x.size, 1))
    tie = ctypes.create_string_buffer(max(x.size, 1))
    pr = problem(params, SimpleNamespace(n_radial=1, n_angular=1, n_arc=0))
    if _load().orc_obstruction(ctypes.byref(pr), x.size, _dp(xr), _dp(xi), int(n_samples), out,
                               tie) != 0:
        raise ValueError("n_samples must be >= 2")
    return (np.frombuffer(out.raw[:x.size], dtype=np.uint8).copy(),
            np.frombuffer(tie.raw[:x.size], dtype=np.uint8).astype(bool))


def taylor(params, quad, n: int, props=None):
    """K_0..K_n of the subtraction at mu^2 by the Cauchy formula, and the
    radius rho of the circle (rounding error of K_i ~ eps max|S| rho^-i)."""
    out = np.zeros(2 * (n + 1))
    rho = ctypes.c_double()
    if _load().orc_taylor(ctypes.byref(problem(params, quad, props)), int(n), _dp(out),
                          ctypes.byref(rho)) != 0:
        raise ValueError("bad problem or order")
    return out[0::2] + 1j * out[1::2], rho.value


def radial_nodes(params, quad, x: complex):
    """Radial nodes r_i and dy weights of the straight part of x's contour."""
    r = np.zeros(quad.n_radial)
    w = np.zeros(quad.n_radial)
    x = complex(x)
    if _load().orc_radial_nodes_at(ctypes.byref(problem(params, quad)), x.real, x.imag, _dp(r),
                                   _dp(w)) != 0:
        raise ValueError("bad problem")
    return r, w


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().orc_threads())


def jmu(params, quad, props=None) -> complex:
    """Unscaled subtraction sum (real-axis contour at x = mu^2)."""
    re = ctypes.c_double()
    im = ctypes.c_double()
    pr = problem(params, quad, props)
    _load().orc_jmu(ctypes.byref(pr), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def classify(params, quad, x, props=None) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).ravel())
    xr = np.ascontiguousarray(x.real)
    xi = np.ascontiguousarray(x.imag)
    cls = ctypes.create_string_buffer(max(x.size, 1))
    pr = problem(params, quad, props)
    lib.orc_classify_points(ctypes.byref(pr), x.size, _dp(xr), _dp(xi), cls)
    return np.frombuffer(cls.raw[:x.size], dtype=np.int8).copy()
