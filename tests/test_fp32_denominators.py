"""Rounding of the FP32C form's folded denominators q = |U^2 - V^2 s|^2, s = z^2.

The FP32 angular sum forms q either directly (D = U^2 - V^2 s from the FP32
values of U^2 and V^2, then |D|^2) or from the quadratic c0 - c1 s + c2 s^2
with c0 = |U^2|^2, c1 = 2 Re(U^2 conj V^2), c2 = |V^2|^2 formed in FP64 and
rounded once.  With the node's ratio r = (|U^2| + |V^2|) / dist(U^2, [0, V^2])
(taken as sqrt(2 (|U^2|^2 + |V^2|^2) |V^2|^2 / (dist^2 |V^2|^2)), the form the
kernels test), the direct form's relative error grows like r eps32 and the
quadratic's like r^2 eps32.  The kernels take the quadratic only for r <= 4,
the direct form up to r = 16 and FP64 beyond, which is sound if the
quadratic's worst case below 4 does not exceed the direct form's below 16.
These tests emulate both FP32 forms (fused multiply-adds as one rounding of
the exact FP64 result) on random scaled U^2, V^2 and s, against |U^2 - V^2 s|^2
in FP64 with the same FP32 s."""
import numpy as np

EPS32 = 2.0 ** -24
F32 = np.float32


def _fma32(a, b, c):
    # a b is exact in FP64 for FP32 a, b; the sum is rounded to FP64, then to FP32
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def _cases(n=200_000, seed=0):
    rng = np.random.default_rng(seed)
    u2 = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    v2 = (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)) * 10 ** rng.uniform(-2, 0.3, n)
    s = rng.uniform(0, 1, n).astype(F32)
    uu, vv = np.abs(u2) ** 2, np.abs(v2) ** 2
    dot = (u2 * np.conj(v2)).real
    cross = (u2 * np.conj(v2)).imag
    d2vv = np.where(dot <= 0, uu * vv, np.where(dot >= vv, (uu - 2 * dot + vv) * vv, cross ** 2))
    ratio = np.sqrt(2 * (uu + vv) * vv / d2vv)
    exact = np.abs(u2 - v2 * s.astype(np.float64)) ** 2
    ur, ui, vr, vi = (x.astype(F32) for x in (u2.real, u2.imag, v2.real, v2.imag))
    dr, di = _fma32(-vr, s, ur), _fma32(-vi, s, ui)
    direct = _fma32(dr, dr, (di.astype(np.float64) * di).astype(F32))
    c0, c1, c2 = uu.astype(F32), (-2 * dot).astype(F32), vv.astype(F32)
    quad = _fma32(_fma32(c2, s, c1), s, c0)
    err_d = np.abs(direct.astype(np.float64) / exact - 1)
    err_q = np.abs(quad.astype(np.float64) / exact - 1)
    return ratio, err_d, err_q


def test_quadratic_below_4_is_no_worse_than_direct_below_16():
    ratio, err_d, err_q = _cases()
    q4 = ratio <= 4
    d16 = (ratio > 4) & (ratio <= 16)
    assert q4.sum() > 10_000 and d16.sum() > 5_000
    assert err_q[q4].max() <= err_d[d16].max(), (err_q[q4].max() / EPS32, err_d[d16].max() / EPS32)


def test_error_growth_with_the_ratio():
    """Direct form: at most ~(2 + r) eps32; quadratic: at most ~(2 + r^2) eps32,
    and beyond r = 8 the quadratic is clearly worse (why it stops at 4)."""
    ratio, err_d, err_q = _cases(seed=1)
    assert np.all(err_d <= (4 + 2 * ratio) * EPS32), np.max(err_d / ((4 + 2 * ratio) * EPS32))
    assert np.all(err_q <= (4 + 2 * ratio ** 2) * EPS32), np.max(err_q / ((4 + 2 * ratio ** 2) * EPS32))
    far = (ratio > 8) & (ratio <= 16)
    assert err_q[far].max() > 4 * err_d[far].max()
