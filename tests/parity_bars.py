"""Parity bars shared by the GPU tests: the HIP path against the oracle,
element by element.

FP64.  Per point the oracle returns a condition number kappa (the sum over
every quadrature term -- each w_j / D over every contour node times its node
coefficient, and the subtraction sum -- of |term| times the term's
first-order sensitivity to relative perturbations of its inputs, divided by
|G|).  Two FP64 evaluations of the same quadrature whose inputs and
operations are each accurate to a few ulp differ by at most c eps kappa |G|
(eps = 2^-53, c = 64); the stated target, 1e-12 relative, is required
wherever kappa <= 1e3.

FP32C (FP32 bulk).  The stated target 1e-6, mixed absolute/relative because
G(mu^2) = 0 makes a pure relative error unbounded near x = mu^2:
|G32 - G| <= 1e-6 max(|G|, s) at every point, no condition gate.  s = 1 for
the four-dimensional integral (the configurations the target is stated for,
and every D = 4 extension); for D = 2 and 3, whose unsubtracted sums are
larger than G itself, s = max |G| over the scan.
"""
import numpy as np

EPS = 2.0 ** -53
EPS32 = 2.0 ** -24
FP64_REL = 1e-12
KAPPA_GOOD = 1e3
FP32C_TOL = 1e-6


def check_fp64(g, g_or, cond, max_bad_share=None):
    """FP64 bar on points the caller has already matched (same class, not
    SINGULAR).  Returns error statistics; `max_bad_share` bounds the share of
    points with kappa > KAPPA_GOOD, the only points the 1e-12 target does not
    cover."""
    g, g_or, cond = (np.asarray(v) for v in (g, g_or, cond))
    assert np.all(np.isfinite(g)), "non-finite GPU value at a point with a contour"
    err = np.abs(g - g_or)
    mag = np.abs(g_or)
    bound = np.maximum(FP64_REL * mag, 64 * EPS * cond * mag)
    assert np.all(err <= bound), float(np.max(err / bound))
    good = cond <= KAPPA_GOOD
    rel = err / mag
    if good.any():
        assert np.max(rel[good]) <= FP64_REL, float(np.max(rel[good]))
    bad_share = float(1.0 - good.mean()) if good.size else 0.0
    if max_bad_share is not None:
        assert bad_share <= max_bad_share, bad_share
    stats = {"n": int(g.size), "max_rel": float(rel.max()) if rel.size else 0.0,
             "median_rel": float(np.median(rel)) if rel.size else 0.0,
             "kappa_gt_1e3_share": bad_share,
             "max_bound_ratio": float(np.max(err / bound)) if err.size else 0.0}
    if (~good).any():
        stats["max_err_over_1e-12_at_kappa_gt_1e3"] = float(np.max(rel[~good]) / FP64_REL)
    return stats


def check_fp32c(g32, g_ref, floor=1.0):
    """FP32C bar: |G32 - G| <= 1e-6 max(|G|, floor) at every point."""
    g32, g_ref = np.asarray(g32), np.asarray(g_ref)
    assert np.all(np.isfinite(g32))
    err = np.abs(g32 - g_ref)
    lim = FP32C_TOL * np.maximum(np.abs(g_ref), floor)
    assert np.all(err <= lim), float(np.max(err / lim))
    return {"n": int(g32.size), "max_abs": float(err.max()) if err.size else 0.0,
            "max_ratio": float(np.max(err / lim)) if err.size else 0.0}


def fp32c_floor(dim, g_ref):
    """The scale s of the FP32C bar for a scan in `dim` dimensions."""
    return 1.0 if dim in (0, 4) else max(1.0, float(np.max(np.abs(g_ref))))


def check(prec, g, g_or, cond, dim=4):
    """The bar of precision `prec` (0 FP64, 1 FP32C)."""
    if prec == 0:
        return check_fp64(g, g_or, cond)
    return check_fp32c(g, g_or, fp32c_floor(dim, g_or))


def band_report(g, g_ref, x, cut_threshold):
    """Max and mean abs/rel error separately within 0.05 of the cut
    x < -cut_threshold and elsewhere."""
    band = (np.abs(x.imag) < 0.05) & (x.real < -cut_threshold)
    out = {}
    for name, m in (("band", band), ("elsewhere", ~band)):
        if not m.any():
            continue
        err = np.abs(g[m] - g_ref[m])
        rel = err / np.abs(g_ref[m])
        out[name] = {"n": int(m.sum()), "max_abs": float(err.max()), "mean_abs": float(err.mean()),
                     "max_rel": float(rel.max()), "mean_rel": float(rel.mean())}
    return out
