"""Rounding of the general integrands against quad precision.

The quad-precision twin evaluates pole sums, numerators and every contour
class (the long way round in D = 3 and 4, residues of several k-leg poles,
t^n) in __float128 on the contours the FP64 oracle chooses (passed as data, so
the comparison measures rounding alone).  CPU: where the single-pole twin
(written separately, with its own contour choice) applies, the two quad
evaluations agree to quad rounding; the FP64 oracle lies within its
condition-number bar 64 eps kappa |G| of the quad values for every general
case.  GPU: the FP64 kernel's errors against the quad values are no larger
than the FP64 oracle's, within a factor 4, in median and maximum."""
import numpy as np
import pytest

import oracle
from paper_1205_0752_amd.workloads import GC2, GL, Grid, Params, Propagators, Quadrature

EPS = 2.0 ** -53
GRIBOV = Propagators(Propagators.conjugate_pair(1.0 + 0.8j, 0.5), ((1.0, 0.6), (3.0, 0.4)))
SWEPT = Propagators(((2.0, 1.0),), ((-0.5 + 0.6j, 0.7), (-0.3 + 1.5j, 0.3 - 0.2j)))
NUM = ((0, 0, 1.0), (1, 0, 0.5), (0, 1, -0.75), (0, 2, 0.25), (1, 2, -0.1))
GRID = Grid(16, 12, -8.0, 4.0, -4.0, 4.0)
CASES = {
    "gribov_long": (Params(1.0, 1.0, 1.0, 1e4), GRIBOV, GC2),
    "gribov_long_d3": (Params(1.0, 1.0, 1.0, 1e4, 1.0, 0, 3), GRIBOV, GL),
    "gribov_long_t2": (Params(1.0, 1.0, 1.0, 1e4, 1.0, 2, 4), GRIBOV, GC2),
    "swept_residues": (Params(1.0, 1.0, 1.0, 1e4), SWEPT, GC2),
    "numerator": (Params(1.0, 1.0, 1.0, 1e4), Propagators(GRIBOV.poles1, GRIBOV.poles2, NUM), GC2),
    "single_long_d3": (Params(1 + 0.8j, 1.0, 1.0, 1e4, 1.0, 0, 3), None, GL),
}


@pytest.mark.parametrize("p,q", [
    (Params(1.0, 1.0, 1.0, 1e4), Quadrature(64, 32, 16)),
    (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e4, 1.0, 2), Quadrature(48, 24, 16)),
    (Params(1.0, 0.25, 2.0, 1e4, 1.0, 0, 3), Quadrature(48, 25, 16, 0, GL))],
    ids=["real", "conjugate_t2", "unequal_d3"])
def test_general_quad_evaluator_equals_the_single_pole_twin(p, q):
    x = oracle.grid_points(GRID)
    g_old, c_old = oracle.eval_points_q(p, q, x)
    g_new = oracle.eval_points_q_sets(p, q, x)
    _, c64 = oracle.eval_points(p, q, x)
    ok = (c_old == c64) & np.isfinite(g_old)
    assert ok.sum() >= 0.9 * x.size
    assert np.max(np.abs(g_new[ok] - g_old[ok]) / np.abs(g_old[ok])) < 1e-28


@pytest.mark.parametrize("case", list(CASES))
def test_fp64_oracle_rounding_for_general_integrands(case):
    p, props, rule = CASES[case]
    q = Quadrature(64, 32, 16, 0, rule)
    x = oracle.grid_points(GRID)
    g, c, cond = oracle.eval_points(p, q, x, want_cond=True, props=props)
    gq = oracle.eval_points_q_sets(p, q, x, props=props)
    ok = c != oracle.SINGULAR
    assert np.all(np.isnan(gq[~ok]))
    err = np.abs(g[ok] - gq[ok])
    assert np.all(err <= 64 * EPS * cond[ok] * np.abs(gq[ok])), np.max(err / (EPS * cond[ok] * np.abs(gq[ok])))
    if case != "gribov_long_t2":  # t^2 leaves a small remainder of its sums
        assert np.median(err / np.abs(gq[ok])) < 1e-14


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(CASES))
def test_gpu_fp64_rounding_for_general_integrands(case):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1205_0752_amd as gf
    p, props, rule = CASES[case]
    q = Quadrature(64, 32, 16, 0, rule)
    plan = gf.Plan(p, q, props=props)
    cls = torch.empty((GRID.n_im, GRID.n_re), dtype=torch.int8, device="cuda")
    g = gf.scan_plan(plan, GRID, cls=cls)
    torch.cuda.synchronize()
    plan.close()
    g = g.cpu().numpy().ravel()
    c = cls.cpu().numpy().ravel()
    x = oracle.grid_points(GRID)
    go, co = oracle.eval_points(p, q, x, props=props)
    gq = oracle.eval_points_q_sets(p, q, x, props=props)
    ok = (c == co) & (co != oracle.SINGULAR)
    assert ok.sum() >= 0.8 * x.size
    ref = np.abs(gq[ok])
    e_gpu = np.abs(g[ok] - gq[ok]) / ref
    e_or = np.abs(go[ok] - gq[ok]) / ref
    assert np.median(e_gpu) <= 4 * np.median(e_or) + 1e-16, (np.median(e_gpu), np.median(e_or))
    assert e_gpu.max() <= 4 * e_or.max() + 1e-16, (e_gpu.max(), e_or.max())
