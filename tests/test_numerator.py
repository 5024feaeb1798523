"""Numerators: the integrand N(k^2, p.k) P1((p-k)^2) P2(k^2) of eq. 4's general
form, with N = sum_{i,j<=2} n_ij (k^2)^i (p.k)^j and pole-sum propagators.

CPU pins of the oracle.  (1) The numerator D1 Q(k^2, p.k), D1 = (p-k)^2 + m1^2,
cancels a single-pole P1 term by term, so the integral is that of Q P2 alone,
whose odd powers of p.k average to zero: G = int_0^Lambda^2 dy y (q00 + q10 y)
P2(y), a closed form, on every contour class (the contour sum of an integrand
analytic up to P2's poles is the real-axis integral, with the swept poles'
residues).  This fixes the placement and sign of every coefficient but n_22,
the factor of p.k = sqrt(x) sqrt(y) z and its branch on rotated contours.
(2) A rotated contour forced where the real axis is valid gives the same
result.  (3) Real coefficients keep G(conj x) = conj G(x) for real-analytic
propagators.  (4) A constant numerator scales the plain result.
GPU: scans against the oracle (FP64, FP32C; D = 4 and 3; orders -1, 0 and 2),
the power-series Taylor coefficients against the oracle's Cauchy-formula ones,
served numerator requests equal to standalone scans, validation."""
import numpy as np
import pytest

import oracle
from parity_bars import check
from paper_1205_0752_amd.workloads import Grid, Params, Propagators, Quadrature

M1 = 1.0
# k-leg poles whose bad rays (-50 and -79 degrees) the rotated contour sweeps
# for points in the lower left quadrant: residues with the numerator in them
SWEPT_K = ((-0.5 + 0.6j, 0.7), (-0.3 + 1.5j, 0.3 - 0.2j))
Q = {(0, 0): 0.7 - 0.2j, (1, 0): 0.3 + 0.1j, (0, 1): -0.4 + 0.5j, (1, 1): 0.25 - 0.3j}
# every coefficient in play, complex
NUM_FULL = ((0, 0, 0.8 - 0.1j), (1, 0, 0.3 + 0.2j), (2, 0, 0.01 - 0.05j), (0, 1, 0.4),
            (1, 1, -0.2 + 0.1j), (2, 1, 0.02), (0, 2, 0.1 - 0.3j), (1, 2, 0.05),
            (2, 2, 0.01 + 0.01j))
# a real numerator (a p.k-dependent tensor structure)
NUM_REAL = ((0, 0, 1.0), (1, 0, 0.5), (0, 1, -0.75), (0, 2, 0.25), (1, 2, -0.1))
REAL = Propagators(((1.0, 1.0), (4.0, -0.5)), ((0.5, 0.7), (2.0, 0.3)), NUM_FULL)
GRIBOV1 = Propagators(Propagators.conjugate_pair(1.0 + 0.8j, 0.5), ((1.0, 0.6), (3.0, 0.4)),
                      NUM_REAL)
SWEPT2 = Propagators(((2.0, 1.0),), SWEPT_K, NUM_FULL)


def d1_times_q(x, m1sq=M1):
    """Coefficients of D1 Q with D1 = (x + m1^2) + k^2 - 2 p.k."""
    c0 = complex(x) + m1sq
    n = {}
    for (i, j), q in Q.items():
        for (di, dj, f) in ((0, 0, c0), (1, 0, 1.0), (0, 1, -2.0)):
            n[(i + di, j + dj)] = n.get((i + di, j + dj), 0) + f * q
    return tuple((i, j, c) for (i, j), c in n.items())


def q_p2_integral(poles2, lam2):
    """int_0^lam2 dy y (q00 + q10 y) sum_b c_b / (y + m_b): per pole
    int y/(y+m) = L - m log(1 + L/m), int y^2/(y+m) = L^2/2 - m L + m^2 log(1 + L/m)."""
    tot = 0.0
    for m, c in poles2:
        m = complex(m)
        lg = np.log((lam2 + m) / m)
        tot += c * (Q[(0, 0)] * (lam2 - m * lg) + Q[(1, 0)] * (lam2 ** 2 / 2 - m * lam2 + m * m * lg))
    return tot


@pytest.mark.parametrize("poles2,xs", [
    (((0.5, 1.0),), [2 + 1j, -3 + 4j, 0.5 - 2j, -6 + 6j, 5 + 0.5j, -0.5 - 3j, 0.3]),
    (SWEPT_K, [-4 - 3j, -1 - 4j, 2 + 1j, -3 + 4j, -6 + 6j]),
], ids=["real_k_pole", "swept_k_poles"])
def test_d1_numerator_cancels_the_first_propagator(poles2, xs):
    lam2 = 1e4
    p = Params(M1, 1.0, 1.0, lam2, 1.0, -1, 4)
    ref = q_p2_integral(poles2, lam2)
    seen = set()
    for x in xs:
        props = Propagators(((M1, 1.0),), poles2, d1_times_q(x))
        g, c = oracle.eval_points(p, Quadrature(128, 32, 16), [x], props=props)
        seen.add(int(c[0]))
        assert abs(g[0] - ref) <= 1e-13 * abs(ref), (x, int(c[0]), g[0], ref)
    # the real axis, rotated rays, and (swept k-leg poles) residues
    assert seen >= ({oracle.R, oracle.Y} if len(poles2) == 1 else {oracle.YRES, oracle.Y})


def test_rotated_contour_agrees_with_the_real_axis():
    p = Params(1.0, 1.0, 1.0, 1e4, 1.0, 0, 4)
    q = Quadrature(256, 64, 32)
    xs = np.array([0.5 + 0.1j, 0.3 - 0.05j, 0.6 + 0.0j])
    for props in (REAL, GRIBOV1):
        g, c = oracle.eval_points(p, q, xs, props=props)
        assert np.all(c == oracle.R)
        gy, cy = oracle.eval_points(p, q, xs, force_class=oracle.Y, props=props)
        assert np.all(np.abs(g - gy) <= 1e-10 * np.abs(g)), np.abs(g - gy) / np.abs(g)


def test_real_numerator_keeps_the_mirror_symmetry():
    p = Params(1.0, 1.0, 1.0, 1e4, 1.0, 0, 4)
    q = Quadrature(128, 64, 16)
    xs = np.array([-4 + 2j, 1.5 + 3j, -0.5 + 0.7j, 3 - 1j])
    g, cls = oracle.eval_points(p, q, xs, props=GRIBOV1)
    gb, _ = oracle.eval_points(p, q, np.conj(xs), props=GRIBOV1)
    ok = cls != oracle.SINGULAR
    assert ok.sum() >= 3
    assert np.allclose(gb[ok], np.conj(g[ok]), rtol=1e-12, atol=0)


def test_constant_numerator_scales_the_plain_result():
    p = Params(1.0, 1.0, 1.0, 1e4, 1.0, 0, 4)
    q = Quadrature(64, 32, 16)
    xs = np.array([-4 + 2j, 1.5 + 3j, -0.5 - 0.7j, 3 - 1j, 0.4])
    plain = Propagators(((1.0, 1.0),), ((0.5, 1.0),))
    c = 0.3 - 1.7j
    g0, c0, cond = oracle.eval_points(p, q, xs, props=plain, want_cond=True)
    g1, c1 = oracle.eval_points(p, q, xs, props=Propagators(plain.poles1, plain.poles2,
                                                            ((0, 0, c),)))
    assert np.array_equal(c0, c1)
    ok = c0 != oracle.SINGULAR
    # the two differ by rounding only: the multiplication by c happens per
    # node, before the subtraction's cancellation (condition number cond)
    ref = c * g0[ok]
    assert np.all(np.abs(g1[ok] - ref) <= 16 * 2.0 ** -53 * cond[ok] * np.abs(ref))


def test_library_validates_numerators():
    import paper_1205_0752_amd as gf
    p = Params(1.0, 1.0, 1.0, 1e6)
    q = Quadrature(32, 16, 8)
    with pytest.raises(gf.GFError) as e:  # the split radial rule takes no numerator
        gf.Plan(p, Quadrature(32, 16, 8, radial_split=1),
                props=Propagators(((1.0, 1.0),), ((1.0, 1.0),), ((0, 1, 1.0),)))
    assert e.value.code == -2
    with pytest.raises(gf.GFError) as e:
        gf.Plan(p, q, props=Propagators(REAL.poles1, REAL.poles2, ((0, 1, float("nan")),)))
    assert e.value.code == -1
    with pytest.raises(ValueError):
        gf.Plan(p, q, props=Propagators(REAL.poles1, REAL.poles2, ((3, 0, 1.0),)))


# ---------------------------------------------------------------- GPU

def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1205_0752_amd as gf
    return torch, gf


@pytest.mark.gpu
@pytest.mark.parametrize("props", [REAL, GRIBOV1, SWEPT2], ids=["real", "gribov1", "swept2"])
@pytest.mark.parametrize("order,dim,lam2", [(0, 4, 1e6), (-1, 4, 1e4), (0, 3, 1e4), (2, 4, 1e4)])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32c"])
def test_gpu_numerator_scan_matches_oracle(props, order, dim, lam2, prec):
    torch, gf = _gpu()
    if order == 2:
        # t^2 with a numerator of degree 4 in k: the sums grow like Lambda^4
        # while G is what the subtraction leaves (condition numbers 1e8 and
        # more), so only the FP64 path resolves it; the FP64 bar is the
        # condition-number bar
        if prec == 1:
            pytest.skip("FP32 sums cannot resolve a remainder 1e8 times smaller than they are")
        props = Propagators(props.poles1, props.poles2, NUM_REAL)
    p = Params(1.0, 1.0, 1.0, lam2, 1.0, order, dim)
    q = Quadrature(64, 32, 16, prec, 3 if dim == 3 else 0)
    for grid in (Grid(37, 29, -8.0, 4.0, -4.0, 4.0), Grid(21, 17, -12.0, 6.0, -6.0, 6.0)):
        plan = gf.Plan(p, q, props=props)
        out = gf.empty_result(grid)
        cls = torch.empty((grid.n_im, grid.n_re), dtype=torch.int8, device="cuda")
        gf.scan_plan(plan, grid, out, cls)
        torch.cuda.synchronize()
        plan.close()
        g = out.cpu().numpy().ravel()
        c = cls.cpu().numpy().ravel()
        go, co, cond = oracle.scan(p, q, grid, want_cond=True, props=props)
        assert (c != co).sum() <= 1
        assert np.all(np.isnan(g[(c == co) & (co == oracle.SINGULAR)]))
        keep = (c == co) & (co != oracle.SINGULAR)
        # every point off the bad rays has a contour (the long way round included)
        assert keep.sum() >= 0.9 * grid.n_points
        check(prec, g[keep], go[keep], cond[keep], dim=dim)


@pytest.mark.gpu
@pytest.mark.parametrize("props", [REAL, GRIBOV1], ids=["real", "gribov1"])
def test_gpu_numerator_taylor_coefficients(props):
    """The library's power-series coefficients with a numerator against the
    oracle's Cauchy-formula ones (an independent method)."""
    import dataclasses
    torch, gf = _gpu()
    p = Params(1.0, 1.0, 1.0, 1e6, 1.0, 3)
    q = Quadrature(128, 64, 16)
    plan = gf.Plan(p, q, props=props)
    K = np.array(plan.taylor())
    plan.close()
    Ko, rho = oracle.taylor(dataclasses.replace(p, taylor_order=0), q, 3, props=props)
    eps = 2.0 ** -53
    for i in range(4):
        tol = 1e-12 * abs(Ko[i]) + 64 * eps * 4 * abs(Ko[0]) * rho ** -i
        assert abs(K[i] - Ko[i]) <= tol, (i, K[i], Ko[i])


@pytest.mark.gpu
def test_gpu_served_numerators_equal_standalone():
    torch, gf = _gpu()
    reqs = [(Params(1.0, 1.0, 1.0, 1e6, 1.0, order), Grid(40, 24, -8.0, 4.0, -4.0, 4.0),
             Quadrature(64, 32, 16, prec), props)
            for order in (-1, 0, 2) for prec in (0, 1) for props in (None, REAL, SWEPT2)]
    with gf.Server(budget_bytes=64 << 20, max_inflight=32, batch_evals=1e7) as srv:
        ts = [srv.submit(*r) for r in reqs]
        for t in ts:
            assert srv.wait(t, 120000.0)
        got = [srv.result(t) for t in ts]
    for (p, grid, q, props), g in zip(reqs, got):
        plan = gf.Plan(p, q, props=props)
        ref = gf.scan_plan(plan, grid, lanes=1)
        torch.cuda.synchronize()
        plan.close()
        ref = ref.cpu().numpy().ravel()
        assert np.array_equal(g.view(np.float64), ref.view(np.float64), equal_nan=True), (p, q)
