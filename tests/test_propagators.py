"""General propagators (the integrand plug-in): F = P1((p-k)^2) P2(k^2) with
each propagator a sum of poles, P(s) = sum_a c_a / (s + m_a^2).

CPU pins of the oracle: real pole sums against the bilinear combination of
Feynman forms (the integral is bilinear in P1, P2); complex pole sums against
the bilinear combination of single-pole oracle results where every term has a
contour; the mirror symmetry of real-analytic propagators (complex-conjugate
pole pairs with conjugate residues); residues of several swept k-leg poles;
the single-pole case reproducing the plain scan.  GPU: pole-sum scans against
the oracle (FP64, FP32C, with t^2 and D = 3), the library's Taylor
coefficients, served pole-sum requests equal to standalone scans."""
import dataclasses

import numpy as np
import pytest

import oracle
from parity_bars import check
from oracle import closed_forms as cf
from paper_1205_0752_amd.workloads import Grid, Params, Propagators, Quadrature

EPS = 2.0 ** -53
REAL = Propagators(((1.0, 1.0), (4.0, -0.5)), ((0.5, 0.7), (2.0, 0.3)))
# a complex-conjugate pole pair on the (p-k) leg (a Gribov-type form
# s / (s^2 + M^4) shifted by a real mass) and a real pole sum on the k leg
GRIBOV1 = Propagators(Propagators.conjugate_pair(1.0 + 0.8j, 0.5), ((1.0, 0.6), (3.0, 0.4)))
# complex k-leg poles whose bad rays (-50 and -79 degrees) the rotated contour
# sweeps for points in the lower left quadrant (residues needed)
SWEPT2 = Propagators(((2.0, 1.0),), ((-0.5 + 0.6j, 0.7), (-0.3 + 1.5j, 0.3 - 0.2j)))
XS = [2 + 1j, -3 + 4j, 0.5 - 2j, -6 + 6j, 5 + 0.5j, -0.5 - 3j, -4 - 3j, -1 - 4j]


def test_real_pole_sums_match_bilinear_feynman_forms():
    p = Params(1.0, 1.0, 1.0, 1e6)
    g, cls = oracle.eval_points(p, Quadrature(512, 256, 16), XS, props=REAL)
    for x, gx in zip(XS, g):
        ref = sum(c1 * c2 * (cf.feynman(x, m1, m2, 1.0) + cf.cutoff_bias(x, m1, 1.0, 1e6))
                  for m1, c1 in REAL.poles1 for m2, c2 in REAL.poles2)
        assert abs(gx - ref) <= 1e-12 * abs(ref), (x, gx, ref)


@pytest.mark.parametrize("props", [GRIBOV1, SWEPT2], ids=["gribov1", "swept2"])
def test_complex_pole_sums_are_bilinear(props):
    """Where every single-pole term has a contour, the pole-sum result equals
    sum_ab c1_a c2_b G(x; m1_a, m2_b) (contours may differ per term: the
    agreement is to the quadrature's accuracy)."""
    p = Params(1.0, 1.0, 1.0, 1e6)
    q = Quadrature(512, 256, 32)
    xs = np.array(XS + [-1.5 + 0.3j, 1.0 + 3.0j, -2.0 - 0.5j])
    g, cls = oracle.eval_points(p, q, xs, props=props)
    tot = np.zeros(xs.size, complex)
    ok = cls != oracle.SINGULAR
    for m1, c1 in props.poles1:
        for m2, c2 in props.poles2:
            gs, cs = oracle.eval_points(Params(m1, m2, 1.0, 1e6), q, xs)
            ok &= cs != oracle.SINGULAR
            tot += c1 * c2 * gs
    assert ok.sum() >= 4
    assert np.all(np.abs(g[ok] - tot[ok]) <= 1e-9 * np.abs(tot[ok])), np.abs(g - tot)


def test_swept_k_leg_poles_add_their_residues():
    """SWEPT2's k-leg bad rays arg(-m2_b^2) lie at -50 and -79 degrees: points
    beyond both take the YRES class with one residue per swept pole, and still
    agree with the bilinear combination (checked above); dropping the residues
    would change the result at O(1)."""
    p = Params(1.0, 1.0, 1.0, 1e6)
    q = Quadrature(256, 128, 16)
    x = np.array([-4 - 3j, -1 - 4j])
    g, cls = oracle.eval_points(p, q, x, props=SWEPT2)
    assert np.all(cls == oracle.YRES)
    gy, cy = oracle.eval_points(p, q, x, force_class=oracle.Y, props=SWEPT2)
    assert np.all(np.abs(g - gy) > 1e-2 * np.abs(g))


def test_mirror_symmetry_of_real_analytic_propagators():
    p = Params(1.0, 1.0, 1.0, 1e6)
    q = Quadrature(128, 64, 16)
    xs = np.array([-4 + 2j, 1.5 + 3j, -0.5 + 0.7j, 3 - 1j])
    g, cls = oracle.eval_points(p, q, xs, props=GRIBOV1)
    gb, _ = oracle.eval_points(p, q, np.conj(xs), props=GRIBOV1)
    ok = cls != oracle.SINGULAR
    assert ok.sum() >= 3
    assert np.allclose(gb[ok], np.conj(g[ok]), rtol=1e-12, atol=0)


def test_single_pole_sum_reproduces_the_plain_scan():
    p = Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6)
    one = Propagators(((1 + 0.5j, 1.0),), ((1 - 0.5j, 1.0),))
    q = Quadrature(64, 32, 16)
    grid = Grid(24, 18, -12.0, 6.0, -6.0, 6.0)
    g0, c0 = oracle.scan(p, q, grid)
    g1, c1 = oracle.scan(p, q, grid, props=one)
    assert np.array_equal(c0, c1)
    ok = c0 != oracle.SINGULAR
    assert np.allclose(g1[ok], g0[ok], rtol=1e-13, atol=0)


def test_library_validates_propagators():
    import paper_1205_0752_amd as gf
    p = Params(1.0, 1.0, 1.0, 1e6)
    bad = Propagators(((-1.0, 1.0),), ((1.0, 1.0),))  # pole on the negative real axis
    with pytest.raises(gf.GFError) as e:
        gf.Plan(p, Quadrature(32, 16, 8), props=bad)
    assert e.value.code == -1
    with pytest.raises(gf.GFError) as e:  # split rule with two poles
        gf.Plan(p, Quadrature(32, 16, 8, radial_split=1), props=REAL)
    assert e.value.code == -2
    with pytest.raises(ValueError):
        gf.Plan(p, Quadrature(32, 16, 8), props=Propagators(tuple((1.0 + k, 1.0) for k in range(9)),
                                                           ((1.0, 1.0),)))


# ---------------------------------------------------------------- GPU

def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1205_0752_amd as gf
    return torch, gf


@pytest.mark.gpu
@pytest.mark.parametrize("props", [REAL, GRIBOV1, SWEPT2], ids=["real", "gribov1", "swept2"])
@pytest.mark.parametrize("order,dim", [(0, 4), (2, 4), (0, 3)])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32c"])
def test_gpu_pole_sum_scan_matches_oracle(props, order, dim, prec):
    torch, gf = _gpu()
    p = Params(1.0, 1.0, 1.0, 1e6, 1.0, order, dim)
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
        check(prec, g[keep], go[keep], cond[keep], dim=dim)


@pytest.mark.gpu
@pytest.mark.parametrize("props", [REAL, GRIBOV1], ids=["real", "gribov1"])
def test_gpu_pole_sum_taylor_coefficients(props):
    torch, gf = _gpu()
    p = Params(1.0, 1.0, 1.0, 1e6, 1.0, 3)
    q = Quadrature(128, 64, 16)
    plan = gf.Plan(p, q, props=props)
    K = np.array(plan.taylor())
    plan.close()
    Ko, rho = oracle.taylor(dataclasses.replace(p, taylor_order=0), q, 3, props=props)
    # the oracle's Cauchy-sum rounding is ~eps max|S| rho^-i on its circle; the
    # pole sums' terms partly cancel, so max|S| is taken as 4 |K_0| here
    for i in range(4):
        tol = 1e-12 * abs(Ko[i]) + 64 * EPS * 4 * abs(Ko[0]) * rho ** -i
        assert abs(K[i] - Ko[i]) <= tol, (i, K[i], Ko[i])


@pytest.mark.gpu
def test_gpu_served_pole_sums_equal_standalone():
    torch, gf = _gpu()
    reqs = [(Params(1.0, 1.0, 1.0, 1e6, 1.0, order), Grid(40, 24, -8.0, 4.0, -4.0, 4.0),
             Quadrature(64, 32, 16, prec), props)
            for order in (0, 2) for prec in (0, 1) for props in (None, REAL, SWEPT2)]
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
