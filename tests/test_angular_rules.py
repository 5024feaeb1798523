"""Angular quadrature rules: Gauss-Chebyshev of the second kind (default),
of the first kind, and tanh-sinh (the paper's main angular rule, section
"Numerical Implementation").

CPU pins of the oracle's rules: the moments <z^2k> = C_k / 4^k (C_k the
Catalan numbers) of the measure (2/pi) sqrt(1-z^2) dz, exact for the Gauss
rules up to their polynomial degree and to rounding for tanh-sinh at the
paper's 49 nodes; the angular average against its continuum closed form; the
whole subtracted integral agreeing across rules.  GPU: scans with each rule
against the oracle with the same rule, FP64 and FP32C."""
from math import comb

import numpy as np
import pytest

import oracle
from parity_bars import check
from oracle import closed_forms as cf
from paper_1205_0752_amd.workloads import GC1, GC2, TANH_SINH, Grid, Params, Quadrature

EPS = 2.0 ** -53


def _catalan_moment(k):
    return comb(2 * k, k) / (k + 1) / 4 ** k


@pytest.mark.parametrize("n", [1, 2, 3, 8, 17, 64])
def test_gauss_rules_exact_moments(n):
    """GC-II integrates z^2k exactly for 2k <= 2n - 1; GC-I (applied to
    f (1 - z^2)) for 2k + 2 <= 2n - 1."""
    for rule, maxdeg in ((GC2, 2 * n - 1), (GC1, 2 * n - 3)):
        z, w = oracle.angular_rule(rule, n)
        for k in range(0, 12):
            if 2 * k > maxdeg:
                break
            assert abs(np.sum(w * z ** (2 * k)) - _catalan_moment(k)) <= 1e-15, (rule, n, k)
        # and the rules are symmetric: odd moments vanish
        assert abs(np.sum(w * z)) <= 1e-15


def test_gauss_rules_not_exact_beyond_degree():
    """A degree past exactness shows a visible error (the exactness claims are
    tight, so a wrong node formula could not hide behind them)."""
    z, w = oracle.angular_rule(GC2, 4)
    assert abs(np.sum(w * z ** 8) - _catalan_moment(4)) > 1e-4
    z, w = oracle.angular_rule(GC1, 4)
    assert abs(np.sum(w * z ** 6) - _catalan_moment(3)) > 1e-4


def test_tanh_sinh_moments_and_convergence():
    """At the paper's 49 nodes (h = 1/8) the double-exponential rule gives the
    low moments to rounding; halving the node count (h = 1/4) loses accuracy
    visibly, as the rule's exp(-c/h) error predicts."""
    z, w = oracle.angular_rule(TANH_SINH, 49)
    for k in range(5):
        assert abs(np.sum(w * z ** (2 * k)) - _catalan_moment(k)) <= 4e-15, k
    assert np.all(w > 0) and np.all(np.abs(z) < 1)
    assert np.allclose(z, -z[::-1], rtol=0, atol=0) and np.array_equal(w, w[::-1])
    assert z[24] == 0.0 and w[24] == 1 / 8
    z, w = oracle.angular_rule(TANH_SINH, 25)
    err = abs(np.sum(w * z ** 4) - _catalan_moment(2))
    assert 1e-10 < err < 1e-5
    with pytest.raises(ValueError):
        oracle.angular_rule(TANH_SINH, 2)


def _uv(x, y, m1sq):
    return x + y + m1sq, 2 * np.sqrt(complex(x)) * np.sqrt(complex(y))


@pytest.mark.parametrize("rule,n", [(GC2, 256), (GC1, 256), (TANH_SINH, 193)])
def test_rules_reach_continuum_angular_average(rule, n):
    """Away from the cut, every rule reproduces 2/(U + sqrt(U^2 - V^2))."""
    rng = np.random.default_rng(11)
    x = 1.5 + 2.0j
    m1 = 1.0
    checked = 0
    z, w = oracle.angular_rule(rule, n)
    for y in rng.uniform(0.5, 8, 40) * np.exp(1j * rng.uniform(-1.2, 1.2, 40)):
        u, v = _uv(x, y, m1)
        if np.min(np.abs(u - v * np.linspace(-1, 1, 2001))) < 0.3 * (abs(u) + abs(v)) / 4:
            continue
        got = np.sum(w / (u - v * z))
        ref = cf.angular_continuum(u, v)
        assert abs(got - ref) <= 1e-12 * abs(ref), (rule, y, abs(got - ref) / abs(ref))
        checked += 1
    assert checked >= 10


def test_subtracted_integral_agrees_across_rules():
    """G(x) with the same radial nodes and GC-II (128), GC-I (128) or tanh-sinh
    (97) angular nodes agrees to 1e-8 at points away from the cut, and matches
    the Feynman closed form plus the cutoff bias."""
    p = Params(1.0, 1.0, 1.0, 1e6)
    xs = np.array([2.0 + 1.0j, -3.0 + 4.0j, 0.5 - 2.0j, -6.0 + 6.0j])
    res = []
    for rule, n in ((GC2, 128), (GC1, 128), (TANH_SINH, 97)):
        g, _ = oracle.eval_points(p, Quadrature(256, n, 32, angular_rule=rule), xs)
        res.append(g)
    for g in res[1:]:
        assert np.all(np.abs(g - res[0]) <= 1e-8 * np.abs(res[0])), np.abs(g - res[0])
    for x, g in zip(xs, res[2]):
        ref = cf.feynman(x, 1.0, 1.0, 1.0) + cf.cutoff_bias(x, 1.0, 1.0, 1e6)
        assert abs(g - ref) <= 1e-6 * abs(ref), (x, g, ref)


def test_library_rejects_bad_rules():
    """Validation happens on the host before any device work."""
    import paper_1205_0752_amd as gf
    p = Params(1.0, 1.0, 1.0, 1e6)
    for q in (Quadrature(64, 32, 16, angular_rule=7), Quadrature(64, 2, 16, angular_rule=TANH_SINH)):
        with pytest.raises(gf.GFError) as e:
            gf.Plan(p, q)
        assert e.value.code == -1


# ---------------------------------------------------------------- GPU parity

def _gpu_scan(gf, torch, params, quad, grid, lanes=0):
    plan = gf.Plan(params, quad)
    out = gf.empty_result(grid)
    cls = torch.empty((grid.n_im, grid.n_re), dtype=torch.int8, device="cuda")
    gf.scan_plan(plan, grid, out, cls, lanes=lanes)
    torch.cuda.synchronize()
    g = out.cpu().numpy().ravel()
    c = cls.cpu().numpy().ravel()
    plan.close()
    return g, c


@pytest.mark.gpu
@pytest.mark.parametrize("rule,n", [(GC1, 32), (GC1, 33), (TANH_SINH, 49), (TANH_SINH, 64)])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32c"])
def test_gpu_scan_with_rule_matches_oracle(rule, n, prec):
    """Every point of a ragged 37 x 29 grid (real masses) and of a 21 x 17 grid
    (conjugate pair: all four contour classes) against the oracle with the same
    angular rule.  FP64: |dG| <= max(1e-12 |G|, 64 eps kappa |G|) and 1e-12
    relative wherever kappa <= 1e3.  FP32C: 1e-6 max(|G|, 1) at every point."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1205_0752_amd as gf
    cases = [(Params(1.0, 1.0, 1.0, 1e4), Grid(37, 29, -8.0, 4.0, -4.0, 4.0)),
             (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6), Grid(21, 17, -12.0, 6.0, -6.0, 6.0))]
    for p, grid in cases:
        q = Quadrature(64, n, 16, prec, rule)
        g, c = _gpu_scan(gf, torch, p, q, grid)
        go, co, cond = oracle.scan(p, q, grid, want_cond=True)
        keep = (c == co) & (co != oracle.SINGULAR)
        assert (c != co).sum() <= 1
        check(prec, g[keep], go[keep], cond[keep], dim=4)


@pytest.mark.gpu
def test_gpu_tanh_sinh_subtraction_constant():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1205_0752_amd as gf
    p, q = Params(2.0, 0.7, 1.5, 1e6), Quadrature(256, 49, 16, angular_rule=TANH_SINH)
    plan = gf.Plan(p, q)
    j = plan.jmu()
    plan.close()
    jo = oracle.jmu(p, q)
    assert abs(j - jo) <= 1e-13 * abs(jo)
