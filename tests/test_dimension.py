"""Dimensions D = 2, 3 besides 4 (the hyperspherical measure of eq. 5-9 in
D dimensions: dy y^{(D-2)/2} and (1-z^2)^{(D-3)/2} dz, the angular part
normalised), and the Gauss-Legendre angular rule (natural for D = 3).

CPU pins of the oracle: the angular moments Gamma(k+1/2) Gamma(D/2) /
(sqrt(pi) Gamma(k+D/2)) (exact for each dimension's natural rule, to rounding
for tanh-sinh); the angular average against direct quadrature in the angle;
the loop sums against their Feynman forms, S_2 = int da / Delta and
S_3 = (pi/2) int da Delta^(-1/2), with and without the subtraction at mu^2,
including the derived cutoff bias (which the test shows is needed).  GPU:
scans in D = 2, 3 against the oracle (FP64, FP32C, several rules and orders),
the y-plane integrand in D = 3, and served results equal to standalone scans."""
import numpy as np
import pytest

import oracle
from parity_bars import check
from oracle import closed_forms as cf
from paper_1205_0752_amd.workloads import GC1, GC2, GL, TANH_SINH, Grid, Params, Quadrature

EPS = 2.0 ** -53
NATURAL = {2: GC1, 3: GL, 4: GC2}


@pytest.mark.parametrize("dim", [2, 3, 4])
@pytest.mark.parametrize("n", [1, 2, 5, 16])
def test_natural_rule_moments_exact(dim, n):
    z, w = oracle.angular_rule(NATURAL[dim], n, dim)
    for k in range(n):  # degree 2k <= 2n - 1
        assert abs(np.sum(w * z ** (2 * k)) - cf.angular_moment(k, dim)) <= 2e-15, (k,)
    z, w = oracle.angular_rule(NATURAL[dim], 3, dim)
    assert abs(np.sum(w * z ** 6) - cf.angular_moment(3, dim)) > 1e-4  # degree 6 > 5


@pytest.mark.parametrize("dim", [2, 3, 4])
def test_tanh_sinh_moments_in_every_dimension(dim):
    z, w = oracle.angular_rule(TANH_SINH, 97, dim)
    for k in range(6):
        assert abs(np.sum(w * z ** (2 * k)) - cf.angular_moment(k, dim)) <= 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_angular_average_matches_direct_quadrature(dim):
    rng = np.random.default_rng(2)
    x = 1.5 + 2.0j
    z, w = oracle.angular_rule(NATURAL[dim], 128, dim)
    checked = 0
    for y in rng.uniform(0.5, 8, 30) * np.exp(1j * rng.uniform(-1.2, 1.2, 30)):
        u, v = x + y + 1.0, 2 * np.sqrt(x) * np.sqrt(y)
        if np.min(np.abs(u - v * np.linspace(-1, 1, 2001))) < 0.1 * (abs(u) + abs(v)):
            continue
        ref = cf.angular_average_dim(u, v, dim)
        assert abs(np.sum(w / (u - v * z)) - ref) <= 1e-12 * abs(ref)
        checked += 1
    assert checked >= 8


MASSES = [(1.0, 1.0, 1.0), (2.0, 0.7, 1.5), (1 + 0.5j, 1 - 0.5j, 1.0)]
XS = [2 + 1j, -3 + 4j, 0.5 - 2j, -6 + 6j, 5 + 0.5j]


def _reference(x, m1, m2, mu2, dim, order, lam2, with_bias=True):
    ref = cf.loop_sum(x, m1, m2, dim)
    if order == 0:
        ref -= cf.loop_sum(mu2, m1, m2, dim)
    if with_bias:
        ref += cf.loop_sum_cutoff_bias(x, m1, m2, mu2, lam2, dim, order == 0)
    return ref


@pytest.mark.parametrize("m1,m2,mu2", MASSES)
@pytest.mark.parametrize("order", [-1, 0])
def test_two_dimensions_matches_feynman_form(m1, m2, mu2, order):
    """D = 2 with its natural rule: the radial integrand is analytic at y = 0,
    so the quadrature reaches rounding level."""
    p = Params(m1, m2, mu2, 1e6, 1.0, order, 2)
    g, _ = oracle.eval_points(p, Quadrature(512, 256, 32, 0, GC1), XS)
    for x, gx in zip(XS, g):
        ref = _reference(x, m1, m2, mu2, 2, order, 1e6)
        assert abs(gx - ref) <= 1e-12 * abs(ref), (x, gx, ref)


@pytest.mark.parametrize("m1,m2,mu2", MASSES)
@pytest.mark.parametrize("order", [-1, 0])
def test_three_dimensions_matches_feynman_form(m1, m2, mu2, order):
    """D = 3: y^(1/2) is not analytic at y = 0 in t = log(1+y), so the radial
    rule converges algebraically (error ~ n_r^-3); 512 nodes give ~1e-7 and
    doubling them cuts the error by at least 4."""
    errs = []
    for nr in (256, 512):
        p = Params(m1, m2, mu2, 1e6, 1.0, order, 3)
        g, _ = oracle.eval_points(p, Quadrature(nr, 128, 32, 0, GL), XS)
        errs.append(max(abs(gx - _reference(x, m1, m2, mu2, 3, order, 1e6)) /
                        abs(_reference(x, m1, m2, mu2, 3, order, 1e6)) for x, gx in zip(XS, g)))
    assert errs[1] <= 3e-7 and errs[1] <= errs[0] / 4, errs


def test_three_dimensions_cutoff_bias_is_needed():
    """Unsubtracted D = 3 misses the tail 2/Lambda of the y integral."""
    p = Params(1.0, 1.0, 1.0, 1e6, 1.0, -1, 3)
    g, _ = oracle.eval_points(p, Quadrature(512, 128, 32, 0, GL), XS)
    for x, gx in zip(XS, g):
        no_bias = _reference(x, 1.0, 1.0, 1.0, 3, -1, 1e6, with_bias=False)
        assert abs(gx - no_bias) > 1e-3
        assert abs(gx - _reference(x, 1.0, 1.0, 1.0, 3, -1, 1e6)) < 1e-6 * abs(no_bias)


def test_four_dimensions_unchanged_by_the_generalisation():
    """D = 4 with the default rule is the same quadrature as before: the
    Feynman form with the Lambda^-4 bias, to 5e-11."""
    p = Params(1.0, 1.0, 1.0, 1e4, 1.0, 0, 4)
    g, _ = oracle.eval_points(p, Quadrature(256, 128, 32), XS[:3])
    for x, gx in zip(XS[:3], g):
        ref = cf.feynman(x, 1.0, 1.0, 1.0) + cf.cutoff_bias(x, 1.0, 1.0, 1e4)
        assert abs(gx - ref) <= 5e-11 * max(abs(ref), 1.0)


# ---------------------------------------------------------------- GPU

def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1205_0752_amd as gf
    return torch, gf


@pytest.mark.gpu
@pytest.mark.parametrize("dim,rule,n_a", [(2, GC1, 32), (2, TANH_SINH, 49), (3, GL, 33),
                                          (3, TANH_SINH, 48), (4, GL, 32)])
@pytest.mark.parametrize("order", [-1, 0, 2])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32c"])
def test_gpu_scan_in_dimension_matches_oracle(dim, rule, n_a, order, prec):
    torch, gf = _gpu()
    cases = [(Params(2.0, 0.7, 1.5, 1e6, 1.0, order, dim), Grid(37, 29, -8.0, 4.0, -4.0, 4.0)),
             (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6, 1.0, order, dim),
              Grid(21, 17, -12.0, 6.0, -6.0, 6.0))]
    for p, grid in cases:
        q = Quadrature(64, n_a, 16, prec, rule)
        plan = gf.Plan(p, q)
        out = gf.empty_result(grid)
        cls = torch.empty((grid.n_im, grid.n_re), dtype=torch.int8, device="cuda")
        gf.scan_plan(plan, grid, out, cls)
        torch.cuda.synchronize()
        plan.close()
        g = out.cpu().numpy().ravel()
        c = cls.cpu().numpy().ravel()
        go, co, cond = oracle.scan(p, q, grid, want_cond=True)
        keep = (c == co) & (co != oracle.SINGULAR)
        assert (c != co).sum() <= 1
        check(prec, g[keep], go[keep], cond[keep], dim=dim)


@pytest.mark.gpu
@pytest.mark.parametrize("dim", [2, 3])
def test_gpu_yscan_integrand_in_dimension(dim):
    torch, gf = _gpu()
    p = Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6, 1.0, 0, dim)
    q = Quadrature(64, 64, 16, 0, NATURAL[dim])
    grid = Grid(40, 33, -6.0, 7.0, -4.0, 6.0)
    plan = gf.Plan(p, q)
    got = gf.yscan_plan(plan, 2.0 + 1.5j, grid, gf.YSCAN_INTEGRAND)
    torch.cuda.synchronize()
    got = got.cpu().numpy().ravel()
    plan.close()
    ys = oracle.grid_points(grid)
    ref = oracle.yscan(p, q, 2.0 + 1.5j, ys, 1)
    z, w = oracle.angular_rule(NATURAL[dim], 64, dim)

    def cond(x):
        # sum_j |w_j / D_j| (1 + (|U| + |V z_j|) / |D_j|) per y, as in the y-plane tests
        u = x + ys[:, None] + complex(p.m1sq)
        v = 2 * np.sqrt(complex(x)) * np.sqrt(ys)[:, None]
        d = u - v * z[None, :]
        return np.sum(np.abs(w / d) * (1 + (np.abs(u) + np.abs(v * z)) / np.abs(d)), axis=1)

    f = np.abs(ys if dim == 4 else (np.sqrt(ys) if dim == 3 else np.ones_like(ys)))
    bound = 64 * EPS * (cond(2.0 + 1.5j) + cond(p.mu2)) * f / np.abs(ys + complex(p.m2sq))
    assert np.all(np.abs(got - ref) <= bound + 1e-14 * np.abs(ref))


@pytest.mark.gpu
def test_gpu_served_dimensions_equal_standalone():
    torch, gf = _gpu()
    reqs = [(Params(1.0, 1.0, 1.0, 1e6, 1.0, order, dim), Grid(40, 24, -8.0, 4.0, -4.0, 4.0),
             Quadrature(64, 32, 16, prec, NATURAL[dim]))
            for dim in (2, 3, 4) for order in (-1, 0) for prec in (0, 1)]
    with gf.Server(budget_bytes=64 << 20, max_inflight=32, batch_evals=1e7) as srv:
        ts = [srv.submit(*r) for r in reqs]
        for t in ts:
            assert srv.wait(t, 120000.0)
        got = [srv.result(t) for t in ts]
    for (p, grid, q), g in zip(reqs, got):
        plan = gf.Plan(p, q)
        ref = gf.scan_plan(plan, grid, lanes=1)
        torch.cuda.synchronize()
        plan.close()
        ref = ref.cpu().numpy().ravel()
        assert np.array_equal(g.view(np.float64), ref.view(np.float64)), (p, q)
