"""y-plane diagnostics at a fixed external x (the paper's Fig. 1 and eq. 25).

CPU: the oracle's angular average <1/D1>(x, y) against the continuum closed
form away from the cut, the subtracted integrand against its definition, and
the cut curve of eq. 25 against the vanishing of the first propagator.
GPU: the y-plane kernel against the oracle on every point of a grid that
crosses the cut, within a bound set by the sum's conditioning."""
import cmath

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from paper_1205_0752_amd.workloads import Grid, Params, Quadrature

X = 2.0 + 1.5j
PARAMS = [Params(1.0, 1.0, 1.0, 1e6), Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6),
          Params(2.0, 0.7, 1.5, 1e6)]


def _gf():
    import paper_1205_0752_amd as gf
    return gf


def _uv(x, y, m1sq):
    """U = x + y + m1^2 and V = 2 sqrt(x) sqrt(y) of D1 = U - V z."""
    return x + y + m1sq, 2 * cmath.sqrt(x) * cmath.sqrt(y)


def _cut_distance(x, y, m1sq):
    """Distance from 0 of the segment {U - V z : z in [-1, 1]} over |U|+|V|."""
    u, v = _uv(x, y, m1sq)
    zs = np.linspace(-1, 1, 4001)
    return np.min(np.abs(u - v * zs)) / (abs(u) + abs(v))


@pytest.mark.parametrize("p", PARAMS, ids=["real", "conj", "unequal"])
def test_oracle_angular_matches_continuum_away_from_cut(p):
    """Where D1 keeps a distance from 0 over z in [-1, 1], the GC-II average
    converges geometrically to 2/(U + sqrt(U^2 - V^2)): at order 256 the
    difference is at rounding level."""
    rng = np.random.default_rng(3)
    ys = rng.uniform(-6, 6, 64) + 1j * rng.uniform(-6, 6, 64)
    ys = np.array([y for y in ys if _cut_distance(X, y, complex(p.m1sq)) > 0.05])
    assert ys.size >= 20
    got = oracle.yscan(p, Quadrature(64, 256, 16), X, ys, 0)
    for y, g in zip(ys, got):
        u, v = _uv(X, y, complex(p.m1sq))
        ref = cf.angular_continuum(u, v)
        assert abs(g - ref) <= 1e-13 * max(abs(ref), 1.0), (y, g, ref)


def test_oracle_integrand_matches_definition():
    """what = 1 is y/(y + m2^2) times the difference of the angular average
    at x and at mu^2 (eq. 14's subtracted integrand)."""
    p = Params(2.0, 0.7, 1.5, 1e6)
    q = Quadrature(64, 64, 16)
    ys = np.array([0.3 + 0.1j, 2.0 - 1.0j, -4.0 + 0.5j, 7.0 + 3.0j])
    a = oracle.yscan(p, q, X, ys, 0)
    ref = []
    for y in ys:
        u, v = _uv(X, y, 2.0)
        um, vm = _uv(p.mu2, y, 2.0)
        ref.append(y / (y + 0.7) * (oracle.angular_sum(u, v, 64) - oracle.angular_sum(um, vm, 64)))
    b = oracle.yscan(p, q, X, ys, 1)
    assert np.allclose(a, [oracle.angular_sum(*_uv(X, y, 2.0), 64) for y in ys], rtol=1e-14)
    assert np.allclose(b, ref, rtol=1e-13, atol=1e-15)


def test_integrand_vanishes_at_subtraction_point():
    """At x = mu^2 the subtracted integrand is identically zero."""
    p = Params(1.0, 1.0, 1.0, 1e6)
    ys = np.array([0.5 + 0.5j, -2 + 1j, 3 - 2j])
    assert np.all(oracle.yscan(p, Quadrature(64, 32, 16), p.mu2, ys, 1) == 0)


@pytest.mark.parametrize("p", PARAMS, ids=["real", "conj", "unequal"])
@pytest.mark.parametrize("x", [X, -1.5 + 0.5j, 0.4 - 2.0j])
def test_cut_curve_roots_zero_first_propagator(p, x):
    """Every point of both branches makes D1 vanish for z = cos t (eq. 25), and
    the branch product is y+ y- = (x + m1^2)^2 (product of the two roots of the
    quadratic in sqrt(y), squared)."""
    gf = _gf()
    n = 65
    yp, ym = gf.cut_curve(p, x, n)
    m1 = complex(p.m1sq)
    sx = cmath.sqrt(x)
    for k in range(n):
        c = np.cos(np.pi * k / (n - 1))
        for y in (yp[k], ym[k]):
            # either square root of y is a root of s^2 - 2 sqrt(x) c s + x + m1^2
            s = cmath.sqrt(y)
            res = min(abs(s * s - 2 * sx * c * s + x + m1), abs(s * s + 2 * sx * c * s + x + m1))
            assert res <= 1e-12 * (abs(y) + abs(x) + abs(m1)), (k, y, res)
        assert abs(yp[k] * ym[k] - (x + m1) ** 2) <= 1e-12 * abs(x + m1) ** 2


def test_cut_curve_rejects_bad_arguments():
    gf = _gf()
    with pytest.raises(gf.GFError):
        gf.cut_curve(Params(1.0, 1.0, 1.0, 1e6), X, 1)


def _cond(x, ys, m1sq, n):
    """sum_j |w_j / D1_j| (1 + (|U| + |V z_j|) / |D1_j|): the sum's absolute
    size times its sensitivity to relative perturbations of U and V."""
    z, w = oracle.gauss_cheb2(n)
    out = np.empty(ys.size)
    for k, y in enumerate(ys):
        u, v = _uv(x, y, m1sq)
        d = u - v * z
        out[k] = np.sum(np.abs(w / d) * (1 + (abs(u) + np.abs(v * z)) / np.abs(d)))
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("p", PARAMS, ids=["real", "conj", "unequal"])
@pytest.mark.parametrize("what", [0, 1])
def test_gpu_yscan_matches_oracle(p, what):
    """The y-plane kernel against the oracle on every point of two grids that
    cross the cut: 72 x 40 (whole 8 x 8 tiles) and 67 x 37 (ragged tiles)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf = _gf()
    q = Quadrature(64, 64, 16)
    for grid in (Grid(72, 40, -8.0, 8.0, -5.0, 5.0), Grid(67, 37, -6.0, 7.0, -4.0, 6.0)):
        plan = gf.Plan(p, q)
        out = gf.yscan_plan(plan, X, grid, what)
        torch.cuda.synchronize()
        got = out.cpu().numpy().ravel()
        plan.close()
        ys = oracle.grid_points(grid)
        ref = oracle.yscan(p, q, X, ys, what)
        m1 = complex(p.m1sq)
        cond = _cond(X, ys, m1, q.n_angular)
        if what == 1:
            cond = (cond + _cond(p.mu2, ys, m1, q.n_angular)) * np.abs(ys / (ys + complex(p.m2sq)))
        err = np.abs(got - ref)
        bound = 64 * 2.0 ** -53 * cond + 1e-14 * np.abs(ref)
        assert np.all(err <= bound), (grid, np.max(err / bound), ys[np.argmax(err / bound)])


@pytest.mark.gpu
def test_gpu_yscan_peaks_on_cut_curve():
    """|<1/D1>| over the y-plane is largest next to the eq. 25 curve: the grid
    point of largest modulus lies within two cells of a point of the curve."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf = _gf()
    p = Params(1.0, 1.0, 1.0, 1e6)
    grid = Grid(256, 256, -8.0, 8.0, -8.0, 8.0)
    plan = gf.Plan(p, Quadrature(64, 64, 16))
    a = gf.yscan_plan(plan, X, grid, 0)
    torch.cuda.synchronize()
    mod = np.abs(a.cpu().numpy().ravel())
    plan.close()
    ys = oracle.grid_points(grid)
    ymax = ys[np.argmax(mod)]
    yp, ym = gf.cut_curve(p, X, 4097)
    dist = np.min(np.abs(np.concatenate([yp, ym]) - ymax))
    assert dist <= 2 * np.hypot(16 / 256, 16 / 256), (ymax, dist)


@pytest.mark.gpu
def test_gpu_yscan_largest_grid():
    """The largest y grid the library takes, 65536 x 32768 = 2^31 points (a
    32 GiB result), at four angular nodes: every point is written, and the
    grid's first and last points, its last row and a spread of others match
    the oracle within the conditioning bound above."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf = _gf()
    p, q = PARAMS[1], Quadrature(16, 4, 4)
    grid = Grid(65536, 32768, -8.0, 8.0, -8.0, 8.0)
    n = grid.n_points
    plan = gf.Plan(p, q)
    out = gf.empty_result(grid)
    out.fill_(complex(float("nan"), 7.0))
    gf.yscan_plan(plan, X, grid, 0, out=out)
    torch.cuda.synchronize()
    plan.close()
    assert int((torch.isnan(out.real) & (out.imag == 7.0)).sum()) == 0
    rng = np.random.default_rng(13)
    idx = np.unique(np.concatenate([
        [0, grid.n_re - 1, n - grid.n_re, n - 1, n // 2 - 1, n // 2],
        n - grid.n_re + rng.choice(grid.n_re, 60, replace=False),
        rng.choice(n, 200, replace=False)]).astype(np.int64))
    got = out.view(-1)[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    ys = oracle.grid_points_at(grid, idx)
    ref = oracle.yscan(p, q, X, ys, 0)
    bound = 64 * 2.0 ** -53 * _cond(X, ys, complex(p.m1sq), q.n_angular) + 1e-14 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)
