"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element on the same cell-centred grid points (GPU tests, MI355X).

Bars (parity_bars): FP64 within max(1e-12 |G|, 64 eps kappa |G|) everywhere
and 1e-12 relative wherever the oracle's condition number kappa <= 1e3 (the
GPU computes sqrt, sincos and the reciprocal with its own, equally accurate,
routines), with at most 3 % of the points of the named workloads above
kappa = 1e3; FP32C within 1e-6 max(|G|, 1) at every point.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1205_0752_amd as gf  # noqa: E402
from paper_1205_0752_amd.workloads import CONFIGS, Grid, Params, Quadrature, sample_points  # noqa: E402
from parity_bars import band_report, check_fp32c, check_fp64  # noqa: E402

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    gf.load()
    yield
    gf.cache_clear()


def _gpu_scan(params, quad, grid, lanes=0):
    plan = gf.Plan(params, quad)
    out = gf.empty_result(grid)
    cls = torch.empty((grid.n_im, grid.n_re), dtype=torch.int8, device="cuda")
    gf.scan_plan(plan, grid, out, cls, lanes=lanes)
    torch.cuda.synchronize()
    g = out.cpu().numpy().ravel()
    c = cls.cpu().numpy().ravel()
    plan.close()
    return g, c


def _compare(g_gpu, c_gpu, params, quad, x, g_or, c_or, cond, max_bad_share=None):
    """Element-wise FP64 check (parity_bars.check_fp64); returns its
    statistics."""
    assert g_gpu.shape == g_or.shape
    # contour class: must agree except where floating point sits on a decision
    # boundary; there the GPU value is compared with the oracle forced to the
    # GPU's class (both contours are valid there)
    mism = np.nonzero(c_gpu != c_or)[0]
    assert mism.size <= max(2, g_or.size // 10000), (mism.size, x[mism][:5])
    if mism.size:
        for k in mism:
            gk, ck = oracle.eval_points(params, quad, [x[k]], force_class=int(c_gpu[k]))
            g_or[k] = gk[0]
    sing = c_or == oracle.SINGULAR
    assert np.all(np.isnan(g_gpu[sing & (c_gpu == oracle.SINGULAR)]))
    ok = ~sing
    return check_fp64(g_gpu[ok], g_or[ok], cond[ok], max_bad_share)


def test_config0_full_grid_matches_oracle():
    """64 x 64 box, m1 = m2 = 1, mu^2 = 1, Lambda^2 = 1e4, 64 x 32 nodes:
    every point against the oracle."""
    p, grid, q = CONFIGS["c0_fp64_64sq"]
    g, c = _gpu_scan(p, q, grid)
    go, co, cond = oracle.scan(p, q, grid, want_cond=True)
    x = oracle.grid_points(grid)
    stats = _compare(g, c, p, q, x, go, co, cond, max_bad_share=0.03)
    print("config0", stats)


@pytest.mark.parametrize("lanes", [1, 2, 4, 16, 64])
def test_ragged_grid_all_lane_splits(lanes):
    """37 x 23 points (ragged against every tile shape), real unequal masses;
    each lanes-per-point split gives the oracle's values."""
    p = Params(1.0, 0.25, 2.0, 1e4, 1.0)
    q = Quadrature(48, 24, 8)
    grid = Grid(37, 23, -7.0, 5.0, -3.0, 4.5)
    g, c = _gpu_scan(p, q, grid, lanes=lanes)
    go, co, cond = oracle.scan(p, q, grid, want_cond=True)
    _compare(g, c, p, q, oracle.grid_points(grid), go, co, cond)


def _tail_case(form):
    from paper_1205_0752_amd.workloads import Propagators
    pair = Propagators(Propagators.conjugate_pair(1.0 + 0.8j, 0.5), ((1.0, 0.6), (3.0, 0.4)))
    p, q, props, n_im = Params(1.0, 1.0, 1.0, 1e6), Quadrature(128, 64, 16), None, 1024
    if form == "fp32c":
        q, n_im = Quadrature(128, 64, 16, gf.FP32C), 1000
    elif form == "t2":
        p = Params(1.0, 1.0, 1.0, 1e6, 1.0, 2)
    elif form == "split":
        q = Quadrature(128, 64, 16, gf.FP64, gf.GC2, 1)
    elif form == "poles":
        props = pair
    elif form == "numerator":
        props = Propagators(pair.poles1, pair.poles2, ((0, 0, 1.0), (1, 0, 0.5), (0, 1, 0.3j), (0, 2, 0.2)))
    return p, q, props, Grid(1030, n_im, -16.0, 8.0, -8.0, 8.0)


@pytest.mark.parametrize("form", ["fp64", "fp32c", "t2", "split", "poles", "numerator"])
def test_tail_rows_on_a_ragged_grid(form):
    """A large scan at the automatic lane count (one lane per point here) runs
    its last rows at 16 lanes per point in the same launch, in every kernel
    form.  On a 1030-wide grid (the tail's tiles hold four points, the last
    one half outside the grid) every point is written, its class equals the
    one-lane scan's and its value the one-lane scan's up to rounding, and
    points of the last 128 rows (the tail and the rows before it) match the
    oracle at the parity bar.  The allocation-free scan, which takes the same
    tail on node tables generated on the device (equal to the plan's to the
    last bits), writes every point too and agrees to rounding."""
    p, q, props, grid = _tail_case(form)
    prec = q.precision
    plan = gf.Plan(p, q, props=props)
    assert plan.auto_lanes(grid) == 1
    auto = gf.empty_result(grid)
    auto.fill_(complex(float("nan"), 7.0))
    cls_a = torch.full((grid.n_im, grid.n_re), 9, dtype=torch.int8, device="cuda")
    gf.scan_plan(plan, grid, auto, cls_a)
    cls_1 = torch.empty_like(cls_a)
    one = gf.scan_plan(plan, grid, cls=cls_1, lanes=1)
    na = None
    if props is None and form in ("fp64", "fp32c"):
        na = gf.empty_result(grid)
        na.fill_(complex(float("nan"), 7.0))
        gf.scan_noalloc(p, grid, q, na)
    torch.cuda.synchronize()
    plan.close()
    g, g1 = auto.cpu().numpy().ravel(), one.cpu().numpy().ravel()
    c, c1 = cls_a.cpu().numpy().ravel(), cls_1.cpu().numpy().ravel()
    assert np.array_equal(c, c1) and not np.any(c == 9)
    sing = c == oracle.SINGULAR
    assert np.all(np.isnan(g[sing])) and np.all(np.isfinite(g[~sing]))
    scale = np.max(np.abs(g1[~sing]))
    # the tail's points are summed over 16 lanes: rounding only (the t^2 sums
    # cancel the most, by ~1e4 on this machine)
    tol = {"fp32c": 1e-6, "t2": 1e-10}.get(form, 1e-12)
    assert np.max(np.abs(g[~sing] - g1[~sing])) <= tol * scale
    if na is not None:
        gn = na.cpu().numpy().ravel()
        assert np.all(np.isnan(gn[sing])) and np.all(np.isfinite(gn[~sing]))
        # the device-generated tables move the quadrature by a few ulp, which
        # the points near the angular cut amplify (kappa): a looser bar, still
        # far below what a misplaced or missing tile would show
        assert np.max(np.abs(gn[~sing] - g[~sing])) <= (1e-9 if prec == 0 else 2e-6) * scale
    rows = np.arange(grid.n_points) // grid.n_re
    rng = np.random.default_rng(5)
    pick = rng.choice(np.nonzero((rows >= grid.n_im - 128) & ~sing)[0], 300, replace=False)
    x = oracle.grid_points(grid)[pick]
    go, co, cond = oracle.eval_points(p, q, x, want_cond=True, props=props)
    assert (co != c[pick]).sum() <= 1
    keep = co == c[pick]
    if prec == 0:
        check_fp64(g[pick][keep], go[keep], cond[keep])
    else:
        check_fp32c(g[pick][keep], go[keep])


def test_paper_worked_example_box_matches_oracle():
    """The paper's worked example (m1^2 = -i/2, m2^2 = +i/2, mu^2 = 0) on its
    display box (128^2 over +-5, STEP 4), all four contour classes."""
    p = Params(-0.5j, 0.5j, 0.0, 1e6, 1.0)
    q = Quadrature(128, 64, 16)
    grid = Grid(128, 128, -5.0, 5.0, -5.0, 5.0)
    g, c = _gpu_scan(p, q, grid)
    go, co, cond = oracle.scan(p, q, grid, want_cond=True)
    assert set(np.unique(c).tolist()) == {0, 1, 2, 3}
    _compare(g, c, p, q, oracle.grid_points(grid), go, co, cond, max_bad_share=0.03)


def test_eq18_on_gpu():
    """The GPU path against the exact solution eq. 18 directly, 1 x 1 grids
    centred on the stored points; 512 x 256 nodes, Lambda^2 = 1e6."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "eq18_points.json")) as f:
        pts = json.load(f)["points"]
    p = Params(-0.5j, 0.5j, 0.0, 1e6, 1.0)
    plan = gf.Plan(p, Quadrature(512, 256, 16))
    h = 2.0 ** -20
    errs = []
    for xr, xi, gr, gi in pts:
        grid = Grid(1, 1, xr - h, xr + h, xi - h, xi + h)
        out = gf.scan_plan(plan, grid)
        torch.cuda.synchronize()
        val = complex(out.cpu().numpy().ravel()[0])
        # rays within 0.3 rad of the bad rays arg x = +-pi/2, outside region R,
        # converge more slowly with the node count (see the oracle's pins)
        delta = abs(abs(math.atan2(xi, xr)) - math.pi / 2)
        near_bad_ray = delta < 0.3 and abs((complex(xr, xi) ** 0.5).imag) >= 0.5
        errs.append((abs(val - complex(gr, gi)), near_bad_ray, (xr, xi)))
    plan.close()
    for e, near, x in errs:
        assert e < (1e-6 if near else 5e-11), (x, e)


def test_config1_full_grid_matches_oracle():
    """The benchmark workload at full size (1024^2 points, 256 x 128 nodes,
    Lambda^2 = 1e6) in the benchmark's launch configuration: every point
    against the oracle (about 14 s of oracle time on 16 host threads), plus
    conjugation symmetry of the whole grid."""
    p, grid, q = CONFIGS["c1_fp64_1024sq"]
    g, c = _gpu_scan(p, q, grid)
    go, co, cond = oracle.scan(p, q, grid, want_cond=True)
    x = oracle.grid_points(grid)
    stats = _compare(g, c, p, q, x, go, co, cond, max_bad_share=0.03)
    print("config1 full grid", stats)
    assert np.all(np.isfinite(g))
    gm = g.reshape(grid.n_im, grid.n_re)
    # the grid is symmetric under Im x -> -Im x (rows b and n_im - 1 - b)
    assert np.max(np.abs(gm - np.conj(gm[::-1])) / np.abs(gm)) < 1e-13


@pytest.mark.parametrize("name", ["c3a_conj_2048sq", "c3b_unequal_2048sq"])
def test_config3_full_size_sampled(name):
    """The 2048^2 workloads at full size and nodes (512 x 256 + 16): complex
    masses m^2 = 1 +- 0.5i (every contour class) and unequal real masses
    m1 = 1, m2 = 0.5 with mu^2 = 2, in the benchmark's launch configuration:
    sampled points against the oracle; NaN exactly at the SINGULAR class.
    With real masses the quadrature at conj x is the mirror image of the one
    at x, so G(conj x) = conj G(x) to rounding, row against row (the grid is
    symmetric under Im x -> -Im x); with conjugate masses conjugation swaps
    the legs, which the continuum function allows but the discretised
    integral only to its quadrature error, so that check is not made."""
    p, grid, q = CONFIGS[name]
    g, c = _gpu_scan(p, q, grid)
    idx = sample_points(grid, 400, seed=3)
    x = oracle.grid_points_at(grid, idx)
    go, co, cond = oracle.eval_points(p, q, x, want_cond=True)
    print(name, _compare(g[idx], c[idx], p, q, x, go, co, cond, max_bad_share=0.03))
    bidx = _band_sample(grid, 300, seed=4)
    xb = oracle.grid_points_at(grid, bidx)
    go, co, cond = oracle.eval_points(p, q, xb, want_cond=True)
    print(name, "cut and pinch band", _compare(g[bidx], c[bidx], p, q, xb, go, co, cond))
    assert np.array_equal(np.isnan(g), c == gf.CLASS_SINGULAR)
    if complex(p.m1sq).imag == 0 and complex(p.m2sq).imag == 0:
        gm = g.reshape(grid.n_im, grid.n_re)
        ok = np.isfinite(gm) & np.isfinite(gm[::-1])
        rel = np.abs(gm - np.conj(gm[::-1]))[ok] / np.abs(gm[ok])
        assert rel.max() < 1e-12, rel.max()


def test_conjugate_masses_sampled():
    """m1^2 = 1 + 0.5i, m2^2 = 1 - 0.5i, mu^2 = 1 on the 2:1 box of the
    complex-mass workload (reduced to 256^2 points, 512 x 256 nodes)."""
    p = Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6, 1.0)
    q = Quadrature(512, 256, 16)
    grid = Grid(256, 256, -12.0, 6.0, -6.0, 6.0)
    g, c = _gpu_scan(p, q, grid)
    assert set(np.unique(c).tolist()) >= {0, 1, 2, 3}
    idx = sample_points(grid, 300, seed=2)
    x = oracle.grid_points_at(grid, idx)
    go, co, cond = oracle.eval_points(p, q, x, want_cond=True)
    _compare(g[idx], c[idx], p, q, x, go, co, cond)


def test_singular_points_nan_and_class():
    """Points exactly on the negative real axis below -m1^2 (real masses) have
    no fixed contour: NaN and class SINGULAR, like the oracle."""
    p = Params(1.0, 1.0, 1.0, 1e4, 1.0)
    q = Quadrature(32, 16, 4)
    grid = Grid(8, 3, -6.0, 2.0, -1.5, 1.5)  # middle row is Im x = 0 exactly
    g, c = _gpu_scan(p, q, grid)
    go, co = oracle.scan(p, q, grid)
    assert np.array_equal(c, co)
    assert np.array_equal(np.isnan(g), np.isnan(go))
    assert np.isnan(g).sum() >= 3


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32c"])
@pytest.mark.parametrize("p", [Params(1.0, 1.0, 0.0, 1e4, 1.0), Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e4, 1.0),
                               Params(-0.5j, 0.5j, 0.0, 1e4, 1.0)], ids=["real_mu0", "conj", "paper"])
def test_degenerate_points_x_zero_and_x_mu2(p, prec):
    """Grid points exactly at x = 0 (V^2 = 0: every angular term is 1/U) and
    exactly at x = mu^2 (G = 0 by the subtraction): a 5 x 5 box of unit
    cells centred on 0 puts both on the grid for mu^2 in {0, 1}.  Every point
    against the oracle at the parity bar; at x = mu^2 |G| stays at rounding
    size next to the subtracted sum."""
    q = Quadrature(64, 32, 16, prec)
    grid = Grid(5, 5, -2.5, 2.5, -2.5, 2.5)
    x = oracle.grid_points(grid)
    assert (x == 0).sum() == 1 and (x == 1.0).sum() == 1
    g, c = _gpu_scan(p, q, grid)
    go, co, cond = oracle.scan(p, q, grid, want_cond=True)
    assert np.array_equal(c, co)
    k = int(np.nonzero(x == complex(p.mu2))[0][0])
    ok = co != oracle.SINGULAR
    assert ok[k] and go[k] == 0
    assert np.all(np.isnan(g[~ok]))
    # every point but x = mu^2 (G = 0, no relative bar) at the parity bar
    ok[k] = False
    if prec == 0:
        check_fp64(g[ok], go[ok], cond[ok])
    else:
        check_fp32c(g[ok], go[ok])
    plan = gf.Plan(p, q)
    jmu = plan.jmu()
    plan.close()
    # the subtracted sum at mu^2 itself: rounding of |J(mu^2)| only
    assert abs(g[k]) <= (1e-12 if prec == 0 else 1e-6) * max(1.0, abs(jmu)), (g[k], jmu)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32c"])
def test_largest_grid_2_31_points(prec):
    """The largest grid the library takes, 65536 x 32768 = 2^31 points (flat
    indices up to 2^31 - 1, a 32 GiB result), at few nodes per point: the
    automatic count (one lane per point, with the 16-lane tail) covers every
    point exactly once -- every class written, every value finite off the
    SINGULAR class and NaN on it -- and the first and last points of the
    grid, of its last row and a spread of others match the oracle at the
    parity bar; the allocation-free scan at the same size writes every
    point and agrees with it.  An explicit lane count whose wave tiles one
    launch cannot hold is refused before anything is enqueued."""
    p, q = Params(1.0, 1.0, 1.0, 1e4), Quadrature(8, 6, 2, prec)
    grid = Grid(65536, 32768, -16.0, 8.0, -8.0, 8.0)
    n = grid.n_points
    assert n == 2 ** 31
    plan = gf.Plan(p, q)
    assert plan.auto_lanes(grid) == 1
    out = gf.empty_result(grid)
    out.fill_(complex(float("nan"), 7.0))
    cls = torch.full((grid.n_im, grid.n_re), 9, dtype=torch.int8, device="cuda")
    gf.scan_plan(plan, grid, out, cls)
    with pytest.raises(Exception, match="one launch holds"):
        gf.scan_plan(plan, grid, out, cls, lanes=2)
    torch.cuda.synchronize()
    plan.close()
    assert int(((cls < 0) | (cls > 5)).sum()) == 0
    sing = cls == oracle.SINGULAR
    assert int((torch.isfinite(out) == sing).sum()) == 0
    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([
        [0, grid.n_re - 1, n - grid.n_re, n - 1, n // 2 - 1, n // 2],
        n - grid.n_re + rng.choice(grid.n_re, 60, replace=False),
        rng.choice(n, 200, replace=False)]).astype(np.int64))
    it = torch.from_numpy(idx).to("cuda")
    g = out.view(-1)[it].cpu().numpy()
    c = cls.view(-1)[it].cpu().numpy()
    # the allocation-free scan (node tables generated on the device) at the
    # same size into the same buffer: every point written, the samples equal
    # to the plan's up to the tables' last bits
    out.fill_(complex(float("nan"), 7.0))
    gf.scan_noalloc(p, grid, q, out)
    torch.cuda.synchronize()
    assert int((torch.isfinite(out) == sing).sum()) == 0
    gn = out.view(-1)[it].cpu().numpy()
    del out, cls, sing, it
    torch.cuda.empty_cache()
    fin = np.isfinite(g)
    assert np.array_equal(fin, np.isfinite(gn))
    assert np.max(np.abs(gn[fin] - g[fin])) <= (1e-9 if prec == 0 else 2e-6) * np.max(np.abs(g[fin]))
    x = oracle.grid_points_at(grid, idx)
    go, co, cond = oracle.eval_points(p, q, x, want_cond=True)
    assert (co != c).sum() <= 1
    keep = (co == c) & (co != oracle.SINGULAR)
    assert keep[np.searchsorted(idx, n - 1)]
    if prec == 0:
        check_fp64(g[keep], go[keep], cond[keep])
    else:
        check_fp32c(g[keep], go[keep])


def test_one_call_scan_matches_plan_scan_and_is_deterministic():
    p, grid, q = CONFIGS["c0_fp64_64sq"]
    a = gf.scan(p, grid, q)
    b = gf.scan(p, grid, q)  # cached plan
    plan = gf.Plan(p, q)
    c = gf.scan_plan(plan, grid)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)
    plan.close()


def test_empty_grid_and_validation_errors():
    p, _, q = CONFIGS["c0_fp64_64sq"]
    plan = gf.Plan(p, q)
    out = gf.scan_plan(plan, Grid(0, 5, -1.0, 1.0, -1.0, 1.0))
    assert out.numel() == 0
    with pytest.raises(gf.GFError):
        gf.scan_plan(plan, Grid(4, 4, 1.0, -1.0, -1.0, 1.0))
    with pytest.raises(gf.GFError):  # Lambda^2 = 1e4 too small for a box reaching |x| ~ 1e4
        gf.scan_plan(plan, Grid(4, 4, -1e4, 1e4, -1.0, 1.0))
    with pytest.raises(gf.GFError):
        gf.scan_plan(plan, Grid(4, 4, -1.0, 1.0, -1.0, 1.0), lanes=3)
    plan.close()


def test_automatic_lanes_follow_the_rounds_and_lane_work_rule():
    """The automatic lanes per point on MI355X (4 resident FP64 waves and 6
    FP32C waves per SIMD): at least 4 rounds of resident waves, pole sums
    included (the long way round leaves no tiles without a contour), no lane
    below 2048 angular pairs (4096 in FP32C), the device filled at least
    once.  The bench grid keeps one lane per point."""
    from paper_1205_0752_amd.workloads import Propagators
    pair = Propagators(Propagators.conjugate_pair(1.0 + 0.8j, 0.5), ((1.0, 0.6), (3.0, 0.4)))
    p = Params(1.0, 1.0, 1.0, 1e6)

    def box(n):
        return Grid(n, n, -16.0, 8.0, -8.0, 8.0)

    cases = [(Quadrature(256, 128, 16), None, 2048, 1), (Quadrature(256, 128, 16), None, 1024, 1),
             (Quadrature(256, 128, 16), None, 512, 4), (Quadrature(256, 128, 16), None, 256, 8),
             (Quadrature(256, 128, 16), None, 128, 16), (Quadrature(64, 32, 16), None, 64, 64),
             (Quadrature(512, 256, 16, gf.FP32C), None, 1024, 2),
             (Quadrature(512, 256, 16, gf.FP32C), None, 512, 8),
             (Quadrature(512, 256, 16, gf.FP32C), None, 256, 16),
             (Quadrature(256, 128, 16), pair, 1024, 1), (Quadrature(256, 128, 16), pair, 512, 4),
             (Quadrature(256, 128, 16), pair, 256, 16)]
    for q, props, n, want in cases:
        plan = gf.Plan(p, q, props=props)
        assert plan.auto_lanes(box(n)) == want, (q, props is not None, n)
        plan.close()


def test_subtraction_constant_matches_oracle():
    for p, q in ((Params(1.0, 1.0, 1.0, 1e6), Quadrature(256, 128, 16)),
                 (Params(-0.5j, 0.5j, 0.0, 1e6), Quadrature(512, 256, 16)),
                 (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6), Quadrature(64, 32, 16))):
        plan = gf.Plan(p, q)
        j = plan.jmu()
        plan.close()
        jo = oracle.jmu(p, q)
        assert abs(j - jo) <= 1e-13 * abs(jo)


@pytest.mark.parametrize("q", [Quadrature(8192, 64, 64), Quadrature(64, 8192, 16),
                               Quadrature(64, 8191, 1024), Quadrature(32, 7, 1)],
                         ids=["n_r_8192", "n_a_8192", "n_a_8191_arc_1024", "tiny"])
def test_large_node_counts(q):
    """The maximum radial order (8192), the maximum angular order (8192, and
    8191: odd, with the middle node), the maximum arc order (1024) and a tiny
    rule (7 angular nodes, one arc node), at a few points."""
    p = Params(1.0, 1.0, 1.0, 1e6, 1.0)
    grid = Grid(4, 2, -6.0, 3.0, -3.0, 3.0)
    g, c = _gpu_scan(p, q, grid)
    go, co, cond = oracle.scan(p, q, grid, want_cond=True)
    _compare(g, c, p, q, oracle.grid_points(grid), go, co, cond)


def test_maximum_taylor_order_and_pole_count():
    """t^8, the highest subtraction order, and eight poles on each leg (real
    pole sums), against the oracle on a small ragged grid."""
    from paper_1205_0752_amd.workloads import Propagators
    for p, props in ((Params(2.0, 0.7, 1.5, 1e6, 1.0, 8), None),
                     (Params(1.0, 1.0, 1.0, 1e6, 1.0),
                      Propagators(tuple((0.5 + 0.4 * k, 1.0 / (k + 1)) for k in range(8)),
                                  tuple((0.3 + 0.5 * k, 0.5 + 0.1 * k) for k in range(8))))):
        q = Quadrature(64, 32, 16)
        grid = Grid(13, 9, -8.0, 4.0, -4.0, 4.0)
        plan = gf.Plan(p, q, props=props)
        out = gf.empty_result(grid)
        cls = torch.empty((grid.n_im, grid.n_re), dtype=torch.int8, device="cuda")
        gf.scan_plan(plan, grid, out, cls)
        torch.cuda.synchronize()
        plan.close()
        g = out.cpu().numpy().ravel()
        c = cls.cpu().numpy().ravel()
        go, co, cond = oracle.scan(p, q, grid, want_cond=True, props=props)
        keep = (c == co) & (co != oracle.SINGULAR)
        assert (c != co).sum() <= 1 and keep.sum() >= 0.5 * c.size
        err = np.abs(g[keep] - go[keep])
        mag = np.abs(go[keep])
        assert np.all(err <= np.maximum(1e-12 * mag, 64 * EPS * cond[keep] * mag)), np.max(err / mag)


@pytest.mark.parametrize("p,grid", [
    (Params(1.0, 1.0, 1.0, 1e6), Grid(32, 32, -16.0, 8.0, -8.0, 8.0)),
    (Params(1.0, 1.0, 1.0, 1e6), Grid(32, 8, -12.0, 0.0, -0.1, 0.1)),
    (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6), Grid(32, 32, -12.0, 6.0, -6.0, 6.0))],
    ids=["bench_box", "cut_band", "conjugate"])
def test_fp64_rounding_against_quad_precision(p, grid):
    """The FP64 kernel (shared reciprocals, the real quadratic for |D|^2 away
    from the angular cut) against the same quadrature in __float128: its
    errors are no larger than the plain FP64 oracle's, within a factor 4, in
    median and maximum over the grid."""
    q = Quadrature(128, 64, 16)
    g, c = _gpu_scan(p, q, grid)
    x = oracle.grid_points(grid)
    gq, cq = oracle.eval_points_q(p, q, x)
    go, co = oracle.eval_points(p, q, x)
    ok = np.isfinite(gq) & (cq == c)
    assert ok.sum() >= 0.5 * x.size
    ref = np.abs(gq[ok])
    e_gpu = np.abs(g[ok] - gq[ok]) / ref
    e_or = np.abs(go[ok] - gq[ok]) / ref
    assert np.median(e_gpu) <= 4 * np.median(e_or) + 1e-16, (np.median(e_gpu), np.median(e_or))
    assert e_gpu.max() <= 4 * e_or.max() + 1e-16, (e_gpu.max(), e_or.max())


@pytest.mark.parametrize("p,q", [
    (Params(1.0, 1.0, 1.0, 1e4), Quadrature(96, 49, 16, gf.FP64, gf.TANH_SINH)),
    (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6), Quadrature(96, 33, 16, gf.FP64, gf.GC1)),
    (Params(2.0, 0.7, 1.5, 1e6, 1.0, 2), Quadrature(96, 48, 16)),
    (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6, 1.0, 4), Quadrature(96, 48, 16)),
    (Params(1.0, 1.0, 1.0, 1e4, 1.0, 0, 3), Quadrature(96, 33, 16, gf.FP64, gf.GL)),
    (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6, 1.0, -1, 2), Quadrature(96, 48, 16, gf.FP64, gf.GC1))],
    ids=["tanh_sinh", "gc1_conj", "taylor2", "taylor4_conj", "dim3", "dim2_conj"])
def test_fp64_rounding_against_quad_precision_rules_orders_dims(p, q):
    """The FP64 kernel's rounding for the other angular rules, Taylor orders
    and dimensions, against the __float128 twin on a 16 x 16 box: its errors
    are no larger than the plain FP64 oracle's, within a factor 4, in median
    and maximum over the box."""
    grid = Grid(16, 16, -12.0, 6.0, -6.0, 6.0)
    g, c = _gpu_scan(p, q, grid)
    x = oracle.grid_points(grid)
    gq, cq = oracle.eval_points_q(p, q, x)
    go, co = oracle.eval_points(p, q, x)
    ok = np.isfinite(gq) & (cq == c)
    assert ok.sum() >= 0.5 * x.size
    ref = np.abs(gq[ok])
    e_gpu = np.abs(g[ok] - gq[ok]) / ref
    e_or = np.abs(go[ok] - gq[ok]) / ref
    assert np.median(e_gpu) <= 4 * np.median(e_or) + 1e-16, (np.median(e_gpu), np.median(e_or))
    assert e_gpu.max() <= 4 * e_or.max() + 1e-16, (e_gpu.max(), e_or.max())


# ---------------------------------------------------------------- FP32C (FP32 bulk)

def _band_sample(grid, n, seed, re_below=-1.0):
    """n flat indices drawn from the points within 0.05 of the real axis with
    Re x < re_below (the cut band and the pinch band of the workloads)."""
    d_im = (grid.im_hi - grid.im_lo) / grid.n_im
    d_re = (grid.re_hi - grid.re_lo) / grid.n_re
    rows = [b for b in range(grid.n_im) if abs(grid.im_lo + (b + 0.5) * d_im) < 0.05]
    cols = [a for a in range(grid.n_re) if grid.re_lo + (a + 0.5) * d_re < re_below]
    cand = np.array([b * grid.n_re + a for b in rows for a in cols], dtype=np.int64)
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(cand, size=min(n, cand.size), replace=False))


def _fp32c_vs_oracle(g32, c32, p, q, x):
    """FP32C values at points x against the FP64 oracle (same class)."""
    go, co = oracle.eval_points(p, q, x)
    keep = (c32 == co) & (co != oracle.SINGULAR)
    assert (~keep & (co != oracle.SINGULAR)).sum() <= 1
    assert np.all(np.isnan(g32[co == oracle.SINGULAR]))
    return check_fp32c(g32[keep], go[keep]), g32[keep], go[keep], x[keep]


def test_fp32c_config2_sampled_and_cut_band():
    """Mixed precision on the 1024^2 box (512 x 256 nodes), unsplit: sampled
    points and a sample of the cut and pinch bands (|Im x| < 0.05, Re x < -1)
    against the FP64 oracle; errors reported inside and outside the cut band."""
    p, grid, q = CONFIGS["c2_fp32c_1024sq"]
    g, c = _gpu_scan(p, q, grid)
    assert np.all(np.isfinite(g))
    for idx in (sample_points(grid, 400, seed=3), _band_sample(grid, 300, seed=6)):
        x = oracle.grid_points_at(grid, idx)
        stats, g32, go, xk = _fp32c_vs_oracle(g[idx], c[idx], p, q, x)
        print("fp32c c2", stats, band_report(g32, go, xk, 4.0))


def test_fp32c_full_grid_against_fp64_gpu():
    """FP32C against the parity-checked FP64 path at every point of the full
    config c2 workload (1024^2 points, 512 x 256 nodes): the FP32-bulk bar
    holds at all 1,048,576 points, in the cut band and elsewhere."""
    p, grid, q32 = CONFIGS["c2_fp32c_1024sq"]
    q64 = Quadrature(q32.n_radial, q32.n_angular, q32.n_arc, gf.FP64)
    g32, c32 = _gpu_scan(p, q32, grid)
    g64, c64 = _gpu_scan(p, q64, grid)
    assert np.array_equal(c32, c64)
    stats = check_fp32c(g32, g64)
    x = oracle.grid_points(grid)
    print("fp32c vs fp64 (all points)", stats, band_report(g32, g64, x, 4.0))


@pytest.mark.parametrize("name", ["c3a_conj_2048sq", "c3b_unequal_2048sq"])
def test_fp32c_config3_full_size_sampled(name):
    """The 2048^2 complex-mass and unequal-mass workloads in FP32C at full
    size and nodes (512 x 256 + 16): a uniform sample and a sample of the cut
    and pinch bands against the FP64 oracle; NaN exactly at SINGULAR."""
    p, grid, q = CONFIGS[name]
    q = Quadrature(q.n_radial, q.n_angular, q.n_arc, gf.FP32C)
    g, c = _gpu_scan(p, q, grid)
    assert np.array_equal(np.isnan(g), c == gf.CLASS_SINGULAR)
    m1, m2 = np.sqrt(complex(p.m1sq)), np.sqrt(complex(p.m2sq))
    thr = abs(m1 + m2) ** 2
    for idx in (sample_points(grid, 400, seed=3), _band_sample(grid, 300, seed=4)):
        x = oracle.grid_points_at(grid, idx)
        stats, g32, go, xk = _fp32c_vs_oracle(g[idx], c[idx], p, q, x)
        print(name, "fp32c", stats, band_report(g32, go, xk, thr))


def test_fp32c_ragged_and_odd_rules():
    """FP32C on a ragged grid with odd angular order (middle node) and several
    lane splits; complex conjugate masses (all four classes)."""
    p = Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6, 1.0)
    q = Quadrature(96, 49, 8, gf.FP32C)
    grid = Grid(29, 19, -12.0, 6.0, -6.0, 6.0)
    go, co = oracle.scan(p, q, grid)
    for lanes in (1, 4, 64):
        g, c = _gpu_scan(p, q, grid, lanes=lanes)
        keep = (c == co) & (co != oracle.SINGULAR)
        assert (c != co).sum() <= 1
        check_fp32c(g[keep], go[keep])


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32c"])
def test_rescaled_sums_at_large_magnitudes(prec):
    """Lambda^2 = 1e10 puts |y| above 2^30, so the FP64 launch rescales U^2
    and V^2 by powers of two (the products of eight denominators would leave
    the double range unscaled): the bench box and a box with |x| ~ 1e6, every
    point against the oracle."""
    p = Params(1.0, 1.0, 1.0, 1e10, 1.0)
    q = Quadrature(64, 32, 16, prec)
    for grid in (Grid(27, 19, -16.0, 8.0, -8.0, 8.0), Grid(23, 17, -2e6, 1e6, -1e6, 1e6)):
        g, c = _gpu_scan(p, q, grid)
        go, co, cond = oracle.scan(p, q, grid, want_cond=True)
        if prec == 0:
            _compare(g, c, p, q, oracle.grid_points(grid), go, co, cond)
        else:
            keep = (c == co) & (co != oracle.SINGULAR)
            assert (c != co).sum() <= 1
            check_fp32c(g[keep], go[keep])


@pytest.mark.parametrize("name", ["c0_fp64_64sq", "paper"])
def test_fp32c_small_boxes_every_point(name):
    """FP32C at every point of the small workload (64^2, 64 x 32 nodes) and of
    the paper's display box with its masses (128^2, 128 x 64 nodes)."""
    if name == "paper":
        p, grid, q = Params(-0.5j, 0.5j, 0.0, 1e6, 1.0), Grid(128, 128, -5.0, 5.0, -5.0, 5.0), \
            Quadrature(128, 64, 16, gf.FP32C)
    else:
        p, grid, q = CONFIGS[name]
        q = Quadrature(q.n_radial, q.n_angular, q.n_arc, gf.FP32C)
    g, c = _gpu_scan(p, q, grid)
    go, co = oracle.scan(p, q, grid)
    keep = (c == co) & (co != oracle.SINGULAR)
    assert (c != co).sum() <= 1
    print(name, check_fp32c(g[keep], go[keep]))
