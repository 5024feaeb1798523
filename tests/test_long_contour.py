"""The long way round (class LONG): the contour for points whose rotation
towards arg x would sweep a (p-k)-leg bad ray where neither the residue class
nor the mirror point applies -- a complex pole on the (p-k) leg without its
conjugate on the k leg, or a complex-conjugate pair on the (p-k) leg (a
Gribov-type propagator), whose two bad rays leave the sector between them
with no short rotation at all.

Each blocked pole's term is continued the other way round the origin, through
the other half plane, sweeping none of its own bad ray (section "Step 3:
Analytic continuation": the contour deformed around what obstructs it, as
the contours of regions 3 and 4 go round the poles).  CPU pins of the oracle:
the class reproduces eq. 18 (forced, at points of the paper's box where its
mirror class applies) and the continued Feynman-parameter form of eq. 17-18
for a complex (p-k)-leg pole inside the curve where the discretised angular
cut meets the k-leg pole; pole sums are the bilinear combination of their
single-pole terms, keep G(conj x) = conj G(x) for real-analytic propagators,
and leave no point off the real axis without a contour in D = 4.  GPU: the
kernel's LONG points against the oracle (FP64 and FP32C, pole sums, t^2,
D = 2 and 3) and served LONG requests equal to standalone scans.  In D = 3 the
long way round converges to the mirror value (the measure sqrt(y) continued
along the long rotation)."""
import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from parity_bars import check
from paper_1205_0752_amd.workloads import GC1, GL, Grid, Params, Propagators, Quadrature

GRIBOV1 = Propagators(Propagators.conjugate_pair(1.0 + 0.8j, 0.5), ((1.0, 0.6), (3.0, 0.4)))
Q = Quadrature(512, 256, 16)


def test_long_class_reproduces_eq18_where_the_mirror_class_applies():
    """The paper's masses (m1^2 = -i/2, m2^2 = +i/2, mu^2 = 0): points of the
    upper left quadrant inside |x| < 1 (the threshold x = -1 and the pinch
    curve from it through x = i) are MIRROR points; forcing the long way
    round there gives eq. 18 as well (Cauchy: two valid contours)."""
    p = Params(-0.5j, 0.5j, 0.0, 1e6)
    xs = [-0.3 + 0.4j, -0.5 + 0.3j, -0.2 + 0.1j, -0.6 + 0.5j, -0.75 + 0.3j]
    g_long, c_long = oracle.eval_points(p, Q, xs, force_class=oracle.LONG)
    g_nat, c_nat = oracle.eval_points(p, Q, xs)
    assert np.all(c_nat == oracle.MIRROR)
    for x, gl, gn in zip(xs, g_long, g_nat):
        ref = complex(cf.eq18(x)) + cf.cutoff_bias(x, -0.5j, 0.0, 1e6)
        assert abs(gl - ref) < 1e-12 * abs(ref) + 5e-13, (x, gl, ref)
        assert abs(gl - gn) < 1e-12 * abs(gn) + 5e-13


@pytest.mark.parametrize("m1", [1 + 0.8j, 1 - 0.8j])
def test_single_complex_pole_matches_continued_feynman_form(m1):
    """m1^2 = 1 +- 0.8i on the (p-k) leg, m2^2 = 1, mu^2 = 1 (no mirror
    symmetry): the sector beyond the bad ray arg(-m1^2) was without a contour;
    the long way round matches the continued Feynman form (plus its cutoff
    bias) inside the pinch curve from the threshold -(sqrt(m1^2) + 1)^2 and
    beyond the threshold's angle."""
    p = Params(m1, 1.0, 1.0, 1e6)
    s = 1.0 if complex(m1).imag < 0 else -1.0   # the blocked sector's half plane
    xs = [complex(-1.5, 0.6 * s), complex(-2.0, 0.5 * s), complex(-2.2, 0.8 * s),
          complex(-6.0, 1.0 * s), complex(-9.0, 1.2 * s)]
    g, c = oracle.eval_points(p, Q, xs)
    assert np.all(c == oracle.LONG), c
    for x, gx in zip(xs, g):
        ref = cf.feynman_continued(x, m1, 1.0, 1.0) + cf.cutoff_bias(x, m1, 1.0, 1e6)
        assert abs(gx - ref) < 5e-10 * abs(ref), (x, gx, ref, abs(gx - ref))


def test_pole_sum_has_a_contour_everywhere_off_the_real_axis():
    """A complex-conjugate pair on the (p-k) leg (1 +- 0.8i, residues 1/2) and
    two real poles on the k leg: on the pole-sum benchmark box no point off
    the real axis is left without a contour (46 % were, before the long way
    round), in D = 4 and in D = 3 with the same classes."""
    grid = Grid(64, 64, -16.0, 8.0, -8.0, 8.0)
    x = oracle.grid_points(grid)
    cls = oracle.classify(Params(1.0, 1.0, 1.0, 1e6), Q, x, props=GRIBOV1)
    assert not np.any(cls == oracle.SINGULAR)
    assert (cls == oracle.LONG).mean() > 0.3
    cls3 = oracle.classify(Params(1.0, 1.0, 1.0, 1e6, 1.0, 0, 3), Quadrature(512, 256, 16, 0, 3),
                           x, props=GRIBOV1)
    assert np.array_equal(cls3, cls)


WEDGE = [-1.5 + 0.6j, -2.0 + 0.5j, -2.2 + 0.8j, -1.6 - 0.5j, -2.1 - 0.7j, -6.0 + 1.0j, -9.0 - 1.2j]


def test_pole_sum_is_bilinear_in_its_single_pole_terms():
    """In the sector beyond both bad rays each term of the pole sum takes its
    own rotation: G = sum_ab c1_a c2_b G_ab with the single-pole oracle's
    G_ab (the short way for the unblocked pole, the long way for the blocked
    one), to rounding."""
    p = Params(1.0, 1.0, 1.0, 1e6)
    g, c = oracle.eval_points(p, Q, WEDGE, props=GRIBOV1)
    assert np.all(c == oracle.LONG)
    ref = np.zeros(len(WEDGE), dtype=complex)
    for m1, c1 in GRIBOV1.poles1:
        for m2, c2 in GRIBOV1.poles2:
            gab, _ = oracle.eval_points(Params(m1, m2, 1.0, 1e6), Q, WEDGE)
            ref += c1 * c2 * gab
    assert np.max(np.abs(g - ref) / np.abs(ref)) < 1e-12


def test_pole_sum_matches_bilinear_continued_feynman_forms():
    """The same points against sum_ab c1_a c2_b (continued Feynman form of
    (m1_a^2, m2_b^2) + its cutoff bias): the points lie inside every term's
    pinch curve or beyond its threshold's angle."""
    p = Params(1.0, 1.0, 1.0, 1e6)
    g, _ = oracle.eval_points(p, Q, WEDGE, props=GRIBOV1)
    for x, gx in zip(WEDGE, g):
        ref = sum(c1 * c2 * (cf.feynman_continued(x, m1, m2, 1.0) + cf.cutoff_bias(x, m1, 1.0, 1e6))
                  for m1, c1 in GRIBOV1.poles1 for m2, c2 in GRIBOV1.poles2)
        assert abs(gx - ref) < 5e-10 * abs(ref), (x, gx, ref)


def test_real_analytic_pole_sum_keeps_the_mirror_symmetry():
    """Conjugating every pole and residue maps the pair onto itself, so
    G(conj x) = conj G(x); the long contour of conj x is the mirror image of
    that of x, so the symmetry holds to rounding."""
    p = Params(1.0, 1.0, 1.0, 1e6)
    xs = np.array(WEDGE)
    g, c = oracle.eval_points(p, Q, xs, props=GRIBOV1)
    gb, cb = oracle.eval_points(p, Q, np.conj(xs), props=GRIBOV1)
    assert np.all(c == oracle.LONG) and np.all(cb == oracle.LONG)
    assert np.max(np.abs(gb - np.conj(g)) / np.abs(g)) < 1e-13


def test_long_class_in_two_dimensions_is_cauchy_consistent():
    """D = 2 (integer power of y, so the long way round stays on the same
    branch): where the mirror class applies (paper's masses, inside the
    threshold), forcing the long way round gives the same value."""
    p = Params(-0.5j, 0.5j, 0.0, 1e6, 1.0, -1, 2)
    q = Quadrature(512, 256, 16, 0, GC1)
    xs = [-0.3 + 0.4j, -0.5 + 0.3j, -0.6 + 0.5j]
    g_long, _ = oracle.eval_points(p, q, xs, force_class=oracle.LONG)
    g_nat, c_nat = oracle.eval_points(p, q, xs)
    assert np.all(c_nat == oracle.MIRROR)
    assert np.max(np.abs(g_long - g_nat) / np.abs(g_nat)) < 1e-11


def test_long_class_in_three_dimensions_converges_to_the_mirror_value():
    """D = 3: the measure sqrt(y) continued along the long rotation has the
    opposite sign on its ray, arc and far residues.  Where the mirror class
    applies (paper's masses, inside the threshold) the forced long way round
    and the mirror value differ only by the radial rule's error, which the
    sqrt(y) end point makes algebraic: 8 times smaller per doubling of n_r
    (order 3), so the two converge to one value.  Without the continuation
    (the principal sqrt(y) on the long rotation) they would differ at O(1)."""
    from paper_1205_0752_amd.workloads import GL
    xs = [-0.3 + 0.4j, -0.5 + 0.3j, -0.6 + 0.5j]
    d = []
    for nr in (256, 512):
        p = Params(-0.5j, 0.5j, 0.0, 1e6, 1.0, -1, 3)
        q = Quadrature(nr, 256, 16, 0, GL)
        g_long, _ = oracle.eval_points(p, q, xs, force_class=oracle.LONG)
        g_nat, c_nat = oracle.eval_points(p, q, xs)
        assert np.all(c_nat == oracle.MIRROR)
        d.append(np.abs(g_long - g_nat) / np.abs(g_nat))
    assert np.all(d[1] < 2e-7)
    assert np.all((d[0] / d[1] > 7.0) & (d[0] / d[1] < 9.0)), d[0] / d[1]


@pytest.mark.parametrize("phi0", [-160.0, 160.0])
def test_long_residues_in_three_dimensions_keep_g_continuous(phi0):
    """D = 3: a (p-k)-leg pole 1 + 0.8i (bad ray -141.3 degrees) and a k-leg
    pole whose bad ray lies at -160 degrees (and the mirror image of the
    setup).  Just inside that ray the long rotation sweeps the k-leg pole past
    the negative real axis, where the continued sqrt(y0) has the opposite sign
    of the principal one; just outside it sweeps no pole.  G is analytic
    across the ray, so the two sides' values, extrapolated to it (split radial
    rule, quadratic in the distance), must meet: they do to 4e-4 (D = 4,
    where the measure has no square root: 2e-4); with the principal sqrt(y0)
    the residue enters with the wrong sign and they miss by O(1)."""
    from paper_1205_0752_amd.workloads import GC2
    m2 = np.exp(1j * np.deg2rad(20.0))
    m1, m2 = (1 + 0.8j, m2) if phi0 < 0 else (1 - 0.8j, np.conj(m2))
    for dim, rule, tol in ((3, GL, 2e-3), (4, GC2, 1e-3)):
        p = Params(m1, m2, 1.0, 1e6, 1.0, 0, dim)
        q = Quadrature(1024, 128, 32, 0, rule, 1)
        side = []
        for sgn in (-1, 1):
            xs = 3.0 * np.exp(1j * (np.deg2rad(phi0) + sgn * np.array([0.02, 0.04, 0.06])))
            g, c = oracle.eval_points(p, q, xs)
            assert np.all(c == oracle.LONG)
            side.append(3 * g[0] - 3 * g[1] + g[2])
        assert abs(side[1] - side[0]) <= tol * abs(side[1]), (dim, abs(side[1] - side[0]) / abs(side[1]))


# ---------------------------------------------------------------- GPU

def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1205_0752_amd as gf
    return torch, gf


def _gpu_scan(gf, torch, p, q, grid, props=None, lanes=0):
    plan = gf.Plan(p, q, props=props)
    out = gf.empty_result(grid)
    cls = torch.empty((grid.n_im, grid.n_re), dtype=torch.int8, device="cuda")
    gf.scan_plan(plan, grid, out, cls, lanes=lanes)
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy().ravel(), cls.cpu().numpy().ravel()


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["gribov1", "gribov1_t2", "gribov1_d2", "gribov1_d3", "single_pole",
                                  "single_pole_d3"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32c"])
def test_gpu_long_points_match_oracle(case, prec):
    """Every point of two ragged grids (one of them the complex-mass box)
    against the oracle, LONG points included: the conjugate pair on the
    (p-k) leg with t^0, t^2 and in D = 2 and 3, and a single complex (p-k)-leg
    pole without mirror symmetry (D = 4 and 3); several lane splits."""
    torch, gf = _gpu()
    props, dim, order, rule = GRIBOV1, 4, 0, 0
    m1 = 1.0
    if case == "gribov1_t2":
        order = 2
    elif case == "gribov1_d2":
        dim, order, rule = 2, -1, GC1
    elif case == "gribov1_d3":
        dim, rule = 3, GL
    elif case.startswith("single_pole"):
        props, m1 = None, 1 + 0.8j
        if case.endswith("d3"):
            dim, rule = 3, GL
    p = Params(m1, 1.0, 1.0, 1e6, 1.0, order, dim)
    q = Quadrature(64, 32, 16, prec, rule)
    n_long = 0
    for grid, lanes in ((Grid(37, 29, -8.0, 4.0, -4.0, 4.0), 0), (Grid(21, 17, -12.0, 6.0, -6.0, 6.0), 4)):
        g, c = _gpu_scan(gf, torch, p, q, grid, props, lanes)
        go, co, cond = oracle.scan(p, q, grid, want_cond=True, props=props)
        assert (c != co).sum() <= 1
        keep = (c == co) & (co != oracle.SINGULAR)
        n_long += int((c[keep] == oracle.LONG).sum())
        check(prec, g[keep], go[keep], cond[keep], dim=dim)
    assert n_long >= 40


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32c"])
def test_gpu_pole_sum_bench_box_long_points(prec):
    """The pole-sum benchmark workload at full size (1024^2 points of the
    bench box, 256 x 128 + 16 nodes, conjugate pair on the (p-k) leg) in the
    benchmark's launch configuration: no point off the real axis without a
    contour, and 300 sampled LONG points plus 200 uniform ones against the
    oracle."""
    torch, gf = _gpu()
    from paper_1205_0752_amd.workloads import sample_points
    p = Params(1.0, 1.0, 1.0, 1e6)
    grid = Grid(1024, 1024, -16.0, 8.0, -8.0, 8.0)
    q = Quadrature(256, 128, 16, prec)
    g, c = _gpu_scan(gf, torch, p, q, grid, GRIBOV1)
    assert not np.any(c == oracle.SINGULAR)
    assert np.all(np.isfinite(g))
    rng = np.random.Generator(np.random.PCG64(9))
    longs = np.nonzero(c == oracle.LONG)[0]
    idx = np.unique(np.concatenate([rng.choice(longs, 300, replace=False),
                                    sample_points(grid, 200, seed=10)]))
    x = oracle.grid_points_at(grid, idx)
    go, co, cond = oracle.eval_points(p, q, x, want_cond=True, props=GRIBOV1)
    keep = c[idx] == co
    assert (~keep).sum() <= 1
    check(prec, g[idx][keep], go[keep], cond[keep])


@pytest.mark.gpu
def test_gpu_served_long_requests_equal_standalone():
    """Served requests with LONG points (pole sums and a single complex
    pole, FP64 and FP32C, t^0 and t^2) are bitwise equal to their standalone
    one-lane scans."""
    torch, gf = _gpu()
    reqs = [(Params(m1, 1.0, 1.0, 1e6, 1.0, order), Grid(40, 24, -12.0, 6.0, -6.0, 6.0),
             Quadrature(64, 32, 16, prec), props)
            for order in (0, 2) for prec in (0, 1)
            for m1, props in ((1.0, GRIBOV1), (1 + 0.8j, None))]
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
