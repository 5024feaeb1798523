"""Seeded synthetic workloads: parameter containers, the named scan
configurations and the serving-trace generator.

This module holds inputs only -- no arithmetic of the method.  Both the HIP
path and the CPU oracle take their inputs from here.

The paper has no dataset: its workload is a box in the complex x = p^2 plane
discretised into M x N points (STEP 4), an integrand with masses, a
subtraction point and a cutoff (eq. 14-16), and a quadrature (section
"Numerical Implementation").  The configurations below fix those numbers.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# precision codes of the quadrature record
FP64 = 0
FP32C = 1
#: angular rules (GF_ANG_*)
GC2 = 0
GC1 = 1
TANH_SINH = 2
GL = 3


@dataclasses.dataclass(frozen=True)
class Params:
    """Integrand parameters: masses on the (p-k) leg (m1sq) and the k leg
    (m2sq), the real subtraction point mu2 >= 0, the cutoff Lambda^2 of eq. 14,
    the output scale (1.0 = rescaled units of eq. 18, 1/(16 pi^2) =
    eq. 17), the order n of the Taylor subtraction t^n (eq. 12-13, about
    x = mu2; -1 subtracts nothing) and the dimension D of the integral (2, 3
    or 4)."""
    m1sq: complex = 1.0
    m2sq: complex = 1.0
    mu2: float = 1.0
    lambda2: float = 1e4
    scale: float = 1.0
    taylor_order: int = 0
    dimension: int = 4


@dataclasses.dataclass(frozen=True)
class Propagators:
    """Pole-sum propagators P1(s) = sum_a c1_a / (s + m1_a^2) on the (p-k) leg
    and P2(s) = sum_b c2_b / (s + m2_b^2) on the k leg: tuples of (m^2, c),
    1 to 8 poles each; optionally a numerator N(k^2, p.k) = sum n_ij (k^2)^i
    (p.k)^j (i, j = 0..2) given as a tuple of (i, j, n_ij), () for N = 1."""
    poles1: tuple
    poles2: tuple
    numerator: tuple = ()

    @staticmethod
    def conjugate_pair(m2: complex, c: complex = 0.5) -> tuple:
        """A pole pair at m^2 and conj(m^2) with residues c and conj(c), e.g. the
        propagator s / (s^2 + M^4) = (1/2)/(s + i M^2) + (1/2)/(s - i M^2)."""
        m2, c = complex(m2), complex(c)
        return ((m2, c), (m2.conjugate(), c.conjugate()))


@dataclasses.dataclass(frozen=True)
class Grid:
    """Cell-centred n_re x n_im box over [re_lo, re_hi] x [im_lo, im_hi];
    results are row-major with the Re index fastest."""
    n_re: int
    n_im: int
    re_lo: float
    re_hi: float
    im_lo: float
    im_hi: float

    @property
    def n_points(self) -> int:
        return self.n_re * self.n_im


@dataclasses.dataclass(frozen=True)
class Quadrature:
    """Node counts: Gauss-Legendre radial nodes in t = log(1+y), angular nodes
    of the rule `angular_rule` (GC2: Gauss-Chebyshev second kind, the default;
    GC1: first kind; TANH_SINH: double exponential; GL: Gauss-Legendre),
    Gauss-Legendre arc nodes; radial_split = 1 cuts the radial rule into four
    Gauss-Legendre pieces at the point's near-singular radii;
    precision FP64 or FP32C (FP32 bulk, FP64 at the sensitive steps)."""
    n_radial: int = 64
    n_angular: int = 32
    n_arc: int = 16
    precision: int = FP64
    angular_rule: int = 0
    radial_split: int = 0


# --------------------------------------------------------------------------
# Named configurations
# --------------------------------------------------------------------------

#: the paper's worked example (eq. 16 with 2 sqrt(2) theta^2 = 1): m1^2 = -i/2
#: on the (p-k) leg, m2^2 = +i/2 on the k leg, subtraction at x = 0 (eq. 20)
PAPER_EXAMPLE = Params(m1sq=-0.5j, m2sq=0.5j, mu2=0.0, lambda2=1e6, scale=1.0)

#: the paper's display box (worked example, STEP 4): 128^2 points over +-5
PAPER_BOX = Grid(128, 128, -5.0, 5.0, -5.0, 5.0)

CONFIGS = {
    # small FP64 case the oracle finishes in seconds
    "c0_fp64_64sq": (Params(1.0, 1.0, 1.0, 1e4, 1.0),
                     Grid(64, 64, -8.0, 4.0, -4.0, 4.0),
                     Quadrature(64, 32, 16, FP64)),
    # large FP64 scan: 1024^2 points, 256 x 128 nodes
    "c1_fp64_1024sq": (Params(1.0, 1.0, 1.0, 1e6, 1.0),
                       Grid(1024, 1024, -16.0, 8.0, -8.0, 8.0),
                       Quadrature(256, 128, 16, FP64)),
    # mixed precision on the same box, 512 x 256 nodes
    "c2_fp32c_1024sq": (Params(1.0, 1.0, 1.0, 1e6, 1.0),
                        Grid(1024, 1024, -16.0, 8.0, -8.0, 8.0),
                        Quadrature(512, 256, 16, FP32C)),
    # conjugate mass pair, 2048^2 points, 512 x 256 nodes
    "c3a_conj_2048sq": (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6, 1.0),
                        Grid(2048, 2048, -12.0, 6.0, -6.0, 6.0),
                        Quadrature(512, 256, 16, FP64)),
    # unequal real masses m1 = 1, m2 = 0.5, mu^2 = 2
    "c3b_unequal_2048sq": (Params(1.0, 0.25, 2.0, 1e6, 1.0),
                           Grid(2048, 2048, -12.0, 6.0, -6.0, 6.0),
                           Quadrature(512, 256, 16, FP64)),
}


# --------------------------------------------------------------------------
# Serving trace
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Request:
    arrival_s: float
    params: Params
    grid: Grid
    quad: Quadrature


SIDES = tuple(range(16, 513, 16))          # grid side in {16, 32, ..., 512}
ORDERS = (32, 64, 128, 256, 512)           # radial / angular orders
SERVING_WINDOW = (-8.0, 4.0, -4.0, 4.0)    # Re lo, Re hi, Im lo, Im hi


def serving_trace(n_requests: int, rate_per_s: float, seed: int = 0,
                  sides=SIDES, orders=ORDERS, lambda2: float = 1e6,
                  n_arc: int = 16) -> list[Request]:
    """Poisson arrivals at `rate_per_s`; per request: grid side uniform in
    `sides`; masses m^2 uniform in [0.25, 4], 30% of requests a conjugate pair
    m1^2 = r + i s, m2^2 = r - i s with s uniform in [0.1, 1]; mu^2 uniform in
    [0.5, 4]; radial and angular orders drawn independently from `orders`;
    FP64 or FP32C with probability 1/2 each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    re_lo, re_hi, im_lo, im_hi = SERVING_WINDOW
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        side = int(rng.choice(sides))
        if rng.random() < 0.3:
            r = rng.uniform(0.25, 4.0)
            s = rng.uniform(0.1, 1.0)
            m1sq, m2sq = complex(r, s), complex(r, -s)
        else:
            m1sq = complex(rng.uniform(0.25, 4.0), 0.0)
            m2sq = complex(rng.uniform(0.25, 4.0), 0.0)
        mu2 = float(rng.uniform(0.5, 4.0))
        nr = int(rng.choice(orders))
        na = int(rng.choice(orders))
        prec = FP64 if rng.random() < 0.5 else FP32C
        out.append(Request(t, Params(m1sq, m2sq, mu2, lambda2, 1.0),
                           Grid(side, side, re_lo, re_hi, im_lo, im_hi),
                           Quadrature(nr, na, n_arc, prec)))
    return out


def sample_points(grid: Grid, n: int, seed: int = 0) -> np.ndarray:
    """`n` distinct flat indices (b * n_re + a) drawn uniformly from the grid,
    sorted, always including the four corners."""
    rng = np.random.Generator(np.random.PCG64(seed))
    total = grid.n_points
    n = min(n, total)
    idx = set(rng.choice(total, size=n, replace=False).tolist())
    for c in (0, grid.n_re - 1, total - grid.n_re, total - 1):
        idx.add(c)
    return np.array(sorted(idx), dtype=np.int64)

