"""Analytic references the oracle is pinned against (test infrastructure).

Nothing here calls the oracle's quadrature; every function is an independent
statement of a result the quadrature must reproduce.

* `eq18`               -- exact subtracted, rescaled worked-example correlator
                          (eq. 17 / eq. 18), masses m1^2 = -i/2, m2^2 = +i/2,
                          subtraction at x = 0.
* `feynman`            -- textbook Feynman-parameter form of the subtracted
                          bubble, int_0^1 log(Delta(a, mu^2) / Delta(a, x)) da,
                          Delta(a, s) = a m1^2 + (1 - a) m2^2 + a (1 - a) s.
* `cutoff_bias`        -- leading effect of the sharp cutoff Lambda^2 of eq. 14.
* `cut_discontinuity`  -- G(-s + i0) - G(-s - i0) from the Kallen function.
* `gc2_discrete`       -- exact value of the n-node Gauss-Chebyshev-II sum
                          sum_j w_j / (U - V z_j).
* `angular_continuum`  -- exact angular average (2/pi) int sqrt(1-z^2)/(U - V z).
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

mp.mp.dps = 40


def eq18(x: complex) -> complex:
    """1 - pi/(2x) + sqrt(1 - x^2) arccos(x) / x (eq. 18, principal branches)."""
    x = mp.mpc(x)
    r = 1 - mp.pi / (2 * x) + mp.sqrt(1 - x * x) * mp.acos(x) / x
    return complex(r)


def delta(a, s, m1sq, m2sq):
    return a * m1sq + (1 - a) * m2sq + a * (1 - a) * s


def feynman(x: complex, m1sq: complex, m2sq: complex, mu2: float) -> complex:
    """int_0^1 [log Delta(a, mu^2) - log Delta(a, x)] da with principal logs.

    Exact for real masses off the real x axis (Delta(a, x) then never crosses
    the negative real axis).  For complex masses it is the analytic function
    only where `feynman_principal_ok` holds."""
    x = mp.mpc(x)
    m1 = mp.mpc(m1sq)
    m2 = mp.mpc(m2sq)
    mu = mp.mpf(mu2)

    def f(a):
        return mp.log(delta(a, mu, m1, m2)) - mp.log(delta(a, x, m1, m2))

    # split at the real parts of the zeros of Delta(a, x) and Delta(a, mu^2)
    # (quadratic in a) so that the quadrature sees smooth pieces
    pts = [mp.mpf(0), mp.mpf(1)]
    for s in (x, mu):
        b = m1 - m2 + s
        if s != 0:
            disc = mp.sqrt(b * b + 4 * s * m2)
            roots = [(b + disc) / (2 * s), (b - disc) / (2 * s)]
        elif b != 0:
            roots = [-m2 / b]
        else:
            roots = []
        for r in roots:
            if 0 < mp.re(r) < 1:
                pts.append(mp.re(r))
    pts = sorted(set(pts))
    return complex(mp.quad(f, pts))


def feynman_taylor(mu2: float, m1sq: complex, m2sq: complex, i: int) -> complex:
    """(1/i!) d^i G/dx^i at x = mu^2 (i >= 1) of the Feynman form: with
    b = a(1-a), d/dx log Delta(a, x) = b/Delta, so the coefficient is
    -((-1)^(i-1)/i) int_0^1 b^i / Delta(a, mu^2)^i da."""
    m1 = mp.mpc(m1sq)
    m2 = mp.mpc(m2sq)
    mu = mp.mpf(mu2)

    def f(a):
        b = a * (1 - a)
        return b ** i / delta(a, mu, m1, m2) ** i

    return complex(-((-1) ** (i - 1)) * mp.quad(f, [0, 0.5, 1]) / i)


def feynman_subtracted(x: complex, m1sq: complex, m2sq: complex, mu2: float, n: int) -> complex:
    """G after the Taylor subtraction t^n about mu^2 (eq. 12-13): the Feynman
    form minus its Taylor polynomial of degree n at mu^2 (whose constant term
    is G(mu^2) = 0)."""
    g = feynman(x, m1sq, m2sq, mu2)
    d = complex(x) - mu2
    for i in range(1, n + 1):
        g -= d ** i * feynman_taylor(mu2, m1sq, m2sq, i)
    return g


def loop_sum(x: complex, m1sq: complex, m2sq: complex, dim: int) -> complex:
    """The unsubtracted rescaled loop sum S_D(x) = int_0^inf dy y^{(D-2)/2} <F>_D
    for D = 2, 3 (convergent), from the Feynman parametrisation of
    int d^D k / ((k^2 + m2^2)((p-k)^2 + m1^2)): with the normalised angular
    averages, int d^2k F = pi S_2 and int d^3k F = 2 pi S_3, so
    S_2 = int_0^1 da / Delta(a, x) and S_3 = (pi/2) int_0^1 da Delta(a, x)^(-1/2)
    (principal branch; valid off the real axis for real masses)."""
    x = mp.mpc(x)
    m1 = mp.mpc(m1sq)
    m2 = mp.mpc(m2sq)
    if dim == 2:
        return complex(mp.quad(lambda a: 1 / delta(a, x, m1, m2), [0, 0.5, 1]))
    if dim == 3:
        return complex(mp.pi / 2 * mp.quad(lambda a: delta(a, x, m1, m2) ** -0.5, [0, 0.5, 1]))
    raise ValueError("dim must be 2 or 3")


def loop_sum_cutoff_bias(x: complex, m1sq: complex, m2sq: complex, mu2: float, lambda2: float,
                         dim: int, subtracted: bool) -> complex:
    """G_Lambda - G_infinity for D = 2, 3 from the large-y expansion of the
    angular averages, <1/D1>_2 = 1/y + (x - m1^2)/y^2 + ..., <1/D1>_3 = 1/y +
    (x/3 - m1^2)/y^2 + ...: the cutoff drops the tail of y^{(D-2)/2} <F>."""
    x = complex(x)
    m1 = complex(m1sq)
    m2 = complex(m2sq)
    L = lambda2 ** 0.5
    if dim == 3:
        if subtracted:
            return -(2.0 / 9.0) * (x - mu2) / L ** 3
        return -2.0 / L - (2.0 / 3.0) * (x / 3.0 - m1 - m2) / L ** 3
    if dim == 2:
        if subtracted:
            return -(x - mu2) / (2.0 * lambda2 ** 2)
        return -1.0 / lambda2 - (x - m1 - m2) / (2.0 * lambda2 ** 2)
    raise ValueError("dim must be 2 or 3")


def angular_moment(k: int, dim: int) -> float:
    """<z^2k> under the normalised D-dimensional measure (1-z^2)^{(D-3)/2} dz / N_D:
    Gamma(k + 1/2) Gamma(D/2) / (sqrt(pi) Gamma(k + D/2))."""
    return float(mp.gamma(k + 0.5) * mp.gamma(dim / 2) / (mp.sqrt(mp.pi) * mp.gamma(k + dim / 2)))


def angular_average_dim(u: complex, v: complex, dim: int) -> complex:
    """<1/(u - v z)> under the normalised D-dimensional measure, by direct
    quadrature in the angle (z = cos t, sin^{D-2} t dt): an independent
    reference for the node rules."""
    u = mp.mpc(u)
    v = mp.mpc(v)
    norm = mp.quad(lambda t: mp.sin(t) ** (dim - 2), [0, mp.pi])
    val = mp.quad(lambda t: mp.sin(t) ** (dim - 2) / (u - v * mp.cos(t)), [0, mp.pi / 2, mp.pi])
    return complex(val / norm)


def feynman_principal_ok(x: complex, m1sq: complex, m2sq: complex, mu2: float,
                         n: int = 4001) -> bool:
    """True when neither Delta(a, x) nor Delta(a, mu^2) crosses the negative real
    axis for a in [0, 1] (sampled), so that the principal-log form is analytic
    in x there."""
    a = np.linspace(0.0, 1.0, n)
    for s in (complex(x), complex(mu2)):
        d = delta(a, s, complex(m1sq), complex(m2sq))
        im = d.imag
        re = d.real
        sign_change = np.nonzero(np.sign(im[1:]) * np.sign(im[:-1]) < 0)[0]
        for k in sign_change:
            if re[k] < 0 or re[k + 1] < 0:
                return False
        if np.any((np.abs(im) < 1e-15) & (re <= 0)):
            return False
    return True


def cutoff_bias(x: complex, m1sq: complex, mu2: float, lambda2: float) -> complex:
    """G_Lambda(x) - G_infinity(x) to leading order, (x - mu^2) m1^2 / (2 Lambda^4).

    From the large-y expansion of the angular average,
    <1/D1> = 1/y - m1^2/y^2 + (m1^4 - x m1^2)/y^3 + O(y^-4): the subtracted
    integrand behaves like (mu^2 - x) m1^2 / y^3, whose tail beyond Lambda^2
    the cutoff drops."""
    return (complex(x) - mu2) * complex(m1sq) / (2.0 * lambda2 * lambda2)


def kallen(a, b, c):
    return a * a + b * b + c * c - 2 * a * b - 2 * b * c - 2 * c * a


def cut_discontinuity(s: float, m1: float, m2: float) -> complex:
    """G(-s + i0) - G(-s - i0) for real masses: -2 pi i sqrt(lambda)/s above the
    threshold s > (m1 + m2)^2, zero below."""
    if s <= (m1 + m2) ** 2:
        return 0.0
    lam = kallen(s, m1 * m1, m2 * m2)
    return -2j * np.pi * np.sqrt(lam) / s


def gc2_discrete(u: complex, v: complex, n: int) -> complex:
    """Exact n-node GC-II sum  sum_j w_j / (u - v z_j),  z_j = cos(j pi/(n+1)),
    w_j = 2 sin^2(j pi/(n+1)) / (n+1):

        2/(u + S) * (1 - q^(2n)) / (1 - q^(2n+2)),  S = sqrt(u^2 - v^2),
        q = v / (u + S),  with the root S chosen so that |u + S| >= |u - S|.

    Evaluated in 40-digit arithmetic; v = 0 gives 1/u."""
    u = mp.mpc(u)
    v = mp.mpc(v)
    if v == 0:
        return complex(1 / u)
    s = mp.sqrt(u * u - v * v)
    if abs(u + s) < abs(u - s):
        s = -s
    q = v / (u + s)
    r = 2 / (u + s) * (1 - q ** (2 * n)) / (1 - q ** (2 * n + 2))
    return complex(r)


def angular_continuum(u: complex, v: complex) -> complex:
    """(2/pi) int_{-1}^{1} sqrt(1-z^2) / (u - v z) dz = 2 / (u + sqrt(u^2 - v^2)),
    root with |u + S| >= |u - S| (u - v z != 0 on [-1, 1])."""
    u = mp.mpc(u)
    v = mp.mpc(v)
    s = mp.sqrt(u * u - v * v)
    if abs(u + s) < abs(u - s):
        s = -s
    return complex(2 / (u + s))


# ---------------------------------------------------------------- complex masses

def _delta_roots(x: complex, m1sq: complex, m2sq: complex):
    """The two roots in a of Delta(a, x) = -x a^2 + (x + m1^2 - m2^2) a + m2^2
    (x != 0): a^2 - b a - c = 0 with b = 1 + (m1^2 - m2^2)/x, c = m2^2/x; the
    larger root from the quadratic formula, the other from the product -c."""
    b = 1.0 + (m1sq - m2sq) / x
    c = m2sq / x
    s = np.sqrt(b * b + 4.0 * c + 0j)
    q = 0.5 * (b + s) if abs(b + s) >= abs(b - s) else 0.5 * (b - s)
    return q, -c / q


def _log_ratio_principal(a):
    """Log(1 - a) - Log(-a): equals int_0^1 da'/(a' - a) along the straight
    segment, analytic in a off [0, 1], where it jumps by 2 pi i."""
    return mp.log(1 - a) - mp.log(-a)


def _segment_crossing(a0: complex, a1: complex):
    """+1 if the straight step a0 -> a1 crosses the open segment (0, 1) from
    above, -1 from below, 0 if it does not cross it; None if the crossing
    lies too close to an end point to decide (the caller refines the step)."""
    if (a0.imag > 0) == (a1.imag > 0) or a0.imag == a1.imag:
        return 0
    t = a0.imag / (a0.imag - a1.imag)
    re = a0.real + t * (a1.real - a0.real)
    step = abs(a1 - a0)
    if abs(re) < 2 * step or abs(re - 1) < 2 * step:
        return None
    if 0 < re < 1:
        return 1 if a0.imag > 0 else -1
    return 0


def _straight_path_ok(s: complex, m1sq: complex, m2sq: complex, n: int = 4001) -> bool:
    a = np.linspace(0.0, 1.0, n)
    d = delta(a, s, m1sq, m2sq)
    cross = np.nonzero((np.sign(d.imag[1:]) * np.sign(d.imag[:-1]) < 0)
                       & ((d.real[1:] < 0) | (d.real[:-1] < 0)))[0]
    return cross.size == 0 and not np.any((np.abs(d.imag) < 1e-15) & (d.real <= 0))


def feynman_continued(x: complex, m1sq: complex, m2sq: complex, mu2: float,
                      base: float | None = None, steps: int = 4000) -> complex:
    """The subtracted bubble int_0^1 [log Delta(a, mu^2) - log Delta(a, x)] da
    analytically continued in x for complex masses, where the principal-log
    form of `feynman` is not the analytic function.

    With the roots a_1, a_2 of Delta(a, x) = 0, integrating by parts gives

        F(x) = int_C log Delta(a, x) da = Log m2^2 - 2 + sum_i (1 - a_i) L(a_i),
        L(a) = int_C da' / (a' - a),

    for an a-contour C from 0 to 1 (log Delta continued along C from its
    principal value at a = 0, where Delta = m2^2).  The continuation in x
    deforms C so that each root stays on the side of C it occupied at a base
    point x0 on the positive real axis, where the straight segment is valid:
    then L(a_i) is Log(1 - a_i) - Log(-a_i) plus 2 pi i times the number of
    times the root has crossed the segment (0, 1) from above, minus those
    from below.  The roots are followed along the path x0 -> x: the circle
    |x'| = x0 from angle 0 to arg x, then the ray to x (so the path stays in
    x's half plane and away from x = 0, where one root runs off to infinity).
    The result is

        G(x) = F_straight(mu^2) - F(x),

    with the subtraction term on the straight segment (mu^2 is real).  Thus G
    is the continuation through x's half plane from the real axis right of the
    cut, the continuation the contour classes of the quadrature follow.  For
    real masses it equals `feynman` off the real axis."""
    x = complex(x)
    m1 = complex(m1sq)
    m2 = complex(m2sq)
    if base is None:
        base = max(1.0, float(mu2))
        while not _straight_path_ok(base, m1, m2):
            base *= 2.0
            if base > 1e8:
                raise ValueError("no base point on the positive real axis")
    r0 = float(base)
    theta = float(np.angle(x))
    # path samples: arc then ray (both parametrised uniformly)
    n_arc = max(2, int(steps * abs(theta) / np.pi) + 2)
    n_ray = max(2, int(steps * abs(np.log(abs(x) / r0))) + 2)
    path = [r0 * np.exp(1j * theta * k / (n_arc - 1)) for k in range(n_arc)]
    ray = np.exp(1j * theta)
    lo, hi = np.log(r0), np.log(abs(x))
    path += [np.exp(lo + (hi - lo) * k / (n_ray - 1)) * ray for k in range(1, n_ray)]
    path[-1] = x
    roots = list(_delta_roots(complex(path[0]), m1, m2))
    wind = [0, 0]

    def advance(xa: complex, xb: complex, ra, depth=0):
        nb = _delta_roots(xb, m1, m2)
        # match the new roots to the old ones by proximity
        if abs(nb[0] - ra[0]) + abs(nb[1] - ra[1]) > abs(nb[1] - ra[0]) + abs(nb[0] - ra[1]):
            nb = (nb[1], nb[0])
        big = max(abs(nb[i] - ra[i]) / (1e-3 + min(abs(ra[i]), abs(ra[i] - 1))) for i in (0, 1))
        cr = [_segment_crossing(ra[i], nb[i]) for i in (0, 1)]
        if (big > 0.05 or None in cr) and depth < 40:
            xm = 0.5 * (xa + xb)
            rm = advance(xa, xm, ra, depth + 1)
            return advance(xm, xb, rm, depth + 1)
        if None in cr:
            raise ValueError(f"a root of Delta passes through an end point near x = {xb}")
        for i in (0, 1):
            wind[i] += cr[i]
        return list(nb)

    for k in range(1, len(path)):
        roots = advance(complex(path[k - 1]), complex(path[k]), roots)

    mp_m2 = mp.mpc(m2)
    F = mp.log(mp_m2) - 2
    for a, w in zip(roots, wind):
        a = mp.mpc(a)
        F += (1 - a) * (_log_ratio_principal(a) + 2j * mp.pi * w)
    mu = mp.mpf(mu2)
    m1m = mp.mpc(m1)
    Fmu = mp.quad(lambda a: mp.log(delta(a, mu, m1m, mp_m2)), _split_points(mu, m1m, mp_m2))
    return complex(Fmu - F)


def _split_points(s, m1, m2):
    pts = [mp.mpf(0), mp.mpf(1)]
    b = m1 - m2 + s
    if s != 0:
        disc = mp.sqrt(b * b + 4 * s * m2)
        roots = [(b + disc) / (2 * s), (b - disc) / (2 * s)]
    elif b != 0:
        roots = [-m2 / b]
    else:
        roots = []
    for r in roots:
        if 0 < mp.re(r) < 1:
            pts.append(mp.re(r))
    return sorted(set(pts))
