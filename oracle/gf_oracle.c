/*
 * CPU FP64 oracle for the subtracted one-loop two-point integral on a grid of
 * complex x = p^2 (Windisch, Alkofer, Haase, Liebmann, "Examining the analytic
 * structure of Green's functions: massive parallel complex integration using
 * GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) never calls it, and the two share no code.
 *
 * What is computed (rescaled units of eq. 18 / eq. 21, times `scale`):
 *
 *   G(x) = scale * ( sum over the contour C of  dy y <F(x,y,.)>
 *                    - sum over the real axis of dy y <F(mu^2,y,.)> )
 *
 *   F(x,y,z)  = 1 / [ (x + y - 2 sqrt(x) sqrt(y) z + m1^2) (y + m2^2) ]
 *               (eq. 10 with the propagators of eq. 16 / eq. 19; m1^2 sits on
 *               the (p-k) leg, m2^2 on the k leg)
 *   <f>       = (2/pi) int_{-1}^{1} dz sqrt(1-z^2) f(z)        (eq. 11, eq. 21)
 *   subtraction at the real point mu^2 >= 0                     (eq. 12-14)
 *   C = deformed y contour from 0 to Lambda^2                   (STEP 3, eq. 15)
 *
 * Quadrature (section "Numerical Implementation"): non-adaptive Gauss rules.
 *   radial : n_radial-point Gauss-Legendre in t = log(1+y) on [0, log(1+Lambda^2)]
 *   angular: n_angular points of one of three rules for the measure
 *            (2/pi) sqrt(1-z^2) dz, chosen by angular_rule:
 *            0 Gauss-Chebyshev, second kind (default): z_j = cos(j pi/(n+1)),
 *              w_j = (2/(n+1)) sin^2(j pi/(n+1)), sum w_j = 1
 *            1 Gauss-Chebyshev, first kind, applied to f(z) (1 - z^2)
 *            2 tanh-sinh (double exponential), the paper's main angular rule
 *   arc    : n_arc-point Gauss-Legendre in the angle
 *
 * Contour per x (STEP 3; the paper's per-region contours of its worked example
 * are replaced by the following reading):
 *   R      real axis [0, Lambda^2]; valid while |Im sqrt(x)| < Re sqrt(m1^2);
 *          chosen when valid and (v < 0.25 v* or 1 - v/v* >= 0.45 delta), with
 *          v = |Im sqrt x|, v* = Re sqrt(m1^2), delta = angular distance from
 *          arg x to the nearest bad ray, or when no rotated contour applies
 *   Y      ray y = r e^{i phi}, phi = arg x, r in [0, Lambda^2], then the arc
 *          |y| = Lambda^2 from angle phi back to 0
 *   YRES   Y plus the residue of the k-leg pole y0 = -m2^2, which the ray has
 *          swept across (+2 pi i for phi > 0, -2 pi i for phi < 0)
 *   MIRROR G(x) = conj G(conj x)  (real masses or a conjugate mass pair)
 * Points on a singular set (x on a "bad ray" or on the negative real axis
 * outside region R) return NaN and class ORC_SINGULAR.
 *
 * Everything here is plain loops in double precision, written for a reader to
 * check against the paper by eye, not for speed.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { ORC_R = 0, ORC_Y = 1, ORC_YRES = 2, ORC_MIRROR = 3, ORC_SINGULAR = 4, ORC_LONG = 5 };

/* Region R is chosen where v = |Im sqrt x| is below ORC_R_NEAR of its bound
 * v* = Re sqrt(m1^2), or where 1 - v/v* is at least ORC_R_SLOPE times the
 * angular distance from arg x to the nearest bad ray. */
#define ORC_R_NEAR 0.25
#define ORC_R_SLOPE 0.45

typedef struct {
    double m1sq_re, m1sq_im;   /* m1^2 on the (p-k) leg */
    double m2sq_re, m2sq_im;   /* m2^2 on the k leg */
    double mu2;                /* real subtraction point, >= 0 */
    double lambda2;            /* cutoff Lambda^2 of eq. 14 */
    double scale;              /* 1 = eq. 18 units, 1/(16 pi^2) = eq. 17 units */
    int n_radial, n_angular, n_arc;
    int angular_rule;          /* 0 GC-II, 1 GC-I, 2 tanh-sinh */
    int taylor_order;          /* n of the subtraction operator t^n (eq. 13), -1..8 */
    int dimension;             /* D = 2, 3 or 4 (0 means 4) */
    int radial_split;          /* 1: split the radial rule at the near-singular radii */
    /* pole-sum propagators P1(s) = sum_a c1_a/(s + m1_a^2), P2(s) = sum_b
     * c2_b/(s + m2_b^2); n1 = 0 means one pole per leg at m1sq, m2sq with
     * residue 1.  Per pole: m^2 re, m^2 im, c re, c im. */
    int n1, n2;
    double p1[32], p2[32];
    /* numerator N(k^2, p.k) = sum_{i,j=0..2} n_ij (k^2)^i (p.k)^j multiplying
     * P1 P2 (eq. 4's general integrand); num_on = 0 means N = 1.  n_ij is
     * num[2(3i + j)] + i num[2(3i + j) + 1]. */
    int num_on;
    double num[18];
} orc_problem;

#define ORC_MAX_TAYLOR 8

static int orc_dim(const orc_problem *p) { return p->dimension == 0 ? 4 : p->dimension; }

/* ------------------------------------------------------------------------ */
/* Quadrature rules                                                          */
/* ------------------------------------------------------------------------ */

/* Gauss-Legendre nodes and weights on [-1,1]: roots of P_n found by Newton's
 * method, P_n and P_n' from the three-term recurrence; w = 2/((1-x^2) P_n'^2).
 * Nodes ascending. */
int orc_gauss_legendre(int n, double *x, double *w)
{
    if (n <= 0) return -1;
    for (int i = 0; i < n; ++i) {
        /* i-th root from the top, initial guess cos(pi (i + 3/4) / (n + 1/2)) */
        double r = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = r;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? r : p1;
            double pnm1 = (n == 1) ? 1.0 : p0;
            dp = n * (r * pn - pnm1) / (r * r - 1.0);
            double step = pn / dp;
            r -= step;
            if (fabs(step) < 1e-16) break;
        }
        /* recompute the derivative at the converged root */
        double p0 = 1.0, p1 = r;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double pn = (n == 1) ? r : p1;
        double pnm1 = (n == 1) ? 1.0 : p0;
        dp = n * (r * pn - pnm1) / (r * r - 1.0);
        x[n - 1 - i] = r;
        w[n - 1 - i] = 2.0 / ((1.0 - r * r) * dp * dp);
    }
    return 0;
}

/* Gauss-Chebyshev of the second kind, normalised so that
 * (2/pi) int_{-1}^{1} sqrt(1-z^2) f(z) dz ~ sum_j w_j f(z_j).  j = 1..n. */
int orc_gauss_cheb2(int n, double *z, double *w)
{
    if (n <= 0) return -1;
    for (int j = 1; j <= n; ++j) {
        double th = j * M_PI / (n + 1);
        double s = sin(th);
        z[j - 1] = cos(th);
        w[j - 1] = 2.0 / (n + 1) * s * s;
    }
    return 0;
}

/* Gauss-Chebyshev of the first kind: int_{-1}^{1} g(z) / sqrt(1-z^2) dz ~
 * (pi/n) sum_j g(z_j), z_j = cos((2j-1) pi/(2n)).  Our measure is
 * (2/pi) sqrt(1-z^2) dz = (2/pi)(1-z^2) dz / sqrt(1-z^2), so g = (2/pi)(1-z^2) f
 * and the weight of f(z_j) is (pi/n)(2/pi)(1-z_j^2). */
int orc_gauss_cheb1(int n, double *z, double *w)
{
    if (n <= 0) return -1;
    for (int j = 1; j <= n; ++j) {
        double zj = cos((2 * j - 1) * M_PI / (2.0 * n));
        z[j - 1] = zj;
        w[j - 1] = (M_PI / n) * (2.0 / M_PI) * (1.0 - zj * zj);
    }
    return 0;
}

/* Tanh-sinh (Takahasi-Mori double exponential) rule: substitute
 * z = tanh((pi/2) sinh t), so dz = (pi/2) cosh t / cosh^2((pi/2) sinh t) dt, and
 * apply the trapezoidal rule with step h on n equispaced t centred on 0,
 * t_k = (k - (n-1)/2) h.  The paper fixes only the node count (49 in well
 * behaved regions); reading: h = 6/(n-1), i.e. t in [-3, 3], where the
 * transformed measure has decayed far below double precision.  The weight of
 * f(z_k) is h dz/dt (2/pi) sqrt(1 - z_k^2); weights are not renormalised. */
int orc_tanh_sinh(int n, double *z, double *w)
{
    if (n < 3) return -1;
    double h = 6.0 / (n - 1);
    for (int k = 0; k < n; ++k) {
        double t = (k - 0.5 * (n - 1)) * h;
        double u = 0.5 * M_PI * sinh(t);
        double zk = tanh(u);
        double dzdt = 0.5 * M_PI * cosh(t) / (cosh(u) * cosh(u));
        z[k] = zk;
        w[k] = h * dzdt * (2.0 / M_PI) * sqrt(fmax(0.0, 1.0 - zk * zk));
    }
    return 0;
}

/* Nodes and weights of the angular rule `rule` (0 GC-II, 1 GC-I, 2 tanh-sinh)
 * for the four-dimensional measure (2/pi) sqrt(1-z^2) dz. */
int orc_angular_rule(int rule, int n, double *z, double *w)
{
    switch (rule) {
    case 0: return orc_gauss_cheb2(n, z, w);
    case 1: return orc_gauss_cheb1(n, z, w);
    case 2: return orc_tanh_sinh(n, z, w);
    default: return -1;
    }
}

/* The angular measure in D dimensions (eq. 5 generalised: the polar angle
 * carries sin^{D-2}(theta) d theta = (1-z^2)^{(D-3)/2} dz), normalised by
 * N_D = int_{-1}^{1} (1-z^2)^{(D-3)/2} dz = pi, 2, pi/2 for D = 2, 3, 4.  Each
 * rule approximates int g(z) omega(z) dz for its own weight function omega
 * (GC-II sqrt(1-z^2), GC-I 1/sqrt(1-z^2), Gauss-Legendre and tanh-sinh 1), so
 * the weight of f(z_j) is its plain weight times (1-z_j^2)^{(D-3)/2} /
 * omega(z_j) / N_D.  Rule 3 is Gauss-Legendre. */
int orc_angular_rule_dim(int rule, int dim, int n, double *z, double *w)
{
    if (n <= 0 || dim < 2 || dim > 4) return -1;
    double ND = dim == 2 ? M_PI : (dim == 3 ? 2.0 : M_PI / 2.0);
    double e = 0.5 * (dim - 3);
    if (rule == 0) {
        for (int j = 1; j <= n; ++j) {
            double th = j * M_PI / (n + 1), zj = cos(th), s2 = sin(th) * sin(th);
            z[j - 1] = zj;
            w[j - 1] = (M_PI / (n + 1)) * s2 * pow(s2, e) / sqrt(s2) / ND;
        }
    } else if (rule == 1) {
        for (int j = 1; j <= n; ++j) {
            double th = (2 * j - 1) * M_PI / (2.0 * n), s2 = sin(th) * sin(th);
            z[j - 1] = cos(th);
            w[j - 1] = (M_PI / n) * pow(s2, e) * sqrt(s2) / ND;
        }
    } else if (rule == 2) {
        /* the trapezoidal grid spans t in [-t_max, t_max] with t_max = 3, 3.5,
         * 4 for D = 4, 3, 2: there the transformed weight h dz/dt (1-z^2)^{(D-3)/2}
         * ~ cosh(t) / cosh^{D-1}((pi/2) sinh t) has fallen below 1e-16 */
        if (n < 3) return -1;
        double tmax = dim == 4 ? 3.0 : (dim == 3 ? 3.5 : 4.0);
        double h = 2.0 * tmax / (n - 1);
        for (int k = 0; k < n; ++k) {
            double t = (k - 0.5 * (n - 1)) * h;
            double u = 0.5 * M_PI * sinh(t);
            double dzdt = 0.5 * M_PI * cosh(t) / (cosh(u) * cosh(u));
            z[k] = tanh(u);
            /* 1 - z^2 = 1/cosh^2(u), exactly, without cancellation near |z| = 1 */
            w[k] = h * dzdt * pow(1.0 / (cosh(u) * cosh(u)), e) / ND;
        }
    } else if (rule == 3) {
        orc_gauss_legendre(n, z, w);
        for (int j = 0; j < n; ++j) w[j] = w[j] * pow(1.0 - z[j] * z[j], e) / ND;
    } else {
        return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The angular integral (eq. 11, inner z integral)                           */
/* ------------------------------------------------------------------------ */

/* <1/D1> for D1 = x + y + m1^2 - 2 sqrt(x) sqrt(y) z, at given sxsy = sqrt(x)sqrt(y).
 * If absum is given, adds sum_j |w_j / D1_j| (1 + (|x + y + m1^2| + |2 sxsy z_j|)/|D1_j|):
 * each term's size times its first-order sensitivity to relative perturbations
 * of its inputs (a conditioning measure, see orc_eval_points). */
static cplx angular_d1(cplx x, cplx y, cplx sxsy, cplx m1sq, int n,
                       const double *z, const double *w, double *absum)
{
    cplx acc = 0.0;
    double a = 0.0;
    /* |x + y + m1^2| and |2 sqrt(x) sqrt(y)| do not depend on j, and
     * |w_j / D1_j| = |w_j| / |D1_j| */
    const double u_abs = absum ? cabs(x + y + m1sq) : 0.0;
    const double v_abs = absum ? cabs(2.0 * sxsy) : 0.0;
    for (int j = 0; j < n; ++j) {
        cplx d1 = x + y - 2.0 * sxsy * z[j] + m1sq;
        cplx t = w[j] / d1;
        acc += t;
        if (absum) {
            const double dabs = sqrt(creal(d1) * creal(d1) + cimag(d1) * cimag(d1));
            a += fabs(w[j]) / dabs * (1.0 + (u_abs + v_abs * fabs(z[j])) / dabs);
        }
    }
    if (absum) *absum += a;
    return acc;
}

/* The same sum with the numerator N(y, p.k) in every term, p.k = sxsy z_j:
 * sum_j w_j N_j / D1_j.  absum adds per term |w_j|/|D1_j| times (the
 * numerator's parts, each times its degree + 1, plus |N_j| times the
 * denominator's sensitivity). */
static cplx angular_d1_num(cplx x, cplx y, cplx sxsy, cplx m1sq, int n, const double *z,
                           const double *w, const double *num, double *absum)
{
    cplx acc = 0.0;
    double a = 0.0;
    const double u_abs = absum ? cabs(x + y + m1sq) : 0.0;
    const double v_abs = absum ? cabs(2.0 * sxsy) : 0.0;
    for (int j = 0; j < n; ++j) {
        cplx d1 = x + y - 2.0 * sxsy * z[j] + m1sq;
        cplx pk = sxsy * z[j];
        cplx nv = 0.0;
        double nabs = 0.0;
        for (int i = 0; i <= 2; ++i)
            for (int q = 0; q <= 2; ++q) {
                cplx c = num[2 * (3 * i + q)] + I * num[2 * (3 * i + q) + 1];
                if (c == 0.0) continue;
                cplx part = c * cpow(y, i) * cpow(pk, q);
                nv += part;
                nabs += cabs(part) * (1.0 + i + q);
            }
        acc += w[j] * nv / d1;
        if (absum) {
            const double dabs = cabs(d1);
            a += fabs(w[j]) / dabs * (nabs + cabs(nv) * (u_abs + v_abs * fabs(z[j])) / dabs);
        }
    }
    if (absum) *absum += a;
    return acc;
}

/* Exported for the pin tests: sum_j w_j / (U - V z_j) with the oracle's GC-II
 * rule of order n. */
void orc_angular_sum(double u_re, double u_im, double v_re, double v_im, int n,
                     double *out_re, double *out_im)
{
    double *z = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    orc_gauss_cheb2(n, z, w);
    /* U - V z = (x + y + m1^2) - 2 sqrt(x)sqrt(y) z with x = U, y = 0, m1^2 = 0,
     * 2 sqrt(x) sqrt(y) = V */
    cplx r = angular_d1(u_re + I * u_im, 0.0, 0.5 * (v_re + I * v_im), 0.0, n, z, w, NULL);
    *out_re = creal(r);
    *out_im = cimag(r);
    free(z);
    free(w);
}

/* ------------------------------------------------------------------------ */
/* Contour choice (STEP 3)                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n1, n2;
    cplx m1[8], c1[8], m2[8], c2[8];  /* poles and residues of P1, P2 */
    double b1[8], b2[8];    /* bad-ray angles arg(-m^2) of every pole */
    cplx m1sq, m2sq;        /* the first pole of each leg */
    double lo, hi;          /* open sector (lo, hi) reachable by rotating the ray */
    double vstar;           /* region-R bound on |Im sqrt(x)|: min_a Re sqrt(m1_a^2) */
    int mirror_ok;          /* G(conj x) = conj G(x) for these propagators */
    int dim;                /* D = 2, 3, 4 */
} orc_geometry;

/* arg(-m^2); a real positive m^2 gives carg(-m^2) = +pi or -pi depending on
 * the sign of the zero imaginary part: it is the negative real axis either
 * way, taken as +pi */
static double orc_bad_ray(cplx m)
{
    return cimag(m) == 0.0 ? M_PI : carg(-m);
}

/* Is the pole multiset (m, c) of `a` (conjugated if conj) equal to that of b? */
static int orc_same_poles(int na, const cplx *ma, const cplx *ca, int nb, const cplx *mb,
                          const cplx *cb, int conj_a)
{
    if (na != nb) return 0;
    int used[8] = {0};
    for (int i = 0; i < na; ++i) {
        cplx m = conj_a ? conj(ma[i]) : ma[i], c = conj_a ? conj(ca[i]) : ca[i];
        int found = 0;
        for (int j = 0; j < nb && !found; ++j)
            if (!used[j] && m == mb[j] && c == cb[j]) used[j] = found = 1;
        if (!found) return 0;
    }
    return 1;
}

static void orc_make_geometry(const orc_problem *p, orc_geometry *g)
{
    if (p->n1 == 0) {
        g->n1 = g->n2 = 1;
        g->m1[0] = p->m1sq_re + I * p->m1sq_im;
        g->m2[0] = p->m2sq_re + I * p->m2sq_im;
        g->c1[0] = g->c2[0] = 1.0;
    } else {
        g->n1 = p->n1;
        g->n2 = p->n2;
        for (int k = 0; k < p->n1; ++k) {
            g->m1[k] = p->p1[4 * k] + I * p->p1[4 * k + 1];
            g->c1[k] = p->p1[4 * k + 2] + I * p->p1[4 * k + 3];
        }
        for (int k = 0; k < p->n2; ++k) {
            g->m2[k] = p->p2[4 * k] + I * p->p2[4 * k + 1];
            g->c2[k] = p->p2[4 * k + 2] + I * p->p2[4 * k + 3];
        }
    }
    g->m1sq = g->m1[0];
    g->m2sq = g->m2[0];
    g->dim = orc_dim(p);
    g->hi = M_PI;
    g->lo = -M_PI;
    g->vstar = INFINITY;
    for (int k = 0; k < g->n1; ++k) {
        g->b1[k] = orc_bad_ray(g->m1[k]);
        g->vstar = fmin(g->vstar, creal(csqrt(g->m1[k])));
    }
    for (int k = 0; k < g->n2; ++k) g->b2[k] = orc_bad_ray(g->m2[k]);
    for (int k = 0; k < g->n1 + g->n2; ++k) {
        double b = k < g->n1 ? g->b1[k] : g->b2[k - g->n1];
        if (b > 0.0 && b < g->hi) g->hi = b;
        if (b <= 0.0 && b > g->lo) g->lo = b;
    }
    /* conjugation maps (P1, P2) onto itself (real-analytic propagators, e.g.
     * real masses) or onto (P2, P1) (e.g. a conjugate mass pair, by the
     * exchange of the two legs) */
    g->mirror_ok = (orc_same_poles(g->n1, g->m1, g->c1, g->n1, g->m1, g->c1, 1) &&
                    orc_same_poles(g->n2, g->m2, g->c2, g->n2, g->m2, g->c2, 1)) ||
                   (orc_same_poles(g->n1, g->m1, g->c1, g->n2, g->m2, g->c2, 1) &&
                    orc_same_poles(g->n2, g->m2, g->c2, g->n1, g->m1, g->c1, 1));
    /* with a numerator N(k^2, p.k): conjugation needs real coefficients, and
     * the exchange k -> p - k of the legs does not leave N as it is */
    if (p->num_on) {
        int real = 1;
        for (int k = 0; k < 9; ++k) real = real && p->num[2 * k + 1] == 0.0;
        g->mirror_ok = real && orc_same_poles(g->n1, g->m1, g->c1, g->n1, g->m1, g->c1, 1) &&
                       orc_same_poles(g->n2, g->m2, g->c2, g->n2, g->m2, g->c2, 1);
    }
}

/* angular distance between two angles, in [0, pi] */
static double ang_dist(double a, double b)
{
    double d = fabs(a - b);
    return d > M_PI ? 2.0 * M_PI - d : d;
}

/* Does rotating the ray from angle 0 to phi sweep across the ray at angle b? */
static int orc_swept(double phi, double b)
{
    return phi > 0.0 ? (b > 0.0 && b < phi) : (b <= 0.0 && b > phi);
}

/* Rotated-contour class of x (Y, YRES, MIRROR, LONG or SINGULAR); for YRES,
 * *res_sign = +1 or -1 and *mask flags the k-leg poles swept across, whose
 * residues the contour picks up.  LONG: the rotation towards arg x sweeps a
 * (p-k)-leg bad ray and neither YRES nor the mirror point applies; each such
 * pole's term is then continued the other way round the origin (see
 * orc_long_sets).  SINGULAR only on a bad ray itself. */
static int orc_rotated_class(const orc_geometry *g, double phi, int *res_sign, int *mask)
{
    *res_sign = 0;
    *mask = 0;
    if (phi > g->lo && phi < g->hi) return ORC_Y;
    int cross1 = 0, on = 0, m = 0;
    for (int k = 0; k < g->n1; ++k) {
        cross1 |= orc_swept(phi, g->b1[k]);
        on |= ang_dist(phi, g->b1[k]) == 0.0;
    }
    for (int k = 0; k < g->n2; ++k) {
        if (orc_swept(phi, g->b2[k])) m |= 1 << k;
        on |= ang_dist(phi, g->b2[k]) == 0.0;
    }
    if (on) return ORC_SINGULAR;
    if (m && !cross1) {
        *res_sign = phi > 0.0 ? 1 : -1;
        *mask = m;
        return ORC_YRES;
    }
    if (cross1 && !m && g->mirror_ok) return ORC_MIRROR;
    return ORC_LONG;
}

/* The two groups of a LONG point.  Rotating the ray from angle 0 to phi the
 * short way (through the half plane of x) is blocked for the (p-k)-leg poles
 * whose bad ray lies in between; each of their terms c1_a <1/(U_a - V z)> is
 * continued by rotating the other way, through the other half plane, by
 * 2 pi - |phi|, which sweeps none of its own bad ray.  Both rotations end on
 * the same ray y = r e^{i phi}; the closing arcs |y| = Lambda^2 run back to
 * angle 0 the short way (terms of the short group) and the long way (terms
 * of the long group), and each group takes the residues of the k-leg poles
 * its own rotation sweeps: the short one with sign sign(phi) (as YRES), the
 * long one with -sign(phi).  In D = 3 the measure sqrt(y) is continued along
 * each rotation: the long one reaches the ray, its arc and its residues with
 * angles shifted by -+ 2 pi, which flips the sign of sqrt(y) there (the
 * short sector holds the cut of sqrt(y)).  *grp_long flags the long group's (p-k)-leg poles,
 * *res_short and *res_long the k-leg poles whose residues each group adds. */
static void orc_long_sets(const orc_geometry *g, double phi, int *grp_long, int *res_short,
                          int *res_long)
{
    *grp_long = *res_short = *res_long = 0;
    for (int a = 0; a < g->n1; ++a)
        if (orc_swept(phi, g->b1[a])) *grp_long |= 1 << a;
    for (int b = 0; b < g->n2; ++b) {
        if (orc_swept(phi, g->b2[b])) *res_short |= 1 << b;
        else if (ang_dist(phi, g->b2[b]) != 0.0) *res_long |= 1 << b;
    }
}

/* Class of x; for YRES, *res_sign = +1 or -1 and *mask the residues due. */
static int orc_classify_m(const orc_geometry *g, cplx x, int *res_sign, int *mask)
{
    double v = fabs(cimag(csqrt(x)));
    double phi = carg(x);
    int rot = orc_rotated_class(g, phi, res_sign, mask);
    if (v < g->vstar) {
        double delta = M_PI;
        for (int k = 0; k < g->n1; ++k) delta = fmin(delta, ang_dist(phi, g->b1[k]));
        for (int k = 0; k < g->n2; ++k) delta = fmin(delta, ang_dist(phi, g->b2[k]));
        if (v < ORC_R_NEAR * g->vstar || 1.0 - v / g->vstar >= ORC_R_SLOPE * delta ||
            rot == ORC_SINGULAR || rot == ORC_LONG) {
            *res_sign = 0;
            *mask = 0;
            return ORC_R;
        }
    }
    return rot;
}

static int orc_classify(const orc_geometry *g, cplx x, int *res_sign)
{
    int mask;
    return orc_classify_m(g, x, res_sign, &mask);
}

/* The class a point is evaluated with: a MIRROR point whose conjugate has no
 * contour of its own (MIRROR, LONG or SINGULAR there) takes the real axis if
 * it is valid at x, else the long way round at x. */
static int orc_final_class(const orc_geometry *g, cplx x, int *res_sign, int *mask)
{
    int cls = orc_classify_m(g, x, res_sign, mask);
    if (cls != ORC_MIRROR) return cls;
    int sb, mb;
    int cb = orc_classify_m(g, conj(x), &sb, &mb);
    if (cb != ORC_MIRROR && cb != ORC_SINGULAR && cb != ORC_LONG) return cls;
    *res_sign = 0;
    *mask = 0;
    if (fabs(cimag(csqrt(x))) < g->vstar) return ORC_R;
    return ORC_LONG;
}

/* ------------------------------------------------------------------------ */
/* One grid point                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_problem *p;
    orc_geometry geo;
    double *gl_t, *gl_w;     /* radial GL on [-1,1] */
    double *arc_x, *arc_w;   /* arc GL on [-1,1] */
    double *z, *w;           /* GC-II */
    double *r, *wr;          /* radial nodes y = r_i, dy weights (incl. Jacobian) */
    double *seg_x, *seg_w;   /* split rule: GL of order n_radial/4 on [-1,1] */
    cplx jmu;                /* subtraction term: real-axis sum at x = mu^2 */
    double jmu_abs;
    cplx taylor[ORC_MAX_TAYLOR + 1]; /* K_i, i >= 1: (1/i!) d^i/dx^i of that sum at mu^2 */
    double taylor_rho;               /* radius of the Cauchy circle the K_i come from */
} orc_ctx;

/* sum over the contour of dy y/(y + m2^2) <1/D1>, for class cls (R, Y, YRES) */
/* The radial measure y^{(D-2)/2} of D dimensions (dy y for D = 4), given y
 * and sqrt(y) on the branch continued along the contour. */
static cplx orc_measure(int dim, cplx y, cplx sy)
{
    return dim == 4 ? y : (dim == 3 ? sy : 1.0);
}

/* Radial nodes r_i and dy weights (Jacobian included) along the straight part
 * of the contour of the point xn.  Without splitting: the plan's GL rule in
 * t = log(1+r) on [0, T], T = log(1 + Lambda^2).  Split (the paper's several
 * sub-contours, section "Numerical Implementation"): [0, T] is cut at
 * t = log(1 + rho) for the radii rho in (0, Lambda^2) where the integrand has
 * near-singularities -- the moduli of the angular cut's end points
 * y(z = +-1) = (sqrt(xn) +- sqrt(-m1^2))^2 (eq. 25 at theta = 0, pi) and of
 * the k-leg pole y = -m2^2 -- and, while fewer than three cuts exist, at the
 * midpoint of the longest piece; each of the four pieces gets n_radial/4 GL
 * nodes.  Tolerances (duplicates within 1e-9 T, "longest" by more than
 * 1e-12 T) keep near-ties decided alike under any rounding. */
static void orc_radial_nodes(const orc_ctx *c, cplx xn, double *r, double *wr)
{
    const orc_problem *p = c->p;
    if (!p->radial_split) {
        memcpy(r, c->r, sizeof(double) * p->n_radial);
        memcpy(wr, c->wr, sizeof(double) * p->n_radial);
        return;
    }
    double T = log1p(p->lambda2);
    cplx sm = csqrt(-c->geo.m1sq), sx = csqrt(xn);
    double cand[3] = {cabs((sx + sm) * (sx + sm)), cabs((sx - sm) * (sx - sm)), cabs(c->geo.m2sq)};
    double b[5];
    int nb = 0;
    b[nb++] = 0.0;
    b[nb++] = T;
    /* cuts within 1e-9 T of one another count once */
    for (int k = 0; k < 3; ++k) {
        if (!(cand[k] > 0.0 && cand[k] < p->lambda2)) continue;
        double t = log1p(cand[k]);
        int dup = 0;
        for (int q = 0; q < nb; ++q) dup |= fabs(b[q] - t) <= 1e-9 * T;
        if (!dup) b[nb++] = t;
    }
    /* sort the boundaries (at most five) */
    for (int i = 1; i < nb; ++i)
        for (int j = i; j > 0 && b[j - 1] > b[j]; --j) {
            double tmp = b[j];
            b[j] = b[j - 1];
            b[j - 1] = tmp;
        }
    while (nb < 5) {
        int wide = 0;
        /* the longest piece, the first one unless another is longer by 1e-12 T */
        for (int i = 1; i < nb - 1; ++i)
            if (b[i + 1] - b[i] > b[wide + 1] - b[wide] + 1e-12 * T) wide = i;
        double mid = 0.5 * (b[wide] + b[wide + 1]);
        for (int j = nb; j > wide + 1; --j) b[j] = b[j - 1];
        b[wide + 1] = mid;
        ++nb;
    }
    int m = p->n_radial / 4;
    for (int s = 0; s < 4; ++s)
        for (int i = 0; i < m; ++i) {
            double h = 0.5 * (b[s + 1] - b[s]);
            double t = b[s] + h * (c->seg_x[i] + 1.0);
            r[s * m + i] = expm1(t);
            wr[s * m + i] = h * c->seg_w[i] * (1.0 + r[s * m + i]);
        }
}

/* <P1(D1)>(x, y) = sum_a c1_a <1/(x + y + m1_a^2 - 2 sqrt(x) sqrt(y) z)>; with
 * sens given, adds sum_a |c1_a| (that pole's absolute angular sum with its
 * sensitivity factor, as angular_d1 counts it). */
static cplx orc_ang_p1_set(const orc_ctx *c, cplx x, cplx y, cplx sxsy, int set, double *sens)
{
    cplx s = 0.0;
    for (int a = 0; a < c->geo.n1; ++a) {
        if (!(set >> a & 1)) continue;
        double t = 0.0;
        s += c->geo.c1[a] *
             (c->p->num_on ? angular_d1_num(x, y, sxsy, c->geo.m1[a], c->p->n_angular, c->z, c->w,
                                            c->p->num, sens ? &t : NULL)
                           : angular_d1(x, y, sxsy, c->geo.m1[a], c->p->n_angular, c->z, c->w,
                                        sens ? &t : NULL));
        if (sens) *sens += cabs(c->geo.c1[a]) * t;
    }
    return s;
}

static cplx orc_ang_p1(const orc_ctx *c, cplx x, cplx y, cplx sxsy, double *sens)
{
    return orc_ang_p1_set(c, x, y, sxsy, ~0, sens);
}

/* P2(y) = sum_b c2_b / (y + m2_b^2); *sens = sum_b |c2_b / (y + m2_b^2)|
 * (1 + |y| / |y + m2_b^2|), its size times its sensitivity to y. */
static cplx orc_p2(const orc_ctx *c, cplx y, double *sens)
{
    cplx s = 0.0;
    *sens = 0.0;
    for (int b = 0; b < c->geo.n2; ++b) {
        cplx t = c->geo.c2[b] / (y + c->geo.m2[b]);
        s += t;
        *sens += cabs(t) * (1.0 + cabs(y) / cabs(y + c->geo.m2[b]));
    }
    return s;
}

/* One contour node of the (p-k)-leg poles in `set`: weight w (dy and the
 * measure) at y with sqrt(y) = sy. */
static cplx orc_node_set(const orc_ctx *c, cplx x, cplx sx, cplx y, cplx sy, cplx w, int set,
                         double *absum)
{
    double a = 0.0, sp = 0.0;
    cplx ang = orc_ang_p1_set(c, x, y, sx * sy, set, absum ? &a : NULL);
    cplx pre = w * orc_measure(orc_dim(c->p), y, sy) * orc_p2(c, y, &sp);
    if (absum) *absum += cabs(w * orc_measure(orc_dim(c->p), y, sy)) * sp * a;
    return pre * ang;
}

static cplx orc_node(const orc_ctx *c, cplx x, cplx sx, cplx y, cplx sy, cplx w, double *absum)
{
    return orc_node_set(c, x, sx, y, sy, w, ~0, absum);
}

/* Residues of the k-leg poles in `res` for the (p-k)-leg poles in `set`: at
 * y0 = -m2_b^2 the residue of y^{(D-2)/2} P2(y) <P1>(y) is
 * c2_b y0^{(D-2)/2} <P1>(y0); each is added times sign 2 pi i. */
static cplx orc_residues(const orc_ctx *c, cplx x, cplx sx, int res, int set, int sign,
                         double long_phi, double *absum)
{
    cplx s = 0.0;
    for (int b = 0; b < c->geo.n2; ++b) {
        if (!(res >> b & 1)) continue;
        cplx y0 = -c->geo.m2[b];
        double a = 0.0;
        cplx ang = orc_ang_p1_set(c, x, y0, sx * csqrt(y0), set, absum ? &a : NULL);
        /* sqrt(y0) continued along the rotation that sweeps y0: the principal
         * one, except for the long rotation (long_phi = arg x != 0), whose
         * angle at y0 is arg(y0) -+ 2 pi past the negative real axis; on that
         * axis it is -pi (long_phi > 0, turning clockwise) or +pi */
        cplx sy0 = csqrt(y0);
        if (long_phi != 0.0) {
            double t = carg(y0);
            if (cimag(y0) == 0.0 && creal(y0) < 0.0) t = long_phi > 0.0 ? -M_PI : M_PI;
            else if (long_phi > 0.0 && t > long_phi) t -= 2.0 * M_PI;
            else if (long_phi < 0.0 && t < long_phi) t += 2.0 * M_PI;
            sy0 = sqrt(cabs(y0)) * cexp(I * 0.5 * t);
        }
        cplx pre = sign * 2.0 * M_PI * I * c->geo.c2[b] * orc_measure(orc_dim(c->p), y0, sy0);
        s += pre * ang;
        if (absum) *absum += cabs(pre) * a;
    }
    return s;
}

/* The contour sum of the point x (class cls, residue flags res_mask for
 * YRES); the straight part's nodes are those of the point xn (x itself, or
 * mu^2 for the subtraction sums). */
static cplx orc_contour_sum(const orc_ctx *c, cplx x, cplx xn, int cls, int res_sign,
                            int res_mask, double *absum)
{
    const int dim = orc_dim(c->p);
    const orc_problem *p = c->p;
    cplx sx = csqrt(x);
    cplx s = 0.0;
    double *rn = malloc(sizeof(double) * p->n_radial), *wn = malloc(sizeof(double) * p->n_radial);
    orc_radial_nodes(c, xn, rn, wn);
    if (cls == ORC_R) {
        for (int i = 0; i < p->n_radial; ++i) s += orc_node(c, x, sx, rn[i], sqrt(rn[i]), wn[i], absum);
        free(rn);
        free(wn);
        return s;
    }
    /* ray at the angle of x: y = r e^{i phi}, dy = e^{i phi} dr */
    double phi = carg(x);
    cplx e = cexp(I * phi);
    cplx eh = cexp(I * 0.5 * phi);
    int grp_long = 0, res_short = res_mask, res_long = 0;
    if (cls == ORC_LONG) orc_long_sets(&c->geo, phi, &grp_long, &res_short, &res_long);
    const int all = (1 << c->geo.n1) - 1, grp_short = all & ~grp_long;
    /* sqrt(y) along each rotation: the long one reaches the ray at angle
     * phi -+ 2 pi, where sqrt(y) = -e^{i phi/2} sqrt(r) (only the measure of
     * D = 3 sees the sign; the angular sums are even in sqrt(y)) */
    const int split_ray = dim == 3 && grp_long;
    for (int i = 0; i < p->n_radial; ++i) {
        if (!split_ray) {
            s += orc_node(c, x, sx, e * rn[i], eh * sqrt(rn[i]), e * wn[i], absum);
        } else {
            if (grp_short)
                s += orc_node_set(c, x, sx, e * rn[i], eh * sqrt(rn[i]), e * wn[i], grp_short, absum);
            s += orc_node_set(c, x, sx, e * rn[i], -eh * sqrt(rn[i]), e * wn[i], grp_long, absum);
        }
    }
    double lam = sqrt(p->lambda2);
    if (grp_short) {
        /* arc |y| = Lambda^2 from angle phi back to 0 the short way:
         * psi(s) = phi (1 - s)/2, dy = i y psi'(s) ds = -i y (phi/2) ds */
        for (int k = 0; k < p->n_arc; ++k) {
            double psi = 0.5 * phi * (1.0 - c->arc_x[k]);
            cplx y = p->lambda2 * cexp(I * psi);
            cplx sy = lam * cexp(I * 0.5 * psi);
            s += orc_node_set(c, x, sx, y, sy, -I * y * (0.5 * phi) * c->arc_w[k], grp_short,
                              absum);
        }
    }
    if (grp_long) {
        /* the long way: psi(s) = phi + L (1 + s)/2 with L = sign(phi) 2 pi - phi,
         * ending at angle +-2 pi, i.e. at y = Lambda^2; dy = i y (L/2) ds */
        double L = (phi > 0.0 ? 2.0 * M_PI : -2.0 * M_PI) - phi;
        for (int k = 0; k < p->n_arc; ++k) {
            double psi = phi + 0.5 * L * (1.0 + c->arc_x[k]);
            cplx y = p->lambda2 * cexp(I * psi);
            /* continued from the ray's angle phi -+ 2 pi: e^{i (psi -+ 2 pi)/2} */
            cplx sy = -lam * cexp(I * 0.5 * psi);
            s += orc_node_set(c, x, sx, y, sy, I * y * (0.5 * L) * c->arc_w[k], grp_long, absum);
        }
    }
    if (cls == ORC_YRES) s += orc_residues(c, x, sx, res_mask, all, res_sign, 0.0, absum);
    if (cls == ORC_LONG) {
        const int sg = phi > 0.0 ? 1 : -1;
        if (grp_short) s += orc_residues(c, x, sx, res_short, grp_short, sg, 0.0, absum);
        s += orc_residues(c, x, sx, res_long, grp_long, -sg, phi, absum);
    }
    free(rn);
    free(wn);
    return s;
}

/* The subtracted polynomial of t^n (eq. 12-13, about x = mu^2):
 * sum_{i=0}^{n} (x - mu^2)^i K_i, K_0 the real-axis sum at mu^2.  If absum is
 * given, adds for i >= 1 |x - mu^2|^i (|K_i| + |K_0| rho^-i): each term's own
 * size, and the rounding of the Cauchy sum that K_i comes from (about
 * eps |S| rho^-i), in units of eps. */
static cplx orc_subtraction(const orc_ctx *c, cplx x, double *absum)
{
    if (c->p->taylor_order < 0) return 0.0;  /* t^-1: nothing subtracted */
    cplx sub = c->jmu, d = x - c->p->mu2, dp = 1.0;
    for (int i = 1; i <= c->p->taylor_order; ++i) {
        dp *= d;
        sub += dp * c->taylor[i];
        if (absum)
            *absum += cabs(dp) * (cabs(c->taylor[i]) + cabs(c->jmu) * pow(c->taylor_rho, -i));
    }
    return sub;
}

/* G at one point; returns the class; *cond as described at orc_eval_points. */
static int orc_point(const orc_ctx *c, cplx x, int force_class, cplx *g, double *cond)
{
    int sign = 0, mask = 0;
    int cls = orc_final_class(&c->geo, x, &sign, &mask);
    if (force_class >= 0) {
        cls = force_class;
        if (cls == ORC_YRES) {
            sign = carg(x) > 0.0 ? 1 : -1;
            mask = 0;
            for (int b = 0; b < c->geo.n2; ++b)
                if (orc_swept(carg(x), c->geo.b2[b])) mask |= 1 << b;
        }
    }
    double absum = c->p->taylor_order < 0 ? 0.0 : c->jmu_abs;
    double *pab = cond ? &absum : NULL;
    cplx s;
    if (cls == ORC_SINGULAR) {
        *g = NAN + I * NAN;
        if (cond) *cond = NAN;
        return cls;
    }
    if (cls == ORC_MIRROR) {
        cplx xb = conj(x);
        int sb = 0, mb = 0;
        int cb = orc_classify_m(&c->geo, xb, &sb, &mb);
        s = orc_contour_sum(c, xb, xb, cb, sb, mb, pab);
        cplx gb = c->p->scale * (s - orc_subtraction(c, xb, pab));
        *g = conj(gb);
        if (cond) *cond = c->p->scale * absum / cabs(gb);
        return cls;
    }
    s = orc_contour_sum(c, x, x, cls, sign, mask, pab);
    *g = c->p->scale * (s - orc_subtraction(c, x, pab));
    if (cond) *cond = c->p->scale * absum / cabs(*g);
    return cls;
}

static void orc_ctx_free(orc_ctx *c);

/* Taylor coefficients K_i = (1/i!) d^i S/dx^i at x = mu^2, i = 0..n, of the
 * real-axis sum S(x) = sum over the radial nodes of W y P2(y) <N P1(D1)>(x, y)
 * (N = 1 without a numerator),
 * by Cauchy's integral formula: K_i = (1/(2 pi i)) contour integral of
 * S(x) / (x - mu^2)^(i+1) over |x - mu^2| = rho, with the trapezoidal rule on
 * 64 equally spaced points (exact up to (rho/R)^64 for S analytic in the disc
 * of radius R).  S is a sum of terms rational in x whose poles are the x where
 * some node's first propagator vanishes, x = (sqrt(y) z +- sqrt(y z^2 - y -
 * m1_a^2))^2 for any pole a of P1; rho is half the distance from mu^2 to the
 * nearest of them. */
static double orc_taylor_cauchy(const orc_ctx *c, int n, cplx *K)
{
    const orc_problem *p = c->p;
    double dmin = INFINITY;
    double *rn = malloc(sizeof(double) * p->n_radial), *wn = malloc(sizeof(double) * p->n_radial);
    orc_radial_nodes(c, p->mu2, rn, wn);
    for (int i = 0; i < p->n_radial; ++i) {
        cplx sy = sqrt(rn[i]);
        for (int j = 0; j < p->n_angular; ++j)
            for (int a = 0; a < c->geo.n1; ++a) {
                cplx root = csqrt(rn[i] * c->z[j] * c->z[j] - rn[i] - c->geo.m1[a]);
                cplx s1 = sy * c->z[j] + root, s2 = sy * c->z[j] - root;
                dmin = fmin(dmin, fmin(cabs(s1 * s1 - p->mu2), cabs(s2 * s2 - p->mu2)));
            }
    }
    free(rn);
    free(wn);
    double rho = 0.5 * dmin;
    const int N = 64;
    for (int i = 0; i <= n; ++i) K[i] = 0.0;
    for (int k = 0; k < N; ++k) {
        cplx e = cexp(I * 2.0 * M_PI * k / N);
        cplx S = orc_contour_sum(c, p->mu2 + rho * e, p->mu2, ORC_R, 0, 0, NULL);
        for (int i = 0; i <= n; ++i) K[i] += S * cpow(rho * e, -i) / N;
    }
    return rho;
}

static int orc_ctx_init(orc_ctx *c, const orc_problem *p)
{
    memset(c, 0, sizeof(*c));
    c->p = p;
    if (p->n_radial <= 0 || p->n_angular <= 0 || p->n_arc < 0) return -1;
    orc_make_geometry(p, &c->geo);
    int nr = p->n_radial, na = p->n_angular, nc = p->n_arc > 0 ? p->n_arc : 1;
    c->gl_t = malloc(sizeof(double) * nr);
    c->gl_w = malloc(sizeof(double) * nr);
    c->r = malloc(sizeof(double) * nr);
    c->wr = malloc(sizeof(double) * nr);
    c->arc_x = malloc(sizeof(double) * nc);
    c->arc_w = malloc(sizeof(double) * nc);
    c->z = malloc(sizeof(double) * na);
    c->w = malloc(sizeof(double) * na);
    orc_gauss_legendre(nr, c->gl_t, c->gl_w);
    if (p->n_arc > 0) orc_gauss_legendre(p->n_arc, c->arc_x, c->arc_w);
    if (p->radial_split) {
        if (nr % 4 != 0 || p->n1 > 1 || p->n2 > 1) {  /* the split rule needs single poles */
            orc_ctx_free(c);
            return -1;
        }
        c->seg_x = malloc(sizeof(double) * (nr / 4));
        c->seg_w = malloc(sizeof(double) * (nr / 4));
        orc_gauss_legendre(nr / 4, c->seg_x, c->seg_w);
    }
    if (orc_angular_rule_dim(p->angular_rule, orc_dim(p), na, c->z, c->w) != 0) {
        orc_ctx_free(c);
        return -1;
    }
    /* t = log(1+y) on [0, T], T = log(1 + Lambda^2): y = e^t - 1, dy = (1+y) dt */
    double T = log1p(p->lambda2);
    for (int i = 0; i < nr; ++i) {
        double t = 0.5 * T * (c->gl_t[i] + 1.0);
        c->r[i] = expm1(t);
        c->wr[i] = 0.5 * T * c->gl_w[i] * (1.0 + c->r[i]);
    }
    /* subtraction term (eq. 14 at x = mu^2, real axis) */
    double a = 0.0;
    c->jmu = orc_contour_sum(c, p->mu2 + 0.0 * I, p->mu2, ORC_R, 0, 0, &a);
    c->jmu_abs = a;
    if (p->taylor_order < -1 || p->taylor_order > ORC_MAX_TAYLOR) {
        orc_ctx_free(c);
        return -1;
    }
    if (p->taylor_order > 0) c->taylor_rho = orc_taylor_cauchy(c, p->taylor_order, c->taylor);
    return 0;
}

static void orc_ctx_free(orc_ctx *c)
{
    free(c->gl_t); free(c->gl_w); free(c->r); free(c->wr);
    free(c->arc_x); free(c->arc_w); free(c->z); free(c->w);
    free(c->seg_x); free(c->seg_w);
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                     */
/* ------------------------------------------------------------------------ */

/* G at n arbitrary points.  force_class < 0: automatic contour choice.
 * g: 2n doubles (re, im interleaved).  cls, cond may be NULL.
 * cond[k] = scale * sum over every term of |term| * (its first-order
 * sensitivity to relative input perturbations) / |G|, with the subtraction sum
 * counted the same way: a second FP64 evaluation of the same quadrature whose
 * inputs and operations are each accurate to a few ulp differs from this one
 * by a small multiple of eps * cond * |G|. */
int orc_eval_points(const orc_problem *p, long n, const double *x_re, const double *x_im,
                    int force_class, double *g, signed char *cls, double *cond)
{
    orc_ctx c;
    if (orc_ctx_init(&c, p) != 0) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < n; ++k) {
        cplx gk;
        double ck = 0.0;
        int cl = orc_point(&c, x_re[k] + I * x_im[k], force_class, &gk, cond ? &ck : NULL);
        g[2 * k] = creal(gk);
        g[2 * k + 1] = cimag(gk);
        if (cls) cls[k] = (signed char)cl;
        if (cond) cond[k] = ck;
    }
    orc_ctx_free(&c);
    return 0;
}

/* Cell-centred grid point (a, b) of an n_re x n_im box (STEP 4):
 * Re x = fma(a + 1/2, (re_hi - re_lo)/n_re, re_lo), likewise Im x.
 * Row-major, a (the Re index) fastest. */
void orc_grid_point(long a, long b, long n_re, long n_im, double re_lo, double re_hi,
                    double im_lo, double im_hi, double *xr, double *xi)
{
    double dre = (re_hi - re_lo) / (double)n_re;
    double dim = (im_hi - im_lo) / (double)n_im;
    *xr = fma((double)a + 0.5, dre, re_lo);
    *xi = fma((double)b + 0.5, dim, im_lo);
}

/* Whole grid: out has 2 n_re n_im doubles, index (b n_re + a). */
int orc_scan(const orc_problem *p, long n_re, long n_im, double re_lo, double re_hi,
             double im_lo, double im_hi, double *g, signed char *cls, double *cond)
{
    long n = n_re * n_im;
    double *xr = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *xi = malloc(sizeof(double) * (n > 0 ? n : 1));
    for (long b = 0; b < n_im; ++b)
        for (long a = 0; a < n_re; ++a)
            orc_grid_point(a, b, n_re, n_im, re_lo, re_hi, im_lo, im_hi,
                           &xr[b * n_re + a], &xi[b * n_re + a]);
    int rc = orc_eval_points(p, n, xr, xi, -1, g, cls, cond);
    free(xr);
    free(xi);
    return rc;
}

/* The subtraction term sum (unscaled), for tests. */
int orc_jmu(const orc_problem *p, double *re, double *im)
{
    orc_ctx c;
    if (orc_ctx_init(&c, p) != 0) return -1;
    *re = creal(c.jmu);
    *im = cimag(c.jmu);
    orc_ctx_free(&c);
    return 0;
}

/* Class of each point without evaluating (for tests). */
/* All Taylor coefficients K_0..K_n of the subtraction by the Cauchy formula
 * (K_0 also by the direct sum, as orc_jmu): out 2(n+1) doubles; *rho the
 * radius of the circle used. */
int orc_taylor(const orc_problem *p, int n, double *out, double *rho)
{
    orc_ctx c;
    orc_problem q = *p;
    q.taylor_order = 0;
    if (orc_dim(p) < 2 || orc_dim(p) > 4) return -1;
    if (n < 0 || n > ORC_MAX_TAYLOR || orc_ctx_init(&c, &q) != 0) return -1;
    cplx K[ORC_MAX_TAYLOR + 1];
    *rho = orc_taylor_cauchy(&c, n, K);
    for (int i = 0; i <= n; ++i) {
        out[2 * i] = creal(K[i]);
        out[2 * i + 1] = cimag(K[i]);
    }
    orc_ctx_free(&c);
    return 0;
}

int orc_classify_points(const orc_problem *p, long n, const double *x_re, const double *x_im,
                        signed char *cls)
{
    orc_geometry g;
    orc_make_geometry(p, &g);
    for (long k = 0; k < n; ++k) {
        int s, m;
        cls[k] = (signed char)orc_final_class(&g, x_re[k] + I * x_im[k], &s, &m);
    }
    return 0;
}

/* The contour each point is evaluated on, for the quad-precision twin:
 * info[7k..7k+6] = {evaluated at conj x (MIRROR), class there, residue sign,
 * k-leg residues of the short rotation, (p-k)-leg poles of the long rotation,
 * k-leg residues of the long rotation, 0}. */
int orc_point_contours(const orc_problem *p, long n, const double *x_re, const double *x_im,
                       int *info)
{
    orc_geometry g;
    orc_make_geometry(p, &g);
    for (long k = 0; k < n; ++k) {
        cplx x = x_re[k] + I * x_im[k];
        int sign = 0, mask = 0, conj_eval = 0;
        int cls = orc_final_class(&g, x, &sign, &mask);
        if (cls == ORC_MIRROR) {
            x = conj(x);
            cls = orc_classify_m(&g, x, &sign, &mask);
            conj_eval = 1;
        }
        int grp_long = 0, res_short = mask, res_long = 0;
        if (cls == ORC_LONG) {
            orc_long_sets(&g, carg(x), &grp_long, &res_short, &res_long);
            sign = carg(x) > 0.0 ? 1 : -1;
        }
        int *o = info + 7 * k;
        o[0] = conj_eval;
        o[1] = cls;
        o[2] = sign;
        o[3] = res_short;
        o[4] = grp_long;
        o[5] = res_long;
        o[6] = 0;
    }
    return 0;
}

/* Threads an OpenMP region of the oracle uses. */
int orc_threads(void) { return omp_get_max_threads(); }

/* y-plane diagnostic at fixed x (the paper's Fig. 1): for each y_k,
 * what = 0: <P1>(x, y_k); what = 1: y^{(D-2)/2} P2(y) (<P1>(x, y) - <P1>(mu^2, y)),
 * the order-0 subtracted y-integrand of eq. 14 (principal sqrt(y) for D = 3;
 * P1 = 1/D1 and P2 = 1/(y + m2^2) for single poles).  out: 2n doubles. */
int orc_yscan(const orc_problem *p, double x_re, double x_im, long n, const double *y_re,
              const double *y_im, int what, double *out)
{
    if (p->n_angular <= 0) return -1;
    double *z = malloc(sizeof(double) * p->n_angular), *w = malloc(sizeof(double) * p->n_angular);
    if (orc_angular_rule_dim(p->angular_rule, orc_dim(p), p->n_angular, z, w) != 0) {
        free(z);
        free(w);
        return -1;
    }
    orc_geometry g;
    orc_make_geometry(p, &g);
    cplx x = x_re + I * x_im;
    cplx sx = csqrt(x), smu = sqrt(p->mu2);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        cplx y = y_re[k] + I * y_im[k];
        cplx sy = csqrt(y);
        cplx a = 0.0, amu = 0.0, p2 = 0.0;
        for (int q = 0; q < g.n1; ++q) {
            a += g.c1[q] * angular_d1(x, y, sx * sy, g.m1[q], p->n_angular, z, w, NULL);
            amu += g.c1[q] * angular_d1(p->mu2 + 0.0 * I, y, smu * sy, g.m1[q], p->n_angular, z, w,
                                        NULL);
        }
        for (int q = 0; q < g.n2; ++q) p2 += g.c2[q] / (y + g.m2[q]);
        if (what == 1) a = orc_measure(orc_dim(p), y, csqrt(y)) * p2 * (a - amu);
        out[2 * k] = creal(a);
        out[2 * k + 1] = cimag(a);
    }
    free(z);
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Obstruction of a contour by the angular cut (the paper's Fig. 2)          */
/* ------------------------------------------------------------------------ */

/* The first propagator x + y + m1^2 - 2 sqrt(x) sqrt(y) z has a zero in z on
 * [-1, 1] exactly when z0 = (x + y + m1^2) / (2 sqrt(x) sqrt(y)) is real with
 * |z0| <= 1, i.e. when zeta = z0^2 = (x + y + m1^2)^2 / (4 x y) is real and in
 * [0, 1].  A contour part is sampled at parameter values u_k; where Im zeta is
 * positive at one sample and not at the next, the zero of Im zeta between them
 * is located by 40 bisection steps on u, and the cut crosses the contour if
 * Re zeta there is in [0, 1].  *tie is raised when that value lies within 1e-9
 * of 0 or 1, or a sample has |Im zeta| <= 1e-13 |zeta|: there, another
 * rounding of the same steps may decide the other way. */
typedef struct {
    cplx x, m1sq;
    int arc;          /* 0: y = (e^u - 1) dir; 1: y = Lambda^2 e^{iu} */
    cplx dir;
    double lambda2;
} orc_cut_part;

static cplx orc_zeta(const orc_cut_part *c, double u)
{
    cplx y = c->arc ? c->lambda2 * cexp(I * u) : expm1(u) * c->dir;
    cplx num = (c->x + y + c->m1sq) * (c->x + y + c->m1sq);
    return num / (4.0 * c->x * y);
}

/* Walks the samples u[0..n-1] of one part; returns 1 if the cut crosses it. */
static int orc_cut_walk(const orc_cut_part *c, const double *u, int n, int *tie)
{
    int hit = 0;
    cplx prev = 0.0;
    for (int k = 0; k < n; ++k) {
        cplx zeta = orc_zeta(c, u[k]);
        if (fabs(cimag(zeta)) <= 1e-13 * cabs(zeta)) *tie = 1;
        if (k > 0 && (cimag(prev) > 0.0) != (cimag(zeta) > 0.0)) {
            double a = u[k - 1], b = u[k];
            int a_pos = cimag(prev) > 0.0;
            for (int it = 0; it < 40; ++it) {
                double m = 0.5 * (a + b);
                if ((cimag(orc_zeta(c, m)) > 0.0) == a_pos) a = m;
                else b = m;
            }
            double re = creal(orc_zeta(c, 0.5 * (a + b)));
            if (re >= 0.0 && re <= 1.0) hit = 1;
            if (fabs(re) < 1e-9 || fabs(re - 1.0) < 1e-9) *tie = 1;
        }
        prev = zeta;
    }
    return hit;
}

/* The real segment: u = T k/(n-1), k = 1..n-1, T = log(1 + Lambda^2). */
static int orc_cut_real(const orc_problem *p, cplx x, int n, int *tie)
{
    orc_cut_part c = {x, p->m1sq_re + I * p->m1sq_im, 0, 1.0, p->lambda2};
    double T = log1p(p->lambda2);
    double *u = malloc(sizeof(double) * n);
    for (int k = 1; k < n; ++k) u[k - 1] = T * k / (n - 1);
    int hit = orc_cut_walk(&c, u, n - 1, tie);
    free(u);
    return hit;
}

/* The ray at phi = arg x (same u), then the arc from phi back to 0 at
 * u = phi (1 - k/(n-1)), k = 0..n-1, or, the long way round the origin, from
 * phi on to +-2 pi at u = phi + L k/(n-1), L = sign(phi) 2 pi - phi. */
static int orc_cut_ray_arc(const orc_problem *p, cplx x, int n, int long_way, int *tie)
{
    double phi = carg(x), T = log1p(p->lambda2);
    orc_cut_part ray = {x, p->m1sq_re + I * p->m1sq_im, 0, cexp(I * phi), p->lambda2};
    orc_cut_part arc = ray;
    arc.arc = 1;
    double *u = malloc(sizeof(double) * n);
    for (int k = 1; k < n; ++k) u[k - 1] = T * k / (n - 1);
    int hit = orc_cut_walk(&ray, u, n - 1, tie);
    double L = (phi > 0.0 ? 2.0 * M_PI : -2.0 * M_PI) - phi;
    for (int k = 0; k < n; ++k)
        u[k] = long_way ? phi + L * k / (n - 1) : phi * (1.0 - (double)k / (n - 1));
    hit |= orc_cut_walk(&arc, u, n, tie);
    free(u);
    return hit;
}

/* Per point: bit 0 the real segment [0, Lambda^2] is crossed; bit 1 the
 * contour of the class rule is crossed (for a mirror point, the contour of
 * conj x); bit 2 no contour (SINGULAR).  tie[k] = 1 where a decision sits
 * within rounding of its threshold. */
int orc_obstruction(const orc_problem *p, long n, const double *x_re, const double *x_im,
                    int n_samples, unsigned char *out, unsigned char *tie)
{
    if (n_samples < 2) return -1;
    orc_geometry g;
    orc_make_geometry(p, &g);
#pragma omp parallel for schedule(dynamic, 64)
    for (long k = 0; k < n; ++k) {
        cplx x = x_re[k] + I * x_im[k];
        int t = 0, s;
        int v = orc_cut_real(p, x, n_samples, &t);
        int m;
        int cls = orc_final_class(&g, x, &s, &m);
        cplx xe = x;
        int ecls = cls;
        if (cls == ORC_MIRROR) {
            xe = conj(x);
            ecls = orc_classify(&g, xe, &s);
        }
        if (cls == ORC_SINGULAR) {
            v |= 4;
        } else {
            int used = ecls == ORC_R ? orc_cut_real(p, xe, n_samples, &t)
                                     : orc_cut_ray_arc(p, xe, n_samples, ecls == ORC_LONG, &t);
            if (used) v |= 2;
        }
        out[k] = (unsigned char)v;
        tie[k] = (unsigned char)t;
    }
    return 0;
}

/* The radial nodes and dy weights the straight part of the contour of x uses
 * (exported for the pin tests of the split rule). */
int orc_radial_nodes_at(const orc_problem *p, double x_re, double x_im, double *r, double *w)
{
    orc_ctx c;
    orc_problem q = *p;
    q.taylor_order = 0;
    if (orc_ctx_init(&c, &q) != 0) return -1;
    orc_radial_nodes(&c, x_re + I * x_im, r, w);
    orc_ctx_free(&c);
    return 0;
}
