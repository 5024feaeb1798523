/*
 * Quad-precision (__float128) brute force of the same quadrature as the FP64
 * oracle: identical rules, contour choice and subtraction, every node, weight
 * and sum carried in 113-bit arithmetic.  Only tiny grids are meant for it.
 *
 * TEST INFRASTRUCTURE ONLY (see the FP64 oracle's header).  It exists to
 * measure the rounding error of the FP64 oracle (and, through it, of the GPU
 * path), not to be fast.
 *
 * Written separately from the FP64 oracle: the two files share no code.
 */
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 qr;
typedef __complex128 qc;

typedef struct {
    double m1sq_re, m1sq_im, m2sq_re, m2sq_im;
    double mu2, lambda2, scale;
    int n_radial, n_angular, n_arc;
    int angular_rule;   /* 0 GC-II, 1 GC-I, 2 tanh-sinh, 3 Gauss-Legendre */
    int taylor_order;   /* n of t^n, -1..8 */
    int dimension;      /* 2, 3, 4 (0 = 4) */
    int radial_split;   /* only 0 is implemented here */
    int n1, n2;         /* only 0 (single poles) is implemented here */
    double p1[32], p2[32];
    int num_on;         /* only 0 (no numerator) is implemented here */
    double num[18];
} orcq_problem;   /* same layout as the FP64 oracle's problem struct */

#define QPI M_PIq

static qc mkc(qr re, qr im)
{
    qc z;
    __real__ z = re;
    __imag__ z = im;
    return z;
}

/* Legendre roots by Newton in quad precision, seeded from the asymptotic guess. */
static void q_gauss_legendre(int n, qr *x, qr *w)
{
    for (int i = 0; i < n; ++i) {
        qr r = cosq(QPI * (i + 0.75Q) / (n + 0.5Q));
        qr dp = 1, pn = 0, pnm1 = 0;
        for (int it = 0; it < 200; ++it) {
            qr p0 = 1, p1 = r;
            for (int k = 2; k <= n; ++k) {
                qr p2 = ((2 * k - 1) * r * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            pn = (n == 1) ? r : p1;
            pnm1 = (n == 1) ? 1 : p0;
            dp = n * (r * pn - pnm1) / (r * r - 1);
            qr step = pn / dp;
            r -= step;
            if (fabsq(step) < 1e-33Q) break;
        }
        qr p0 = 1, p1 = r;
        for (int k = 2; k <= n; ++k) {
            qr p2 = ((2 * k - 1) * r * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        pn = (n == 1) ? r : p1;
        pnm1 = (n == 1) ? 1 : p0;
        dp = n * (r * pn - pnm1) / (r * r - 1);
        x[n - 1 - i] = r;
        w[n - 1 - i] = 2 / ((1 - r * r) * dp * dp);
    }
}

/* The angular rule for the normalised D-dimensional angular measure
 * (1 - z^2)^{(D-3)/2} dz / N_D, N_D = pi, 2, pi/2 for D = 2, 3, 4: each rule
 * integrates g against its own weight omega(z) and is applied to
 * g = f (1 - z^2)^{(D-3)/2} / omega.  Gauss-Chebyshev II (omega = sqrt(1-z^2),
 * z = cos(j pi/(n+1))), Gauss-Chebyshev I (omega = 1/sqrt(1-z^2),
 * z = cos((2j-1) pi/(2n))), tanh-sinh (z = tanh((pi/2) sinh t) on n
 * equispaced t in [-t_max, t_max], t_max = 3, 3.5, 4 for D = 4, 3, 2),
 * Gauss-Legendre (omega = 1).  Returns -1 for an unknown rule. */
static int q_angular_rule(int rule, int dim, int n, qr *z, qr *w)
{
    const qr norm = dim == 2 ? QPI : (dim == 3 ? 2 : QPI / 2);
    const qr ex = (qr)(dim - 3) / 2;   /* exponent of (1 - z^2) in the measure */
    if (rule == 0 || rule == 1) {
        for (int j = 1; j <= n; ++j) {
            qr th = rule == 0 ? j * QPI / (n + 1) : (2 * j - 1) * QPI / (2 * n);
            qr s = sinq(th);
            z[j - 1] = cosq(th);
            /* omega^-1 (1-z^2)^ex = sin^{D-4} (GC-II) or sin^{D-2} (GC-I), times
             * the rule's own weight pi/(n+1) sin^2 or pi/n */
            w[j - 1] = (rule == 0 ? QPI / (n + 1) * s * s * powq(s, dim - 4)
                                  : QPI / n * powq(s, dim - 2)) / norm;
        }
        return 0;
    }
    if (rule == 2) {
        if (n < 3) return -1;
        const qr tmax = dim == 4 ? 3 : (dim == 3 ? 3.5Q : 4);
        const qr h = 2 * tmax / (n - 1);
        for (int k = 0; k < n; ++k) {
            qr t = (k - (n - 1) / 2.0Q) * h;
            qr u = QPI / 2 * sinhq(t);
            qr cu = coshq(u);
            z[k] = tanhq(u);
            /* dz = (pi/2) cosh t / cosh^2 u dt, 1 - z^2 = 1/cosh^2 u */
            w[k] = h * QPI / 2 * coshq(t) / (cu * cu) * powq(cu, -2 * ex) / norm;
        }
        return 0;
    }
    if (rule == 3) {
        q_gauss_legendre(n, z, w);
        for (int k = 0; k < n; ++k) w[k] = w[k] * powq(1 - z[k] * z[k], ex) / norm;
        return 0;
    }
    return -1;
}

/* sum_j w_j / (x + y + m1^2 - 2 sxsy z_j) with the problem's angular rule */
static qc q_angular(qc x, qc y, qc sxsy, qc m1sq, int n, const qr *z, const qr *w)
{
    qc acc = 0;
    for (int j = 0; j < n; ++j) acc += w[j] / (x + y - 2 * sxsy * z[j] + m1sq);
    return acc;
}

/* Contour classes, numbered as in the FP64 oracle */
enum { Q_R = 0, Q_Y = 1, Q_YRES = 2, Q_MIRROR = 3, Q_SINGULAR = 4 };

typedef struct {
    const orcq_problem *p;
    qc m1sq, m2sq;
    qr beta1, beta2, lo, hi, vstar;
    int mirror_ok;
    qr *r, *wr, *ax, *aw, *az, *azw;
    int dim;
    qc jmu;
    qc taylor[9];   /* K_0..K_n of the subtraction at mu^2 */
} qctx;

static qr q_angdist(qr a, qr b)
{
    qr d = fabsq(a - b);
    return d > QPI ? 2 * QPI - d : d;
}

static int q_classify(const qctx *c, qc x, int *sign)
{
    qr v = fabsq(cimagq(csqrtq(x)));
    qr phi = cargq(x);
    int rot;
    *sign = 0;
    if (phi > c->lo && phi < c->hi) {
        rot = Q_Y;
    } else {
        int c1, c2;
        if (phi > 0) {
            c1 = c->beta1 > 0 && c->beta1 < phi;
            c2 = c->beta2 > 0 && c->beta2 < phi;
        } else {
            c1 = c->beta1 <= 0 && c->beta1 > phi;
            c2 = c->beta2 <= 0 && c->beta2 > phi;
        }
        int on = q_angdist(phi, c->beta1) == 0 || q_angdist(phi, c->beta2) == 0;
        if (on) rot = Q_SINGULAR;
        else if (c2 && !c1) { rot = Q_YRES; *sign = phi > 0 ? 1 : -1; }
        else if (c1 && !c2 && c->mirror_ok) rot = Q_MIRROR;
        else rot = Q_SINGULAR;
    }
    if (v < c->vstar) {
        qr d1 = q_angdist(phi, c->beta1), d2 = q_angdist(phi, c->beta2);
        qr delta = d1 < d2 ? d1 : d2;
        if (v < 0.25Q * c->vstar || 1 - v / c->vstar >= 0.45Q * delta || rot == Q_SINGULAR) {
            *sign = 0;
            return Q_R;
        }
    }
    return rot;
}

/* y^{(D-2)/2} with the square root continued along the contour from y = 0:
 * on the ray y = e^{i phi} r it is e^{i phi/2} sqrt(r), |phi| < pi */
static qc q_ypow(int dim, qc y)
{
    return dim == 4 ? y : (dim == 3 ? csqrtq(y) : mkc(1, 0));
}

static qc q_contour(const qctx *c, qc x, int cls, int sign)
{
    const orcq_problem *p = c->p;
    const int na = p->n_angular;
    qc sx = csqrtq(x);
    qc s = 0;
    if (cls == Q_R) {
        for (int i = 0; i < p->n_radial; ++i) {
            qc y = mkc(c->r[i], 0);
            qc a = q_angular(x, y, sx * sqrtq(c->r[i]), c->m1sq, na, c->az, c->azw);
            s += c->wr[i] * q_ypow(c->dim, y) / (y + c->m2sq) * a;
        }
        return s;
    }
    qr phi = cargq(x);
    qc e = mkc(cosq(phi), sinq(phi));
    qc eh = mkc(cosq(phi / 2), sinq(phi / 2));
    for (int i = 0; i < p->n_radial; ++i) {
        qc y = e * c->r[i];
        qc a = q_angular(x, y, sx * eh * sqrtq(c->r[i]), c->m1sq, na, c->az, c->azw);
        s += e * c->wr[i] * q_ypow(c->dim, y) / (y + c->m2sq) * a;
    }
    qr L2 = p->lambda2, L = sqrtq(L2);
    for (int k = 0; k < p->n_arc; ++k) {
        qr psi = phi * (1 - c->ax[k]) / 2;
        qc y = L2 * mkc(cosq(psi), sinq(psi));
        qc sy = L * mkc(cosq(psi / 2), sinq(psi / 2));
        qc a = q_angular(x, y, sx * sy, c->m1sq, na, c->az, c->azw);
        qc dy = mkc(0, -1) * y * (phi / 2) * c->aw[k];
        s += dy * q_ypow(c->dim, y) / (y + c->m2sq) * a;
    }
    if (cls == Q_YRES) {
        qc y0 = -c->m2sq;
        qc a = q_angular(x, y0, sx * csqrtq(y0), c->m1sq, na, c->az, c->azw);
        s += sign * 2 * QPI * mkc(0, 1) * q_ypow(c->dim, y0) * a;
    }
    return s;
}

/* Taylor coefficients K_1..K_n of the real-axis sum S(x) about mu^2 by
 * Cauchy's formula, trapezoidal rule on 64 points of the circle of radius half
 * the distance from mu^2 to the nearest x where a node's first propagator
 * vanishes (aliasing below 2^-64 of the coefficients' size). */
static void q_taylor(qctx *c)
{
    const orcq_problem *p = c->p;
    const int n = p->taylor_order;
    qr dmin = 1e300Q;
    for (int i = 0; i < p->n_radial; ++i) {
        qr sy = sqrtq(c->r[i]);
        for (int j = 0; j < p->n_angular; ++j) {
            qc root = csqrtq(c->r[i] * c->az[j] * c->az[j] - c->r[i] - c->m1sq);
            qc s1 = sy * c->az[j] + root, s2 = sy * c->az[j] - root;
            qr d1 = cabsq(s1 * s1 - p->mu2), d2 = cabsq(s2 * s2 - p->mu2);
            if (d1 < dmin) dmin = d1;
            if (d2 < dmin) dmin = d2;
        }
    }
    const qr rho = dmin / 2;
    const int N = 64;
    for (int i = 1; i <= n; ++i) c->taylor[i] = 0;
    for (int k = 0; k < N; ++k) {
        qc e = mkc(cosq(2 * QPI * k / N), sinq(2 * QPI * k / N));
        qc S = q_contour(c, p->mu2 + rho * e, Q_R, 0);
        qc pw = 1;
        for (int i = 1; i <= n; ++i) {
            pw *= rho * e;
            c->taylor[i] += S / pw / N;
        }
    }
}

/* The subtracted sum at the evaluated point xe (conj x for a mirror point):
 * S(xe) - sum_{i=0}^{n} (xe - mu^2)^i K_i (nothing for n = -1). */
static qc q_subtracted(const qctx *c, qc xe, qc S)
{
    const int n = c->p->taylor_order;
    if (n < 0) return S;
    qc sub = c->jmu, d = xe - c->p->mu2, pw = 1;
    for (int i = 1; i <= n; ++i) {
        pw *= d;
        sub += pw * c->taylor[i];
    }
    return S - sub;
}

/* G at n points in quad precision, rounded to double on output (g: 2n doubles). */
int orcq_eval_points(const orcq_problem *p, long n, const double *x_re, const double *x_im,
                     double *g, signed char *cls)
{
    qctx c;
    memset(&c, 0, sizeof(c));
    c.p = p;
    c.m1sq = mkc(p->m1sq_re, p->m1sq_im);
    c.m2sq = mkc(p->m2sq_re, p->m2sq_im);
    c.beta1 = (p->m1sq_im == 0) ? QPI : cargq(-c.m1sq);
    c.beta2 = (p->m2sq_im == 0) ? QPI : cargq(-c.m2sq);
    c.hi = QPI;
    c.lo = -QPI;
    qr b[2] = {c.beta1, c.beta2};
    for (int k = 0; k < 2; ++k) {
        if (b[k] > 0 && b[k] < c.hi) c.hi = b[k];
        if (b[k] <= 0 && b[k] > c.lo) c.lo = b[k];
    }
    c.vstar = crealq(csqrtq(c.m1sq));
    c.mirror_ok = (p->m1sq_im == 0 && p->m2sq_im == 0) ||
                  (p->m1sq_re == p->m2sq_re && p->m1sq_im == -p->m2sq_im);
    if (p->radial_split || p->n1 > 1 || p->n2 > 1 || p->num_on || p->taylor_order < -1 ||
        p->taylor_order > 8)
        return -1;
    c.dim = p->dimension == 0 ? 4 : p->dimension;
    if (c.dim < 2 || c.dim > 4) return -1;
    int nr = p->n_radial, nc = p->n_arc > 0 ? p->n_arc : 1;
    c.az = malloc(sizeof(qr) * p->n_angular);
    c.azw = malloc(sizeof(qr) * p->n_angular);
    if (q_angular_rule(p->angular_rule, c.dim, p->n_angular, c.az, c.azw) != 0) {
        free(c.az);
        free(c.azw);
        return -1;
    }
    qr *t = malloc(sizeof(qr) * nr), *tw = malloc(sizeof(qr) * nr);
    c.r = malloc(sizeof(qr) * nr);
    c.wr = malloc(sizeof(qr) * nr);
    c.ax = malloc(sizeof(qr) * nc);
    c.aw = malloc(sizeof(qr) * nc);
    q_gauss_legendre(nr, t, tw);
    if (p->n_arc > 0) q_gauss_legendre(p->n_arc, c.ax, c.aw);
    qr T = log1pq((qr)p->lambda2);
    for (int i = 0; i < nr; ++i) {
        qr tt = T * (t[i] + 1) / 2;
        c.r[i] = expm1q(tt);
        c.wr[i] = T / 2 * tw[i] * (1 + c.r[i]);
    }
    c.jmu = q_contour(&c, mkc(p->mu2, 0), Q_R, 0);
    if (p->taylor_order > 0) q_taylor(&c);
#pragma omp parallel for schedule(dynamic, 1)
    for (long k = 0; k < n; ++k) {
        qc x = mkc(x_re[k], x_im[k]);
        int sign;
        int cl = q_classify(&c, x, &sign);
        qc gk;
        if (cl == Q_SINGULAR) {
            gk = mkc(NAN, NAN);
        } else if (cl == Q_MIRROR) {
            qc xb = conjq(x);
            int sb;
            int cb = q_classify(&c, xb, &sb);
            if (cb == Q_MIRROR || cb == Q_SINGULAR) {
                gk = mkc(NAN, NAN);
                cl = Q_SINGULAR;
            } else {
                gk = conjq((qr)p->scale * q_subtracted(&c, xb, q_contour(&c, xb, cb, sb)));
            }
        } else {
            gk = (qr)p->scale * q_subtracted(&c, x, q_contour(&c, x, cl, sign));
        }
        g[2 * k] = (double)crealq(gk);
        g[2 * k + 1] = (double)cimagq(gk);
        if (cls) cls[k] = (signed char)cl;
    }
    free(t); free(tw); free(c.r); free(c.wr); free(c.ax); free(c.aw); free(c.az); free(c.azw);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* General integrands: pole sums, numerators, the long way round             */
/* ------------------------------------------------------------------------ */

/* The same quadrature for pole-sum propagators P1 = sum_a c1_a/(s + m1_a^2),
 * P2 = sum_b c2_b/(s + m2_b^2), an optional numerator N(k^2, p.k), every
 * contour class including the long way round, in quad precision.  The
 * contour of each point is not chosen here: it is given (class, residue
 * sign and pole sets, as the FP64 oracle chose them; a discrete choice, not
 * a rounding), so that the comparison measures rounding alone.  Per point,
 * info[7k..7k+6] = {evaluated at conj x (MIRROR), class at the evaluated
 * point, residue sign, k-leg residues of the short rotation, (p-k)-leg poles
 * of the long rotation, k-leg residues of the long rotation, 0}. */
typedef struct {
    const orcq_problem *p;
    int n1, n2, dim;
    qc m1[8], c1[8], m2[8], c2[8];
    qc num[9];
    int num_on;
    qr *r, *wr, *ax, *aw, *az, *azw;
    qc jmu;
    qc taylor[9];
} qgen;

static qc q_meas(int dim, qc y, qc sy)
{
    return dim == 4 ? y : (dim == 3 ? sy : mkc(1, 0));
}

/* sum over the (p-k)-leg poles in `set` of c1_a sum_j w_j N_j / D1_j,
 * D1_j = x + y + m1_a^2 - 2 sxsy z_j, N_j = N(y, sxsy z_j) (1 without one) */
static qc q_ang_set(const qgen *g, qc x, qc y, qc sxsy, int set)
{
    const int na = g->p->n_angular;
    qc s = 0;
    for (int a = 0; a < g->n1; ++a) {
        if (!(set >> a & 1)) continue;
        qc acc = 0;
        for (int j = 0; j < na; ++j) {
            qc d = x + y - 2 * sxsy * g->az[j] + g->m1[a];
            qc nv = 1;
            if (g->num_on) {
                qc pk = sxsy * g->az[j];
                nv = 0;
                qc yi = 1;
                for (int i = 0; i <= 2; ++i) {
                    qc pj = 1;
                    for (int q = 0; q <= 2; ++q) {
                        nv += g->num[3 * i + q] * yi * pj;
                        pj *= pk;
                    }
                    yi *= y;
                }
            }
            acc += g->azw[j] * nv / d;
        }
        s += g->c1[a] * acc;
    }
    return s;
}

static qc q_p2(const qgen *g, qc y)
{
    qc s = 0;
    for (int b = 0; b < g->n2; ++b) s += g->c2[b] / (y + g->m2[b]);
    return s;
}

/* the contour sum at the evaluated point x for the given class and sets */
static qc q_contour_gen(const qgen *g, qc x, int cls, int sign, int res_short, int grp_long,
                        int res_long)
{
    const orcq_problem *p = g->p;
    const int all = (1 << g->n1) - 1, grp_short = all & ~grp_long;
    qc sx = csqrtq(x);
    qc s = 0;
    if (cls == Q_R) {
        for (int i = 0; i < p->n_radial; ++i) {
            qc y = mkc(g->r[i], 0), sy = mkc(sqrtq(g->r[i]), 0);
            s += g->wr[i] * q_meas(g->dim, y, sy) * q_p2(g, y) * q_ang_set(g, x, y, sx * sy, all);
        }
        return s;
    }
    qr phi = cargq(x);
    qc e = mkc(cosq(phi), sinq(phi)), eh = mkc(cosq(phi / 2), sinq(phi / 2));
    for (int i = 0; i < p->n_radial; ++i) {
        qc y = e * g->r[i], sy = eh * sqrtq(g->r[i]);
        qc pre = e * g->wr[i] * q_p2(g, y);
        if (grp_short)
            s += pre * q_meas(g->dim, y, sy) * q_ang_set(g, x, y, sx * sy, grp_short);
        /* the long rotation reaches the ray at phi -+ 2 pi: sqrt(y) changes sign */
        if (grp_long)
            s += pre * q_meas(g->dim, y, -sy) * q_ang_set(g, x, y, sx * sy, grp_long);
    }
    qr L2 = p->lambda2, Lm = sqrtq(L2);
    if (grp_short)
        for (int k = 0; k < p->n_arc; ++k) {
            qr psi = phi * (1 - g->ax[k]) / 2;
            qc y = L2 * mkc(cosq(psi), sinq(psi)), sy = Lm * mkc(cosq(psi / 2), sinq(psi / 2));
            qc dy = mkc(0, -1) * y * (phi / 2) * g->aw[k];
            s += dy * q_meas(g->dim, y, sy) * q_p2(g, y) * q_ang_set(g, x, y, sx * sy, grp_short);
        }
    if (grp_long) {
        qr Lr = (phi > 0 ? 2 * QPI : -2 * QPI) - phi;
        for (int k = 0; k < p->n_arc; ++k) {
            qr psi = phi + Lr * (1 + g->ax[k]) / 2;
            qc y = L2 * mkc(cosq(psi), sinq(psi)), sy = -Lm * mkc(cosq(psi / 2), sinq(psi / 2));
            qc dy = mkc(0, 1) * y * (Lr / 2) * g->aw[k];
            s += dy * q_meas(g->dim, y, sy) * q_p2(g, y) * q_ang_set(g, x, y, sx * sy, grp_long);
        }
    }
    /* residues: the short rotation's with `sign`, the long one's with -sign
     * and sqrt(y0) at the long rotation's angle */
    for (int b = 0; b < g->n2; ++b) {
        qc y0 = -g->m2[b];
        if (res_short >> b & 1) {
            qc sy0 = csqrtq(y0);
            s += sign * 2 * QPI * mkc(0, 1) * g->c2[b] * q_meas(g->dim, y0, sy0) *
                 q_ang_set(g, x, y0, sx * sy0, grp_short);
        }
        if (res_long >> b & 1) {
            qr t = cargq(y0);
            if (cimagq(y0) == 0 && crealq(y0) < 0) t = phi > 0 ? -QPI : QPI;
            else if (phi > 0 && t > phi) t -= 2 * QPI;
            else if (phi < 0 && t < phi) t += 2 * QPI;
            qc sy0 = sqrtq(cabsq(y0)) * mkc(cosq(t / 2), sinq(t / 2));
            s += -sign * 2 * QPI * mkc(0, 1) * g->c2[b] * q_meas(g->dim, y0, sy0) *
                 q_ang_set(g, x, y0, sx * sy0, grp_long);
        }
    }
    return s;
}

/* Taylor coefficients K_1..K_n of the real-axis sum about mu^2 by Cauchy's
 * formula on 64 points of a circle of half the distance from mu^2 to the
 * nearest x where a node's first propagator (any pole) vanishes. */
static void q_taylor_gen(qgen *g)
{
    const orcq_problem *p = g->p;
    const int n = p->taylor_order;
    qr dmin = 1e300Q;
    for (int i = 0; i < p->n_radial; ++i) {
        qr sy = sqrtq(g->r[i]);
        for (int j = 0; j < p->n_angular; ++j)
            for (int a = 0; a < g->n1; ++a) {
                qc root = csqrtq(g->r[i] * g->az[j] * g->az[j] - g->r[i] - g->m1[a]);
                qc s1 = sy * g->az[j] + root, s2 = sy * g->az[j] - root;
                qr d1 = cabsq(s1 * s1 - p->mu2), d2 = cabsq(s2 * s2 - p->mu2);
                if (d1 < dmin) dmin = d1;
                if (d2 < dmin) dmin = d2;
            }
    }
    const qr rho = dmin / 2;
    const int N = 64;
    for (int i = 1; i <= n; ++i) g->taylor[i] = 0;
    for (int k = 0; k < N; ++k) {
        qc e = mkc(cosq(2 * QPI * k / N), sinq(2 * QPI * k / N));
        qc S = q_contour_gen(g, p->mu2 + rho * e, Q_R, 0, 0, 0, 0);
        qc pw = 1;
        for (int i = 1; i <= n; ++i) {
            pw *= rho * e;
            g->taylor[i] += S / pw / N;
        }
    }
}

int orcq_eval_points_sets(const orcq_problem *p, long n, const double *x_re, const double *x_im,
                          const int *info, double *out)
{
    qgen g;
    memset(&g, 0, sizeof(g));
    g.p = p;
    if (p->radial_split || p->taylor_order < -1 || p->taylor_order > 8) return -1;
    g.dim = p->dimension == 0 ? 4 : p->dimension;
    if (g.dim < 2 || g.dim > 4) return -1;
    if (p->n1 == 0) {
        g.n1 = g.n2 = 1;
        g.m1[0] = mkc(p->m1sq_re, p->m1sq_im);
        g.m2[0] = mkc(p->m2sq_re, p->m2sq_im);
        g.c1[0] = g.c2[0] = 1;
    } else {
        if (p->n1 < 1 || p->n1 > 8 || p->n2 < 1 || p->n2 > 8) return -1;
        g.n1 = p->n1;
        g.n2 = p->n2;
        for (int a = 0; a < g.n1; ++a) {
            g.m1[a] = mkc(p->p1[4 * a], p->p1[4 * a + 1]);
            g.c1[a] = mkc(p->p1[4 * a + 2], p->p1[4 * a + 3]);
        }
        for (int b = 0; b < g.n2; ++b) {
            g.m2[b] = mkc(p->p2[4 * b], p->p2[4 * b + 1]);
            g.c2[b] = mkc(p->p2[4 * b + 2], p->p2[4 * b + 3]);
        }
    }
    g.num_on = p->num_on;
    for (int k = 0; k < 9; ++k) g.num[k] = mkc(p->num[2 * k], p->num[2 * k + 1]);
    int nr = p->n_radial, nc = p->n_arc > 0 ? p->n_arc : 1;
    g.az = malloc(sizeof(qr) * p->n_angular);
    g.azw = malloc(sizeof(qr) * p->n_angular);
    if (q_angular_rule(p->angular_rule, g.dim, p->n_angular, g.az, g.azw) != 0) {
        free(g.az);
        free(g.azw);
        return -1;
    }
    qr *t = malloc(sizeof(qr) * nr), *tw = malloc(sizeof(qr) * nr);
    g.r = malloc(sizeof(qr) * nr);
    g.wr = malloc(sizeof(qr) * nr);
    g.ax = malloc(sizeof(qr) * nc);
    g.aw = malloc(sizeof(qr) * nc);
    q_gauss_legendre(nr, t, tw);
    if (p->n_arc > 0) q_gauss_legendre(p->n_arc, g.ax, g.aw);
    qr T = log1pq((qr)p->lambda2);
    for (int i = 0; i < nr; ++i) {
        qr tt = T * (t[i] + 1) / 2;
        g.r[i] = expm1q(tt);
        g.wr[i] = T / 2 * tw[i] * (1 + g.r[i]);
    }
    g.jmu = q_contour_gen(&g, mkc(p->mu2, 0), Q_R, 0, 0, 0, 0);
    if (p->taylor_order > 0) q_taylor_gen(&g);
#pragma omp parallel for schedule(dynamic, 1)
    for (long k = 0; k < n; ++k) {
        const int *in = info + 7 * k;
        qc x = mkc(x_re[k], in[0] ? -x_im[k] : x_im[k]);
        qc gk;
        if (in[1] == Q_SINGULAR) {
            gk = mkc(NAN, NAN);
        } else {
            qc S = q_contour_gen(&g, x, in[1], in[2], in[3], in[4], in[5]);
            qc sub = 0;
            if (p->taylor_order >= 0) {
                sub = g.jmu;
                qc d = x - p->mu2, pw = 1;
                for (int i = 1; i <= p->taylor_order; ++i) {
                    pw *= d;
                    sub += pw * g.taylor[i];
                }
            }
            gk = (qr)p->scale * (S - sub);
            if (in[0]) gk = conjq(gk);
        }
        out[2 * k] = (double)crealq(gk);
        out[2 * k + 1] = (double)cimagq(gk);
    }
    free(t); free(tw); free(g.r); free(g.wr); free(g.ax); free(g.aw); free(g.az); free(g.azw);
    return 0;
}
