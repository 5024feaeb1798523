// Host side of the gf C ABI: validation, quadrature tables (STEP 4
// preparation, done on the host in FP64 as in the paper's initialisation
// phase), plan objects, the plan cache and kernel launches.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gf.h"
#include "gf_internal.h"

struct gf_plan {
    int device = -1;
    gf_params params{};
    gf_quadrature quad{};
    gf_propagators props{};
    bool has_props = false;
    void *d_mem = nullptr;       // one allocation holding every table
    gf::ScanArgs base{};         // kernel arguments minus the grid and outputs
    double jmu[2 * (GF_MAX_TAYLOR + 1)] = {};  // host copy of K_0..K_n
};

namespace gf {

namespace {
// fixed-size so that recording an error never allocates
thread_local char g_error[512];

bool finite(double v) { return std::isfinite(v); }

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double *pn, double *dpn)
{
    double pkm1 = 1.0, pk = x;  // P_0, P_1
    if (n == 0) {
        *pn = 1.0;
        *dpn = 0.0;
        return;
    }
    for (int k = 1; k < n; ++k) {
        double pkp1 = ((2 * k + 1) * x * pk - k * pkm1) / (k + 1);
        pkm1 = pk;
        pk = pkp1;
    }
    *pn = pk;
    *dpn = n * (pkm1 - x * pk) / (1.0 - x * x);
}

double bad_ray(double re, double im)
{
    // arg(-m^2); a real positive m^2 gives the negative real axis, angle +pi
    return im == 0.0 ? M_PI : std::atan2(-im, -re);
}

int tiles_for(const gf_grid &g, int lanes, int *tiles_a, long long *n_tiles)
{
    int tw, th;
    tile_shape(lanes, &tw, &th);
    long long ta = (g.n_re + tw - 1) / tw;
    long long tb = (g.n_im + th - 1) / th;
    *tiles_a = (int)ta;
    *n_tiles = ta * tb;
    return GF_OK;
}
}  // namespace

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_error, sizeof(g_error), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(GF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

const char *last_error() { return g_error; }

// n-point Gauss-Legendre rule on [-1, 1], ascending nodes.  The positive
// roots are found by Newton's method from Tricomi's asymptotic estimate and
// mirrored.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const int half = (n + 1) / 2;
    for (int i = 1; i <= half; ++i) {
        double th = M_PI * (4.0 * i - 1.0) / (4.0 * n + 2.0);
        double r = std::cos(th) * (1.0 - (n - 1.0) / (8.0 * n * n * n));
        double pn = 0.0, dpn = 1.0;
        // Newton to convergence, then one polishing step
        for (int it = 0, extra = 0; it < 64 && extra < 2; ++it) {
            legendre(n, r, &pn, &dpn);
            double dr = pn / dpn;
            r -= dr;
            if (std::fabs(dr) < 1e-15) ++extra;
        }
        legendre(n, r, &pn, &dpn);
        double wt = 2.0 / ((1.0 - r * r) * dpn * dpn);
        // root i (counted from the top) and its mirror image
        x[n - i] = r;
        w[n - i] = wt;
        x[i - 1] = -r;
        w[i - 1] = wt;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;  // exact centre node
}

void radial_table(int nr, double lambda2, int dim, int split, std::vector<double> &rad)
{
    if (split) {
        // base rule of the four pieces: GL of order n_r/4 on [-1, 1], (xi | w)
        std::vector<double> gx, gw;
        const int m = nr / 4;
        gauss_legendre(m, gx, gw);
        rad.assign(3 * (size_t)nr, 0.0);
        for (int i = 0; i < m; ++i) {
            rad[i] = gx[i];
            rad[m + i] = gw[i];
        }
        return;
    }
    // GL in t = log(1+y) on [0, T], y = e^t - 1, dy = (1 + y) dt; the weight
    // column carries the radial measure y^{(D-2)/2} of D dimensions
    std::vector<double> gx, gw;
    gauss_legendre(nr, gx, gw);
    const double T = std::log1p(lambda2);
    rad.assign(3 * (size_t)nr, 0.0);
    for (int i = 0; i < nr; ++i) {
        double t = 0.5 * T * (gx[i] + 1.0);
        double y = std::expm1(t);
        double dy = 0.5 * T * gw[i] * (1.0 + y);
        rad[i] = y;
        rad[nr + i] = std::sqrt(y);
        rad[2 * nr + i] = dim == 4 ? dy * y : (dim == 3 ? dy * std::sqrt(y) : dy);
    }
}

void angular_tables(int na, int rule, int dim, std::vector<double> &ang,
                    std::vector<float> &ang32, double *wmid)
{
    // Stored folded over the symmetric pairs (z_j, -z_j), j running over the
    // positive nodes as (z_j^2, 2 w_j, 2 w_j z_j^2), in FP64 and rounded to FP32;
    // an odd rule's middle node z = 0 keeps its weight apart.  Weights follow the normalised D-dimensional angular
    // measure (1 - z^2)^{(D-3)/2} dz / N_D, N_D = pi (D = 2), 2 (D = 3),
    // pi/2 (D = 4).  Each rule integrates g(z) against its own weight function
    // omega(z) and is applied to g = f (1 - z^2)^{(D-3)/2} / omega.
    const int npair = na / 2;
    ang.assign(3 * (size_t)std::max(npair, 1), 0.0);
    ang32.assign(3 * (size_t)std::max(npair, 1), 0.0f);
    *wmid = 0.0;
    const double norm = dim == 2 ? M_PI : (dim == 3 ? 2.0 : M_PI_2);
    auto put = [&](int j, double zsq, double w) {
        ang[3 * j] = zsq;
        ang[3 * j + 1] = 2.0 * w;
        ang[3 * j + 2] = 2.0 * w * zsq;
        ang32[3 * j] = (float)zsq;
        ang32[3 * j + 1] = (float)(2.0 * w);
        ang32[3 * j + 2] = (float)(2.0 * w * zsq);
    };
    // s^{D-2} for s = sin(theta) = sqrt(1 - z^2)
    auto sinpow = [&](double s) { return dim == 4 ? s * s : (dim == 3 ? s : 1.0); };
    if (rule == GF_ANG_GC2) {
        // omega = sqrt(1 - z^2): weights (pi/(n+1)) sin^2(theta) sin^{D-4}(theta)
        for (int j = 1; j <= npair; ++j) {
            const double th = j * M_PI / (na + 1);
            const double s = std::sin(th), c = std::cos(th);
            put(j - 1, c * c, M_PI / (na + 1) * sinpow(s) / norm);
        }
        if (na % 2 == 1) *wmid = M_PI / (na + 1) / norm;
    } else if (rule == GF_ANG_GC1) {
        // omega = 1/sqrt(1 - z^2): weights (pi/n) sin^{D-2}(theta)
        for (int j = 1; j <= npair; ++j) {
            const double th = (2 * j - 1) * M_PI / (2.0 * na);
            const double s = std::sin(th), c = std::cos(th);
            put(j - 1, c * c, M_PI / na * sinpow(s) / norm);
        }
        if (na % 2 == 1) *wmid = M_PI / na / norm;
    } else if (rule == GF_ANG_GL) {
        // omega = 1: Gauss-Legendre weights times (1 - z^2)^{(D-3)/2}
        std::vector<double> gx, gw;
        gauss_legendre(na, gx, gw);
        for (int j = 0; j < npair; ++j) {
            const double z = gx[na - 1 - j];  // positive nodes, descending
            const double s2 = 1.0 - z * z;
            const double m = dim == 4 ? std::sqrt(s2) : (dim == 3 ? 1.0 : 1.0 / std::sqrt(s2));
            put(j, z * z, gw[na - 1 - j] * m / norm);
        }
        if (na % 2 == 1) *wmid = gw[na / 2] / norm;
    } else {
        // tanh-sinh: z = tanh(u), u = (pi/2) sinh t, dz = (pi/2) cosh t / cosh^2 u dt,
        // (1 - z^2)^{(D-3)/2} = cosh^{3-D} u; t_k = (k - (n-1)/2) h, h = 2 t_max/(n-1),
        // t_max = 3, 3.5, 4 for D = 4, 3, 2 (the weight at t_max is below 1e-16)
        const double tmax = dim == 4 ? 3.0 : (dim == 3 ? 3.5 : 4.0);
        const double h = 2.0 * tmax / (na - 1);
        for (int j = 0; j < npair; ++j) {
            const double t = (na % 2 == 1) ? (j + 1) * h : (j + 0.5) * h;
            const double u = M_PI_2 * std::sinh(t);
            const double z = std::tanh(u), cu = std::cosh(u);
            const double meas = dim == 4 ? 1.0 / (cu * cu * cu) : (dim == 3 ? 1.0 / (cu * cu) : 1.0 / cu);
            put(j, z * z, h * M_PI_2 * std::cosh(t) * meas / norm);
        }
        if (na % 2 == 1) *wmid = h * M_PI_2 / norm;
    }
}

void arc_table(int nc, std::vector<double> &arc)
{
    std::vector<double> ax, aw;
    if (nc > 0) gauss_legendre(nc, ax, aw);
    arc.assign(2 * (size_t)std::max(nc, 1), 0.0);
    for (int k = 0; k < nc; ++k) {
        arc[k] = ax[k];
        arc[nc + k] = aw[k];
    }
}

namespace {

// A propagator as a multiset of (m^2 re, m^2 im, c re, c im), optionally
// conjugated: the first n entries, sorted (a fixed-size array, no allocation).
struct PoleSet {
    std::array<std::array<double, 4>, GF_MAX_POLES> v{};
    int n = 0;
    bool operator==(const PoleSet &o) const
    {
        return n == o.n && std::equal(v.begin(), v.begin() + n, o.v.begin());
    }
};

PoleSet pole_set(const double *p, int n, bool conj)
{
    PoleSet s;
    s.n = n;
    for (int k = 0; k < n; ++k) {
        const double c = conj ? -1.0 : 1.0;
        // + 0.0 turns -0.0 into +0.0 so that equal values compare equal
        s.v[k] = {p[4 * k] + 0.0, c * p[4 * k + 1] + 0.0, p[4 * k + 2] + 0.0,
                  c * p[4 * k + 3] + 0.0};
    }
    std::sort(s.v.begin(), s.v.begin() + n);
    return s;
}

}  // namespace

void fill_constants(ScanArgs &a, const gf_params &p, const gf_propagators *props,
                    const gf_quadrature &q)
{
    a.n_r = q.n_radial;
    a.n_a = q.n_angular;
    a.n_arc = q.n_arc;
    // poles: from props, or one pole per leg at the masses of p with residue 1
    a.poles = props ? 1 : 0;
    a.n1 = props ? props->n1 : 1;
    a.n2 = props ? props->n2 : 1;
    for (int k = 0; k < GF_MAX_POLES; ++k) {
        for (int c = 0; c < 4; ++c) a.p1[4 * k + c] = a.p2[4 * k + c] = 0.0;
        a.b1[k] = a.b2[k] = 0.0;
    }
    for (int k = 0; k < a.n1; ++k) {
        a.p1[4 * k] = props ? props->m1sq_re[k] : p.m1sq_re;
        a.p1[4 * k + 1] = props ? props->m1sq_im[k] : p.m1sq_im;
        a.p1[4 * k + 2] = props ? props->c1_re[k] : 1.0;
        a.p1[4 * k + 3] = props ? props->c1_im[k] : 0.0;
        a.b1[k] = bad_ray(a.p1[4 * k], a.p1[4 * k + 1]);
    }
    for (int k = 0; k < a.n2; ++k) {
        a.p2[4 * k] = props ? props->m2sq_re[k] : p.m2sq_re;
        a.p2[4 * k + 1] = props ? props->m2sq_im[k] : p.m2sq_im;
        a.p2[4 * k + 2] = props ? props->c2_re[k] : 1.0;
        a.p2[4 * k + 3] = props ? props->c2_im[k] : 0.0;
        a.b2[k] = bad_ray(a.p2[4 * k], a.p2[4 * k + 1]);
    }
    a.num = props && props->numerator ? 1 : 0;
    for (int k = 0; k < 9; ++k) {
        a.nc[2 * k] = a.num ? props->num_re[k] : 0.0;
        a.nc[2 * k + 1] = a.num ? props->num_im[k] : 0.0;
    }
    a.m1_re = a.p1[0];
    a.m1_im = a.p1[1];
    a.m2_re = a.p2[0];
    a.m2_im = a.p2[1];
    a.lam2 = p.lambda2;
    a.lam = std::sqrt(p.lambda2);
    const std::complex<double> sy0 = std::sqrt(std::complex<double>(-a.m2_re, -a.m2_im));
    a.sy0_re = sy0.real();
    a.sy0_im = sy0.imag();
    a.scale = p.scale;
    a.n_taylor = p.taylor_order;
    a.dim = p.dimension == 0 ? 4 : p.dimension;
    a.split = q.radial_split;
    a.T = std::log1p(p.lambda2);
    const std::complex<double> sm1 = std::sqrt(std::complex<double>(-a.m1_re, -a.m1_im));
    a.sm1_re = sm1.real();
    a.sm1_im = sm1.imag();
    a.mu2 = p.mu2;
    // bad rays arg(-m^2) of every pole and the open sector (lo, hi) around the
    // positive real axis that the ray can sweep without crossing one
    a.beta1 = a.b1[0];
    a.beta2 = a.b2[0];
    a.hi = M_PI;
    a.lo = -M_PI;
    a.vstar = INFINITY;
    for (int k = 0; k < a.n1 + a.n2; ++k) {
        const double b = k < a.n1 ? a.b1[k] : a.b2[k - a.n1];
        if (b > 0.0 && b < a.hi) a.hi = b;
        if (b <= 0.0 && b > a.lo) a.lo = b;
    }
    // the real axis is valid below the smallest Re sqrt(m1_a^2)
    for (int k = 0; k < a.n1; ++k)
        a.vstar = std::min(a.vstar,
                           std::real(std::sqrt(std::complex<double>(a.p1[4 * k], a.p1[4 * k + 1]))));
    // G(conj x) = conj G(x) when conjugation maps (P1, P2) onto itself or onto (P2, P1)
    const auto P1 = pole_set(a.p1, a.n1, false), P2 = pole_set(a.p2, a.n2, false);
    const auto C1 = pole_set(a.p1, a.n1, true), C2 = pole_set(a.p2, a.n2, true);
    a.mirror_ok = (C1 == P1 && C2 == P2) || (C1 == P2 && C2 == P1);
    // a numerator keeps the first symmetry only if its coefficients are real;
    // the exchange k -> p - k changes N(k^2, p.k), so it is not used
    if (a.num) {
        bool real = true;
        for (int k = 0; k < 9; ++k) real = real && a.nc[2 * k + 1] == 0.0;
        a.mirror_ok = real && C1 == P1 && C2 == P2;
    }
}

int validate_props(const gf_propagators *props, const gf_quadrature &q)
{
    if (!props) return GF_OK;
    if (props->n1 < 1 || props->n1 > GF_MAX_POLES || props->n2 < 1 || props->n2 > GF_MAX_POLES)
        return fail(GF_EINVAL, "n1, n2 must be in [1, %d], got %d, %d", GF_MAX_POLES, props->n1,
                    props->n2);
    for (int leg = 0; leg < 2; ++leg) {
        const int n = leg ? props->n2 : props->n1;
        const double *mr = leg ? props->m2sq_re : props->m1sq_re;
        const double *mi = leg ? props->m2sq_im : props->m1sq_im;
        const double *cr = leg ? props->c2_re : props->c1_re;
        const double *ci = leg ? props->c2_im : props->c1_im;
        for (int k = 0; k < n; ++k) {
            if (!finite(mr[k]) || !finite(mi[k]) || !finite(cr[k]) || !finite(ci[k]))
                return fail(GF_EINVAL, "pole positions and residues must be finite");
            if (mi[k] == 0.0 && mr[k] <= 0.0)
                return fail(GF_EINVAL, "pole %d of leg %d lies on the non-positive real axis", k,
                            leg + 1);
        }
    }
    if (q.radial_split && (props->n1 > 1 || props->n2 > 1))
        return fail(GF_EUNSUPPORTED, "the split radial rule needs one pole per leg");
    if (props->numerator != 0 && props->numerator != 1)
        return fail(GF_EINVAL, "numerator must be 0 or 1");
    if (props->numerator) {
        for (int k = 0; k < 9; ++k)
            if (!finite(props->num_re[k]) || !finite(props->num_im[k]))
                return fail(GF_EINVAL, "numerator coefficients must be finite");
        if (q.radial_split)
            return fail(GF_EUNSUPPORTED, "the split radial rule takes no numerator");
    }
    return GF_OK;
}

int validate_params(const gf_params *p, const gf_quadrature *q)
{
    if (!p || !q) return fail(GF_EINVAL, "params and quadrature must not be NULL");
    if (q->n_radial < 1 || q->n_radial > 8192)
        return fail(GF_EINVAL, "n_radial must be in [1, 8192], got %d", q->n_radial);
    if (q->n_angular < 1 || q->n_angular > 8192)
        return fail(GF_EINVAL, "n_angular must be in [1, 8192], got %d", q->n_angular);
    // every ray contour closes with the arc |y| = Lambda^2 back to the real
    // axis; without arc nodes its points would silently miss that part
    if (q->n_arc < 1 || q->n_arc > 1024)
        return fail(GF_EINVAL, "n_arc must be in [1, 1024], got %d", q->n_arc);
    if (q->precision != GF_PREC_FP64 && q->precision != GF_PREC_FP32C)
        return fail(GF_EINVAL, "precision must be GF_PREC_FP64 or GF_PREC_FP32C");
    if (q->angular_rule != GF_ANG_GC2 && q->angular_rule != GF_ANG_GC1 &&
        q->angular_rule != GF_ANG_TANH_SINH && q->angular_rule != GF_ANG_GL)
        return fail(GF_EINVAL,
                    "angular_rule must be GF_ANG_GC2, GF_ANG_GC1, GF_ANG_TANH_SINH or GF_ANG_GL");
    if (q->radial_split != 0 && q->radial_split != 1)
        return fail(GF_EINVAL, "radial_split must be 0 or 1");
    if (q->radial_split && q->n_radial % 4 != 0)
        return fail(GF_EINVAL, "radial_split needs n_radial divisible by 4, got %d", q->n_radial);
    if (q->angular_rule == GF_ANG_TANH_SINH && q->n_angular < 3)
        return fail(GF_EINVAL, "the tanh-sinh rule needs n_angular >= 3, got %d", q->n_angular);
    const double vals[] = {p->m1sq_re, p->m1sq_im, p->m2sq_re, p->m2sq_im,
                           p->mu2,     p->lambda2, p->scale};
    for (double v : vals)
        if (!finite(v)) return fail(GF_EINVAL, "parameters must be finite");
    if (!(p->lambda2 > 0.0)) return fail(GF_EINVAL, "lambda2 must be > 0");
    if (!(p->lambda2 <= 1e30)) return fail(GF_EINVAL, "lambda2 must be <= 1e30");
    if (!(p->mu2 >= 0.0)) return fail(GF_EINVAL, "mu2 must be >= 0");
    if (!(p->mu2 < p->lambda2)) return fail(GF_EINVAL, "mu2 must be below lambda2");
    if (p->taylor_order < -1 || p->taylor_order > GF_MAX_TAYLOR)
        return fail(GF_EINVAL, "taylor_order must be in [-1, %d], got %d", GF_MAX_TAYLOR,
                    p->taylor_order);
    if (p->dimension != 0 && (p->dimension < 2 || p->dimension > 4))
        return fail(GF_EINVAL, "dimension must be 2, 3, 4 or 0 (= 4), got %d", p->dimension);
    if (p->m1sq_im == 0.0 && p->m1sq_re <= 0.0)
        return fail(GF_EINVAL, "m1^2 must not lie on the non-positive real axis");
    if (p->m2sq_im == 0.0 && p->m2sq_re <= 0.0)
        return fail(GF_EINVAL, "m2^2 must not lie on the non-positive real axis");
    return GF_OK;
}

int validate_grid(const gf_params &p, const gf_propagators *props, const gf_grid *g)
{
    if (!g) return fail(GF_EINVAL, "grid must not be NULL");
    if (g->n_re < 0 || g->n_im < 0) return fail(GF_EINVAL, "grid sizes must be >= 0");
    if ((long long)g->n_re * (long long)g->n_im > (1LL << 31))
        return fail(GF_EINVAL, "grid has more than 2^31 points");
    const double v[] = {g->re_lo, g->re_hi, g->im_lo, g->im_hi};
    for (double x : v)
        if (!finite(x)) return fail(GF_EINVAL, "grid bounds must be finite");
    if (!(g->re_lo < g->re_hi) || !(g->im_lo < g->im_hi))
        return fail(GF_EINVAL, "grid bounds must satisfy lo < hi");
    // the closing arc |y| = Lambda^2 must clear the angular cut, which reaches
    // out to |y| = (sqrt|x| + sqrt(|x| + |m1^2|))^2 (largest |m1_a^2| of a pole sum)
    double m1abs = std::hypot(p.m1sq_re, p.m1sq_im);
    if (props) {
        m1abs = 0.0;
        for (int k = 0; k < props->n1; ++k)
            m1abs = std::max(m1abs, std::hypot(props->m1sq_re[k], props->m1sq_im[k]));
    }
    const double cr[2] = {g->re_lo, g->re_hi}, ci[2] = {g->im_lo, g->im_hi};
    for (double a : cr)
        for (double b : ci) {
            double ax = std::hypot(a, b);
            double reach = std::sqrt(ax) + std::sqrt(ax + m1abs);
            if (!(reach * reach < p.lambda2))
                return fail(GF_EINVAL,
                            "lambda2 = %g is too small for the grid box: the closing arc "
                            "needs lambda2 > %g",
                            p.lambda2, reach * reach);
        }
    return GF_OK;
}

// Lanes per point, the smallest count that meets three aims:
//  * several rounds of the kernel's resident waves per launch, since the last
//    round drains with SIMDs left one or two waves that cannot hide latency:
//    kRounds rounds (a launch at one lane per point, FP32C also at two, then
//    runs its last rows as a tail of short waves, set_tail);
//  * but no count that leaves a lane fewer than kMinLanePairs angular pairs
//    (its share of a point's contour nodes x pairs per node x (p-k)-leg
//    poles), since every lane repeats its point's setup and the nodes split
//    unevenly; FP32C pairs are cheaper next to that setup, so it keeps twice
//    as many (measured: FP32C on 256^2 9 % faster at 4224 pairs per lane than
//    at 2176; FP64 at 1152 within 1 % of 2240);
//  * and never fewer lanes than fill the device once.
constexpr long long kRounds = 4;
constexpr long long kMinLanePairs[2] = {2048, 4096};  // FP64, FP32C

int auto_lanes(const ScanArgs &base, int precision, const gf_grid &g)
{
    const bool taylor = base.n_taylor > 0, split = base.split != 0, poles = base.poles != 0;
    const long long rounds = kRounds;
    const long long pairs = (long long)((base.n_a + 1) / 2) * (poles ? base.n1 : 1);
    const long long nodes = (long long)base.n_r + base.n_arc + (poles ? base.n2 : 1);
    int fill = 0, want = 0, work = 1;
    for (int l = 1; l <= 64; l *= 2) {
        int ta;
        long long nt;
        tiles_for(g, l, &ta, &nt);
        const long long slots = scan_resident_waves(precision, l, taylor, split, poles);
        if (!fill && nt >= slots) fill = l;
        if (!want && nt >= rounds * slots) want = l;
        if (l > 1 && (nodes + l - 1) / l * pairs >= kMinLanePairs[precision == 1]) work = l;
    }
    if (!fill) fill = 64;
    if (!want) want = 64;
    return std::max(fill, std::min(want, work));
}

// Every tile is one 64-wide block of a one-dimensional launch (the y-plane
// scan packs four to a 256-wide block), and a dispatch counts its work-items
// in 32 bits: a launch holds at most (2^32 - 256) / 64 tiles.  At one lane
// per point the largest grid (2^31 points) takes 2^25 tiles; more lanes per
// point on a grid that large are refused rather than launched.
constexpr long long kMaxLaunchTiles = ((1LL << 32) - 256) / 64;

int set_grid(ScanArgs &a, const gf_grid &g, int lanes)
{
    a.n_re = g.n_re;
    a.n_im = g.n_im;
    a.re_lo = g.re_lo;
    a.im_lo = g.im_lo;
    a.d_re = (g.re_hi - g.re_lo) / (double)g.n_re;
    a.d_im = (g.im_hi - g.im_lo) / (double)g.n_im;
    long long nt;
    tiles_for(g, lanes, &a.tiles_a, &nt);
    if (nt > kMaxLaunchTiles)
        return fail(GF_EINVAL,
                    "grid too large for %d lanes per point: %lld wave tiles, one launch holds "
                    "at most %lld (fewer lanes per point)",
                    lanes, nt, kMaxLaunchTiles);
    a.n_tiles = (int)nt;
    a.tail_tiles = a.tail_row0 = a.tail_tiles_a = 0;
    // The FP64 angular sums multiply eight denominators |U^2 - V^2 s|^2 <=
    // 25 M^4, M = |x| + |y| + |m1^2|, into one reciprocal; below M = 2^30 the
    // product stays under 2^1000 without the rescaling by 2^-e.
    double m1max = 0.0;
    for (int k = 0; k < a.n1; ++k) m1max = std::max(m1max, std::hypot(a.p1[4 * k], a.p1[4 * k + 1]));
    const double xmax = std::max(std::hypot(g.re_lo, g.im_lo), std::hypot(g.re_hi, g.im_hi));
    const double xmax2 = std::max(std::hypot(g.re_lo, g.im_hi), std::hypot(g.re_hi, g.im_lo));
    a.unscaled = std::max(xmax, xmax2) + a.lam2 + m1max < std::ldexp(1.0, 30) ? 1 : 0;
    return GF_OK;
}

// The tail of a large automatically-laned scan: every kernel form (t^n, split
// rule, pole sums and numerators alike) at one lane per point, FP32C also at
// two, with at least kTailMinRounds rounds of its resident waves, gets its last
// rows as tiles of kTailLanes lanes per point: about a quarter round of the
// bulk's work (16 / lanes points per resident wave), with the rows before them
// a whole number of bulk tiles.  Measured (one box per line, ms): FP64 1024^2
// bench grid (256 x 128 + 16 nodes, one lane) no tail 4.37-4.41; 64 rows at 16
// lanes 4.27-4.29, at 4 lanes 4.32-4.34, at 8 lanes 4.33-4.34, at 32 lanes
// 4.34; 32 rows at 16 lanes 4.39-4.40 (too few to cover the drain), 128 rows
// 4.34 (every lane repeats its point's setup).  FP32C 1024^2 at 512 x 256 + 16
// nodes (two lanes): 11.97-11.98 without, 11.65-11.66 with 32-64 rows, 11.69-11.73
// with 96; 2048^2 (one lane): 45.9-46.1 without, 45.1-45.2 with 32-64 rows.
// The other forms on the bench grid and nodes (one box): t^2 4.38 -> 4.25,
// split rule 5.07 -> 4.83; pole sums (a conjugate pair on the (p-k) leg, two
// k-leg poles) at four lanes without a tail 9.33, at one lane with it 8.99,
// and with a numerator 13.25 -> 12.57.
constexpr long long kTailMinRounds = 2;
constexpr long long kTailPoints = 16;  // per resident wave, at one lane per point

void set_tail(ScanArgs &a, const gf_grid &g, int precision, int lanes)
{
    a.tail_tiles = a.tail_row0 = a.tail_tiles_a = 0;
    if (!(lanes == 1 || (precision == 1 && lanes == 2))) return;
    const long long slots =
        scan_resident_waves(precision, lanes, a.n_taylor > 0, a.split != 0, a.poles != 0);
    if (a.n_tiles < kTailMinRounds * slots || g.n_re <= 0) return;
    int twb, thb, twt, tht;
    tile_shape(lanes, &twb, &thb);
    tile_shape(kTailLanes, &twt, &tht);
    const long long points = kTailPoints * slots / lanes;
    const long long rows = std::max(1LL, (points + g.n_re / 2) / g.n_re);
    const long long row0 = (g.n_im - rows) / thb * thb;  // whole bulk tiles before it
    if (row0 < thb) return;
    const long long ta = (g.n_re + twt - 1) / twt;
    const long long tt = ta * ((g.n_im - row0 + tht - 1) / tht);
    const long long bulk = (long long)a.tiles_a * (row0 / thb);
    if (bulk + tt > kMaxLaunchTiles) return;
    a.tail_row0 = (int)row0;
    a.tail_tiles_a = (int)ta;
    a.tail_tiles = (int)tt;
    a.n_tiles = (int)(bulk + tt);
}

int current_device(int *dev)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    return GF_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace gf

namespace {

std::mutex g_cache_mu;
std::map<std::string, gf_plan_t *> g_cache;

std::string cache_key(const gf_params *p, const gf_quadrature *q, int dev)
{
    std::string k(reinterpret_cast<const char *>(p), sizeof(*p));
    k.append(reinterpret_cast<const char *>(q), sizeof(*q));
    k.append(reinterpret_cast<const char *>(&dev), sizeof(dev));
    return k;
}

}  // namespace

using gf::fail;
using gf::hip_fail;

extern "C" {

const char *gf_last_error(void) { return gf::last_error(); }

const char *gf_version(void) { return "gf 0.2 (gfx950)"; }

int gf_plan(const gf_params *params, const gf_quadrature *quad, gf_plan_t **out)
{
    return gf_plan_ex(params, nullptr, quad, out);
}

int gf_plan_ex(const gf_params *params, const gf_propagators *props, const gf_quadrature *quad,
               gf_plan_t **out)
{
    if (!out) return fail(GF_EINVAL, "out must not be NULL");
    *out = nullptr;
    int rc = gf::validate_params(params, quad);
    if (rc != GF_OK) return rc;
    if ((rc = gf::validate_props(props, *quad)) != GF_OK) return rc;
    int dev;
    if ((rc = gf::current_device(&dev)) != GF_OK) return rc;

    std::vector<double> rad, ang, arc;
    std::vector<float> ang32;
    double wmid = 0.0;
    const int dim = params->dimension == 0 ? 4 : params->dimension;
    gf::radial_table(quad->n_radial, params->lambda2, dim, quad->radial_split, rad);
    gf::angular_tables(quad->n_angular, quad->angular_rule, dim, ang, ang32, &wmid);
    gf::arc_table(quad->n_arc, arc);

    const size_t off_rad = 0;
    const size_t off_ang = off_rad + gf::align256(rad.size() * sizeof(double));
    const size_t off_arc = off_ang + gf::align256(ang.size() * sizeof(double));
    const size_t off_jmu = off_arc + gf::align256(arc.size() * sizeof(double));
    const size_t off_a32 = off_jmu + 256;
    const size_t total = off_a32 + gf::align256(ang32.size() * sizeof(float));

    gf_plan_t *plan = new (std::nothrow) gf_plan_t();
    if (!plan) return fail(GF_ENOMEM, "host allocation failed");
    plan->device = dev;
    plan->params = *params;
    plan->quad = *quad;
    hipError_t e = hipMalloc(&plan->d_mem, total);
    if (e != hipSuccess) {
        delete plan;
        return fail(GF_ENOMEM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
    }
    char *base = static_cast<char *>(plan->d_mem);
    struct Up {
        size_t off;
        const void *src;
        size_t bytes;
    } ups[] = {{off_rad, rad.data(), rad.size() * sizeof(double)},
               {off_ang, ang.data(), ang.size() * sizeof(double)},
               {off_arc, arc.data(), arc.size() * sizeof(double)},
               {off_a32, ang32.data(), ang32.size() * sizeof(float)}};
    for (const Up &u : ups) {
        e = hipMemcpy(base + u.off, u.src, u.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            gf_free(plan);
            return hip_fail(e, "hipMemcpy (tables)");
        }
    }

    if (props) {
        plan->props = *props;
        plan->has_props = true;
    }
    gf::ScanArgs &a = plan->base;
    gf::fill_constants(a, *params, props, *quad);
    a.rad = reinterpret_cast<const double *>(base + off_rad);
    a.ang = reinterpret_cast<const double *>(base + off_ang);
    a.arc = reinterpret_cast<const double *>(base + off_arc);
    a.ang32 = reinterpret_cast<const float *>(base + off_a32);
    a.wmid = wmid;

    // Taylor coefficients of the subtraction at mu^2 (FP64, real axis), once per plan
    double *d_jmu = reinterpret_cast<double *>(base + off_jmu);
    a.jmu = d_jmu;
    hipStream_t s;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        gf_free(plan);
        return hip_fail(e, "hipStreamCreate");
    }
    e = gf::launch_jmu(a, params->mu2, d_jmu, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(plan->jmu, d_jmu,
                           2 * sizeof(double) * (std::max(params->taylor_order, 0) + 1),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (e != hipSuccess) {
        gf_free(plan);
        return hip_fail(e, "subtraction-term kernel");
    }
    *out = plan;
    return GF_OK;
}

void gf_free(gf_plan_t *plan)
{
    if (!plan) return;
    if (plan->d_mem) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != plan->device) (void)hipSetDevice(plan->device);
        (void)hipFree(plan->d_mem);
        if (cur != plan->device && cur >= 0) (void)hipSetDevice(cur);
    }
    delete plan;
}

int gf_plan_jmu(const gf_plan_t *plan, double *re, double *im)
{
    if (!plan || !re || !im) return fail(GF_EINVAL, "NULL argument");
    *re = plan->jmu[0];
    *im = plan->jmu[1];
    return GF_OK;
}

int gf_plan_taylor(const gf_plan_t *plan, double *coeffs)
{
    if (!plan || !coeffs) return fail(GF_EINVAL, "NULL argument");
    for (int i = 0; i < 2 * (std::max(plan->params.taylor_order, 0) + 1); ++i)
        coeffs[i] = plan->jmu[i];
    return GF_OK;
}

int gf_plan_auto_lanes(const gf_plan_t *plan, const gf_grid *grid)
{
    if (!plan || !grid) return fail(GF_EINVAL, "NULL argument");
    return gf::auto_lanes(plan->base, plan->quad.precision, *grid);
}

int gf_scan_plan_ex(const gf_plan_t *plan, const gf_grid *grid, void *out, int8_t *cls_out,
                    int lanes_per_point, void *stream)
{
    if (!plan) return fail(GF_EINVAL, "plan must not be NULL");
    int rc = gf::validate_grid(plan->params, plan->has_props ? &plan->props : nullptr, grid);
    if (rc != GF_OK) return rc;
    if ((long long)grid->n_re * grid->n_im == 0) return GF_OK;
    if (!out) return fail(GF_EINVAL, "out must not be NULL");
    int lanes = lanes_per_point;
    if (lanes == 0) lanes = gf::auto_lanes(plan->base, plan->quad.precision, *grid);
    if (lanes < 1 || lanes > 64 || (lanes & (lanes - 1)) != 0)
        return fail(GF_EINVAL, "lanes_per_point must be 0 or a power of two <= 64, got %d",
                    lanes_per_point);
    int dev;
    if ((rc = gf::current_device(&dev)) != GF_OK) return rc;
    if (dev != plan->device)
        return fail(GF_EINVAL, "plan was built on device %d, current device is %d", plan->device,
                    dev);
    gf::ScanArgs a = plan->base;
    if ((rc = gf::set_grid(a, *grid, lanes)) != GF_OK) return rc;
    if (lanes_per_point == 0) gf::set_tail(a, *grid, plan->quad.precision, lanes);
    a.out = static_cast<double *>(out);
    a.cls = cls_out;
    hipError_t e = gf::launch_scan(a, plan->quad.precision, lanes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "scan kernel launch");
    return GF_OK;
}

int gf_scan_plan(const gf_plan_t *plan, const gf_grid *grid, void *out, int8_t *cls_out,
                 void *stream)
{
    return gf_scan_plan_ex(plan, grid, out, cls_out, 0, stream);
}

int gf_yscan_plan(const gf_plan_t *plan, double x_re, double x_im, const gf_grid *ygrid, int what,
                  void *out, void *stream)
{
    if (!plan) return fail(GF_EINVAL, "plan must not be NULL");
    if (what != GF_YSCAN_ANGULAR && what != GF_YSCAN_INTEGRAND)
        return fail(GF_EINVAL, "what must be GF_YSCAN_ANGULAR or GF_YSCAN_INTEGRAND");
    if (!std::isfinite(x_re) || !std::isfinite(x_im)) return fail(GF_EINVAL, "x must be finite");
    if (!ygrid) return fail(GF_EINVAL, "grid must not be NULL");
    if (ygrid->n_re < 0 || ygrid->n_im < 0 ||
        (long long)ygrid->n_re * (long long)ygrid->n_im > (1LL << 31))
        return fail(GF_EINVAL, "grid sizes must be >= 0 with at most 2^31 points");
    const double v[] = {ygrid->re_lo, ygrid->re_hi, ygrid->im_lo, ygrid->im_hi};
    for (double x : v)
        if (!std::isfinite(x)) return fail(GF_EINVAL, "grid bounds must be finite");
    if (!(ygrid->re_lo < ygrid->re_hi) || !(ygrid->im_lo < ygrid->im_hi))
        return fail(GF_EINVAL, "grid bounds must satisfy lo < hi");
    if ((long long)ygrid->n_re * ygrid->n_im == 0) return GF_OK;
    if (!out) return fail(GF_EINVAL, "out must not be NULL");
    int dev, rc;
    if ((rc = gf::current_device(&dev)) != GF_OK) return rc;
    if (dev != plan->device)
        return fail(GF_EINVAL, "plan was built on device %d, current device is %d", plan->device,
                    dev);
    gf::ScanArgs a = plan->base;
    if ((rc = gf::set_grid(a, *ygrid, 1)) != GF_OK) return rc;
    a.out = static_cast<double *>(out);
    a.cls = nullptr;
    hipError_t e = gf::launch_yscan(a, x_re, x_im, plan->params.mu2, what,
                                    static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "y-plane kernel launch");
    return GF_OK;
}

int gf_cut_curve(const gf_params *params, double x_re, double x_im, int n, double *out)
{
    // eq. 25: the first propagator x + y + m1^2 - 2 sqrt(x) sqrt(y) cos t vanishes
    // at sqrt(y) = sqrt(x) cos t +- sqrt(x cos^2 t - x - m1^2), t in [0, pi]
    if (!params || !out || n < 2) return fail(GF_EINVAL, "need params, out and n >= 2");
    const std::complex<double> x(x_re, x_im), m1(params->m1sq_re, params->m1sq_im);
    const std::complex<double> sx = std::sqrt(x);
    for (int k = 0; k < n; ++k) {
        const double t = M_PI * k / (n - 1);
        const double c = std::cos(t);
        const std::complex<double> root = std::sqrt(x * (c * c - 1.0) - m1);
        const std::complex<double> p = sx * c + root, m = sx * c - root;
        const std::complex<double> yp = p * p, ym = m * m;
        out[4 * k] = yp.real();
        out[4 * k + 1] = yp.imag();
        out[4 * k + 2] = ym.real();
        out[4 * k + 3] = ym.imag();
    }
    return GF_OK;
}

int gf_obstruction_map(const gf_params *params, const gf_grid *grid, int n_samples, uint8_t *out,
                       void *stream)
{
    const gf_quadrature q1 = {1, 1, 1, GF_PREC_FP64, GF_ANG_GC2, 0};  // the map needs no nodes
    int rc = gf::validate_params(params, &q1);
    if (rc != GF_OK) return rc;
    if ((rc = gf::validate_grid(*params, nullptr, grid)) != GF_OK) return rc;
    if (n_samples < 2 || n_samples > (1 << 20))
        return fail(GF_EINVAL, "n_samples must be in [2, 2^20], got %d", n_samples);
    if ((long long)grid->n_re * grid->n_im == 0) return GF_OK;
    if (!out) return fail(GF_EINVAL, "out must not be NULL");
    gf::ScanArgs a{};
    gf::fill_constants(a, *params, nullptr, q1);
    if ((rc = gf::set_grid(a, *grid, 1)) != GF_OK) return rc;
    hipError_t e = gf::launch_obstruction(a, n_samples, std::log1p(params->lambda2), out,
                                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "obstruction-map kernel launch");
    return GF_OK;
}

int gf_scan(const gf_params *params, const gf_grid *grid, const gf_quadrature *quad, void *out,
            void *stream)
{
    int rc = gf::validate_params(params, quad);
    if (rc != GF_OK) return rc;
    int dev;
    if ((rc = gf::current_device(&dev)) != GF_OK) return rc;
    const std::string key = cache_key(params, quad, dev);
    gf_plan_t *plan = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            plan = it->second;
        } else {
            rc = gf_plan(params, quad, &plan);
            if (rc != GF_OK) return rc;
            g_cache[key] = plan;
        }
    }
    return gf_scan_plan(plan, grid, out, nullptr, stream);
}

void gf_cache_clear(void)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (auto &kv : g_cache) gf_free(kv.second);
    g_cache.clear();
}

}  // extern "C"
