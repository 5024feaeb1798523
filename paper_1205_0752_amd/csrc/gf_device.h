// Device-side building blocks shared by the gfx950 kernels: complex FP64
// arithmetic, the hardware reciprocal with one Newton step, reads through the
// constant address space, the contour-class rule, per-point set-up and
// per-node coefficients, and the folded angular sums in FP64 and FP32C.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "gf_internal.h"

namespace gf {
namespace {

struct cd {
    double r, i;
};

__device__ __forceinline__ cd mk(double r, double i)
{
    cd z;
    z.r = r;
    z.i = i;
    return z;
}
__device__ __forceinline__ cd cadd(cd a, cd b) { return mk(a.r + b.r, a.i + b.i); }
__device__ __forceinline__ cd cmul(cd a, cd b)
{
    return mk(a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r);
}
__device__ __forceinline__ cd cscale(cd a, double s) { return mk(a.r * s, a.i * s); }
__device__ __forceinline__ double rcp64(double q)
{
    // hardware reciprocal estimate (24 bits on gfx950) + one Newton-Raphson step
    double r = __builtin_amdgcn_rcp(q);
    return fma(fma(-q, r, 1.0), r, r);
}
// a / b = a conj(b) / |b|^2 with the refined reciprocal
__device__ __forceinline__ cd cdiv(cd a, cd b)
{
    double inv = rcp64(b.r * b.r + b.i * b.i);
    return mk((a.r * b.r + a.i * b.i) * inv, (a.i * b.r - a.r * b.i) * inv);
}

// Plan tables and argument tables are read-only while a kernel runs.  Reading
// them through the constant address space tells the compiler so: wave-uniform
// reads then become scalar loads into SGPR operands even in the serving
// kernel, whose stores of earlier work items would otherwise count as
// possible clobbers.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *ro(const T *p)
{
    return (const __attribute__((address_space(4))) T *)(uintptr_t)p;
}

// principal square root; follows the sign of a zero imaginary part
__device__ cd csqrt_principal(double a, double b)
{
    if (a == 0.0 && b == 0.0) return mk(0.0, b);
    double r = hypot(a, b);
    if (a >= 0.0) {
        double t = sqrt(0.5 * (r + a));
        return mk(t, b / (2.0 * t));
    }
    double t = sqrt(0.5 * (r - a));
    return mk(fabs(b) / (2.0 * t), copysign(t, b));
}

__device__ __forceinline__ double angle_between(double a, double b)
{
    double d = fabs(a - b);
    return d > M_PI ? 2.0 * M_PI - d : d;
}

// Contour class of x (STEP 3).  Rotating the ray from angle 0 to phi = arg x
// is free inside (lo, hi); sweeping across the k-leg pole rays arg(-m2_b^2)
// adds their residues (sign of phi); across a ray arg(-m1_a^2) the conjugate
// point is used instead where the propagators allow it.  Otherwise (kLong)
// every (p-k)-leg pole whose bad ray the rotation would sweep has its term
// continued the other way round the origin, through the other half plane:
// that rotation, by 2 pi - |phi|, sweeps none of its own bad ray and ends on
// the same ray at angle phi; its closing arc runs back the long way and it
// takes the residues of the k-leg poles it sweeps, with the opposite sign.
// In D = 3 the measure sqrt(y) is continued along each rotation: the long
// one reaches the ray, its arc and its residues at angles shifted by -+ 2 pi,
// where sqrt(y) has the opposite sign (its cut lies in the short sector,
// which the long rotation does not sweep).  Points on a bad ray itself are
// kSingular.  The real
// axis is preferred where it is valid (|Im sqrt x| < v*) and either
// comfortably inside (v < kRNear v*), closer to its own edge than the ray is
// to a bad ray, or the alternative is the long way round.
//
// *info packs the contour's pole sets (kInfo* below): the k-leg residues of
// the short rotation's terms (YRES; a single pole flags bit 0), those of the
// long rotation's terms, the (p-k)-leg poles of the long rotation, and
// whether the real axis is valid at x.  For kMirror it holds the kLong sets
// of x, the contour to fall back on when the conjugate point has none.
constexpr int kInfoResLong = 8;    // bits 8-15: k-leg residues of the long rotation
constexpr int kInfoGrpLong = 16;   // bits 16-23: (p-k)-leg poles of the long rotation
constexpr int kInfoRValid = 1 << 24;

template <bool POLES = false, class Args>
__device__ int classify(const Args &a, double xr, double xi, int *res_sign, int *info = nullptr)
{
    cd sx = csqrt_principal(xr, xi);
    double v = fabs(sx.i);
    double phi = atan2(xi, xr);
    int rot;
    int mask = 0, lng = 0;  // residues of the short rotation; the kLong sets
    *res_sign = 0;
    double delta;
    if (!POLES) {
        delta = fmin(angle_between(phi, a.beta1), angle_between(phi, a.beta2));
        if (phi > a.lo && phi < a.hi) {
            rot = kY;
        } else {
            bool past1, past2;
            if (phi > 0.0) {
                past1 = a.beta1 > 0.0 && a.beta1 < phi;
                past2 = a.beta2 > 0.0 && a.beta2 < phi;
            } else {
                past1 = a.beta1 <= 0.0 && a.beta1 > phi;
                past2 = a.beta2 <= 0.0 && a.beta2 > phi;
            }
            bool on_bad = angle_between(phi, a.beta1) == 0.0 || angle_between(phi, a.beta2) == 0.0;
            // the long rotation of the single (p-k)-leg pole sweeps the k-leg
            // ray exactly when the short one does not
            lng = (1 << kInfoGrpLong) | (past2 ? 0 : 1 << kInfoResLong);
            if (on_bad) {
                rot = kSingular;
            } else if (past2 && !past1) {
                rot = kYRes;
                mask = 1;
            } else if (past1 && !past2 && a.mirror_ok) {
                rot = kMirror;
            } else {
                rot = kLong;
            }
        }
    } else {
        // swept means: on the way from angle 0 to phi
        auto swept = [phi](double b) {
            return phi > 0.0 ? (b > 0.0 && b < phi) : (b <= 0.0 && b > phi);
        };
        bool past1 = false, on_bad = false;
        delta = M_PI;
        for (int k = 0; k < a.n1; ++k) {
            if (swept(a.b1[k])) {
                past1 = true;
                lng |= 1 << (kInfoGrpLong + k);
            }
            on_bad = on_bad || angle_between(phi, a.b1[k]) == 0.0;
            delta = fmin(delta, angle_between(phi, a.b1[k]));
        }
        for (int k = 0; k < a.n2; ++k) {
            if (swept(a.b2[k]))
                mask |= 1 << k;
            else
                lng |= 1 << (kInfoResLong + k);
            on_bad = on_bad || angle_between(phi, a.b2[k]) == 0.0;
            delta = fmin(delta, angle_between(phi, a.b2[k]));
        }
        if (phi > a.lo && phi < a.hi) {
            rot = kY;
            mask = 0;
        } else if (on_bad) {
            rot = kSingular;
        } else if (mask != 0 && !past1) {
            rot = kYRes;
        } else if (past1 && mask == 0 && a.mirror_ok) {
            rot = kMirror;
        } else {
            rot = kLong;
        }
    }
    const bool r_valid = v < a.vstar;
    if (r_valid) {
        if (v < kRNear * a.vstar || 1.0 - v / a.vstar >= kRSlope * delta || rot == kSingular ||
            rot == kLong) {
            if (info) *info = kInfoRValid;
            return kR;
        }
    }
    if (rot == kYRes || rot == kLong || rot == kMirror) *res_sign = phi > 0.0 ? 1 : -1;
    if (info)
        *info = rot == kYRes ? mask
                : (rot == kLong || rot == kMirror) ? (mask | lng | (r_valid ? kInfoRValid : 0))
                                                   : 0;
    return rot;
}

// Per-point quantities hoisted out of the node loop.  V^2 = 4 x y for every
// node whatever the branches of sqrt(x) sqrt(y), and the angular sum depends
// on V only through V^2 (symmetric rule), so no square root of y is needed.
struct PointCtx {
    cd x1;    // x + m1^2
    cd dir;   // e^{i phi} (ray) or 1 (real axis)
    cd dirD;  // e^{i phi D/2}: the phase of dy y^{(D-2)/2} along the ray
    double phi;
    int nodes;  // contour nodes of this point
    int res_sign;
    int info;      // the contour's pole sets, packed as by classify
    double tb[5];  // split radial rule: piece boundaries in t = log(1+r)
};

// (p-k)-leg poles whose terms rotate the short way, given the packed sets
// (all of them for kY and kYRes; a single pole counts as pole 0).
template <bool POLES, class Args>
__device__ __forceinline__ int short_group(const Args &a, int info)
{
    const int all = POLES ? (1 << a.n1) - 1 : 1;
    return all & ~(info >> kInfoGrpLong & 0xFF);
}

// Split radial rule: the straight part [0, T] in t = log(1+r) is cut at the
// radii where the integrand is nearly singular -- |(sqrt x +- sqrt(-m1^2))^2|,
// the moduli of the angular cut's end points (eq. 25 at z = +-1), and |m2^2|,
// the k-leg pole's -- then, while fewer than three cuts exist, at the middle
// of the longest piece; each of the four pieces carries n_r/4 GL nodes.  Cuts
// within 1e-9 T of one another count once, and a piece only replaces the
// longest one found so far if longer by 1e-12 T, so near-ties are decided the
// same way whatever the rounding.
template <class Args>
__device__ void split_boundaries(const Args &a, double xr, double xi, double *b)
{
    const cd sx = csqrt_principal(xr, xi);
    const cd sp = cadd(sx, mk(a.sm1_re, a.sm1_im)), sn = mk(sx.r - a.sm1_re, sx.i - a.sm1_im);
    const double cand[3] = {sp.r * sp.r + sp.i * sp.i, sn.r * sn.r + sn.i * sn.i,
                            sqrt(a.m2_re * a.m2_re + a.m2_im * a.m2_im)};
    const double T = a.T, tol = 1e-9 * T;
    int nb = 2;
    b[0] = 0.0;
    b[1] = T;
    for (int k = 0; k < 3; ++k) {
        if (!(cand[k] > 0.0 && cand[k] < a.lam2)) continue;
        const double t = log1p(cand[k]);
        bool dup = false;
        for (int q = 0; q < nb; ++q) dup = dup || fabs(b[q] - t) <= tol;
        if (!dup) {
            int j = nb++;
            while (j > 0 && b[j - 1] > t) {  // insertion keeps b sorted
                b[j] = b[j - 1];
                --j;
            }
            b[j] = t;
        }
    }
    while (nb < 5) {
        int wide = 0;
        for (int i = 1; i < nb - 1; ++i)
            if (b[i + 1] - b[i] > b[wide + 1] - b[wide] + 1e-12 * T) wide = i;
        for (int j = nb; j > wide + 1; --j) b[j] = b[j - 1];
        b[wide + 1] = 0.5 * (b[wide] + b[wide + 2]);
        ++nb;
    }
}

template <bool SPLIT = false, bool POLES = false, class Args>
__device__ PointCtx point_setup(const Args &a, double xr, double xi, int cls, int res_sign,
                                int info = 0)
{
    PointCtx P;
    P.x1 = mk(xr + a.m1_re, xi + a.m1_im);
    P.res_sign = res_sign;
    P.info = info;
    if (SPLIT) {
        double b[5];
        split_boundaries(a, xr, xi, b);
#pragma unroll
        for (int i = 0; i < 5; ++i) P.tb[i] = b[i];
    }
    if (cls == kY || cls == kYRes || cls == kLong) {
        double phi = atan2(xi, xr);
        double s, c;
        sincos(phi, &s, &c);
        P.dir = mk(c, s);
        if (a.dim == 4) {
            P.dirD = cmul(P.dir, P.dir);
        } else if (a.dim == 3) {
            sincos(0.5 * phi, &s, &c);
            P.dirD = cmul(P.dir, mk(c, s));
        } else {
            P.dirD = P.dir;
        }
        P.phi = phi;
        // the closing arcs (short, long or both) and the residue nodes of
        // each rotation; the short rotation's residues need its terms
        const int grp_long = info >> kInfoGrpLong & 0xFF, grp_short = short_group<POLES>(a, info);
        if (!grp_short) P.info &= ~0xFF;
        // D = 3: the long rotation meets the ray at angle phi -+ 2 pi, where
        // sqrt(y) = -e^{i phi/2} sqrt(r); when every term rotates the long
        // way that is the ray's measure (mixed groups: ray_neg per term)
        if (a.dim == 3 && cls == kLong && !grp_short) P.dirD = mk(-P.dirD.r, -P.dirD.i);
        const int arcs = grp_long && grp_short ? 2 : 1;
        P.nodes = a.n_r + arcs * a.n_arc + __popc(P.info & 0xFF) +
                  __popc(P.info >> kInfoResLong & 0xFF);
    } else {
        P.dir = mk(1.0, 0.0);
        P.dirD = P.dir;
        P.phi = 0.0;
        P.nodes = cls == kR ? a.n_r : 0;
    }
    return P;
}

// Coefficients of contour node k -- radial (ray or real axis), closing arc,
// or residue of the k-leg pole: U = x + y + m1^2, V^2 = 4 x y and the node's
// weight omega = dy y^{(D-2)/2} / (y + m2^2) (the D-dimensional radial measure;
// y for D = 4), or +-2 pi i y0^{(D-2)/2} at the residue.  Along the ray
// y = e^{i phi} r, dy y^{(D-2)/2} = e^{i phi D/2} dr r^{(D-2)/2}; the table holds
// the real weight dr r^{(D-2)/2}.
// Radial node k of the straight part: r and the real weight dr r^{(D-2)/2}.
// Unsplit, from the plan's table; split, from the base GL rule of order n_r/4
// (table: xi[m], w[m]) mapped onto piece k / m of the point's boundaries.
template <bool SPLIT, class Args>
__device__ __forceinline__ void radial_node(const Args &a, const PointCtx &P, int k, double &r,
                                            double &g)
{
    const auto *rad = ro(a.rad);
    if (!SPLIT) {
        r = rad[k];
        g = rad[2 * a.n_r + k];
        return;
    }
    const int m = a.n_r >> 2;
    const int s = k / m, i = k - s * m;
    double lo = P.tb[0], hi = P.tb[1];
    for (int q = 1; q <= 3; ++q)  // select piece s without indexing registers dynamically
        if (s == q) {
            lo = P.tb[q];
            hi = P.tb[q + 1];
        }
    const double h = 0.5 * (hi - lo);
    r = expm1(fma(h, rad[i] + 1.0, lo));
    const double dr = h * rad[m + i] * (1.0 + r);
    g = a.dim == 4 ? dr * r : (a.dim == 3 ? dr * sqrt(r) : dr);
}

// The k-leg pole sum P2(y) = sum_b c2_b / (y + m2_b^2).
template <class Args>
__device__ __forceinline__ cd prop2(const Args &a, cd y)
{
    cd p = mk(0.0, 0.0);
    for (int b = 0; b < a.n2; ++b) {
        const auto *q = &a.p2[4 * b];
        p = cadd(p, cdiv(mk(q[2], q[3]), cadd(y, mk(q[0], q[1]))));
    }
    return p;
}

// Node k < n_r: the straight part (real axis or ray).
template <bool SPLIT, bool POLES, class Args>
__device__ __forceinline__ void radial_coeffs(const Args &a, const PointCtx &P, int k, cd &U,
                                              cd &V2, cd &w)
{
    // 4 x, recovered from x + m1^2 (recomputing it per node keeps fewer
    // registers live across the node loop than carrying it)
    const cd x4 = mk(4.0 * (P.x1.r - a.m1_re), 4.0 * (P.x1.i - a.m1_im));
    double r, g;
    radial_node<SPLIT>(a, P, k, r, g);
    const cd y = cscale(P.dir, r);                         // y = e^{i phi} r
    U = cadd(P.x1, y);
    V2 = cmul(x4, y);                                      // 4 x y
    if (POLES)
        w = cmul(cscale(P.dirD, g), prop2(a, y));
    else
        w = cdiv(cscale(P.dirD, g), cadd(y, mk(a.m2_re, a.m2_im)));
}

// Node k >= n_r: the closing arcs |y| = Lambda^2, then the residue nodes
// (returns true for a residue node); *set flags the (p-k)-leg poles whose
// terms the node belongs to.  The short
// arc runs from phi back to 0 through the half plane of x, the long arc
// (kLong) from phi on to +-2 pi through the other one; the short rotation's
// residues carry the sign of phi, the long rotation's the opposite sign.
template <bool POLES, class Args>
__device__ __forceinline__ bool outer_coeffs(const Args &a, const PointCtx &P, int k, cd &U,
                                             cd &V2, cd &w, int &set)
{
    const cd m2 = mk(a.m2_re, a.m2_im);
    const cd x4 = mk(4.0 * (P.x1.r - a.m1_re), 4.0 * (P.x1.i - a.m1_im));
    const int grp_long = P.info >> kInfoGrpLong & 0xFF, grp_short = short_group<POLES>(a, P.info);
    const int arcs = grp_long && grp_short ? 2 : 1;
    const int q = k - a.n_r;
    if (q < arcs * a.n_arc) {
        const bool second = q >= a.n_arc;
        const int i = second ? q - a.n_arc : q;
        const bool lng = second || !grp_short;
        set = lng ? grp_long : grp_short;
        const auto *arc = ro(a.arc);
        const double xi = arc[i];
        const double wa = arc[a.n_arc + i];
        double psi, h;
        if (!lng) {
            psi = 0.5 * P.phi * (1.0 - xi);                // from phi back to 0
            h = -0.5 * P.phi * wa;
        } else {
            const double L = (P.phi > 0.0 ? 2.0 * M_PI : -2.0 * M_PI) - P.phi;
            psi = fma(0.5 * L, 1.0 + xi, P.phi);           // from phi on to +-2 pi
            h = 0.5 * L * wa;
        }
        double s, c;
        sincos(psi, &s, &c);
        const cd y = mk(a.lam2 * c, a.lam2 * s);
        U = cadd(P.x1, y);
        V2 = cmul(x4, y);
        const cd dy = mk(-y.i * h, y.r * h);              // dy = i y psi'(xi) dxi
        cd f = y;                                         // y^{(D-2)/2}
        if (a.dim == 3) {
            // the long arc's angle runs from phi -+ 2 pi back to 0 along the
            // contour: sqrt(y) = e^{i (psi -+ 2 pi)/2} Lambda = -e^{i psi/2} Lambda
            sincos(0.5 * psi, &s, &c);
            const double lam = lng ? -a.lam : a.lam;
            f = mk(lam * c, lam * s);
        } else if (a.dim == 2) {
            f = mk(1.0, 0.0);
        }
        if (POLES)
            w = cmul(cmul(dy, f), prop2(a, y));
        else
            w = cdiv(cmul(dy, f), cadd(y, m2));
        return false;
    }
    // residue node j: the short rotation's flagged k-leg poles, then the long one's
    int j = q - arcs * a.n_arc;
    const int rs = P.info & 0xFF, rl = P.info >> kInfoResLong & 0xFF;
    const int ns = __popc(rs);
    int m = rs, sg = P.res_sign;
    bool long_rot = false;
    set = grp_short;
    if (j >= ns) {
        j -= ns;
        m = rl;
        sg = -sg;
        set = grp_long;
        long_rot = true;
    }
    const double f = sg * 2.0 * M_PI;                     // +-2 pi i Res
    // D = 3: sqrt(y0) continued along the rotation that sweeps y0.  The long
    // rotation turns clockwise for phi > 0: its angle at y0 is arg(y0) - 2 pi
    // past the negative real axis and -pi on it; counter-clockwise for
    // phi < 0: arg(y0) + 2 pi past it and +pi on it
    auto long_sqrt = [&](cd y0) {
        double t = atan2(y0.i, y0.r);
        if (y0.i == 0.0 && y0.r < 0.0) t = P.phi > 0.0 ? -M_PI : M_PI;
        else if (P.phi > 0.0 && t > P.phi) t -= 2.0 * M_PI;
        else if (P.phi < 0.0 && t < P.phi) t += 2.0 * M_PI;
        double s, c;
        sincos(0.5 * t, &s, &c);
        const double m = sqrt(hypot(y0.r, y0.i));
        return mk(m * c, m * s);
    };
    if (!POLES) {
        const cd y0 = mk(-a.m2_re, -a.m2_im);
        U = cadd(P.x1, y0);
        V2 = cmul(x4, y0);
        cd fy = a.dim == 4 ? y0 : (a.dim == 3 ? mk(a.sy0_re, a.sy0_im) : mk(1.0, 0.0));
        if (a.dim == 3 && long_rot) fy = long_sqrt(y0);
        w = mk(-fy.i * f, fy.r * f);
    } else {
        for (int it = 0; it < j; ++it) m &= m - 1;  // drop the j lowest flags
        const int b = m ? __ffs(m) - 1 : 0;
        const auto *q2 = &a.p2[4 * b];
        const cd y0 = mk(-q2[0], -q2[1]);
        U = cadd(P.x1, y0);
        V2 = cmul(x4, y0);
        cd sq = a.dim == 4 ? y0 : (a.dim == 3 ? csqrt_principal(y0.r, y0.i) : mk(1.0, 0.0));
        if (a.dim == 3 && long_rot) sq = long_sqrt(y0);
        const cd fy = cmul(mk(q2[2], q2[3]), sq);
        w = mk(-fy.i * f, fy.r * f);                      // +-2 pi i c2_b y0^{(D-2)/2}
    }
    return true;
}

// The numerator's polynomials in y = k^2 at a node (pole sums with a.num):
// N_j(y) = sum_i n_ij y^i for the powers j = 0, 1, 2 of p.k; y = U - (x + m1^2).
template <class Args>
__device__ __forceinline__ void numerator_at(const Args &a, cd U, cd x1, cd *N)
{
    const cd y = mk(U.r - x1.r, U.i - x1.i);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const auto *c = &a.nc[2 * j];  // n_ij at 2 (3i + j)
        cd v = mk(c[12], c[13]);       // i = 2
        v = cadd(cmul(v, y), mk(c[6], c[7]));
        N[j] = cadd(cmul(v, y), mk(c[0], c[1]));
    }
}

template <bool SPLIT = false, bool POLES = false, class Args>
__device__ __forceinline__ void node_coeffs(const Args &a, const PointCtx &P, int k, cd &U,
                                            cd &V2, cd &w)
{
    int set;
    if (k < a.n_r)
        radial_coeffs<SPLIT, POLES>(a, P, k, U, V2, w);
    else
        outer_coeffs<POLES>(a, P, k, U, V2, w, set);
}

// Angular sum A = sum_j w_j / (U - V z_j) over the GC-II rule.  The rule is
// symmetric (z_{n+1-j} = -z_j, equal weights), so each node pair is folded:
//   w/(U - V z) + w/(U + V z) = 2 w U / (U^2 - V^2 z^2),
// one complex denominator per two integrand evaluations; the middle node of an
// odd rule (z = 0) adds w/U.  U^2 and V^2 are scaled by an exact power of two
// 2^-e (e = exponent of their largest component), which changes no rounding
// and keeps every |D|^2 of order 1 or below, so several denominators can share
// one reciprocal (1/q0 = q1 q2 ... / (q0 q1 q2 ...)) without overflow.
__device__ __forceinline__ int scale_exponent(cd U2, cd V2)
{
    const double big = fmax(fmax(fabs(U2.r), fabs(U2.i)), fmax(fabs(V2.r), fabs(V2.i)));
    int e = 0;
    frexp(big, &e);
    return e;
}

// Near the angular cut: the folded denominators U^2 - V^2 s, s = z^2 in (0, 1),
// come within dist(U^2, [0, V^2]) of zero.  The ratio (|U^2| + |V^2|) / dist
// bounds how much rounding in U^2, V^2 or s is amplified in a denominator:
// by the ratio itself for D computed directly, by its square for |D|^2 taken
// from the quadratic in s.  A node is "near" when the ratio exceeds
// kCutSensitivity; the FP32 sums take the quadratic only below
// kQuad32Sensitivity, the square root of kCutSensitivity, so their worst
// case stays that of the direct form at the near threshold.  The tests
// depend on the node alone, so results stay reproducible.
constexpr double kCutSensitivity = 16.0;
constexpr double kQuad32Sensitivity = 4.0;

// 2 (|U^2|^2 + |V^2|^2) |V^2|^2 and dist^2 |V^2|^2 (no division), on U^2 = (ar, ai),
// V^2 = (br, bi): the squared ratio, up to a factor of at most 2, is lhs / d2vv.
// With dot = Re(U^2 conj V^2) and t = dot clamped to [0, |V^2|^2] (the nearest
// point of the segment [0, V^2] to U^2 is V^2 t / |V^2|^2),
//   dist^2 |V^2|^2 = |U^2|^2 |V^2|^2 - 2 dot t + t^2,
// which is |U^2|^2 |V^2|^2 before the segment, |U^2 - V^2|^2 |V^2|^2 beyond it and
// Im(U^2 conj V^2)^2 beside it, without a branch.  Beside the segment it is a
// difference whose rounding, ~eps |U^2|^2 |V^2|^2, is far below the threshold's
// lhs / kCutSensitivity^2: a near node stays near.
__device__ __forceinline__ void cut_measure(double ar, double ai, double br, double bi,
                                            double &lhs, double &d2vv)
{
    const double vv = br * br + bi * bi;
    const double uu = ar * ar + ai * ai;
    const double dot = ar * br + ai * bi;
    const double t = fmin(fmax(dot, 0.0), vv);
    d2vv = fma(t, fma(-2.0, dot, t), uu * vv);
    lhs = 2.0 * (uu + vv) * vv;  // 0 when V^2 = 0: the sum is exactly 1/U, never near
}

__device__ __forceinline__ bool near_cut_sq(double ar, double ai, double br, double bi)
{
    double lhs, d2vv;
    cut_measure(ar, ai, br, bi, lhs, d2vv);
    return lhs > kCutSensitivity * kCutSensitivity * d2vv;
}

// Sums T0 = sum 2w_j / q_j and T1 = sum 2w_j z_j^2 / q_j of the folded pairs,
// q_j = |U^2 - V^2 s_j|^2 (s_j = z_j^2), on the scaled U^2 = (ur, ui), V^2 = (vr, vi).
// QUAD: q_j from the real quadratic c0 - c1 s + c2 s^2 (c0 = |U^2|^2,
// c1 = 2 Re(U^2 conj V^2), c2 = |V^2|^2), two FMAs; its rounding, relative
// ~eps (|U^2| + |V^2| s)^2 / q_j, is taken only away from the cut (below
// kCutSensitivity^2 eps).  Otherwise q_j = |D_j|^2 from D_j itself.  Eight (then
// four) denominators share one reciprocal of their product, refined by one
// Newton step; each 1/q_k is unfolded by multiplying out the others (the
// scaling keeps every q_k, and so the product, in range).
template <bool QUAD, bool NUM = false>
__device__ __forceinline__ void pair_sums64(const double *table, int npair, double ur, double ui,
                                            double vr, double vi, double &T0, double &T1,
                                            double *T2 = nullptr)
{
    // NUM: also T2 = sum 2w_j z_j^4 / q_j, for numerators in p.k
    const auto *tab = ro(table);
    const double c0 = fma(ur, ur, ui * ui), c2 = fma(vr, vr, vi * vi);
    const double c1 = -2.0 * fma(ur, vr, ui * vi);
    auto qof = [&](double s) {
        if (QUAD) return fma(fma(c2, s, c1), s, c0);
        const double dr = fma(-vr, s, ur), di = fma(-vi, s, ui);
        return fma(dr, dr, di * di);
    };
    double s0 = 0.0, s1 = 0.0, z0 = 0.0, z1 = 0.0;  // T0 and T1, two partial sums each
    double y0 = 0.0, y1 = 0.0;                      // T2 (NUM)
    int p = 0;
    for (; p + 8 <= npair; p += 8) {
        const auto *t = tab + 3 * p;
        double q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) q[k] = qof(t[3 * k]);
        const double p01 = q[0] * q[1], p23 = q[2] * q[3], p45 = q[4] * q[5], p67 = q[6] * q[7];
        const double p03 = p01 * p23, p47 = p45 * p67;
        const double inv = rcp64(p03 * p47);
        const double i03 = p47 * inv, i47 = p03 * inv;
        const double i01 = p23 * i03, i23 = p01 * i03, i45 = p67 * i47, i67 = p45 * i47;
        const double r[8] = {q[1] * i01, q[0] * i01, q[3] * i23, q[2] * i23,
                             q[5] * i45, q[4] * i45, q[7] * i67, q[6] * i67};
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
            s0 = fma(t[3 * k + 1], r[k], s0);
            z0 = fma(t[3 * k + 2], r[k], z0);
            s1 = fma(t[3 * k + 4], r[k + 1], s1);
            z1 = fma(t[3 * k + 5], r[k + 1], z1);
            if (NUM) {
                y0 = fma(t[3 * k + 2] * t[3 * k], r[k], y0);
                y1 = fma(t[3 * k + 5] * t[3 * k + 3], r[k + 1], y1);
            }
        }
    }
    for (; p + 4 <= npair; p += 4) {
        const auto *t = tab + 3 * p;
        const double q0 = qof(t[0]), q1 = qof(t[3]), q2 = qof(t[6]), q3 = qof(t[9]);
        const double p01 = q0 * q1, p23 = q2 * q3;
        const double inv = rcp64(p01 * p23);
        const double i01 = p23 * inv, i23 = p01 * inv;
        const double r0 = q1 * i01, r1 = q0 * i01, r2 = q3 * i23, r3 = q2 * i23;  // 1 / q_k
        s0 = fma(t[1], r0, s0);
        z0 = fma(t[2], r0, z0);
        s1 = fma(t[4], r1, s1);
        z1 = fma(t[5], r1, z1);
        s0 = fma(t[7], r2, s0);
        z0 = fma(t[8], r2, z0);
        s1 = fma(t[10], r3, s1);
        z1 = fma(t[11], r3, z1);
        if (NUM) {
            y0 = fma(t[2] * t[0], r0, y0);
            y1 = fma(t[5] * t[3], r1, y1);
            y0 = fma(t[8] * t[6], r2, y0);
            y1 = fma(t[11] * t[9], r3, y1);
        }
    }
    for (; p < npair; ++p) {
        const auto *t = tab + 3 * p;
        const double r0 = rcp64(qof(t[0]));
        s0 = fma(t[1], r0, s0);
        z0 = fma(t[2], r0, z0);
        if (NUM) y0 = fma(t[2] * t[0], r0, y0);
    }
    T0 = s0 + s1;
    T1 = z0 + z1;
    if (NUM) *T2 = y0 + y1;
}

template <int SCALE = 1>
__device__ __forceinline__ cd angular_sum64(const double *table, int npair, double wmid, cd U,
                                            cd V2in, bool scale_rt = true)
{
    // SCALE 1: always rescale; 0: never; -1: as scale_rt says
    const bool scale = SCALE == 1 || (SCALE == -1 && scale_rt);
    // sum_j 2w_j / D_j = sum_j 2w_j conj(D_j) / |D_j|^2 with D_j = U^2 - V^2 z_j^2,
    // and conj(D_j) = conj(U^2) - conj(V^2) z_j^2, so the pair sum is
    // conj(U^2) T0 - conj(V^2) T1 with the real sums T0 = sum 2w_j / |D_j|^2 and
    // T1 = sum 2w_j z_j^2 / |D_j|^2; the table holds (z_j^2, 2w_j, 2w_j z_j^2).
    // scale = false (wave-uniform): the magnitudes are known to be small
    // enough that the products of eight denominators stay in range unscaled.
    const cd U2in = cmul(U, U);
    int e = 0;
    double u2r = U2in.r, u2i = U2in.i, v2r = V2in.r, v2i = V2in.i;
    if (scale) {
        e = scale_exponent(U2in, V2in);
        u2r = ldexp(u2r, -e);
        u2i = ldexp(u2i, -e);
        v2r = ldexp(v2r, -e);
        v2i = ldexp(v2i, -e);
    }
    double T0, T1;
    if (near_cut_sq(u2r, u2i, v2r, v2i))
        pair_sums64<false>(table, npair, u2r, u2i, v2r, v2i, T0, T1);
    else
        pair_sums64<true>(table, npair, u2r, u2i, v2r, v2i, T0, T1);
    // the pair sum (scaled by 2^e): conj(U^2) T0 - conj(V^2) T1, then times U
    double sr = fma(u2r, T0, -(v2r * T1)), si = fma(u2i, T0, -(v2i * T1));
    if (scale) {
        sr = ldexp(sr, -e);
        si = ldexp(si, -e);
    }
    cd A = cmul(U, mk(sr, -si));
    if (wmid != 0.0) A = cadd(A, cdiv(mk(wmid, 0.0), U));
    return A;
}

// Numerators in p.k: with p.k = (V/2) z, each folded pair gives
//   (V/2) z [w/(U - Vz) - w/(U + Vz)]      = (V^2/2)   2w s / D(s),
//   (V/2)^2 z^2 [w/(U - Vz) + w/(U + Vz)]  = (V^2 U/4) 2w s / D(s),
// s = z^2, D(s) = U^2 - V^2 s (the middle node z = 0 adds nothing), and
// sum 2w s / D = conj(U^2) T1 - conj(V^2) T2 with T2 = sum 2w s^2 / |D|^2: one
// more real sum of positive terms, so no cancellation is introduced.
// Returns A = <1/(U - Vz)> and S1 = sum_pairs 2w s / D(s).
template <int SCALE = -1>
__device__ __forceinline__ void angular_sums64_num(const double *table, int npair, double wmid,
                                                   cd U, cd V2in, bool scale_rt, cd &A, cd &S1)
{
    const bool scale = SCALE == 1 || (SCALE == -1 && scale_rt);
    const cd U2in = cmul(U, U);
    int e = 0;
    double u2r = U2in.r, u2i = U2in.i, v2r = V2in.r, v2i = V2in.i;
    if (scale) {
        e = scale_exponent(U2in, V2in);
        u2r = ldexp(u2r, -e);
        u2i = ldexp(u2i, -e);
        v2r = ldexp(v2r, -e);
        v2i = ldexp(v2i, -e);
    }
    double T0, T1, T2;
    if (near_cut_sq(u2r, u2i, v2r, v2i))
        pair_sums64<false, true>(table, npair, u2r, u2i, v2r, v2i, T0, T1, &T2);
    else
        pair_sums64<true, true>(table, npair, u2r, u2i, v2r, v2i, T0, T1, &T2);
    double sr = fma(u2r, T0, -(v2r * T1)), si = fma(u2i, T0, -(v2i * T1));
    double tr = fma(u2r, T1, -(v2r * T2)), ti = fma(u2i, T1, -(v2i * T2));
    if (scale) {
        sr = ldexp(sr, -e);
        si = ldexp(si, -e);
        tr = ldexp(tr, -e);
        ti = ldexp(ti, -e);
    }
    A = cmul(U, mk(sr, -si));
    if (wmid != 0.0) A = cadd(A, cdiv(mk(wmid, 0.0), U));
    S1 = mk(tr, -ti);
}

// FP32 angular sum with blocked accumulation, on U^2 and V^2 formed in FP64
// and scaled by the exact power of two 2^-e (e = exponent of their largest
// component), so every FP32 denominator is O(1) and the shared-reciprocal
// product q0 q1 stays in range.  As in the FP64 sum, the pair sum is
// conj(U^2) T0 - conj(V^2) T1 with the real sums T0 = sum 2w_j/|D_j|^2 and
// T1 = sum 2w_j z_j^2/|D_j|^2 (positive terms); each is summed in FP32 blocks
// of kBlock pairs whose block sums are added in FP64 (for sums of positive
// terms this bounds the error by the block's, like a two-sum accumulator of
// the block sums, at two instructions per block and sum).  QUAD: q_j from the
// quadratic c0 - c1 s + c2 s^2 with its coefficients formed in FP64 and
// rounded once, so the denominators are those of the FP64 U^2, V^2, which the
// final combination (in FP64) then takes.  Otherwise q_j = |D_j|^2 from D_j
// in FP32, and the combination takes the FP32 values of U^2, V^2 (exact in
// FP64) that D_j was formed from.  The table holds (z_j^2, 2w_j, 2w_j z_j^2) in FP32.
constexpr int kBlock = 16;

template <bool QUAD, bool NUM = false>
__device__ __forceinline__ cd angular_sum32c(const float *table, int npair, double wmid, cd U,
                                             double u2r, double u2i, double v2r, double v2i, int e,
                                             cd *S1 = nullptr)
{
    const auto *tab = ro(table);
    const float fu2r = (float)u2r, fu2i = (float)u2i, fv2r = (float)v2r, fv2i = (float)v2i;
    const float c0 = (float)fma(u2r, u2r, u2i * u2i), c2 = (float)fma(v2r, v2r, v2i * v2i);
    const float c1 = (float)(-2.0 * fma(u2r, v2r, u2i * v2i));
    auto qof = [&](float s) {
        if (QUAD) return fmaf(fmaf(c2, s, c1), s, c0);
        const float dr = fmaf(-fv2r, s, fu2r), di = fmaf(-fv2i, s, fu2i);
        return fmaf(dr, dr, di * di);
    };
    double T0 = 0.0, T1 = 0.0, T2 = 0.0;  // FP32 block sums added in FP64
    int p = 0;
    while (p < npair) {
        const int pe = min(p + kBlock, npair);
        float b0 = 0.0f, d0 = 0.0f, b1 = 0.0f, d1 = 0.0f, f0 = 0.0f, f1 = 0.0f;
        const auto *t = tab + 3 * p;
        // four pairs per step, two shared reciprocals (of q0 q1 and q2 q3)
        for (; p + 4 <= pe; p += 4, t += 12) {
            const float q0 = qof(t[0]), q1 = qof(t[3]), q2 = qof(t[6]), q3 = qof(t[9]);
            const float inv01 = __builtin_amdgcn_rcpf(q0 * q1);
            const float inv23 = __builtin_amdgcn_rcpf(q2 * q3);
            const float r0 = q1 * inv01, r1 = q0 * inv01;  // 1 / q_k
            const float r2 = q3 * inv23, r3 = q2 * inv23;
            b0 = fmaf(t[1], r0, b0);
            d0 = fmaf(t[2], r0, d0);
            b1 = fmaf(t[4], r1, b1);
            d1 = fmaf(t[5], r1, d1);
            b0 = fmaf(t[7], r2, b0);
            d0 = fmaf(t[8], r2, d0);
            b1 = fmaf(t[10], r3, b1);
            d1 = fmaf(t[11], r3, d1);
            if (NUM) {
                f0 = fmaf(t[2] * t[0], r0, f0);
                f1 = fmaf(t[5] * t[3], r1, f1);
                f0 = fmaf(t[8] * t[6], r2, f0);
                f1 = fmaf(t[11] * t[9], r3, f1);
            }
        }
        for (; p < pe; ++p, t += 3) {
            const float r0 = __builtin_amdgcn_rcpf(qof(t[0]));
            b0 = fmaf(t[1], r0, b0);
            d0 = fmaf(t[2], r0, d0);
            if (NUM) f0 = fmaf(t[2] * t[0], r0, f0);
        }
        T0 += (double)(b0 + b1);
        T1 += (double)(d0 + d1);
        if (NUM) T2 += (double)(f0 + f1);
    }
    const double ar = QUAD ? u2r : (double)fu2r, ai = QUAD ? u2i : (double)fu2i;
    const double br = QUAD ? v2r : (double)fv2r, bi = QUAD ? v2i : (double)fv2i;
    const double sr = fma(ar, T0, -(br * T1)), si = fma(ai, T0, -(bi * T1));
    cd A = cmul(U, mk(ldexp(sr, -e), -ldexp(si, -e)));
    if (wmid != 0.0) A = cadd(A, cdiv(mk(wmid, 0.0), U));
    if (NUM) {
        const double tr = fma(ar, T1, -(br * T2)), ti = fma(ai, T1, -(bi * T2));
        *S1 = mk(ldexp(tr, -e), -ldexp(ti, -e));
    }
    return A;
}

// FP32C: by the node's ratio (|U^2| + |V^2|) / dist, the FP64 sum near the cut
// (rounding U^2, V^2 and s to FP32 perturbs a denominator by ~eps32 times the
// ratio), the FP32 sum with direct denominators below that, and with the
// quadratic below kQuad32Sensitivity.
template <class Args>
__device__ __forceinline__ cd angular_sum_fp32c(const Args &a, cd U, cd V2)
{
    const cd U2 = cmul(U, U);
    const int e = scale_exponent(U2, V2);
    const double u2r = ldexp(U2.r, -e), u2i = ldexp(U2.i, -e);
    const double v2r = ldexp(V2.r, -e), v2i = ldexp(V2.i, -e);
    double lhs, d2vv;
    cut_measure(u2r, u2i, v2r, v2i, lhs, d2vv);
    if (lhs > kCutSensitivity * kCutSensitivity * d2vv)
        return angular_sum64<-1>(a.ang, a.n_a / 2, a.wmid, U, V2, !a.unscaled);
    if (lhs > kQuad32Sensitivity * kQuad32Sensitivity * d2vv)
        return angular_sum32c<false>(a.ang32, a.n_a / 2, a.wmid, U, u2r, u2i, v2r, v2i, e);
    return angular_sum32c<true>(a.ang32, a.n_a / 2, a.wmid, U, u2r, u2i, v2r, v2i, e);
}

// SCALE (FP64 only): -1 rescales as the launch's `unscaled` flag says; 0 or 1
// fix it at compile time for a caller that has branched on the flag.
// The numerator form of the angular sums: A = <1/(U - Vz)> and
// S1 = sum_pairs 2w s / D(s), in FP64 or (as angular_sum_fp32c chooses by the
// node's distance from the cut) FP32C.
template <int PREC, class Args>
__device__ __forceinline__ void angular_sums_num(const Args &a, cd U, cd V2, cd &A, cd &S1)
{
    if (PREC == 0) {
        angular_sums64_num<-1>(a.ang, a.n_a / 2, a.wmid, U, V2, !a.unscaled, A, S1);
        return;
    }
    const cd U2 = cmul(U, U);
    const int e = scale_exponent(U2, V2);
    const double u2r = ldexp(U2.r, -e), u2i = ldexp(U2.i, -e);
    const double v2r = ldexp(V2.r, -e), v2i = ldexp(V2.i, -e);
    double lhs, d2vv;
    cut_measure(u2r, u2i, v2r, v2i, lhs, d2vv);
    if (lhs > kCutSensitivity * kCutSensitivity * d2vv)
        angular_sums64_num<-1>(a.ang, a.n_a / 2, a.wmid, U, V2, !a.unscaled, A, S1);
    else if (lhs > kQuad32Sensitivity * kQuad32Sensitivity * d2vv)
        A = angular_sum32c<false, true>(a.ang32, a.n_a / 2, a.wmid, U, u2r, u2i, v2r, v2i, e, &S1);
    else
        A = angular_sum32c<true, true>(a.ang32, a.n_a / 2, a.wmid, U, u2r, u2i, v2r, v2i, e, &S1);
}

template <int PREC, int SCALE = -1, class Args>
__device__ __forceinline__ cd angular_sum(const Args &a, cd U, cd V2)
{
    if (PREC == 0) return angular_sum64<SCALE>(a.ang, a.n_a / 2, a.wmid, U, V2, !a.unscaled);
    return angular_sum_fp32c(a, U, V2);
}

// Pole sums: <P1(D1)> = sum_a c1_a <1/(U_a - V z)>, U_a = U + m1_a^2 - m1_0^2
// (U carries pole 0); one folded angular sum per pole of `set`.
// Numerator (pole sums with a.num): N(k^2, p.k) = N0(y) + N1(y) p.k + N2(y) (p.k)^2
// at the node's y (N: the three polynomials' values), so per pole
//   <N / (U_a - Vz)> = N0 A_a + N1 (V^2/2) S1_a + N2 (V^2 U_a/4) S1_a.
// neg flags the poles whose terms enter with the opposite sign (the D = 3
// measure on a ray shared by the short and the long rotation).
template <int PREC, bool POLES, class Args>
__device__ __forceinline__ cd angular_sum_p(const Args &a, cd U, cd V2, int set = ~0,
                                            const cd *N = nullptr, int neg = 0)
{
    if (!POLES) return angular_sum<PREC>(a, U, V2);
    cd A = mk(0.0, 0.0);
    if (N) {
        for (int p = 0; p < a.n1; ++p) {
            if (!(set >> p & 1)) continue;
            const auto *q = &a.p1[4 * p];
            const cd Ua = mk(U.r + (q[0] - a.m1_re), U.i + (q[1] - a.m1_im));
            cd Aa, S1;
            angular_sums_num<PREC>(a, Ua, V2, Aa, S1);
            const cd half_v2 = cscale(V2, 0.5);
            const cd val = cadd(cmul(N[0], Aa),
                                cmul(cadd(N[1], cmul(N[2], cscale(Ua, 0.5))), cmul(half_v2, S1)));
            const double sg = neg >> p & 1 ? -1.0 : 1.0;
            A = cadd(A, cmul(mk(sg * q[2], sg * q[3]), val));
        }
        return A;
    }
    for (int p = 0; p < a.n1; ++p) {
        if (!(set >> p & 1)) continue;
        const auto *q = &a.p1[4 * p];
        const cd Ua = mk(U.r + (q[0] - a.m1_re), U.i + (q[1] - a.m1_im));
        const double sg = neg >> p & 1 ? -1.0 : 1.0;
        A = cadd(A, cmul(mk(sg * q[2], sg * q[3]), angular_sum<PREC>(a, Ua, V2)));
    }
    return A;
}

}  // namespace
}  // namespace gf
