// gfx950 diagnostic kernels: the y-plane scan at fixed x (the paper's Fig. 1)
// and the obstruction map of the original contour (Fig. 2).  Both reuse the
// device building blocks of the scan kernels.
#include "gf_device.h"

namespace gf {
namespace {

// y-plane diagnostic (the paper's Fig. 1): at fixed x, the angular average
// <1/D1>(x, y) over a cell-centred grid of complex y (what = 0), or the
// order-0 subtracted y-integrand y^{(D-2)/2}/(y + m2^2) (<1/D1>(x, y) -
// <1/D1>(mu^2, y)) of eq. 14 (what = 1); with pole sums, <P1> and P2(y) in
// place of <1/D1> and 1/(y + m2^2).  One lane per y point, 8 x 8 tiles, FP64.
__global__ void __launch_bounds__(256) yscan_kernel(ScanArgs a, double xr, double xi, double mu2,
                                                    int what)
{
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= a.n_tiles) return;
    const int lane = threadIdx.x & 63;
    const int ia = (wave % a.tiles_a) * 8 + lane % 8;
    const int ib = (wave / a.tiles_a) * 8 + lane / 8;
    if (ia >= a.n_re || ib >= a.n_im) return;
    const cd y = mk(fma((double)ia + 0.5, a.d_re, a.re_lo), fma((double)ib + 0.5, a.d_im, a.im_lo));
    const cd x = mk(xr, xi);
    const cd m1 = mk(a.m1_re, a.m1_im);
    const cd V2 = cmul(mk(4.0 * xr, 4.0 * xi), y);
    cd A;
    if (!a.poles) {
        A = angular_sum64(a.ang, a.n_a / 2, a.wmid, cadd(cadd(x, y), m1), V2);
    } else {
        A = angular_sum_p<0, true>(a, cadd(cadd(x, y), m1), V2);  // <P1((p-k)^2)>
    }
    if (what == 1) {
        const cd Umu = cadd(mk(mu2 + y.r, y.i), m1), V2mu = cscale(y, 4.0 * mu2);
        const cd Amu = a.poles ? angular_sum_p<0, true>(a, Umu, V2mu)
                               : angular_sum64(a.ang, a.n_a / 2, a.wmid, Umu, V2mu);
        // the radial measure y^{(D-2)/2} (principal sqrt(y) for D = 3)
        const cd f = a.dim == 4 ? y : (a.dim == 3 ? csqrt_principal(y.r, y.i) : mk(1.0, 0.0));
        if (!a.poles)
            A = cdiv(cmul(f, mk(A.r - Amu.r, A.i - Amu.i)), cadd(y, mk(a.m2_re, a.m2_im)));
        else
            A = cmul(cmul(f, mk(A.r - Amu.r, A.i - Amu.i)), prop2(a, y));
    }
    const size_t idx = (size_t)ib * (size_t)a.n_re + (size_t)ia;
    reinterpret_cast<double2 *>(a.out)[idx] = make_double2(A.r, A.i);
}

// Obstruction map (the paper's Fig. 2).  The first propagator
// x + y + m1^2 - 2 sqrt(x) sqrt(y) z vanishes for some z in [-1, 1] exactly when
// zeta(y) = (x + y + m1^2)^2 / (4 x y) is real and lies in [0, 1].  Each straight
// part of a contour is sampled at y = (e^t - 1) dir, the closing arc at
// y = Lambda^2 e^{i psi}; where Im zeta changes sign between two consecutive
// samples, 40 bisection steps on the part's parameter locate the zero of
// Im zeta, and the cut crosses the contour there if Re zeta lies in [0, 1].
struct CutWalk {
    cd x1, x4;  // x + m1^2, 4x
    cd dir;     // direction of a straight part
    double lam2;
    bool arc;   // current part: false = straight, true = arc
    bool hit;
};

__device__ __forceinline__ cd cut_zeta(const CutWalk &w, double u)
{
    cd y;
    if (w.arc) {
        double s, c;
        sincos(u, &s, &c);
        y = mk(w.lam2 * c, w.lam2 * s);
    } else {
        y = cscale(w.dir, expm1(u));
    }
    const cd U = cadd(w.x1, y);
    return cdiv(cmul(U, U), cmul(w.x4, y));
}

// A sign change of Im zeta between the samples at parameters lo and hi (Im
// zeta positive at lo when lo_pos): 40 bisection steps on the part's
// parameter (with zeta itself) locate its zero, and the cut crosses the
// contour there if Re zeta lies in [0, 1].
__device__ void cut_bisect(CutWalk &w, double lo, double hi, bool lo_pos)
{
    for (int it = 0; it < 40; ++it) {
        const double mid = 0.5 * (lo + hi);
        if ((cut_zeta(w, mid).i > 0.0) == lo_pos)
            lo = mid;
        else
            hi = mid;
    }
    const cd zc = cut_zeta(w, 0.5 * (lo + hi));
    if (zc.r >= 0.0 && zc.r <= 1.0) w.hit = true;
}

// The walks below take their samples in chunks of 64 from a fresh anchor,
// eight samples at a time, each group's first sample carried over from the
// one before as one more step of the same recurrence.  The eight signs are
// compared with one branch per group (sign changes are rare: at most one per
// real-segment walk on the bench box); inside it a loop kept rolled bisects
// each change in order, so a walk holds one copy of the bisection.  The
// comparison starts from the sign of the walk's first sample, which has no
// predecessor; only a walk's last group can reach past its last sample
// (k + j >= k_end: those signs are not compared, and nothing reads them after
// it).  Once every point of
// the wave has met the cut, the rest of the part cannot change the map: the
// wave leaves the part at the next chunk (wave-uniform).  Positions, signs,
// brackets and their order are those of a one-sample-at-a-time walk.
constexpr int kGroup = 8;

__device__ __forceinline__ bool group_changes(bool prev, const bool (&p)[kGroup], int k, int k_end)
{
    bool any = p[0] != prev;
#pragma unroll
    for (int j = 1; j < kGroup; ++j) any |= (k + j < k_end) & (p[j] != p[j - 1]);  // no short cut
    return any;
}

__device__ __forceinline__ void group_bisect(CutWalk &w, bool prev, const bool (&p)[kGroup], int k,
                                             int k_end, double step, double base)
{
#pragma unroll 1
    for (int j = 0; j < kGroup && k + j < k_end; ++j) {
        bool a = prev, b = p[0];
#pragma unroll
        for (int i = 1; i < kGroup; ++i)  // p[j - 1], p[j] without indexing registers dynamically
            if (i == j) {
                a = p[i - 1];
                b = p[i];
            }
        if (b != a)
            cut_bisect(w, fma((double)(k + j - 1), step, base), fma((double)(k + j), step, base), a);
    }
}

// Samples along the straight part, y_k = dir e_k, e_k = e^{u_k} - 1, u_k = k h,
// h = T/(n-1), k = 1..n-1: e follows e_{k+1} = e_k c + e_k + c (c = e^h - 1),
// taken afresh from expm1 every 64 samples, so each sample sits within ~64
// ulp of its exact position (far inside the oracle's tie band).  Im zeta has
// the sign of Im(U^2 conj(4 x y)) (|4 x y|^2 > 0), and with 4 x y = (4 x dir) e,
// e > 0, of Im(U^2 conj(4 x dir)) = ur (2 ui c_r - ur c_i) + ui^2 c_i, U = x1 + dir e:
// no division and no product with e.  On the real segment (REAL, dir = 1) ui is
// x1.i itself, as fma(0, e, x1.i) gives for finite e.
template <bool REAL>
__device__ void cut_walk_straight(CutWalk &w, int n, double T)
{
    const double h = T / (n - 1);
    const double c = expm1(h);
    const cd c4 = cmul(w.x4, w.dir);
    const double c4r2 = 2.0 * c4.r;
    auto pos_at = [&](double e) {
        const double ur = fma(w.dir.r, e, w.x1.r);
        const double ui = REAL ? w.x1.i : fma(w.dir.i, e, w.x1.i);
        return fma(ur, fma(ui, c4r2, -(ur * c4.i)), ui * (ui * c4.i)) > 0.0;
    };
    bool prev = pos_at(expm1(h));  // the first sample, k = 1
    for (int k0 = 1; k0 < n; k0 += 64) {
        if (__all(w.hit)) break;
        const int kend = min(k0 + 64, n);
        double e0 = expm1(k0 * h);
        for (int k = k0; k < kend; k += kGroup) {
            double e[kGroup];
            bool p[kGroup];
            e[0] = e0;
#pragma unroll
            for (int j = 1; j < kGroup; ++j) e[j] = fma(e[j - 1], c, e[j - 1] + c);
#pragma unroll
            for (int j = 0; j < kGroup; ++j) p[j] = pos_at(e[j]);
            if (group_changes(prev, p, k, kend)) group_bisect(w, prev, p, k, kend, h, 0.0);
            prev = p[kGroup - 1];
            e0 = fma(e[kGroup - 1], c, e[kGroup - 1] + c);
        }
    }
}

// Samples along an arc from angle phi, psi_k = phi + span k/(n-1), k = 0..n-1
// (span = -phi: back to 0 the short way; the long way: to +-2 pi): the unit
// vector e = e^{i psi} rotates by e^{i span/(n-1)} per sample, taken afresh
// from sincos every 64 samples.  With y = Lambda^2 e and e conj(e) = 1,
//   U^2 conj(4 x y) = Lambda^2 conj(4x) (x1^2 conj(e) + 2 Lambda^2 x1 + Lambda^4 e),
// so Im zeta has the sign of alpha + b_c cos psi + b_s sin psi with
// A = conj(4x) x1^2, B = Lambda^4 conj(4x), alpha = Im(2 Lambda^2 conj(4x) x1),
// b_c = Im A + Im B, b_s = Re B - Re A: two FMAs a sample.  Its terms add up to
// at most ((Lambda^2 + |x1|) / (Lambda^2 - |x1|))^2 times the value's own scale,
// so the rounding stays that of the direct product.
__device__ void cut_walk_arc(CutWalk &w, int n, double phi, double span)
{
    const double dpsi = span / (n - 1);
    double s, c;
    sincos(dpsi, &s, &c);
    const cd rot = mk(c, s);
    const cd cx4 = mk(w.x4.r, -w.x4.i);
    const double l2 = w.lam2, l4 = l2 * l2;
    const cd A = cmul(cx4, cmul(w.x1, w.x1));
    const cd B = cscale(cx4, l4);
    const double alpha = 2.0 * l2 * fma(cx4.r, w.x1.i, cx4.i * w.x1.r);
    const double bc = A.i + B.i, bs = B.r - A.r;
    auto pos_at = [&](cd e) { return fma(bc, e.r, fma(bs, e.i, alpha)) > 0.0; };
    bool prev;
    {
        sincos(fma(0.0, dpsi, phi), &s, &c);  // the first sample, k = 0, as the walk takes it
        prev = pos_at(mk(c, s));
    }
    for (int k0 = 0; k0 < n; k0 += 64) {
        if (__all(w.hit)) break;
        const int kend = min(k0 + 64, n);
        sincos(fma((double)k0, dpsi, phi), &s, &c);
        cd e0 = mk(c, s);
        for (int k = k0; k < kend; k += kGroup) {
            cd e[kGroup];
            bool p[kGroup];
            e[0] = e0;
#pragma unroll
            for (int j = 1; j < kGroup; ++j) e[j] = cmul(e[j - 1], rot);
#pragma unroll
            for (int j = 0; j < kGroup; ++j) p[j] = pos_at(e[j]);
            if (group_changes(prev, p, k, kend)) group_bisect(w, prev, p, k, kend, dpsi, phi);
            prev = p[kGroup - 1];
            e0 = cmul(e[kGroup - 1], rot);
        }
    }
}

__device__ CutWalk cut_walk_begin(const ScanArgs &a, double xr, double xi)
{
    CutWalk w;
    w.x1 = mk(xr + a.m1_re, xi + a.m1_im);
    w.x4 = mk(4.0 * xr, 4.0 * xi);
    w.dir = mk(1.0, 0.0);
    w.lam2 = a.lam2;
    w.arc = false;
    w.hit = false;
    return w;
}

// Real segment: t = T k/(n-1), k = 1..n-1, T = log(1 + Lambda^2).
__device__ bool cut_hits_real_axis(const ScanArgs &a, double xr, double xi, int n, double T)
{
    CutWalk w = cut_walk_begin(a, xr, xi);
    cut_walk_straight<true>(w, n, T);
    return w.hit;
}

// Ray at phi = arg x (same t samples), then the closing arc, which starts
// where the ray ends: psi = phi (1 - k/(n-1)), k = 0..n-1, back to 0 the
// short way, or (the long way round) psi = phi + L k/(n-1),
// L = sign(phi) 2 pi - phi.
__device__ bool cut_hits_ray_arc(const ScanArgs &a, double xr, double xi, int n, double T,
                                 bool long_way)
{
    CutWalk w = cut_walk_begin(a, xr, xi);
    const double phi = atan2(xi, xr);
    double s, c;
    sincos(phi, &s, &c);
    w.dir = mk(c, s);
    cut_walk_straight<false>(w, n, T);
    w.arc = true;
    cut_walk_arc(w, n, phi, long_way ? (phi > 0.0 ? 2.0 * M_PI : -2.0 * M_PI) - phi : -phi);
    return w.hit;
}

// One wave (one 8x8 tile) per workgroup: a tile walks one contour part (class
// R) or three (ray classes), so a four-wave workgroup would hold the slots of
// its finished waves until its slowest one ends.
__global__ void __launch_bounds__(64) obstruction_kernel(ScanArgs a, int n, double T, uint8_t *out)
{
    const int wave = blockIdx.x;
    if (wave >= a.n_tiles) return;
    const int lane = threadIdx.x & 63;
    const int ia = (wave % a.tiles_a) * 8 + lane % 8;
    const int ib = (wave / a.tiles_a) * 8 + lane / 8;
    if (ia >= a.n_re || ib >= a.n_im) return;
    const double xr = fma((double)ia + 0.5, a.d_re, a.re_lo);
    const double xi = fma((double)ib + 0.5, a.d_im, a.im_lo);
    const bool real_hit = cut_hits_real_axis(a, xr, xi, n, T);
    int sign = 0, info = 0;
    int cls = classify(a, xr, xi, &sign, &info);
    double ei = xi;
    int ecls = cls;
    if (cls == kMirror) {  // the scan evaluates the conjugate point, if it has a contour
        ecls = classify(a, xr, -xi, &sign);
        if (ecls == kMirror || ecls == kSingular || ecls == kLong)
            cls = ecls = (info & kInfoRValid) ? kR : kLong;
        else
            ei = -xi;
    }
    int v = real_hit ? 1 : 0;
    if (cls == kSingular) {
        v |= 4;
    } else {
        const bool used_hit = ecls == kR ? (ei == xi ? real_hit : cut_hits_real_axis(a, xr, ei, n, T))
                                         : cut_hits_ray_arc(a, xr, ei, n, T, ecls == kLong);
        if (used_hit) v |= 2;
    }
    out[(size_t)ib * (size_t)a.n_re + (size_t)ia] = (uint8_t)v;
}

}  // namespace

hipError_t launch_yscan(const ScanArgs &a, double xr, double xi, double mu2, int what,
                        hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(yscan_kernel, dim3((a.n_tiles + 3) / 4), dim3(256), 0, s, a, xr, xi, mu2,
                       what);
    return hipGetLastError();
}

hipError_t launch_obstruction(const ScanArgs &a, int n, double T, uint8_t *out, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(obstruction_kernel, dim3(a.n_tiles), dim3(64), 0, s, a, n, T, out);
    return hipGetLastError();
}

}  // namespace gf
