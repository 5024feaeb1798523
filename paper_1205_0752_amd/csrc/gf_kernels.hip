// gfx950 kernels of the complex-plane scan (STEP 4 + STEP 5 fused).
//
// One 64-wide wavefront owns a tile of grid points; each point is handled by
// L lanes (L = 1 for large grids).  Per point, in FP64: the grid coordinate,
// sqrt(x), arg x and the contour class (STEP 3), then per contour node the
// hoisted coefficients (U, V, omega) of
//
//     omega * sum_j w_j / (U - V z_j),   U = x + y + m1^2,  V = 2 sqrt(x) sqrt(y),
//     omega = dy-weight * y / (y + m2^2),
//
// i.e. eq. 11's angular integral of the first propagator times the y-only
// factor of eq. 19.  The angular nodes are wave-uniform, so their table is
// read through the scalar cache into SGPR operands; each lane keeps its point's
// (U, V) in registers.  Partial sums of the L lanes of a point are combined
// with cross-lane shuffles, the real-axis subtraction sum at mu^2 (eq. 14) is
// removed, the result scaled, conjugated for mirror points, and written once.
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
__device__ __forceinline__ cd cdiv(cd a, cd b)
{
    double inv = 1.0 / (b.r * b.r + b.i * b.i);
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
// is free inside (lo, hi); sweeping across the k-leg pole ray arg(-m2^2) adds
// its residue (sign of phi); across the ray arg(-m1^2) the conjugate point is
// used instead.  The real axis is preferred where it is valid (|Im sqrt x| <
// v*) and either comfortably inside (v < kRNear v*) or closer to its own edge
// than the ray is to a bad ray.
template <class Args>
__device__ int classify(const Args &a, double xr, double xi, int *res_sign)
{
    cd sx = csqrt_principal(xr, xi);
    double v = fabs(sx.i);
    double phi = atan2(xi, xr);
    int rot;
    *res_sign = 0;
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
        if (on_bad) {
            rot = kSingular;
        } else if (past2 && !past1) {
            rot = kYRes;
            *res_sign = phi > 0.0 ? 1 : -1;
        } else if (past1 && !past2 && a.mirror_ok) {
            rot = kMirror;
        } else {
            rot = kSingular;
        }
    }
    if (v < a.vstar) {
        double delta = fmin(angle_between(phi, a.beta1), angle_between(phi, a.beta2));
        if (v < kRNear * a.vstar || 1.0 - v / a.vstar >= kRSlope * delta || rot == kSingular) {
            *res_sign = 0;
            return kR;
        }
    }
    return rot;
}

// Per-point quantities hoisted out of the node loop.
struct PointCtx {
    cd x1;       // x + m1^2
    cd sx2dir;   // 2 sqrt(x) e^{i phi/2} (ray) or 2 sqrt(x) (real axis)
    cd sx2;      // 2 sqrt(x)
    cd dir;      // e^{i phi} (ray) or 1 (real axis)
    double phi;
    int nodes;   // contour nodes of this point
    int res_sign;
};

template <class Args>
__device__ PointCtx point_setup(const Args &a, double xr, double xi, int cls, int res_sign)
{
    PointCtx P;
    cd sx = csqrt_principal(xr, xi);
    P.x1 = mk(xr + a.m1_re, xi + a.m1_im);
    P.sx2 = cscale(sx, 2.0);
    P.res_sign = res_sign;
    if (cls == kR) {
        P.dir = mk(1.0, 0.0);
        P.sx2dir = P.sx2;
        P.phi = 0.0;
        P.nodes = a.n_r;
    } else if (cls == kY || cls == kYRes) {
        double phi = atan2(xi, xr);
        double s, c, sh, ch;
        sincos(phi, &s, &c);
        sincos(0.5 * phi, &sh, &ch);
        P.dir = mk(c, s);
        P.sx2dir = cmul(P.sx2, mk(ch, sh));
        P.phi = phi;
        P.nodes = a.n_r + a.n_arc + (cls == kYRes ? 1 : 0);
    } else {
        P.dir = mk(1.0, 0.0);
        P.sx2dir = P.sx2;
        P.phi = 0.0;
        P.nodes = 0;
    }
    return P;
}

// Coefficients of contour node k: radial (ray or real axis), closing arc, or
// residue of the k-leg pole.
template <class Args>
__device__ __forceinline__ void node_coeffs(const Args &a, const PointCtx &P, int k, cd &U,
                                            cd &V, cd &w)
{
    const cd m2 = mk(a.m2_re, a.m2_im);
    if (k < a.n_r) {
        const auto *rad = ro(a.rad);
        double r = rad[k];
        double sr = rad[a.n_r + k];
        double wr = rad[2 * a.n_r + k];
        cd y = cscale(P.dir, r);                      // y = e^{i phi} r
        U = cadd(P.x1, y);
        V = cscale(P.sx2dir, sr);                     // 2 sqrt(x) sqrt(y)
        w = cdiv(cscale(cmul(P.dir, y), wr), cadd(y, m2));  // dy y / (y + m2^2)
    } else if (k < a.n_r + a.n_arc) {
        int q = k - a.n_r;
        const auto *arc = ro(a.arc);
        double xi = arc[q];
        double wa = arc[a.n_arc + q];
        double psi = 0.5 * P.phi * (1.0 - xi);        // from phi back to 0
        double s, c, sh, ch;
        sincos(psi, &s, &c);
        sincos(0.5 * psi, &sh, &ch);
        cd y = mk(a.lam2 * c, a.lam2 * s);
        U = cadd(P.x1, y);
        V = cmul(P.sx2, mk(a.lam * ch, a.lam * sh));
        double h = 0.5 * P.phi * wa;
        cd dy = mk(y.i * h, -y.r * h);                // dy = -i y (phi/2) dxi
        w = cdiv(cmul(dy, y), cadd(y, m2));
    } else {
        cd y0 = mk(-a.m2_re, -a.m2_im);
        U = cadd(P.x1, y0);
        V = cmul(P.sx2, mk(a.sy0_re, a.sy0_im));
        double f = P.res_sign * 2.0 * M_PI;          // +-2 pi i Res
        w = mk(-y0.i * f, y0.r * f);
    }
}

__device__ __forceinline__ double rcp64(double q)
{
    // hardware reciprocal estimate (24 bits on gfx950) + one Newton-Raphson step
    double r = __builtin_amdgcn_rcp(q);
    return fma(fma(-q, r, 1.0), r, r);
}

// Angular sum A = sum_j w_j / (U - V z_j) over the GC-II rule.  The rule is
// symmetric (z_{n+1-j} = -z_j, equal weights), so each node pair is folded:
//   w/(U - V z) + w/(U + V z) = 2 w U / (U^2 - V^2 z^2),
// one complex denominator per two integrand evaluations; the middle node of an
// odd rule (z = 0) adds w/U.  Two denominators share one reciprocal
// (1/q0 = q1/(q0 q1)).  Table: (z^2, 2w) per pair, FP64.
__device__ __forceinline__ cd angular_sum64(const double *table, int npair, double wmid, cd U,
                                            cd V)
{
    const auto *tab = ro(table);
    const cd U2 = cmul(U, U);
    const cd V2 = cmul(V, V);
    double ar0 = 0.0, ai0 = 0.0, ar1 = 0.0, ai1 = 0.0;
    int p = 0;
#pragma unroll 2
    for (; p + 2 <= npair; p += 2) {
        const double zz0 = tab[2 * p], ww0 = tab[2 * p + 1];
        const double zz1 = tab[2 * p + 2], ww1 = tab[2 * p + 3];
        const double dr0 = fma(-V2.r, zz0, U2.r), di0 = fma(-V2.i, zz0, U2.i);
        const double dr1 = fma(-V2.r, zz1, U2.r), di1 = fma(-V2.i, zz1, U2.i);
        const double q0 = fma(dr0, dr0, di0 * di0);
        const double q1 = fma(dr1, dr1, di1 * di1);
        const double inv = rcp64(q0 * q1);
        const double t0 = ww0 * (q1 * inv);
        const double t1 = ww1 * (q0 * inv);
        ar0 = fma(t0, dr0, ar0);
        ai0 = fma(t0, di0, ai0);
        ar1 = fma(t1, dr1, ar1);
        ai1 = fma(t1, di1, ai1);
    }
    if (p < npair) {
        const double zz0 = tab[2 * p], ww0 = tab[2 * p + 1];
        const double dr0 = fma(-V2.r, zz0, U2.r), di0 = fma(-V2.i, zz0, U2.i);
        const double t0 = ww0 * rcp64(fma(dr0, dr0, di0 * di0));
        ar0 = fma(t0, dr0, ar0);
        ai0 = fma(t0, di0, ai0);
    }
    // sum 2w / D = sum 2w conj(D) / |D|^2, then times U
    cd A = cmul(U, mk(ar0 + ar1, -(ai0 + ai1)));
    if (wmid != 0.0) A = cadd(A, cdiv(mk(wmid, 0.0), U));
    return A;
}

// Knuth's two-sum: s + e == a + b exactly (round-to-nearest, no contraction).
__device__ __forceinline__ void two_sum(float &hi, float &lo, float b)
{
    const float s = hi + b;
    const float bb = s - hi;
    const float e = (hi - (s - bb)) + (b - bb);
    hi = s;
    lo += e;
}

// FP32 angular sum with compensated accumulation.  U^2 and V^2 are formed in
// FP64 and scaled by an exact power of two 2^-e (e = exponent of their largest
// component) before rounding to FP32, so every FP32 denominator is O(1) and the
// shared-reciprocal product q0 q1 stays in range.  Terms are summed in FP32
// blocks of kBlock pairs; block sums enter a (hi, lo) two-sum accumulator; the
// node's sum leaves in FP64 as U 2^-e (hi + lo).
constexpr int kBlock = 16;

__device__ __forceinline__ cd angular_sum32c(const float *table, int npair, double wmid, cd U,
                                             cd V)
{
    const auto *tab = ro(table);
    const cd U2 = cmul(U, U);
    const cd V2 = cmul(V, V);
    const double big = fmax(fmax(fabs(U2.r), fabs(U2.i)), fmax(fabs(V2.r), fabs(V2.i)));
    int e = 0;
    frexp(big, &e);
    const float u2r = (float)ldexp(U2.r, -e), u2i = (float)ldexp(U2.i, -e);
    const float v2r = (float)ldexp(V2.r, -e), v2i = (float)ldexp(V2.i, -e);
    float hr = 0.0f, lr = 0.0f, hi = 0.0f, li = 0.0f;
    int p = 0;
    while (p < npair) {
        const int pe = min(p + kBlock, npair);
        float br0 = 0.0f, bi0 = 0.0f, br1 = 0.0f, bi1 = 0.0f;
        for (; p + 2 <= pe; p += 2) {
            const float zz0 = tab[2 * p], ww0 = tab[2 * p + 1];
            const float zz1 = tab[2 * p + 2], ww1 = tab[2 * p + 3];
            const float dr0 = fmaf(-v2r, zz0, u2r), di0 = fmaf(-v2i, zz0, u2i);
            const float dr1 = fmaf(-v2r, zz1, u2r), di1 = fmaf(-v2i, zz1, u2i);
            const float q0 = fmaf(dr0, dr0, di0 * di0);
            const float q1 = fmaf(dr1, dr1, di1 * di1);
            const float inv = __builtin_amdgcn_rcpf(q0 * q1);
            const float t0 = ww0 * (q1 * inv);
            const float t1 = ww1 * (q0 * inv);
            br0 = fmaf(t0, dr0, br0);
            bi0 = fmaf(t0, di0, bi0);
            br1 = fmaf(t1, dr1, br1);
            bi1 = fmaf(t1, di1, bi1);
        }
        if (p < pe) {
            const float zz0 = tab[2 * p], ww0 = tab[2 * p + 1];
            const float dr0 = fmaf(-v2r, zz0, u2r), di0 = fmaf(-v2i, zz0, u2i);
            const float t0 = ww0 * __builtin_amdgcn_rcpf(fmaf(dr0, dr0, di0 * di0));
            br0 = fmaf(t0, dr0, br0);
            bi0 = fmaf(t0, di0, bi0);
            ++p;
        }
        two_sum(hr, lr, br0 + br1);
        two_sum(hi, li, bi0 + bi1);
    }
    const double sr = ldexp((double)hr + (double)lr, -e);
    const double si = ldexp((double)hi + (double)li, -e);
    cd A = cmul(U, mk(sr, -si));
    if (wmid != 0.0) A = cadd(A, cdiv(mk(wmid, 0.0), U));
    return A;
}

template <int PREC, class Args>
__device__ __forceinline__ cd angular_sum(const Args &a, cd U, cd V)
{
    if (PREC == 0) return angular_sum64(a.ang, a.n_a / 2, a.wmid, U, V);
    return angular_sum32c(a.ang32, a.n_a / 2, a.wmid, U, V);
}

// One wave's tile of grid points: STEP 4 (the point) and STEP 5 (eq. 15 on
// the point's contour), shared by the one-grid scan and the serving kernel so a
// point's result does not depend on which launch computes it.
template <int PREC, int L, class Args>
__device__ __forceinline__ void process_tile(const Args &a, int tile, int lane)
{
    constexpr int P = 64 / L;
    constexpr int TW = P < 8 ? P : 8;
    constexpr int TH = P / TW;
    const int p = lane / L;
    const int s = lane % L;
    const int ia = (tile % a.tiles_a) * TW + p % TW;
    const int ib = (tile / a.tiles_a) * TH + p / TW;
    const bool valid = ia < a.n_re && ib < a.n_im;

    double xr = fma((double)ia + 0.5, a.d_re, a.re_lo);
    double xi = fma((double)ib + 0.5, a.d_im, a.im_lo);
    int sign = 0;
    int cls = valid ? classify(a, xr, xi, &sign) : kSingular;
    int ecls = cls;
    if (cls == kMirror) {
        xi = -xi;  // evaluate at conj x, conjugate the result
        ecls = classify(a, xr, xi, &sign);
        if (ecls == kMirror || ecls == kSingular) {
            cls = kSingular;
            ecls = kSingular;
        }
    }
    const PointCtx pc = point_setup(a, xr, xi, ecls, sign);

    double sr = 0.0, si = 0.0;
    for (int k = s; k < pc.nodes; k += L) {
        cd U, V, w;
        node_coeffs(a, pc, k, U, V, w);
        cd A = angular_sum<PREC>(a, U, V);
        cd t = cmul(w, A);
        sr += t.r;
        si += t.i;
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off);
        si += __shfl_xor(si, off);
    }
    if (valid && s == 0) {
        double gr, gi;
        if (cls == kSingular) {
            gr = __builtin_nan("");
            gi = __builtin_nan("");
        } else {
            gr = a.scale * (sr - a.jmu[0]);
            gi = a.scale * (si - a.jmu[1]);
            if (cls == kMirror) gi = -gi;
        }
        const size_t idx = (size_t)ib * (size_t)a.n_re + (size_t)ia;
        reinterpret_cast<double2 *>(a.out)[idx] = make_double2(gr, gi);
        if (a.cls) a.cls[idx] = (int8_t)cls;
    }
}

template <int PREC, int L>
__global__ void __launch_bounds__(256) scan_kernel(ScanArgs a)
{
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= a.n_tiles) return;  // uniform per wave
    process_tile<PREC, L>(a, wave, threadIdx.x & 63);
}

// Serving: a persistent launch over a packed list of (request, tile) items of
// many requests.  Each wave takes the next item from a device counter (one
// lane's atomic, broadcast) until the list is exhausted, so every wave exits.
template <int PREC, int L>
__global__ void __launch_bounds__(256) serve_kernel(const ScanArgs *__restrict__ reqs,
                                                   const WorkItem *__restrict__ items, int n_items,
                                                   unsigned *counter)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned w = 0;
        if (lane == 0) w = atomicAdd(counter, 1u);
        w = __builtin_amdgcn_readlane(w, 0);  // wave-uniform item index
        if (w >= (unsigned)n_items) break;
        const int req = ro(items)[w].req;
        const int tile = ro(items)[w].tile;
        process_tile<PREC, L>(ro(reqs)[req], tile, lane);
    }
}

// Subtraction sum at the real point mu^2 on the real axis, by one wavefront.
template <class Args>
__device__ __forceinline__ void jmu_wave(const Args &a, double mu2, double *dst, int lane)
{
    const PointCtx pc = point_setup(a, mu2, 0.0, kR, 0);
    double sr = 0.0, si = 0.0;
    for (int k = lane; k < pc.nodes; k += 64) {
        cd U, V, w;
        node_coeffs(a, pc, k, U, V, w);
        cd A = angular_sum<0>(a, U, V);
        cd t = cmul(w, A);
        sr += t.r;
        si += t.i;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off);
        si += __shfl_xor(si, off);
    }
    if (lane == 0) {
        dst[0] = sr;
        dst[1] = si;
    }
}

__global__ void __launch_bounds__(64) jmu_kernel(ScanArgs a, double mu2, double *dst)
{
    jmu_wave(a, mu2, dst, threadIdx.x);
}

// One wave per request: J_mu of request i into its args' jmu slot.
__global__ void __launch_bounds__(64) jmu_batch_kernel(const ScanArgs *__restrict__ reqs,
                                                       const int *__restrict__ slots,
                                                       const double *__restrict__ mu2, int n)
{
    const int i = blockIdx.x;
    if (i >= n) return;
    const auto &a = ro(reqs)[__builtin_amdgcn_readfirstlane(slots[i])];
    jmu_wave(a, mu2[i], const_cast<double *>(a.jmu), threadIdx.x);
}

template <int L>
hipError_t launch_l(const ScanArgs &a, int precision, hipStream_t s)
{
    const int blocks = (a.n_tiles + 3) / 4;
    if (precision == 0) {
        hipLaunchKernelGGL((scan_kernel<0, L>), dim3(blocks), dim3(256), 0, s, a);
    } else if (precision == 1) {
        hipLaunchKernelGGL((scan_kernel<1, L>), dim3(blocks), dim3(256), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L>
hipError_t serve_l(const ScanArgs *reqs, const WorkItem *items, int n_items, unsigned *counter,
                   int precision, int waves, hipStream_t s)
{
    const int blocks = (waves + 3) / 4;
    if (precision == 0) {
        hipLaunchKernelGGL((serve_kernel<0, L>), dim3(blocks), dim3(256), 0, s, reqs, items,
                           n_items, counter);
    } else if (precision == 1) {
        hipLaunchKernelGGL((serve_kernel<1, L>), dim3(blocks), dim3(256), 0, s, reqs, items,
                           n_items, counter);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_scan(const ScanArgs &a, int precision, int lanes, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    switch (lanes) {
    case 1: return launch_l<1>(a, precision, s);
    case 2: return launch_l<2>(a, precision, s);
    case 4: return launch_l<4>(a, precision, s);
    case 8: return launch_l<8>(a, precision, s);
    case 16: return launch_l<16>(a, precision, s);
    case 32: return launch_l<32>(a, precision, s);
    case 64: return launch_l<64>(a, precision, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_jmu(const ScanArgs &a, double mu2, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(jmu_kernel, dim3(1), dim3(64), 0, s, a, mu2, dst);
    return hipGetLastError();
}

hipError_t launch_jmu_batch(const ScanArgs *reqs, const int *slots, const double *mu2, int n,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(jmu_batch_kernel, dim3(n), dim3(64), 0, s, reqs, slots, mu2, n);
    return hipGetLastError();
}

hipError_t launch_serve(const ScanArgs *reqs, const WorkItem *items, int n_items,
                        unsigned *counter, int precision, int lanes, int waves, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    switch (lanes) {
    case 1: return serve_l<1>(reqs, items, n_items, counter, precision, waves, s);
    case 2: return serve_l<2>(reqs, items, n_items, counter, precision, waves, s);
    case 4: return serve_l<4>(reqs, items, n_items, counter, precision, waves, s);
    case 8: return serve_l<8>(reqs, items, n_items, counter, precision, waves, s);
    case 16: return serve_l<16>(reqs, items, n_items, counter, precision, waves, s);
    case 32: return serve_l<32>(reqs, items, n_items, counter, precision, waves, s);
    case 64: return serve_l<64>(reqs, items, n_items, counter, precision, waves, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gf
