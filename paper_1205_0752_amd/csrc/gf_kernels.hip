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
#include <atomic>
#include <type_traits>

#include "gf_device.h"

namespace gf {
namespace {

// One wave's tile of grid points: STEP 4 (the point) and STEP 5 (eq. 15 on
// the point's contour), shared by the one-grid scan and the serving kernel so a
// point's result does not depend on which launch computes it.
// TAYLOR = false compiles out the t^n (n >= 1) epilogue, so the order-0 scan
// carries no extra live values; both forms compute order 0 identically.
// Tiles are numbered row-major over the rows from row0 on, tiles_a per row.
template <int PREC, int L, bool TAYLOR, bool SPLIT, bool POLES, class Args>
__device__ __forceinline__ void process_tile(const Args &a, int tile, int lane, int row0,
                                             int tiles_a)
{
    constexpr int P = 64 / L;
    constexpr int TW = P < 8 ? P : 8;
    constexpr int TH = P / TW;
    const int p = lane / L;
    const int s = lane % L;
    const int ia = (tile % tiles_a) * TW + p % TW;
    const int ib = row0 + (tile / tiles_a) * TH + p / TW;
    const bool valid = ia < a.n_re && ib < a.n_im;

    double xr = fma((double)ia + 0.5, a.d_re, a.re_lo);
    double xi = fma((double)ib + 0.5, a.d_im, a.im_lo);
    int sign = 0, info = 0;
    int cls = valid ? classify<POLES>(a, xr, xi, &sign, &info) : kSingular;
    int ecls = cls;
    if (cls == kMirror) {
        // evaluate at conj x and conjugate the result; if conj x has no
        // contour of its own, the real axis where it is valid at x, else the
        // long way round at x (info holds its sets)
        int sign_b = 0, info_b = 0;
        ecls = classify<POLES>(a, xr, -xi, &sign_b, &info_b);
        if (ecls == kMirror || ecls == kSingular || ecls == kLong) {
            cls = ecls = (info & kInfoRValid) ? kR : kLong;
            if (cls == kR) sign = info = 0;
        } else {
            xi = -xi;
            sign = sign_b;
            info = info_b;
        }
    }
    const PointCtx pc = point_setup<SPLIT, POLES>(a, xr, xi, ecls, sign, info);

    // The straight part's nodes, then the arc and residue nodes, in one
    // sequence k = s, s + L, ... per lane: two loops so that the arc's sine
    // and cosine constants are live only in the second.
    double sr = 0.0, si = 0.0;
    int k = s;
    const int n_straight = min(pc.nodes, a.n_r);
    if (!POLES) {
        // On the straight part y = e^{i phi} r the node weight is
        //   dirD g / (e^{i phi} r + m2^2) = F g / (r + c),  c = m2^2 e^{-i phi},
        // F = dirD e^{-i phi}: F comes out of the sum, and 1/(r + c) takes one
        // real reciprocal of (r + Re c)^2 + (Im c)^2.  U = x + m1^2 + e^{i phi} r
        // and V^2 = (4x e^{i phi}) r are one FMA or product per component.
        // The FP64 sums skip their rescaling when the launch allows it
        // (wave-uniform): the loop is compiled once with and once without.
        const double cr = fma(a.m2_re, pc.dir.r, a.m2_im * pc.dir.i);
        const double ci = fma(a.m2_im, pc.dir.r, -(a.m2_re * pc.dir.i));
        const cd x4d = cmul(mk(4.0 * (pc.x1.r - a.m1_re), 4.0 * (pc.x1.i - a.m1_im)), pc.dir);
        auto straight = [&](auto scale) {
            constexpr int SC = decltype(scale)::value;
            for (; k < n_straight; k += L) {
                double r, g;
                radial_node<SPLIT>(a, pc, k, r, g);
                const cd U = mk(fma(pc.dir.r, r, pc.x1.r), fma(pc.dir.i, r, pc.x1.i));
                const cd A = angular_sum<PREC, SC>(a, U, mk(x4d.r * r, x4d.i * r));
                const double br = r + cr;
                const double gq = g * rcp64(fma(br, br, ci * ci));
                const double wr = gq * br, wi = -(gq * ci);  // g / (r + c)
                sr = fma(wr, A.r, fma(-wi, A.i, sr));
                si = fma(wr, A.i, fma(wi, A.r, si));
            }
        };
        if (PREC == 0 && a.unscaled)
            straight(std::integral_constant<int, 0>{});
        else
            straight(std::integral_constant<int, 1>{});
        const cd F = cmul(pc.dirD, mk(pc.dir.r, -pc.dir.i));
        const double tr = sr;
        sr = fma(F.r, tr, -(F.i * si));
        si = fma(F.r, si, F.i * tr);
    } else {
        // D = 3 with both rotations: the long group's terms see the opposite
        // sign of sqrt(y) on the shared ray (a long group alone has it in dirD)
        const int grp_long = pc.info >> kInfoGrpLong & 0xFF;
        const int ray_neg =
            a.dim == 3 && ecls == kLong && short_group<POLES>(a, pc.info) ? grp_long : 0;
        for (; k < n_straight; k += L) {
            cd U, V2, w;
            radial_coeffs<SPLIT, POLES>(a, pc, k, U, V2, w);
            cd N[3];
            if (a.num) numerator_at(a, U, pc.x1, N);
            cd A = angular_sum_p<PREC, POLES>(a, U, V2, ~0, a.num ? N : nullptr, ray_neg);
            cd t = cmul(w, A);
            sr += t.r;
            si += t.i;
        }
    }
    for (; k < pc.nodes; k += L) {
        cd U, V2, w;
        int set;
        // a residue node carries a whole 2 pi i Res with no quadrature weight
        // to shrink it, and its k-leg pole can sit near the angular cut: its
        // angular sum is taken in FP64 in every precision
        const bool res = outer_coeffs<POLES>(a, pc, k, U, V2, w, set);
        cd N[3];
        const bool num = POLES && a.num;
        if (num) numerator_at(a, U, pc.x1, N);
        cd A = PREC != 0 && res ? angular_sum_p<0, POLES>(a, U, V2, set, num ? N : nullptr)
                                : angular_sum_p<PREC, POLES>(a, U, V2, set, num ? N : nullptr);
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
            double kr = a.jmu[0], ki = a.jmu[1];
            if (TAYLOR && a.n_taylor > 0) {
                // t^n: subtract sum_i (x - mu^2)^i K_i at the evaluated point
                // (conj x for a mirror point), by Horner's rule
                const double er = fma((double)ia + 0.5, a.d_re, a.re_lo) - a.mu2;
                const double yi = fma((double)ib + 0.5, a.d_im, a.im_lo);
                const cd d = mk(er, cls == kMirror ? -yi : yi);
                cd sub = mk(a.jmu[2 * a.n_taylor], a.jmu[2 * a.n_taylor + 1]);
                for (int i = a.n_taylor - 1; i >= 0; --i)
                    sub = cadd(cmul(sub, d), mk(a.jmu[2 * i], a.jmu[2 * i + 1]));
                kr = sub.r;
                ki = sub.i;
            }
            gr = a.scale * (sr - kr);
            gi = a.scale * (si - ki);
            if (cls == kMirror) gi = -gi;
        }
        const size_t idx = (size_t)ib * (size_t)a.n_re + (size_t)ia;
        reinterpret_cast<double2 *>(a.out)[idx] = make_double2(gr, gi);
        if (a.cls) a.cls[idx] = (int8_t)cls;
    }
}

// Register budgets: the FP64 kernel runs best at 4 waves per SIMD (109 VGPRs,
// nothing spilled; 5 waves spill and are 2 % slower), the FP32C kernel at 6
// (measured; its few spills sit outside the inner loop).  One wave (one tile)
// per workgroup: a tile's cost depends on its points' classes (a tile of
// points without a contour ends at once), and a one-wave workgroup frees its
// slot for the next tile by itself, where a four-wave workgroup would hold
// the slots of its finished waves until the last one ends.
//
// The tail of a large scan at one lane per point (FP32C: one or two), in every
// kernel form: its last rows run as tiles of 64 / 16 points at 16 lanes per
// point, a sixteenth of a one-lane wave's work each, dispatched after every
// other tile.  They fill the slots that the last round of long waves leaves as
// it drains (waves sharing a SIMD progress oldest first, so a SIMD's last
// waves end one by one), where otherwise SIMDs would run one or two waves that
// cannot hide the reciprocal's latency.
template <int L, bool TAYLOR, bool SPLIT, bool POLES>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
scan_kernel_fp64(ScanArgs a)
{
    const int wave = blockIdx.x;
    if (wave >= a.n_tiles) return;  // uniform per wave
    // (written as one if-else: an early return gave the tail's pair loop
    // scalar-register spills)
    if (L == 1 && a.tail_tiles > 0 && wave >= a.n_tiles - a.tail_tiles)
        process_tile<0, kTailLanes, TAYLOR, SPLIT, POLES>(a, wave - (a.n_tiles - a.tail_tiles),
                                                          threadIdx.x & 63, a.tail_row0,
                                                          a.tail_tiles_a);
    else
        process_tile<0, L, TAYLOR, SPLIT, POLES>(a, wave, threadIdx.x & 63, 0, a.tiles_a);
}

template <int L, bool TAYLOR, bool SPLIT, bool POLES>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6)))
scan_kernel_fp32c(ScanArgs a)
{
    const int wave = blockIdx.x;
    if (wave >= a.n_tiles) return;  // uniform per wave
    if ((L == 1 || L == 2) && a.tail_tiles > 0 && wave >= a.n_tiles - a.tail_tiles)
        process_tile<1, kTailLanes, TAYLOR, SPLIT, POLES>(a, wave - (a.n_tiles - a.tail_tiles),
                                                          threadIdx.x & 63, a.tail_row0,
                                                          a.tail_tiles_a);
    else
        process_tile<1, L, TAYLOR, SPLIT, POLES>(a, wave, threadIdx.x & 63, 0, a.tiles_a);
}

// Serving: a persistent launch over a packed list of (request, tile) items of
// many requests.  Each wave takes the next item from a device counter (one
// lane's atomic, broadcast) until the list is exhausted, so every wave exits.
template <int PREC, int L, bool SPLIT, bool POLES>
__device__ __forceinline__ void serve_loop(const ScanArgs *reqs, const WorkItem *items, int n_items,
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
        const auto &r = ro(reqs)[req];  // keeps the constant address space
        process_tile<PREC, L, true, SPLIT, POLES>(r, tile, lane, 0, r.tiles_a);
    }
}

template <int L, bool SPLIT, bool POLES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
serve_kernel_fp64(const ScanArgs *__restrict__ reqs, const WorkItem *__restrict__ items,
                  int n_items, unsigned *counter)
{
    serve_loop<0, L, SPLIT, POLES>(reqs, items, n_items, counter);
}

template <int L, bool SPLIT, bool POLES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6)))
serve_kernel_fp32c(const ScanArgs *__restrict__ reqs, const WorkItem *__restrict__ items,
                   int n_items, unsigned *counter)
{
    serve_loop<1, L, SPLIT, POLES>(reqs, items, n_items, counter);
}

// Subtraction sum at the real point mu^2 on the real axis, by one wavefront.
// Higher Taylor coefficients of one folded angular sum about x = mu^2 on the
// real axis (y = r real): with delta = x - mu^2, each symmetric pair
// contributes A(delta) / D(delta) with D = U^2 - 4 x y z^2 = D0 + D1 delta +
// delta^2 (U = U0 + delta), whose power series q_i follows from D q = A term
// by term.  Without a numerator A = 2w U.  With one (N: its polynomials N_j(y)
// in p.k, the same for every pole), the pair carries
//   2w U N0 + 2w z^2 (V^2/2) N1 + 2w z^2 (V^2 U/4) N2,   V^2 = 4 (mu^2 + delta) y,
// a quadratic A = a0 + a1 delta + a2 delta^2 in delta.  The middle node
// (z = 0) w_mid N0 / (U0 + delta) has q_i = w_mid N0 (-1)^i / U0^(i+1).
// acc[i] += omega q_i for i = 1..n.
template <class Args>
__device__ void taylor_node(const Args &a, cd U0, double y, cd omega, int n, cd *acc,
                            const cd *N = nullptr)
{
    const double *tab = a.ang;
    const double mu2 = a.mu2;
    for (int j = 0; j < a.n_a / 2; ++j) {
        const double z2 = ro(tab)[3 * j], w2 = ro(tab)[3 * j + 1];
        const cd D0 = mk(U0.r * U0.r - U0.i * U0.i - 4.0 * mu2 * y * z2, 2.0 * U0.r * U0.i);
        const cd D1 = mk(2.0 * U0.r - 4.0 * y * z2, 2.0 * U0.i);
        cd a0 = cscale(U0, w2), a1 = mk(w2, 0.0), a2 = mk(0.0, 0.0);
        if (N) {
            // a0 = 2w N0 U0 + 2w z^2 y mu^2 (2 N1 + U0 N2)
            // a1 = 2w N0 + 2w z^2 y (2 N1 + (mu^2 + U0) N2)
            // a2 = 2w z^2 y N2
            const double wy = w2 * z2 * y;
            const cd n2u = cmul(N[2], U0);
            a0 = cadd(cmul(a0, N[0]), cscale(cadd(cscale(N[1], 2.0), n2u), wy * mu2));
            a1 = cadd(cscale(N[0], w2),
                      cscale(cadd(cadd(cscale(N[1], 2.0), cscale(N[2], mu2)), n2u), wy));
            a2 = cscale(N[2], wy);
        }
        const cd rD = cdiv(mk(1.0, 0.0), D0);
        cd qm2 = mk(0.0, 0.0);
        cd qm1 = cmul(a0, rD);  // q_0
        for (int i = 1; i <= n; ++i) {
            cd rhs = mk(-(D1.r * qm1.r - D1.i * qm1.i) - qm2.r, -(D1.r * qm1.i + D1.i * qm1.r) - qm2.i);
            if (i == 1) rhs = cadd(rhs, a1);
            if (i == 2) rhs = cadd(rhs, a2);
            const cd q = cmul(rhs, rD);
            acc[i] = cadd(acc[i], cmul(omega, q));
            qm2 = qm1;
            qm1 = q;
        }
    }
    if (a.wmid != 0.0) {
        const cd rU = cdiv(mk(1.0, 0.0), U0);
        cd p = cscale(rU, a.wmid);
        if (N) p = cmul(p, N[0]);
        for (int i = 1; i <= n; ++i) {
            p = cscale(cmul(p, rU), -1.0);
            acc[i] = cadd(acc[i], cmul(omega, p));
        }
    }
}

// Subtraction coefficients at the real point mu^2 on the real axis, by one
// wavefront: K_0 = the subtraction sum of eq. 14 (the order-0 operator t^0),
// and for t^n with n >= 1 the Taylor coefficients K_i = (1/i!) d^i/dx^i of the
// same sum (eq. 13 about x = mu^2).
template <bool SPLIT, bool POLES, class Args>
__device__ __forceinline__ void jmu_wave_impl(const Args &a, double mu2, double *dst, int lane)
{
    const PointCtx pc = point_setup<SPLIT, POLES>(a, mu2, 0.0, kR, 0, 0);
    double sr = 0.0, si = 0.0;
    cd acc[GF_MAX_TAYLOR + 1];
    for (int i = 0; i <= GF_MAX_TAYLOR; ++i) acc[i] = mk(0.0, 0.0);
    for (int k = lane; k < pc.nodes; k += 64) {
        cd U, V2, w;
        node_coeffs<SPLIT, POLES>(a, pc, k, U, V2, w);
        cd N[3];
        const bool num = POLES && a.num;
        if (num) numerator_at(a, U, pc.x1, N);
        cd A = angular_sum_p<0, POLES>(a, U, V2, ~0, num ? N : nullptr);
        cd t = cmul(w, A);
        sr += t.r;
        si += t.i;
        if (a.n_taylor > 0) {
            double r, g;
            radial_node<SPLIT>(a, pc, k, r, g);
            if (!POLES) {
                taylor_node(a, U, r, w, a.n_taylor, acc);
            } else {
                for (int p = 0; p < a.n1; ++p) {  // pole a of P1: U_a, weight c1_a omega
                    const auto *q = &a.p1[4 * p];
                    const cd Ua = mk(U.r + (q[0] - a.m1_re), U.i + (q[1] - a.m1_im));
                    taylor_node(a, Ua, r, cmul(w, mk(q[2], q[3])), a.n_taylor, acc,
                                num ? N : nullptr);
                }
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off);
        si += __shfl_xor(si, off);
    }
    for (int i = 1; i <= a.n_taylor; ++i) {
        double ar = acc[i].r, ai = acc[i].i;
        for (int off = 32; off > 0; off >>= 1) {
            ar += __shfl_xor(ar, off);
            ai += __shfl_xor(ai, off);
        }
        if (lane == 0) {
            dst[2 * i] = ar;
            dst[2 * i + 1] = ai;
        }
    }
    if (lane == 0) {
        // t^-1 (no subtraction) leaves K_0 = 0
        dst[0] = a.n_taylor < 0 ? 0.0 : sr;
        dst[1] = a.n_taylor < 0 ? 0.0 : si;
    }
}

template <class Args>
__device__ __forceinline__ void jmu_wave(const Args &a, double mu2, double *dst, int lane)
{
    if (a.poles)
        jmu_wave_impl<false, true>(a, mu2, dst, lane);  // split needs single poles
    else if (a.split)
        jmu_wave_impl<true, false>(a, mu2, dst, lane);
    else
        jmu_wave_impl<false, false>(a, mu2, dst, lane);
}

__global__ void __launch_bounds__(64) jmu_kernel(ScanArgs a, double mu2, double *dst)
{
    jmu_wave(a, mu2, dst, threadIdx.x);
}

// One wave per request: installs request i's argument record (staged[i]) in
// its slot of the request table, and writes J_mu (and the Taylor
// coefficients) of that request into the record's jmu slot.
__global__ void __launch_bounds__(64) jmu_batch_kernel(ScanArgs *__restrict__ reqs,
                                                       const ScanArgs *__restrict__ staged,
                                                       const int *__restrict__ slots,
                                                       const double *__restrict__ mu2, int n)
{
    static_assert(sizeof(ScanArgs) % sizeof(unsigned long long) == 0, "record size");
    const int i = blockIdx.x;
    if (i >= n) return;
    const int slot = __builtin_amdgcn_readfirstlane(slots[i]);
    constexpr int words = sizeof(ScanArgs) / sizeof(unsigned long long);
    const auto *src = reinterpret_cast<const unsigned long long *>(staged + i);
    auto *dst = reinterpret_cast<unsigned long long *>(reqs + slot);
    for (int k = threadIdx.x; k < words; k += 64) dst[k] = src[k];
    const auto &a = ro(staged)[i];
    jmu_wave(a, mu2[i], const_cast<double *>(a.jmu), threadIdx.x);
}

template <int L>
hipError_t launch_l(const ScanArgs &a, int precision, hipStream_t s)
{
    const int blocks = a.n_tiles;
    const bool taylor = a.n_taylor > 0, split = a.split != 0;
    const dim3 g(blocks), b(64);
    // pole sums run one kernel form (t^n epilogue compiled in; the split rule
    // needs single poles); single poles pick the form without unused parts
    if (precision == 0) {
        if (a.poles)
            hipLaunchKernelGGL((scan_kernel_fp64<L, true, false, true>), g, b, 0, s, a);
        else if (taylor && split)
            hipLaunchKernelGGL((scan_kernel_fp64<L, true, true, false>), g, b, 0, s, a);
        else if (taylor)
            hipLaunchKernelGGL((scan_kernel_fp64<L, true, false, false>), g, b, 0, s, a);
        else if (split)
            hipLaunchKernelGGL((scan_kernel_fp64<L, false, true, false>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((scan_kernel_fp64<L, false, false, false>), g, b, 0, s, a);
    } else if (precision == 1) {
        if (a.poles)
            hipLaunchKernelGGL((scan_kernel_fp32c<L, true, false, true>), g, b, 0, s, a);
        else if (taylor && split)
            hipLaunchKernelGGL((scan_kernel_fp32c<L, true, true, false>), g, b, 0, s, a);
        else if (taylor)
            hipLaunchKernelGGL((scan_kernel_fp32c<L, true, false, false>), g, b, 0, s, a);
        else if (split)
            hipLaunchKernelGGL((scan_kernel_fp32c<L, false, true, false>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((scan_kernel_fp32c<L, false, false, false>), g, b, 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L>
hipError_t serve_l(const ScanArgs *reqs, const WorkItem *items, int n_items, unsigned *counter,
                   int precision, int split, int poles, int waves, hipStream_t s)
{
    const dim3 g((waves + 3) / 4), b(256);
    if (precision == 0) {
        if (poles)
            hipLaunchKernelGGL((serve_kernel_fp64<L, false, true>), g, b, 0, s, reqs, items,
                               n_items, counter);
        else if (split)
            hipLaunchKernelGGL((serve_kernel_fp64<L, true, false>), g, b, 0, s, reqs, items,
                               n_items, counter);
        else
            hipLaunchKernelGGL((serve_kernel_fp64<L, false, false>), g, b, 0, s, reqs, items,
                               n_items, counter);
    } else if (precision == 1) {
        if (poles)
            hipLaunchKernelGGL((serve_kernel_fp32c<L, false, true>), g, b, 0, s, reqs, items,
                               n_items, counter);
        else if (split)
            hipLaunchKernelGGL((serve_kernel_fp32c<L, true, false>), g, b, 0, s, reqs, items,
                               n_items, counter);
        else
            hipLaunchKernelGGL((serve_kernel_fp32c<L, false, false>), g, b, 0, s, reqs, items,
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

hipError_t launch_jmu_batch(ScanArgs *reqs, const ScanArgs *staged, const int *slots,
                            const double *mu2, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(jmu_batch_kernel, dim3(n), dim3(64), 0, s, reqs, staged, slots, mu2, n);
    return hipGetLastError();
}

namespace {

// The scan kernel instance launch_l runs for these flags.
template <int L>
const void *scan_fn(int precision, bool taylor, bool split, bool poles)
{
    if (precision == 0)
        return poles ? reinterpret_cast<const void *>(scan_kernel_fp64<L, true, false, true>)
               : taylor && split
                   ? reinterpret_cast<const void *>(scan_kernel_fp64<L, true, true, false>)
               : taylor ? reinterpret_cast<const void *>(scan_kernel_fp64<L, true, false, false>)
               : split  ? reinterpret_cast<const void *>(scan_kernel_fp64<L, false, true, false>)
                        : reinterpret_cast<const void *>(scan_kernel_fp64<L, false, false, false>);
    if (precision == 1)
        return poles ? reinterpret_cast<const void *>(scan_kernel_fp32c<L, true, false, true>)
               : taylor && split
                   ? reinterpret_cast<const void *>(scan_kernel_fp32c<L, true, true, false>)
               : taylor ? reinterpret_cast<const void *>(scan_kernel_fp32c<L, true, false, false>)
               : split  ? reinterpret_cast<const void *>(scan_kernel_fp32c<L, false, true, false>)
                        : reinterpret_cast<const void *>(scan_kernel_fp32c<L, false, false, false>);
    return nullptr;
}

template <int L>
const void *serve_fn(int precision, int split, int poles)
{
    if (precision == 0)
        return poles ? reinterpret_cast<const void *>(serve_kernel_fp64<L, false, true>)
               : split ? reinterpret_cast<const void *>(serve_kernel_fp64<L, true, false>)
                       : reinterpret_cast<const void *>(serve_kernel_fp64<L, false, false>);
    if (precision == 1)
        return poles ? reinterpret_cast<const void *>(serve_kernel_fp32c<L, false, true>)
               : split ? reinterpret_cast<const void *>(serve_kernel_fp32c<L, true, false>)
                       : reinterpret_cast<const void *>(serve_kernel_fp32c<L, false, false>);
    return nullptr;
}

}  // namespace

int scan_resident_waves(int precision, int lanes, bool taylor, bool split, bool poles)
{
    // cached per device and kernel form: [device][precision][log2 lanes][taylor][split][poles]
    constexpr int kDevices = 16;
    static std::atomic<int> cache[kDevices][2][7][2][2][2];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 4096;
    int lg = 0;
    while (lg < 7 && (1 << lg) != lanes) ++lg;
    if (lg == 7 || precision < 0 || precision > 1) return 4096;
    std::atomic<int> *slot = dev >= 0 && dev < kDevices
                                 ? &cache[dev][precision][lg][taylor][split][poles]
                                 : nullptr;
    if (slot) {
        const int v = slot->load(std::memory_order_relaxed);
        if (v > 0) return v;
    }
    const void *f = nullptr;
    switch (lanes) {
    case 1: f = scan_fn<1>(precision, taylor, split, poles); break;
    case 2: f = scan_fn<2>(precision, taylor, split, poles); break;
    case 4: f = scan_fn<4>(precision, taylor, split, poles); break;
    case 8: f = scan_fn<8>(precision, taylor, split, poles); break;
    case 16: f = scan_fn<16>(precision, taylor, split, poles); break;
    case 32: f = scan_fn<32>(precision, taylor, split, poles); break;
    case 64: f = scan_fn<64>(precision, taylor, split, poles); break;
    default: break;
    }
    int cus = 0, blocks = 0;
    if (!f || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, 64, 0) != hipSuccess ||
        cus <= 0 || blocks <= 0)
        return 4096;
    const int waves = cus * blocks;  // one wave per workgroup
    if (slot) slot->store(waves, std::memory_order_relaxed);
    return waves;
}

int serve_resident_waves(int precision, int lanes, int split, int poles)
{
    const void *f = nullptr;
    switch (lanes) {
    case 1: f = serve_fn<1>(precision, split, poles); break;
    case 2: f = serve_fn<2>(precision, split, poles); break;
    case 4: f = serve_fn<4>(precision, split, poles); break;
    case 8: f = serve_fn<8>(precision, split, poles); break;
    case 16: f = serve_fn<16>(precision, split, poles); break;
    case 32: f = serve_fn<32>(precision, split, poles); break;
    case 64: f = serve_fn<64>(precision, split, poles); break;
    default: break;
    }
    int dev = 0, cus = 0, blocks = 0;
    if (!f || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, 256, 0) != hipSuccess ||
        cus <= 0 || blocks <= 0)
        return 4096;
    return cus * blocks * 4;
}

hipError_t launch_serve(const ScanArgs *reqs, const WorkItem *items, int n_items,
                        unsigned *counter, int precision, int lanes, int split, int poles,
                        int waves, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    switch (lanes) {
    case 1: return serve_l<1>(reqs, items, n_items, counter, precision, split, poles, waves, s);
    case 2: return serve_l<2>(reqs, items, n_items, counter, precision, split, poles, waves, s);
    case 4: return serve_l<4>(reqs, items, n_items, counter, precision, split, poles, waves, s);
    case 8: return serve_l<8>(reqs, items, n_items, counter, precision, split, poles, waves, s);
    case 16: return serve_l<16>(reqs, items, n_items, counter, precision, split, poles, waves, s);
    case 32: return serve_l<32>(reqs, items, n_items, counter, precision, split, poles, waves, s);
    case 64: return serve_l<64>(reqs, items, n_items, counter, precision, split, poles, waves, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gf
