// gf_scan_noalloc: the one-call scan of gf_scan without any allocation, for
// callers that cannot allocate device memory.
//
// gf_scan keeps the node tables and the subtraction constant of each
// (params, quadrature) pair in a cached plan, a device allocation of its own.
// This entry point instead builds them, on the caller's stream, in one
// file-scope device array (`scratch`, kScratchBytes per device, held until the
// process ends): a kernel generates the radial, angular and arc nodes and
// weights (the same rules as the host tables of a plan: Gauss-Legendre by
// Newton's method on the Legendre recurrence, the closed-form Chebyshev and
// tanh-sinh nodes), the subtraction kernel writes K_0..K_n next to them, and
// the scan kernel of gf_scan_plan_ex reads them.  Nothing is copied from the
// host, so the call is asynchronous like gf_scan_plan.  Every table entry the
// scan reads is rewritten by each call; nothing needs clearing.
//
// The array is shared by every call on a device: calls on one device must be
// ordered (one stream, or synchronised), since overlapping calls overwrite
// each other's tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "gf_internal.h"

namespace gf {
namespace {

// Largest table set of a valid quadrature (8192 radial nodes, 8192 angular
// nodes, 1024 arc nodes): 3*8192 + 3*4096 doubles, 2*1024 doubles, 256 bytes of
// Taylor coefficients and 3*4096 floats, each part 256-byte aligned, is about
// 360 KiB.
constexpr size_t kScratchBytes = 512 * 1024;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// The device address of this device's copy of `scratch` (the host-side name
// of the array is only a stand-in), looked up once per device.
int scratch_address(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(GF_EUNSUPPORTED, "device %d is beyond the %d devices supported", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(GF_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return GF_OK;
}

// Node k (ascending) of the n-point Gauss-Legendre rule on [-1, 1] and its
// weight: the root counted i-th from the top by Newton's method on the
// three-term recurrence from Tricomi's estimate, mirrored for the lower half;
// an odd rule's middle node is exactly 0.
__device__ void gl_node(int n, int k, double *x, double *w)
{
    const int i = 2 * k < n ? k + 1 : n - k;
    double r = cos(M_PI * (4.0 * i - 1.0) / (4.0 * n + 2.0)) * (1.0 - (n - 1.0) / (8.0 * n * n * n));
    double pk = 1.0, pkm1 = 1.0;
    auto legendre = [&](double t) {
        pkm1 = 1.0;
        pk = t;
        for (int m = 1; m < n; ++m) {
            const double next = ((2 * m + 1) * t * pk - m * pkm1) / (m + 1);
            pkm1 = pk;
            pk = next;
        }
    };
    for (int it = 0, extra = 0; it < 64 && extra < 2; ++it) {
        legendre(r);
        const double dr = pk / (n * (pkm1 - r * pk) / (1.0 - r * r));
        r -= dr;
        if (fabs(dr) < 1e-15) ++extra;
    }
    legendre(r);
    const double dp = n == 0 ? 0.0 : n * (pkm1 - r * pk) / (1.0 - r * r);
    *w = 2.0 / ((1.0 - r * r) * dp * dp);
    *x = (n % 2 == 1 && 2 * k + 1 == n) ? 0.0 : (2 * k < n ? -r : r);
}

struct TableArgs {
    double *rad;
    double *ang;
    float *ang32;
    double *arc;
    int n_r, n_a, n_arc;
    int rule, dim, split;
    double T;  // log(1 + Lambda^2)
};

// Row 0: the radial table [r | sqrt r | dr r^{(D-2)/2}] of GL in t = log(1+y)
// on [0, T] (split rule: the base GL rule of order n_r/4 as [xi | w], the
// rest zero); row 1: the angular pair table (z^2, 2w, 2w z^2) of the
// normalised D-dimensional measure, in FP64 and FP32; row 2: the arc table
// [xi | w] of GL on [-1, 1].
__global__ void __launch_bounds__(256) table_kernel(TableArgs t)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.y == 0) {
        if (i >= t.n_r) return;
        const int nr = t.n_r;
        if (t.split) {
            const int m = nr / 4;
            double x, w;
            double v = 0.0;
            if (i < 2 * m) {
                gl_node(m, i % m, &x, &w);
                v = i < m ? x : w;
            }
            t.rad[i] = v;
            t.rad[nr + i] = 0.0;
            t.rad[2 * nr + i] = 0.0;
            return;
        }
        double x, w;
        gl_node(nr, i, &x, &w);
        const double y = expm1(0.5 * t.T * (x + 1.0));
        const double dy = 0.5 * t.T * w * (1.0 + y);
        t.rad[i] = y;
        t.rad[nr + i] = sqrt(y);
        t.rad[2 * nr + i] = t.dim == 4 ? dy * y : (t.dim == 3 ? dy * sqrt(y) : dy);
    } else if (blockIdx.y == 1) {
        const int na = t.n_a, npair = na / 2;
        if (i >= (npair > 0 ? npair : 1)) return;
        double zsq = 0.0, wt = 0.0;
        if (npair > 0) {
            const double norm = t.dim == 2 ? M_PI : (t.dim == 3 ? 2.0 : M_PI_2);
            auto sinpow = [&](double s) { return t.dim == 4 ? s * s : (t.dim == 3 ? s : 1.0); };
            const int j = i;
            if (t.rule == GF_ANG_GC2) {
                const double th = (j + 1) * M_PI / (na + 1);
                const double c = cos(th);
                zsq = c * c;
                wt = M_PI / (na + 1) * sinpow(sin(th)) / norm;
            } else if (t.rule == GF_ANG_GC1) {
                const double th = (2 * j + 1) * M_PI / (2.0 * na);
                const double c = cos(th);
                zsq = c * c;
                wt = M_PI / na * sinpow(sin(th)) / norm;
            } else if (t.rule == GF_ANG_GL) {
                double z, w;
                gl_node(na, na - 1 - j, &z, &w);  // positive nodes, descending
                const double s2 = 1.0 - z * z;
                const double m = t.dim == 4 ? sqrt(s2) : (t.dim == 3 ? 1.0 : 1.0 / sqrt(s2));
                zsq = z * z;
                wt = w * m / norm;
            } else {
                const double tmax = t.dim == 4 ? 3.0 : (t.dim == 3 ? 3.5 : 4.0);
                const double h = 2.0 * tmax / (na - 1);
                const double tt = (na % 2 == 1) ? (j + 1) * h : (j + 0.5) * h;
                const double u = M_PI_2 * sinh(tt);
                const double z = tanh(u), cu = cosh(u);
                const double meas = t.dim == 4 ? 1.0 / (cu * cu * cu)
                                    : (t.dim == 3 ? 1.0 / (cu * cu) : 1.0 / cu);
                zsq = z * z;
                wt = h * M_PI_2 * cosh(tt) * meas / norm;
            }
        }
        t.ang[3 * i] = zsq;
        t.ang[3 * i + 1] = 2.0 * wt;
        t.ang[3 * i + 2] = 2.0 * wt * zsq;
        t.ang32[3 * i] = (float)zsq;
        t.ang32[3 * i + 1] = (float)(2.0 * wt);
        t.ang32[3 * i + 2] = (float)(2.0 * wt * zsq);
    } else {
        if (i >= t.n_arc) return;
        double x, w;
        gl_node(t.n_arc, i, &x, &w);
        t.arc[i] = x;
        t.arc[t.n_arc + i] = w;
    }
}

// Weight of the middle node z = 0 of an odd angular rule (0 for even rules).
// Gauss-Legendre: 2 / P_n'(0)^2 with P_n'(0) = n P_{n-1}(0).
double middle_weight(int na, int rule, int dim)
{
    if (na % 2 == 0) return 0.0;
    const double norm = dim == 2 ? M_PI : (dim == 3 ? 2.0 : M_PI_2);
    if (rule == GF_ANG_GC2) return M_PI / (na + 1) / norm;
    if (rule == GF_ANG_GC1) return M_PI / na / norm;
    if (rule == GF_ANG_GL) {
        double pkm1 = 1.0, pk = 0.0;  // P_0(0), P_1(0)
        for (int m = 1; m < na - 1; ++m) {
            const double next = -m * pkm1 / (m + 1);
            pkm1 = pk;
            pk = next;
        }
        const double dp = na == 1 ? 1.0 : na * pk;
        return 2.0 / (dp * dp) / norm;
    }
    const double tmax = dim == 4 ? 3.0 : (dim == 3 ? 3.5 : 4.0);
    return 2.0 * tmax / (na - 1) * M_PI_2 / norm;
}

}  // namespace
}  // namespace gf

extern "C" int gf_scan_noalloc(const gf_params *params, const gf_grid *grid,
                               const gf_quadrature *quad, void *out, void *stream)
{
    using namespace gf;
    int rc = validate_params(params, quad);
    if (rc != GF_OK) return rc;
    if ((rc = validate_grid(*params, nullptr, grid)) != GF_OK) return rc;
    if ((long long)grid->n_re * grid->n_im == 0) return GF_OK;
    if (!out) return fail(GF_EINVAL, "out must not be NULL");

    const int dim = params->dimension == 0 ? 4 : params->dimension;
    const int npair = std::max(quad->n_angular / 2, 1);
    const size_t off_rad = 0;
    const size_t off_ang = off_rad + align256(3 * (size_t)quad->n_radial * sizeof(double));
    const size_t off_arc = off_ang + align256(3 * (size_t)npair * sizeof(double));
    const size_t off_jmu = off_arc + align256(2 * (size_t)quad->n_arc * sizeof(double));
    const size_t off_a32 = off_jmu + 256;
    const size_t total = off_a32 + align256(3 * (size_t)npair * sizeof(float));
    if (total > kScratchBytes)
        return fail(GF_EINVAL, "node tables need %zu bytes, more than the %zu of the static buffer",
                    total, kScratchBytes);

    int dev;
    if ((rc = current_device(&dev)) != GF_OK) return rc;
    char *base = nullptr;
    if ((rc = scratch_address(dev, &base)) != GF_OK) return rc;

    ScanArgs a{};
    fill_constants(a, *params, nullptr, *quad);
    a.rad = reinterpret_cast<const double *>(base + off_rad);
    a.ang = reinterpret_cast<const double *>(base + off_ang);
    a.arc = reinterpret_cast<const double *>(base + off_arc);
    a.ang32 = reinterpret_cast<const float *>(base + off_a32);
    a.jmu = reinterpret_cast<const double *>(base + off_jmu);
    a.wmid = middle_weight(quad->n_angular, quad->angular_rule, dim);
    const int lanes = auto_lanes(a, quad->precision, *grid);
    if ((rc = set_grid(a, *grid, lanes)) != GF_OK) return rc;
    set_tail(a, *grid, quad->precision, lanes);
    a.out = static_cast<double *>(out);
    a.cls = nullptr;

    TableArgs t;
    t.rad = reinterpret_cast<double *>(base + off_rad);
    t.ang = reinterpret_cast<double *>(base + off_ang);
    t.ang32 = reinterpret_cast<float *>(base + off_a32);
    t.arc = reinterpret_cast<double *>(base + off_arc);
    t.n_r = quad->n_radial;
    t.n_a = quad->n_angular;
    t.n_arc = quad->n_arc;
    t.rule = quad->angular_rule;
    t.dim = dim;
    t.split = quad->radial_split;
    t.T = a.T;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int items = std::max(std::max(quad->n_radial, npair), quad->n_arc);
    hipLaunchKernelGGL(table_kernel, dim3((items + 255) / 256, 3), dim3(256), 0, s, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "node-table kernel launch");
    e = launch_jmu(a, params->mu2, const_cast<double *>(a.jmu), s);
    if (e != hipSuccess) return hip_fail(e, "subtraction-term kernel launch");
    e = launch_scan(a, quad->precision, lanes, s);
    if (e != hipSuccess) return hip_fail(e, "scan kernel launch");
    return GF_OK;
}
