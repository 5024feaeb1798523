// Internal interface between the host library (plan, validation, cache) and
// the gfx950 kernels.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/gf.h"

namespace gf {

// Contour classes (same values as GF_CLASS_*).
enum : int { kR = 0, kY = 1, kYRes = 2, kMirror = 3, kSingular = 4, kLong = 5 };

// Region-R preference: take the real-axis contour where it is valid and
// either |Im sqrt x| < kRNear * v*, or 1 - |Im sqrt x| / v* >= kRSlope * delta
// (delta = angular distance from arg x to the nearest bad ray).
constexpr double kRNear = 0.25;
constexpr double kRSlope = 0.45;

// Everything a scan kernel needs, passed by value.
struct ScanArgs {
    // Device tables:
    //   rad: r[n_r], sqrt_r[n_r], g[n_r]   (y nodes of GL in log(1+y), dy r^{(D-2)/2}
    //                                       weights), FP64
    //   ang: (z^2, 2w, 2w z^2) for the n_a/2 symmetric pairs of the angular rule, FP64
    //   arc: xi[n_arc], w[n_arc]           (GL on [-1, 1]), FP64
    //   ang32: the pair table rounded to FP32
    const double *rad;
    const double *ang;
    const double *arc;
    const float *ang32;
    int n_r, n_a, n_arc;
    double wmid;  // weight of the middle node z = 0 (odd n_a), else 0

    double m1_re, m1_im, m2_re, m2_im;  // m1^2, m2^2
    double lam2, lam;                    // Lambda^2, Lambda
    double sy0_re, sy0_im;               // sqrt(-m2^2) (residue node)
    const double *jmu;                   // device: Taylor coefficients K_0..K_n of the
                                         // subtraction at mu^2, (re, im) interleaved
    int n_taylor;                        // n of t^n (-1: no subtraction)
    int dim;                             // space-time dimension D (2, 3 or 4)
    int split;                           // split radial rule (rad then holds GL xi, w)
    double T;                            // log(1 + Lambda^2)
    double sm1_re, sm1_im;               // sqrt(-m1^2), principal

    // general propagators: n1, n2 poles, per pole (m^2 re, m^2 im, c re, c im),
    // and each pole's bad ray arg(-m^2); pole 0 is also in m1_*, m2_*
    int poles;  // 0: one pole per leg with residue 1 (the fields above suffice)
    int n1, n2;
    double p1[4 * GF_MAX_POLES];
    double p2[4 * GF_MAX_POLES];
    double b1[GF_MAX_POLES], b2[GF_MAX_POLES];
    int num;          // pole sums: a numerator polynomial N(k^2, p.k) multiplies P1 P2
    double nc[18];    // its coefficients n_ij of (k^2)^i (p.k)^j, (re, im) at 2 (3i + j)
    double mu2;
    double scale;

    // contour geometry
    double beta1, beta2;  // arg(-m1^2), arg(-m2^2)
    double lo, hi;        // open sector of directly reachable ray angles
    double vstar;         // region-R bound on |Im sqrt x|: Re sqrt(m1^2)
    int mirror_ok;        // real masses or a conjugate pair

    // grid
    int n_re, n_im;
    double re_lo, d_re, im_lo, d_im;
    int tiles_a;  // wave tiles along Re
    int n_tiles;  // total wave tiles
    // large scans at one lane per point (FP32C: one or two): the last
    // tail_tiles tiles cover the rows from tail_row0 on at kTailLanes lanes per
    // point (tail_tiles_a of them per row)
    int tail_tiles, tail_row0, tail_tiles_a;
    int unscaled;  // every |x| + |y| + |m1^2| of the scan is below 2^30: the FP64
                   // angular sums skip their power-of-two rescaling

    double *out;   // interleaved complex128
    int8_t *cls;   // optional class map
};

// One unit of serving work: tile `tile` of the request whose arguments sit in
// slot `req` of the device argument array.
struct WorkItem {
    int32_t req;
    int32_t tile;
};

// Launches the scan of one grid (FP64 or FP32C angular sum) with `lanes`
// lanes per point.
hipError_t launch_scan(const ScanArgs &a, int precision, int lanes, hipStream_t s);

// y-plane diagnostic over a grid of y (fields of `a` set as for a one-lane
// scan): <1/D1>(x, y) (what = 0) or the subtracted y-integrand (what = 1).
hipError_t launch_yscan(const ScanArgs &a, double xr, double xi, double mu2, int what,
                        hipStream_t s);
hipError_t launch_obstruction(const ScanArgs &a, int n, double T, uint8_t *out, hipStream_t s);

// Computes the unscaled real-axis sum at x = mu^2 (FP64) into dst[0..1].
hipError_t launch_jmu(const ScanArgs &a, double mu2, double *dst, hipStream_t s);

// The same for n requests at once (device pointers): copies staged[i] into
// reqs[slots[i]] and writes request i's coefficients, at mu2[i], into the jmu
// slot that staged[i] names.
hipError_t launch_jmu_batch(ScanArgs *reqs, const ScanArgs *staged, const int *slots,
                            const double *mu2, int n, hipStream_t s);

// Persistent launch of `waves` wavefronts over n_items work items (device
// arrays); *counter must be 0 on entry.  All items share precision, lanes,
// the split flag of the radial rule and the pole-sum flag.
hipError_t launch_serve(const ScanArgs *reqs, const WorkItem *items, int n_items,
                        unsigned *counter, int precision, int lanes, int split, int poles,
                        int waves, hipStream_t s);

// Wavefronts of that group's persistent kernel the current device holds at
// once (occupancy x compute units x 4 waves per 256-thread block); 4096 if
// the runtime cannot say.
int serve_resident_waves(int precision, int lanes, int split, int poles);
// Wavefronts of the scan kernel for these flags the current device holds at
// once (occupancy x compute units; one wave per workgroup), cached per device
// and kernel form; 4096 if the runtime cannot say.
int scan_resident_waves(int precision, int lanes, bool taylor, bool split, bool poles);

// ---- host helpers shared by plans and the server (gf_host.cpp) ----------

// Sets the thread-local error message; returns code.
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
const char *last_error();

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
// radial table [r | sqrt r | W], angular pair tables, arc table [xi | w]
void radial_table(int n_r, double lambda2, int dim, int split, std::vector<double> &rad);
void angular_tables(int n_a, int rule, int dim, std::vector<double> &ang,
                    std::vector<float> &ang32, double *wmid);
void arc_table(int n_arc, std::vector<double> &arc);
// masses, cutoff, scale and contour geometry of a (params, quadrature)
void fill_constants(ScanArgs &a, const gf_params &p, const gf_propagators *props,
                    const gf_quadrature &q);
int validate_props(const gf_propagators *props, const gf_quadrature &q);
int validate_params(const gf_params *p, const gf_quadrature *q);
int validate_grid(const gf_params &p, const gf_propagators *props, const gf_grid *g);
// lanes per point the automatic choice uses for a grid scanned with a plan's
// arguments and precision
int auto_lanes(const ScanArgs &base, int precision, const gf_grid &g);
// grid fields and wave tiles of a ScanArgs for `lanes` lanes per point
int set_grid(ScanArgs &a, const gf_grid &g, int lanes);
// for an automatically chosen lane count: give a large scan at one lane per
// point (FP32C: one or two) its tail of short waves (no change otherwise)
void set_tail(ScanArgs &a, const gf_grid &g, int precision, int lanes);
int current_device(int *dev);
size_t align256(size_t b);

// Lanes per point of the tail of a one-lane scan.
constexpr int kTailLanes = 16;

// Tile geometry of a wave for `lanes` lanes per point: tw x th points.
inline void tile_shape(int lanes, int *tw, int *th)
{
    int p = 64 / lanes;
    *tw = p < 8 ? p : 8;
    *th = p / *tw;
}

}  // namespace gf
