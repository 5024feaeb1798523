/*
 * gf -- complex-plane scans of a BPHZ-subtracted one-loop two-point function
 * on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, at every point x = p^2 of a cell-centred box in the
 * complex plane,
 *
 *   G(x) = scale * [ int_C dy y <F(x,y,.)> - int_0^{Lambda^2} dy y <F(mu^2,y,.)> ]
 *
 *   F(x,y,z) = 1 / [ (x + y - 2 sqrt(x) sqrt(y) z + m1^2) (y + m2^2) ]
 *   <f>      = (2/pi) int_{-1}^{1} dz sqrt(1 - z^2) f(z)
 *
 * which is the hyperspherical form of a 4-D Euclidean loop integral (STEP 1,
 * eq. 5-11 of Windisch, Alkofer, Haase, Liebmann, "Examining the analytic
 * structure of Green's functions: massive parallel complex integration using
 * GPUs"), regularised by a zeroth-order Taylor subtraction at the real point
 * mu^2 (STEP 2, eq. 12-14, taken at x = 0 in the paper's worked example,
 * eq. 20) with the cutoff Lambda^2 of eq. 14, and analytically continued by
 * deforming the y contour C per point (STEP 3, eq. 15).  Scale 1 gives the
 * rescaled units of eq. 18 / eq. 21; scale 1/(16 pi^2) gives eq. 17.
 *
 * Quadrature (section "Numerical Implementation"): Gauss-Legendre in
 * t = log(1 + y) on [0, log(1 + Lambda^2)] for the radial integral,
 * Gauss-Chebyshev of the second kind (nodes cos(j pi/(n+1)), weight
 * sin^2) for the angular integral, Gauss-Legendre in the angle on the closing
 * arc |y| = Lambda^2.
 *
 * Contours (STEP 3): real axis (region R), ray at arg x plus the closing arc,
 * the same plus the residue of the k-leg pole y = -m2^2, the conjugate
 * mirror G(x) = conj G(conj x) for real masses and conjugate mass pairs, or,
 * where none of these applies, the long way round the origin (GF_CLASS_LONG).
 * Points with no valid contour (x on a bad ray arg x = arg(-m^2) outside
 * region R, e.g. the negative real axis below -m1^2 for real masses) are
 * returned as NaN + i NaN with class GF_CLASS_SINGULAR.
 *
 * All entry points return GF_OK or a negative error code and never throw;
 * gf_last_error() gives a thread-local message for the last failure.
 * Validation errors return before anything is enqueued on a stream.
 */
#ifndef GF_H
#define GF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define GF_OK 0
#define GF_EINVAL (-1)        /* an argument is out of range */
#define GF_EUNSUPPORTED (-2)  /* valid but not implemented */
#define GF_ENOMEM (-3)        /* device or host allocation failed */
#define GF_EDEVICE (-4)       /* a HIP runtime call failed */
#define GF_EBUDGET (-5)       /* a serving request can never fit the budget */
#define GF_ENOTFOUND (-6)     /* unknown serving ticket */

/* ---- precision of the angular (hot) sum -------------------------------- */
#define GF_PREC_FP64 0   /* everything in FP64 */
#define GF_PREC_FP32C 1  /* angular sum in FP32, its blocks of 16 pairs
                            accumulated in FP64; nodes near the angular cut
                            in FP64, nodes far from it with |D|^2 taken from
                            its quadratic in z^2 (coefficients rounded once
                            from FP64); sqrt(x), contour choice, per-node
                            coefficients, radial sum, mu^2 subtraction and
                            scaling in FP64 */

/* ---- angular quadrature rule for the normalised angular average
 * <f> = int_{-1}^{1} (1-z^2)^{(D-3)/2} f(z) dz / N_D (the z integral of eq. 11
 * in D dimensions; N_D = pi, 2, pi/2 for D = 2, 3, 4).  The paper uses
 * tanh-sinh as its main rule and the two Gauss-Chebyshev rules as checks,
 * choosing between them by dimension (section "Numerical Implementation").
 * Each rule integrates g against its own weight omega(z) and is applied to
 * g = f (1-z^2)^{(D-3)/2} / omega; every rule is symmetric in z, so the kernels
 * sum node pairs (z, -z). */
#define GF_ANG_GC2 0        /* Gauss-Chebyshev, second kind, omega = sqrt(1-z^2):
                               z_j = cos(j pi/(n+1)); natural for D = 4 (exact for
                               polynomial f of degree <= 2n-1) */
#define GF_ANG_GC1 1        /* Gauss-Chebyshev, first kind, omega = 1/sqrt(1-z^2):
                               z_j = cos((2j-1) pi/(2n)); natural for D = 2 */
#define GF_ANG_TANH_SINH 2  /* double exponential: z = tanh((pi/2) sinh t) on the
                               equispaced t_k = (k - (n-1)/2) h, h = 2 t_max/(n-1),
                               t_max = 3, 3.5, 4 for D = 4, 3, 2, weight
                               h dz/dt (1-z^2)^{(D-3)/2} / N_D; n >= 3, weights not
                               renormalised */
#define GF_ANG_GL 3         /* Gauss-Legendre, omega = 1; natural for D = 3 */

/* ---- contour classes (values of the optional class map) ---------------- */
#define GF_CLASS_R 0         /* real axis [0, Lambda^2] */
#define GF_CLASS_Y 1         /* ray at arg x + arc |y| = Lambda^2 */
#define GF_CLASS_YRES 2      /* ray + arc + residue at y = -m2^2 */
#define GF_CLASS_MIRROR 3    /* conj of the value at conj x */
#define GF_CLASS_SINGULAR 4  /* no valid contour: NaN */
#define GF_CLASS_LONG 5      /* the rotation towards arg x would sweep a (p-k)-leg
                                bad ray arg(-m1^2) and neither the residue class
                                nor the mirror point applies (a complex (p-k)-leg
                                pole without its conjugate on the k leg; a
                                complex-conjugate pair on the (p-k) leg): each
                                blocked pole's term is continued the other way
                                round the origin, by 2 pi - |arg x| through the
                                other half plane, which sweeps none of its own
                                bad ray and ends on the same ray y = r e^{i arg x};
                                its closing arc runs back the long way, to angle
                                +-2 pi, and it adds the residues of the k-leg
                                poles that rotation sweeps (sign -sign(arg x));
                                the other poles' terms keep the short rotation.
                                Inside the curve where the discretised angular
                                cut meets a k-leg pole (from the threshold
                                -(sqrt(m1^2) + sqrt(m2^2))^2) this is the analytic
                                continuation; beyond it the term's cut runs along
                                that curve and then the bad ray.  In D = 3 the
                                measure sqrt(y) is continued along the long
                                rotation, which meets the ray, its arc and its
                                residues at angles shifted by -+ 2 pi (the
                                opposite sign of sqrt(y) there) */

/* Integrand parameters (eq. 14-16).  m1^2 sits on the (p-k) leg, m2^2 on the
 * k leg; neither may lie on the non-positive real axis.  mu2 is the real
 * subtraction point (>= 0), lambda2 the cutoff Lambda^2 (> 0), scale the
 * output multiplier.  taylor_order n (-1..GF_MAX_TAYLOR) is the order of the
 * Taylor subtraction operator t^n of eq. 12-13, taken about x = mu2 (eq. 13
 * expands about x = 0, i.e. mu2 = 0): the result is
 *   scale * ( S(x) - sum_{i=0}^{n} (x - mu2)^i K_i ),
 * S the contour sum of y^{(D-2)/2} <F(x, y, .)>, K_i = (1/i!) d^i/dx^i of the
 * real-axis sum at x = mu2 (K_0 is the subtraction sum of order 0); n = -1
 * subtracts nothing (for integrals that converge without it, D < 4).  The
 * angular average is an analytic function of x (V^2 = 4xy enters, not
 * sqrt(x)), so its derivatives exist at x = 0.  dimension D (2, 3 or 4; 0
 * means 4) sets the hyperspherical measure of eq. 5-9 in D dimensions:
 * dy y^{(D-2)/2} (1-z^2)^{(D-3)/2} dz, the angular part normalised (see
 * GF_ANG_*). */
#define GF_MAX_TAYLOR 8
typedef struct {
    double m1sq_re, m1sq_im;
    double m2sq_re, m2sq_im;
    double mu2;
    double lambda2;
    double scale;
    int32_t taylor_order;
    int32_t dimension;
} gf_params;

/* Node counts: n_radial Gauss-Legendre nodes in log(1+y) (1..8192),
 * n_angular angular nodes (1..8192; >= 3 for tanh-sinh) of the rule
 * angular_rule (GF_ANG_*), n_arc Gauss-Legendre nodes on the closing arc
 * (1..1024: every ray contour needs its arc; real-axis points do not use
 * them), precision GF_PREC_*.  radial_split = 1 uses,
 * like the paper's several sub-contour node arrays (section "Numerical
 * Implementation"), four Gauss-Legendre pieces of n_radial/4 nodes each
 * (n_radial a multiple of 4) along the straight part of every point's
 * contour, cut in t = log(1+|y|) at the point's near-singular radii: the
 * moduli |(sqrt(x) +- sqrt(-m1^2))^2| of the angular cut's end points (eq. 25
 * at z = +-1) and |m2^2| of the k-leg pole, those inside (0, Lambda^2), cuts
 * within 1e-9 T (T = log(1 + Lambda^2)) of each other counted once; while
 * fewer than three cuts exist, the longest piece (by more than 1e-12 T, the
 * first on ties) is halved.  The subtraction sums use the cuts of x = mu^2. */
typedef struct {
    int32_t n_radial;
    int32_t n_angular;
    int32_t n_arc;
    int32_t precision;
    int32_t angular_rule;
    int32_t radial_split;
} gf_quadrature;

/* Cell-centred n_re x n_im box (STEP 4): point (a, b), 0 <= a < n_re,
 * 0 <= b < n_im, is
 *   Re x = fma(a + 0.5, (re_hi - re_lo) / n_re, re_lo)
 *   Im x = fma(b + 0.5, (im_hi - im_lo) / n_im, im_lo)
 * and its result is element b * n_re + a (Re index fastest).  Requires
 * re_lo < re_hi, im_lo < im_hi, finite; n_re, n_im >= 0 with
 * n_re * n_im <= 2^31. */
typedef struct {
    int32_t n_re, n_im;
    double re_lo, re_hi, im_lo, im_hi;
} gf_grid;

/* Opaque plan: device-resident node tables and the subtraction constant for
 * one (params, quadrature) pair, bound to the device current at creation. */
typedef struct gf_plan gf_plan_t;

/* Builds a plan (STEP 4 preparation): generates the nodes and weights on the
 * host in FP64 (radial, angular, arc), uploads them, and computes the
 * subtraction sum at x = mu^2 on the device (eq. 14's subtracted term on the
 * real axis).  Synchronous.  *out receives the plan; free it with gf_free.
 * Errors: GF_EINVAL (counts, masses, mu2, lambda2, scale out of range),
 * GF_ENOMEM, GF_EDEVICE. */
int gf_plan(const gf_params *params, const gf_quadrature *quad, gf_plan_t **out);

/* ---- general propagators (the integrand plug-in) ------------------------
 * The integrand F = P1((p-k)^2) P2(k^2) with each propagator a sum of poles,
 *   P1(s) = sum_{a < n1} c1_a / (s + m1_a^2),   P2(s) = sum_{b < n2} c2_b / (s + m2_b^2),
 * a form that covers propagators given by a spectral or pole decomposition
 * (complex-conjugate pole pairs included), the inputs the method is meant
 * for (the correlators of the introduction built from different propagators).
 * gf_params' m1^2, m2^2 with residues 1 is the case n1 = n2 = 1.  Each pole
 * position obeys the rule for m1^2, m2^2 (not on the non-positive real axis);
 * 1 <= n1, n2 <= GF_MAX_POLES.  The contour rule generalises: the real axis is
 * valid below the smallest Re sqrt(m1_a^2); the ray sector is bounded by every
 * pole's bad ray; crossing only k-leg bad rays adds the residue of each
 * crossed pole; crossing only (p-k)-leg bad rays uses the mirror point when
 * G(conj x) = conj G(x) holds, i.e. when conjugating every pole position and
 * residue maps (P1, P2) onto itself or onto (P2, P1) (as pole multisets), and
 * the mirror point has a contour of its own; everywhere else off the bad rays
 * GF_CLASS_LONG, with the short and the long rotation chosen per (p-k)-leg
 * pole. */
#define GF_MAX_POLES 8
typedef struct {
    int32_t n1, n2;
    double m1sq_re[GF_MAX_POLES], m1sq_im[GF_MAX_POLES];
    double c1_re[GF_MAX_POLES], c1_im[GF_MAX_POLES];
    double m2sq_re[GF_MAX_POLES], m2sq_im[GF_MAX_POLES];
    double c2_re[GF_MAX_POLES], c2_im[GF_MAX_POLES];
    /* Numerator (the tensor structure of eq. 4's general integrand): with
     * numerator = 1 the integrand is N(k^2, p.k) P1((p-k)^2) P2(k^2),
     *   N = sum_{i,j=0..2} num[3i + j] (k^2)^i (p.k)^j,  p.k = sqrt(x) sqrt(y) z,
     * complex coefficients num_re/num_im; numerator = 0 means N = 1.  Each
     * power of p.k folds exactly into the symmetric angular sums (one more
     * real pair sum, no cancellation).  A polynomial numerator adds no
     * singularity, so the contour classes are those of P1 P2 (MIRROR only
     * with real coefficients); it is subtracted at mu^2 like the rest (any
     * taylor_order), and raises the integrand's growth at large y, so the
     * subtracted integral can need the cutoff to stay finite. */
    int32_t numerator;
    int32_t reserved;            /* alignment of num_re; ignored, set it to 0 */
    double num_re[9], num_im[9]; /* read only when numerator = 1 */
} gf_propagators;

/* gf_plan with general propagators: props replaces the masses of params
 * (props = NULL is gf_plan).  The split radial rule needs n1 = n2 = 1
 * (GF_EUNSUPPORTED otherwise). */
int gf_plan_ex(const gf_params *params, const gf_propagators *props, const gf_quadrature *quad,
               gf_plan_t **out);

/* Tabulated propagators (the integrand plug-in of the introduction and
 * conclusions, for propagators known only as numbers at Euclidean momenta):
 * fits the pole sum P(s) = sum_a c_a / (s + m_a^2) of gf_propagators to n
 * samples (s_i, P(s_i)), s_i >= 0, so that P can be continued to the complex
 * arguments the contours reach.  Host only (no GPU, no device memory).
 *   s[n]            distinct finite sample points >= 0 (any order)
 *   p_re[n], p_im   P(s_i); p_im may be NULL (real data)
 *   weight[n]       positive weights W_i of the error measure, or NULL for 1
 *                   (W_i = 1/|P(s_i)| fits relative errors, for data that
 *                   spans decades)
 *   max_poles       1..GF_MAX_POLES; n >= 2 (max_poles + 1)
 *   tol             stop once max_i W_i |P(s_i) - r(s_i)| <= tol max_i W_i |P(s_i)|
 *                   for the rational approximant r (e.g. 1e-12)
 * Method: the AAA rational approximation (Nakatsukasa, Sete, Trefethen 2018;
 * at most max_poles + 1 support points), its poles as the zeros of the
 * barycentric denominator, then the residues c_a of the pole sum (no constant
 * term) by weighted least squares over all samples; poles on the sampled
 * half-line s >= 0 (spurious: AAA places them when it starts to fit noise)
 * and poles whose weighted term stays below 1e-3 tol max_i W_i |P(s_i)| on
 * every sample are dropped.  With noisy data choose tol above the noise.  Real data give real poles and
 * exactly conjugate pole pairs with conjugate residues, so the propagator
 * keeps G(conj x) = conj G(x).
 * Out: *n_poles <= max_poles; m2_re/m2_im/c_re/c_im (caller arrays of
 * max_poles) hold m_a^2 and c_a; *max_err (may be NULL) = max_i W_i |P(s_i) -
 * fit(s_i)| / max_i W_i |P(s_i)|.  Errors: GF_EINVAL for bad arguments or no
 * pole found. */
int gf_fit_poles(const double *s, const double *p_re, const double *p_im, const double *weight,
                 int n, int max_poles, double tol, int *n_poles, double *m2_re, double *m2_im,
                 double *c_re, double *c_im, double *max_err);

/* Scans a grid with a plan (STEP 5, eq. 15 at every point): launches the
 * fused grid/contour/quadrature kernel on `stream` (a hipStream_t, NULL for
 * the default stream) and returns without waiting.
 *   out      caller-owned device buffer of n_re * n_im complex128
 *            (interleaved re, im doubles), written once per point
 *   cls_out  optional caller-owned device buffer of n_re * n_im int8 contour
 *            classes (GF_CLASS_*), or NULL
 * The plan and buffers must stay valid until the stream has executed the
 * scan.  The current device must be the plan's device.
 * Errors (nothing enqueued): GF_EINVAL (bad grid, NULL out, Lambda^2 too
 * small for the box: it must exceed (sqrt|x| + sqrt(|x| + |m1^2|))^2 at every
 * corner so the closing arc stays clear of the angular cut), GF_EDEVICE. */
int gf_scan_plan(const gf_plan_t *plan, const gf_grid *grid, void *out, int8_t *cls_out,
                 void *stream);

/* As gf_scan_plan with an explicit number of lanes per grid point
 * (1, 2, 4, ..., 64; 0 = automatic).  Each point's quadrature nodes are
 * split across that many lanes of a 64-wide wavefront and the partial sums
 * reduced with cross-lane shuffles.  Automatic takes the smallest count whose
 * wave tiles make at least 4 rounds of the kernel's resident waves, but none
 * that leaves a lane fewer than 2048 angular pairs (4096 in FP32C), and never
 * fewer lanes than fill the GPU once: 1 for large grids, more for smaller
 * ones.  A large scan at one lane per point (FP32C: one or two; at least two
 * rounds of resident waves) runs its last rows, about a quarter round of its
 * work, at 16 lanes per point in the same launch, which shortens the end of
 * the launch.  Results depend on the lane count only through rounding.
 * One launch holds at most 2^26 - 4 wave tiles (a tile is 64 / lanes points,
 * 64 at one lane per point): an explicit count that needs more returns
 * GF_EINVAL before anything is enqueued (2 lanes on a grid of 2^31 points,
 * 64 lanes on one of more than 2^26 - 4); the automatic count never does. */
int gf_scan_plan_ex(const gf_plan_t *plan, const gf_grid *grid, void *out, int8_t *cls_out,
                    int lanes_per_point, void *stream);

/* One-call scan: looks up (or builds and caches) the plan for
 * (params, quadrature) on the current device, then behaves as gf_scan_plan.
 * Cached plans live until gf_cache_clear() or process exit. */
int gf_scan(const gf_params *params, const gf_grid *grid, const gf_quadrature *quad,
            void *out, void *stream);

/* gf_scan for callers that cannot allocate device memory (code that must not
 * call hipMalloc, such as tight serving loops or work recorded into a HIP
 * graph).  Same arguments, validation and result as gf_scan (lanes per point
 * chosen automatically), but no plan is built or cached: the node tables and
 * the subtraction coefficients are generated on `stream` by the library's
 * kernels into one static device buffer of 512 KiB per device (enough for
 * every valid quadrature; sizes beyond it return GF_EINVAL), held until the
 * process ends, and the scan reads them there.  Nothing is allocated, on the
 * device or the host, and nothing is copied from the host: the call only
 * enqueues three kernels and returns (so it can be recorded into a graph;
 * the first call on a device also looks up the buffer's device address, a
 * host-side query: make it outside the recording).  Every call on a device shares that
 * buffer, so calls on one device must be ordered (one stream, or
 * synchronised streams): calls that overlap on a device race and may return
 * wrong results.  The tables are generated on the device, so results can
 * differ from gf_scan's in the last bits.  Errors as gf_scan
 * (nothing enqueued on a validation error). */
int gf_scan_noalloc(const gf_params *params, const gf_grid *grid, const gf_quadrature *quad,
                    void *out, void *stream);

/* Releases a plan.  The caller must have synchronised every stream that uses
 * it.  NULL is ignored. */
void gf_free(gf_plan_t *plan);

/* Frees every plan cached by gf_scan.  Same synchronisation rule. */
void gf_cache_clear(void);

/* Plan introspection: the unscaled subtraction sum at mu^2 (K_0), all
 * taylor_order + 1 Taylor coefficients K_0..K_n of the subtraction
 * (coeffs: 2(n+1) doubles, re/im interleaved), and the lanes per point the
 * automatic choice would use for a grid.  Errors: GF_EINVAL. */
int gf_plan_jmu(const gf_plan_t *plan, double *re, double *im);
int gf_plan_taylor(const gf_plan_t *plan, double *coeffs);
int gf_plan_auto_lanes(const gf_plan_t *plan, const gf_grid *grid);

/* ---- y-plane diagnostics (the paper's Fig. 1 and eq. 23-25) -------------
 *
 * At a fixed external point x, the angular integral produces a cut in the
 * complex y = k^2 plane where the first propagator vanishes for some
 * z = cos(theta1) in [-1, 1]; whether that cut blocks the real y axis decides
 * the contour (STEP 3).  gf_yscan_plan evaluates, with the plan's angular rule
 * in FP64, at every point of a cell-centred grid of complex y:
 *   GF_YSCAN_ANGULAR    <1/D1>(x, y) = sum_j w_j / (x + y + m1^2 - 2 sqrt(x) sqrt(y) z_j)
 *   GF_YSCAN_INTEGRAND  y^{(D-2)/2}/(y + m2^2) (<1/D1>(x, y) - <1/D1>(mu^2, y)),
 *                       the order-0 subtracted y-integrand of eq. 14 (eq. 22
 *                       in the worked example, up to the factor 2/pi; D = 4
 *                       gives y, D = 3 the principal sqrt(y))
 * into `out` (complex128 [n_im][n_re], caller-owned device memory),
 * asynchronously on `stream`.  Errors: GF_EINVAL, GF_EDEVICE. */
#define GF_YSCAN_ANGULAR 0
#define GF_YSCAN_INTEGRAND 1
int gf_yscan_plan(const gf_plan_t *plan, double x_re, double x_im, const gf_grid *ygrid, int what,
                  void *out, void *stream);

/* The continuum cut of eq. 25 for the first propagator: the y where
 * x + y + m1^2 - 2 sqrt(x) sqrt(y) cos(t) = 0, both roots, for n angles
 * t = pi k/(n-1), k = 0..n-1 (n >= 2).  out: 4n doubles per k as
 * (re y+, im y+, re y-, im y-).  Host only.  Errors: GF_EINVAL. */
int gf_cut_curve(const gf_params *params, double x_re, double x_im, int n, double *out);

/* Obstruction map (the paper's Fig. 2 and the figure that follows it): for
 * every point x of a cell-centred grid, whether the angular cut -- the y
 * where x + y + m1^2 - 2 sqrt(x) sqrt(y) z = 0 for some z in [-1, 1], i.e.
 * where zeta = (x + y + m1^2)^2 / (4xy) is real and in [0, 1] -- crosses
 *   bit 0: the original contour, the real segment [0, Lambda^2];
 *   bit 1: the contour the scan uses at x (the contour class rule; for a
 *          mirror point, the contour of conj x);
 *   bit 2: x has no contour (class SINGULAR; bit 1 is then 0).
 * The contour is sampled (each straight part at t = log(1+|y|) = T k/(n-1),
 * k = 1..n-1, T = log(1 + Lambda^2); the closing arc at n equally spaced
 * angles); where Im zeta changes sign between consecutive samples, the sign
 * change is located by 40 bisection steps on the contour parameter (t, or the
 * arc angle), and a crossing is counted when Re zeta at the midpoint of the
 * final interval lies in [0, 1].  Points with
 * bit 0 clear form the region where the real-axis contour is unharmed.  out:
 * caller-owned device memory, n_re * n_im bytes [n_im][n_re]; asynchronous on
 * `stream`.  n_samples in [2, 2^20].  Errors: GF_EINVAL (also for the grid
 * checks of gf_scan_plan), GF_EDEVICE. */
int gf_obstruction_map(const gf_params *params, const gf_grid *grid, int n_samples, uint8_t *out,
                       void *stream);

/* ---- serving: continuous batching of scan requests ----------------------
 *
 * A server owns three HIP streams (one for staging and subtraction sums, two
 * that take the persistent launches in turn), a device-memory arena of
 * `device_budget_bytes` and a scheduler thread.  Submitted requests wait in
 * FIFO order until their output (16 bytes per point) and any node tables not
 * yet resident fit in the arena and a slot is free; admitted requests run
 * concurrently: each scheduler iteration packs wave tiles of every running
 * request (shares of `batch_evals` integrand evaluations that grow with the
 * square of each request's age, then the rest oldest first, topped up with
 * further tiles to half the tiles still to run, at
 * least 1.5 and at most 6 tiles per wave slot of the device: short batches
 * while little waits, long ones under load) into persistent kernel launches, most
 * expensive tiles first, and keeps three such batches in flight; a launch's
 * last long tiles overlap the next launch on the other stream.  A request completes
 * when its last tile has run; its result stays in the arena until
 * gf_server_release.  Every point is computed by the same device code and
 * tables as gf_scan_plan_ex with one lane per point, so a served result is
 * bitwise identical to that standalone scan of the same request, whatever else
 * was in flight.  Node tables are cached by (n_radial, lambda2), n_angular and
 * n_arc and shared by requests.
 *
 * Thread safety: all gf_server_* calls may be made from any thread. */
typedef struct gf_server gf_server_t;

typedef struct {
    size_t device_budget_bytes;  /* arena for outputs + node tables (>= 1 MiB) */
    int32_t max_inflight;        /* admitted requests at once, 1..65536 */
    double batch_evals;          /* target integrand evaluations per batch (0 = 4e10) */
} gf_server_config;

#define GF_REQ_QUEUED 0
#define GF_REQ_RUNNING 1
#define GF_REQ_DONE 2

typedef struct {
    int64_t submitted, completed, released, rejected;
    int64_t queued, running;
    int64_t bytes_in_use, bytes_peak, bytes_budget;
    int64_t batches, work_items, points_done;
    double nominal_evals_done;  /* points x (n_radial + n_arc) x n_angular */
    double latency_mean_ms, latency_p50_ms, latency_p90_ms, latency_p99_ms, latency_max_ms;
    double first_submit_to_last_done_s;
} gf_server_stats;

/* Creates a server on the current device.  Errors: GF_EINVAL, GF_ENOMEM,
 * GF_EDEVICE. */
int gf_server_create(const gf_server_config *cfg, gf_server_t **out);

/* Queues a scan request; *ticket identifies it.  Validation as gf_plan and
 * gf_scan_plan.  GF_EBUDGET if its output alone exceeds the arena. */
int gf_server_submit(gf_server_t *srv, const gf_params *params, const gf_grid *grid,
                     const gf_quadrature *quad, uint64_t *ticket);

/* gf_server_submit with general propagators (as gf_plan_ex; NULL = the
 * masses of params). */
int gf_server_submit_ex(gf_server_t *srv, const gf_params *params, const gf_propagators *props,
                        const gf_grid *grid, const gf_quadrature *quad, uint64_t *ticket);

/* *state = GF_REQ_QUEUED / RUNNING / DONE.  GF_ENOTFOUND for unknown tickets. */
int gf_server_poll(gf_server_t *srv, uint64_t ticket, int *state);

/* Blocks until the request is done or timeout_ms passes (< 0: no limit).
 * Returns 1 if done, 0 on timeout, < 0 on error. */
int gf_server_wait(gf_server_t *srv, uint64_t ticket, double timeout_ms);

/* Pops the oldest completed-but-not-yet-reported ticket, waiting up to
 * timeout_ms.  Returns 1 and sets *ticket, or 0 on timeout. */
int gf_server_wait_any(gf_server_t *srv, double timeout_ms, uint64_t *ticket);

/* Device pointer to a done request's complex128 result [n_im][n_re] (valid
 * until gf_server_release) and its point count. */
int gf_server_result(gf_server_t *srv, uint64_t ticket, const void **dev_ptr, int64_t *n_points);

/* Copies a done request's result to host memory (n_points complex128). */
int gf_server_copy_result(gf_server_t *srv, uint64_t ticket, void *host_dst);

/* Frees a done request's output and slot (its memory returns to the arena). */
int gf_server_release(gf_server_t *srv, uint64_t ticket);

int gf_server_stats_get(gf_server_t *srv, gf_server_stats *stats);

/* Stops the scheduler after in-flight batches finish and frees everything.
 * Requests not yet done are dropped. */
int gf_server_destroy(gf_server_t *srv);

/* Thread-local description of the last error on this thread ("" if none). */
const char *gf_last_error(void);

/* Library version string. */
const char *gf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GF_H */
