// Tabulated propagators: a pole sum P(s) = sum_a c_a / (s + m_a^2) fitted to
// samples of P on the real axis s >= 0, so that tabulated input (a propagator
// known only at Euclidean momenta) can be continued to the complex arguments
// the contours need.  Host code, FP64, run once before a plan is made.
//
// Steps: the AAA rational approximation (Nakatsukasa, Sete and Trefethen,
// SIAM J. Sci. Comput. 40 (2018) A1494) in barycentric form
//   r(s) = sum_k w_k f_k / (s - z_k)  /  sum_k w_k / (s - z_k),
// support points z_k picked greedily where the error is largest and weights w
// from the smallest right singular vector of the Loewner matrix; the poles of
// r as the zeros of its denominator (Aberth's simultaneous iteration on the
// denominator times prod_k (s - z_k), evaluated in barycentric form); then
// the residues of the pole sum, which has no constant term, by linear least
// squares over every sample with the poles fixed.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/gf.h"
#include "gf_internal.h"

namespace gf {
namespace {

using cplx = std::complex<double>;

// Right singular vector of the smallest singular value of A (rows x cols,
// column-major), by one-sided Jacobi rotations (Hestenes): pairs of columns
// are rotated until every pair is orthogonal; the product of the rotations is
// V, and the final column norms are the singular values.
std::vector<cplx> min_right_singular_vector(std::vector<cplx> A, int rows, int cols)
{
    std::vector<cplx> V((size_t)cols * cols, 0.0);
    for (int k = 0; k < cols; ++k) V[(size_t)k * cols + k] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        bool rotated = false;
        for (int p = 0; p + 1 < cols; ++p)
            for (int q = p + 1; q < cols; ++q) {
                cplx *ap = &A[(size_t)p * rows], *aq = &A[(size_t)q * rows];
                double alpha = 0.0, beta = 0.0;
                cplx gamma = 0.0;
                for (int i = 0; i < rows; ++i) {
                    alpha += std::norm(ap[i]);
                    beta += std::norm(aq[i]);
                    gamma += std::conj(ap[i]) * aq[i];
                }
                const double g = std::abs(gamma);
                if (g == 0.0 || g <= 1e-15 * std::sqrt(alpha * beta)) continue;
                rotated = true;
                // column q times ph makes the pair's inner product the real |gamma|;
                // then the real rotation tan = t with t^2 + 2 zeta t - 1 = 0
                const cplx ph = std::conj(gamma) / g;
                const double zeta = (beta - alpha) / (2.0 * g);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::hypot(1.0, zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < rows; ++i) {
                    const cplx x = ap[i], y = aq[i] * ph;
                    ap[i] = c * x - s * y;
                    aq[i] = s * x + c * y;
                }
                cplx *vp = &V[(size_t)p * cols], *vq = &V[(size_t)q * cols];
                for (int i = 0; i < cols; ++i) {
                    const cplx x = vp[i], y = vq[i] * ph;
                    vp[i] = c * x - s * y;
                    vq[i] = s * x + c * y;
                }
            }
        if (!rotated) break;
    }
    int kmin = 0;
    double smin = INFINITY;
    for (int k = 0; k < cols; ++k) {
        double nk = 0.0;
        for (int i = 0; i < rows; ++i) nk += std::norm(A[(size_t)k * rows + i]);
        if (nk < smin) {
            smin = nk;
            kmin = k;
        }
    }
    return std::vector<cplx>(V.begin() + (size_t)kmin * cols, V.begin() + (size_t)(kmin + 1) * cols);
}

struct Barycentric {
    std::vector<double> z;  // support points
    std::vector<cplx> f, w;
};

// AAA: at most mmax support points, stopping once max W |F - r| <= tol_abs;
// the Loewner rows carry the sample weights W as well
Barycentric aaa(const std::vector<double> &Z, const std::vector<cplx> &F,
                const std::vector<double> &W, int mmax, double tol_abs)
{
    const int M = (int)Z.size();
    std::vector<char> used(M, 0);
    cplx mean = 0.0;
    for (const cplx &v : F) mean += v;
    std::vector<cplx> R(M, mean / (double)M);
    Barycentric b;
    for (int m = 1; m <= mmax; ++m) {
        int j = -1;
        double e = -1.0;
        for (int i = 0; i < M; ++i)
            if (!used[i] && W[i] * std::abs(F[i] - R[i]) > e) {
                e = W[i] * std::abs(F[i] - R[i]);
                j = i;
            }
        if (j < 0) break;
        used[j] = 1;
        b.z.push_back(Z[j]);
        b.f.push_back(F[j]);
        std::vector<int> J;
        for (int i = 0; i < M; ++i)
            if (!used[i]) J.push_back(i);
        const int rows = (int)J.size();
        std::vector<cplx> A((size_t)rows * m);
        for (int k = 0; k < m; ++k)
            for (int r = 0; r < rows; ++r)
                A[(size_t)k * rows + r] = W[J[r]] * (F[J[r]] - b.f[k]) / (Z[J[r]] - b.z[k]);
        b.w = rows > 0 ? min_right_singular_vector(A, rows, m) : std::vector<cplx>(m, 1.0);
        double err = 0.0;
        for (int r = 0; r < rows; ++r) {
            cplx num = 0.0, den = 0.0;
            for (int k = 0; k < m; ++k) {
                const cplx t = b.w[k] / (Z[J[r]] - b.z[k]);
                num += t * b.f[k];
                den += t;
            }
            R[J[r]] = num / den;
            err = std::max(err, W[J[r]] * std::abs(F[J[r]] - R[J[r]]));
        }
        for (int i = 0; i < M; ++i)
            if (used[i]) R[i] = F[i];
        if (err <= tol_abs) break;
    }
    return b;
}

// Zeros of d(s) = sum_k w_k / (s - z_k): the roots of the polynomial
// q(s) = d(s) prod_k (s - z_k) of degree m - 1, by Aberth's iteration with
// q'/q = d'/d + sum_k 1/(s - z_k).  Roots that run off to infinity (a degree
// below m - 1) are dropped.
std::vector<cplx> denominator_zeros(const Barycentric &b)
{
    const int m = (int)b.z.size(), nd = m - 1;
    if (nd <= 0) return {};
    double lo = b.z[0], hi = b.z[0];
    for (double v : b.z) {
        lo = std::min(lo, v);
        hi = std::max(hi, v);
    }
    const cplx centre = 0.5 * (lo + hi);
    const double radius = std::max(0.5 * (hi - lo), 1.0);
    std::vector<cplx> s(nd);
    for (int k = 0; k < nd; ++k) s[k] = centre + std::polar(radius, 2.0 * M_PI * k / nd + 0.7);
    for (int it = 0; it < 2000; ++it) {
        double worst = 0.0;
        for (int k = 0; k < nd; ++k) {
            cplx d = 0.0, dp = 0.0, sz = 0.0;
            bool on_support = false;
            for (int j = 0; j < m; ++j) {
                const cplx diff = s[k] - b.z[j];
                if (diff == 0.0) {
                    on_support = true;
                    break;
                }
                const cplx inv = 1.0 / diff;
                d += b.w[j] * inv;
                dp -= b.w[j] * inv * inv;
                sz += inv;
            }
            if (on_support) {  // nudge off a support point (q does not vanish there)
                s[k] += cplx(0.0, 1e-8 * radius);
                worst = 1.0;
                continue;
            }
            if (d == 0.0) continue;
            cplx others = 0.0;
            for (int l = 0; l < nd; ++l)
                if (l != k) others += 1.0 / (s[k] - s[l]);
            const cplx corr = 1.0 / (dp / d + sz - others);
            s[k] -= corr;
            worst = std::max(worst, std::abs(corr) / (std::abs(s[k]) + radius));
        }
        if (worst < 1e-15) break;
    }
    std::vector<cplx> out;
    const double far = 1e8 * (std::abs(centre) + radius);
    for (const cplx &v : s)
        if (std::isfinite(v.real()) && std::isfinite(v.imag()) && std::abs(v) < far) out.push_back(v);
    return out;
}

// Residues c of sum_a c_a / (Z_i - p_a) ~ F_i in the weighted least-squares
// sense (rows times W_i): QR of the Cauchy matrix by modified Gram-Schmidt,
// each column orthogonalised twice.  Returns false if the columns are
// numerically dependent.
bool residues_lsq(const std::vector<double> &Z, const std::vector<cplx> &F,
                  const std::vector<double> &W, const std::vector<cplx> &p, std::vector<cplx> &c)
{
    const int M = (int)Z.size(), n = (int)p.size();
    std::vector<cplx> Q((size_t)M * n), Rm((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a) {
        cplx *q = &Q[(size_t)a * M];
        for (int i = 0; i < M; ++i) q[i] = W[i] / (Z[i] - p[a]);
        double n0 = 0.0;
        for (int i = 0; i < M; ++i) n0 += std::norm(q[i]);
        for (int pass = 0; pass < 2; ++pass)
            for (int b = 0; b < a; ++b) {
                const cplx *qb = &Q[(size_t)b * M];
                cplx dot = 0.0;
                for (int i = 0; i < M; ++i) dot += std::conj(qb[i]) * q[i];
                for (int i = 0; i < M; ++i) q[i] -= dot * qb[i];
                Rm[(size_t)a * n + b] += dot;  // R(b, a)
            }
        double nn = 0.0;
        for (int i = 0; i < M; ++i) nn += std::norm(q[i]);
        if (!(nn > 1e-28 * n0)) return false;
        const double inv = 1.0 / std::sqrt(nn);
        for (int i = 0; i < M; ++i) q[i] *= inv;
        Rm[(size_t)a * n + a] = std::sqrt(nn);
    }
    std::vector<cplx> y(n, 0.0);
    for (int a = 0; a < n; ++a) {
        const cplx *q = &Q[(size_t)a * M];
        for (int i = 0; i < M; ++i) y[a] += std::conj(q[i]) * (W[i] * F[i]);
    }
    c.assign(n, 0.0);
    for (int a = n - 1; a >= 0; --a) {
        cplx v = y[a];
        for (int b = a + 1; b < n; ++b) v -= Rm[(size_t)b * n + a] * c[b];
        c[a] = v / Rm[(size_t)a * n + a];
    }
    return true;
}

}  // namespace
}  // namespace gf

extern "C" int gf_fit_poles(const double *s, const double *p_re, const double *p_im,
                            const double *weight, int n, int max_poles, double tol, int *n_poles,
                            double *m2_re, double *m2_im, double *c_re, double *c_im,
                            double *max_err)
{
    using gf::cplx;
    using gf::fail;
    if (!s || !p_re || !n_poles || !m2_re || !m2_im || !c_re || !c_im)
        return fail(GF_EINVAL, "NULL argument");
    if (max_poles < 1 || max_poles > GF_MAX_POLES)
        return fail(GF_EINVAL, "max_poles must be in [1, %d], got %d", GF_MAX_POLES, max_poles);
    if (n < 2 * (max_poles + 1))
        return fail(GF_EINVAL, "%d samples are too few for %d poles (need %d)", n, max_poles,
                    2 * (max_poles + 1));
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(GF_EINVAL, "tol must be positive");
    std::vector<double> Z(s, s + n);
    std::vector<cplx> F(n);
    std::vector<double> W(n, 1.0);
    bool real = true;
    double fmax = 0.0;
    for (int i = 0; i < n; ++i) {
        const double im = p_im ? p_im[i] : 0.0;
        if (weight) {
            if (!std::isfinite(weight[i]) || !(weight[i] > 0.0))
                return fail(GF_EINVAL, "sample %d: the weight must be finite and positive", i);
            W[i] = weight[i];
        }
        if (!std::isfinite(Z[i]) || Z[i] < 0.0)
            return fail(GF_EINVAL, "sample %d: s must be finite and >= 0", i);
        if (!std::isfinite(p_re[i]) || !std::isfinite(im))
            return fail(GF_EINVAL, "sample %d: P(s) must be finite", i);
        F[i] = cplx(p_re[i], im);
        real = real && im == 0.0;
        fmax = std::max(fmax, W[i] * std::abs(F[i]));
    }
    {
        std::vector<double> sorted = Z;
        std::sort(sorted.begin(), sorted.end());
        for (int i = 1; i < n; ++i)
            if (sorted[i] == sorted[i - 1]) return fail(GF_EINVAL, "sample points must be distinct");
    }
    if (fmax == 0.0) return fail(GF_EINVAL, "P vanishes at every sample");

    const double tol_abs = tol * fmax;
    const gf::Barycentric b = gf::aaa(Z, F, W, max_poles + 1, tol_abs);
    std::vector<cplx> p = gf::denominator_zeros(b);
    if (real) {
        // real data: real weights, so the poles are real or come in conjugate
        // pairs; make that exact (the mirror symmetry tests it exactly)
        double scale = 1.0;
        for (double v : Z) scale = std::max(scale, std::fabs(v));
        std::vector<char> paired(p.size(), 0);
        for (size_t k = 0; k < p.size(); ++k)
            if (std::fabs(p[k].imag()) <= 1e-9 * (std::abs(p[k]) + 1e-6 * scale)) {
                p[k] = p[k].real();
                paired[k] = 1;
            }
        for (size_t k = 0; k < p.size(); ++k) {
            if (paired[k] || p[k].imag() < 0.0) continue;
            size_t best = p.size();
            double bd = INFINITY;
            for (size_t l = 0; l < p.size(); ++l)
                if (!paired[l] && p[l].imag() < 0.0 && std::abs(p[l] - std::conj(p[k])) < bd) {
                    bd = std::abs(p[l] - std::conj(p[k]));
                    best = l;
                }
            if (best < p.size()) {
                const cplx avg = 0.5 * (p[k] + std::conj(p[best]));
                p[k] = avg;
                p[best] = std::conj(avg);
                paired[k] = paired[best] = 1;
            }
        }
    }
    // A pole on the sampled half-line s >= 0 cannot belong to data that are
    // finite there: it is one of the spurious poles AAA places when it
    // starts to fit the data's noise (below the level tol asked for), and it
    // is dropped.
    {
        double scale = 1.0;
        for (double v : Z) scale = std::max(scale, std::fabs(v));
        std::vector<cplx> kept;
        for (const cplx &v : p)
            if (!(v.real() >= 0.0 && std::fabs(v.imag()) <= 1e-9 * (std::abs(v) + 1e-6 * scale)))
                kept.push_back(v);
        p.swap(kept);
    }
    // residues, then drop poles whose term stays below 1e-3 tol_abs on every
    // sample (the spurious pole-zero pairs AAA can leave), and fit again
    std::vector<cplx> c;
    for (int round = 0; round < 2 * GF_MAX_POLES + 2; ++round) {
        if (p.empty()) return fail(GF_EINVAL, "the fit found no pole");
        if (!gf::residues_lsq(Z, F, W, p, c))
            return fail(GF_EINVAL, "the fitted poles are numerically dependent");
        size_t weakest = p.size();
        double wmin = INFINITY;
        for (size_t a = 0; a < p.size(); ++a) {
            double big = 0.0;
            for (int i = 0; i < n; ++i) big = std::max(big, W[i] * std::abs(c[a] / (Z[i] - p[a])));
            if (big < wmin) {
                wmin = big;
                weakest = a;
            }
        }
        if (wmin >= 1e-3 * tol_abs) break;
        // real data: a complex pole goes together with its conjugate
        const cplx partner = std::conj(p[weakest]);
        p.erase(p.begin() + weakest);
        if (real && partner.imag() != 0.0)
            for (size_t l = 0; l < p.size(); ++l)
                if (p[l] == partner) {
                    p.erase(p.begin() + l);
                    break;
                }
    }
    if (real) {
        for (size_t a = 0; a < p.size(); ++a) {
            if (p[a].imag() == 0.0) {
                c[a] = c[a].real();
            } else if (p[a].imag() > 0.0) {
                for (size_t l = 0; l < p.size(); ++l)
                    if (p[l] == std::conj(p[a])) {
                        const cplx avg = 0.5 * (c[a] + std::conj(c[l]));
                        c[a] = avg;
                        c[l] = std::conj(avg);
                    }
            }
        }
    }
    for (size_t a = 0; a < p.size(); ++a)
        if (p[a].imag() == 0.0 && p[a].real() >= 0.0)
            return fail(GF_EINVAL, "the fit puts a pole at s = %g on the integration path",
                        p[a].real());
    double err = 0.0;
    for (int i = 0; i < n; ++i) {
        cplx v = 0.0;
        for (size_t a = 0; a < p.size(); ++a) v += c[a] / (Z[i] - p[a]);
        err = std::max(err, W[i] * std::abs(F[i] - v));
    }
    *n_poles = (int)p.size();
    for (size_t a = 0; a < p.size(); ++a) {
        // c / (s - p) = c / (s + m^2) with m^2 = -p
        m2_re[a] = -p[a].real();
        m2_im[a] = p[a].imag() == 0.0 ? 0.0 : -p[a].imag();
        c_re[a] = c[a].real();
        c_im[a] = c[a].imag();
    }
    if (max_err) *max_err = err / fmax;
    return GF_OK;
}
