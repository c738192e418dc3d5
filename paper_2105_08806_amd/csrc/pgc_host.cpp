// Host side of the library: descriptor validation, the FP64 plan tables
// (nodes, maps, sphere rules, Chebyshev and cosine-transform matrices, the
// spreading kernel and its Fourier transform, moment functionals), device
// allocation and the extern "C" entry points declared in pgc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "pgc.h"
#include "pgc_internal.h"

namespace pgc {
namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------- small math

// Gauss-Legendre rule on [-1, 1] by Newton iteration on P_n (three-term
// recurrence), started from the asymptotic node positions.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double t = std::cos(kPi * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double pn = 0.0, dpn = 1.0;
        for (int it = 0; it < 60; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            pn = (n == 0) ? 1.0 : p1;
            const double pm = (n == 1) ? 1.0 : p0;
            dpn = n * (pm - t * pn) / (1.0 - t * t);
            const double step = pn / dpn;
            t -= step;
            if (std::fabs(step) <= 1e-16 * std::fabs(t) + 1e-300) break;
        }
        x[n - 1 - i] = t;
        x[i] = -t;
        const double wi = 2.0 / ((1.0 - t * t) * dpn * dpn);
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
}

// exponential of semicircle kernel on [-1, 1]
double es_kernel(double y, double beta)
{
    if (std::fabs(y) >= 1.0) return 0.0;
    return std::exp(beta * (std::sqrt(1.0 - y * y) - 1.0));
}

// Accuracy of the folded cosine transform at upsampling 2 and 3, measured on
// random points against the direct sum (max error over modes / sum |q|), for
// W = 4..16; entries at 2.5e-14 sit at the FP64 rounding floor.
const double kErrSigma2[] = {1.3e-5, 1.2e-6, 2.3e-7, 2.3e-8, 1.8e-9, 2.4e-10, 3.2e-11,
                             3.4e-12, 2.1e-13, 3.3e-14, 2.5e-14, 2.5e-14, 2.5e-14};
const double kErrSigma3[] = {5.1e-6, 2.5e-7, 2.6e-8, 2.6e-9, 1.9e-10, 1.7e-11, 8.9e-13,
                             9.9e-14, 2.5e-14, 2.5e-14, 2.5e-14, 2.5e-14, 2.5e-14};

double estimated_error(int W, double upsample)
{
    if (std::fabs(upsample - 2.0) < 1e-12) return 3.0 * kErrSigma2[W - 4];
    if (std::fabs(upsample - 3.0) < 1e-12) return 3.0 * kErrSigma3[W - 4];
    // exp(-pi W sqrt(1 - 1/sigma)) decay of the ES kernel, with a safety factor
    return 10.0 * std::exp(-kPi * W * std::sqrt(1.0 - 1.0 / upsample));
}

double beta_for(int W, double upsample)
{
    // beta = 0.98 pi W (1 - 1/(2 sigma)): the shape rule of the ES kernel
    // (2.30 W at sigma = 2)
    return 0.98 * kPi * W * (1.0 - 0.5 / upsample);
}

// Directions per chunk of a streamed point index: as many as the budget holds
// (at least one), spread evenly over the chunks, each chunk under 2^32 ids so
// that 32-bit cursors address it; -1 when one direction alone exceeds that.
int stream_dirs(const Plan& p, int64_t budget)
{
    const int64_t per_dir = p.n_points / p.n_sigma;
    const int64_t max32 = 0xffffffffll / per_dir;
    if (max32 < 1) return -1;
    const int64_t dpc = std::min(max32, std::max<int64_t>(1, budget / (8 * per_dir)));
    const int64_t chunks = (p.n_sigma + dpc - 1) / dpc;
    return (int)((p.n_sigma + chunks - 1) / chunks);
}

int width_for(double tol, double upsample)
{
    for (int W = 4; W <= kMaxWidth; ++W)
        if (estimated_error(W, upsample) <= tol) return W;
    return kMaxWidth;
}

// Monomial coefficients (in s on [-1, 1]) of the degree terms-1 Chebyshev
// interpolant of g on the Chebyshev points of the first kind.
template <class F>
void cheb_interp_monomial(F g, int terms, double* mono)
{
    const int n = terms;
    std::vector<double> fx(n), cc(n, 0.0);
    for (int j = 0; j < n; ++j) fx[j] = g(std::cos(kPi * (j + 0.5) / n));
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += fx[j] * std::cos(kPi * k * (j + 0.5) / n);
        cc[k] = (k == 0 ? 1.0 : 2.0) * s / n;
    }
    // sum_k cc_k T_k(s) -> monomials, T_{k+1} = 2 s T_k - T_{k-1}
    std::vector<double> tm(n, 0.0), t(n, 0.0), tn(n, 0.0);
    for (int d = 0; d < n; ++d) mono[d] = 0.0;
    tm[0] = 1.0;
    mono[0] += cc[0];
    if (n > 1) {
        t[1] = 1.0;
        mono[1] += cc[1];
    }
    for (int k = 2; k < n; ++k) {
        for (int d = 0; d < n; ++d) tn[d] = -tm[d] + (d > 0 ? 2.0 * t[d - 1] : 0.0);
        for (int d = 0; d < n; ++d) mono[d] += cc[k] * tn[d];
        tm = t;
        t = tn;
    }
}

// v(xi) for xi = cos(theta') written with the angle, for accuracy near +-1:
// r = 0: S atanh(cos a) = S ln(cot(a/2)); r = 1: S cos a / sin a.
double v_of_angle(int map, double S, double a)
{
    if (map == 0) return S * std::log(1.0 / std::tan(0.5 * a));
    return S * std::cos(a) / std::sin(a);
}

double cheb_norm_sqrt(int k) { return std::sqrt(k == 0 ? kPi : 0.5 * kPi); }

// ---------------------------------------------------------------- validation

pgc_status resolve(const pgc_plan_desc& d, Plan& p)
{
    if (d.dim != 2 && d.dim != 3) return PGC_ERR_INVALID_ARG;
    if (d.n_modes < 3) return PGC_ERR_INVALID_ARG;
    if (d.map != PGC_MAP_LOG && d.map != PGC_MAP_ALGEBRAIC) return PGC_ERR_INVALID_ARG;
    if (!(d.scale > 0.0) || !std::isfinite(d.scale)) return PGC_ERR_INVALID_ARG;
    if (d.scale_mode != PGC_SCALE_DIRECT && d.scale_mode != PGC_SCALE_FROM_DOMAIN)
        return PGC_ERR_INVALID_ARG;
    if (d.kernel != PGC_KERNEL_MAXWELL && d.kernel != PGC_KERNEL_VHS && d.kernel != PGC_KERNEL_ANISO)
        return PGC_ERR_INVALID_ARG;
    if (d.kernel != PGC_KERNEL_MAXWELL && !(d.kernel_gamma >= 0.0 && d.kernel_gamma <= 1.0))
        return PGC_ERR_INVALID_ARG;
    if (d.kernel == PGC_KERNEL_ANISO && !(d.kernel_aniso >= -1.0 && d.kernel_aniso <= 10.0))
        return PGC_ERR_INVALID_ARG;
    if (d.kernel_b0 < 0.0 || !std::isfinite(d.kernel_b0)) return PGC_ERR_INVALID_ARG;
    if (d.precision != PGC_PRECISION_FP64 && d.precision != PGC_PRECISION_FP32)
        return PGC_ERR_INVALID_ARG;
    if (d.nufft_tol < 0.0 || d.upsample < 0.0) return PGC_ERR_INVALID_ARG;
    if (d.upsample != 0.0 && (d.upsample < 1.5 || d.upsample > 4.0)) return PGC_ERR_INVALID_ARG;
    if (d.kernel_width != 0 && (d.kernel_width < 4 || d.kernel_width > kMaxWidth))
        return PGC_ERR_INVALID_ARG;
    if (d.slab_planes < 0 || d.n_chunks < 0) return PGC_ERR_INVALID_ARG;
    if (d.block_threads != 0 && d.block_threads != 256 && d.block_threads != 512 &&
        d.block_threads != 1024)
        return PGC_ERR_INVALID_ARG;
    if (d.gain_mode < 0 || d.gain_mode > 3) return PGC_ERR_INVALID_ARG;
    if (d.deterministic != 0 && d.deterministic != 1) return PGC_ERR_INVALID_ARG;
    if (d.index_bytes < 0) return PGC_ERR_INVALID_ARG;

    p.dim = d.dim;
    p.N = d.n_modes;
    p.m_v = d.m_v == 0 ? d.n_modes + 1 : d.m_v;
    if (p.m_v < 3) return PGC_ERR_INVALID_ARG;
    p.ni = p.m_v - 2;
    p.map = d.map;
    p.kernel = d.kernel;
    p.precision = d.precision;
    p.gamma = d.kernel == PGC_KERNEL_MAXWELL ? 0.0 : d.kernel_gamma;
    p.aniso = d.kernel == PGC_KERNEL_ANISO ? d.kernel_aniso : 0.0;
    p.elt = p.precision == PGC_PRECISION_FP64 ? sizeof(double) : sizeof(float);

    // map scale: direct, or the adaptive choice v(xi_2) = -L, v(xi_{m_v-1}) = L
    const double a1 = kPi / (p.m_v - 1);  // angle of the second node from the end
    if (d.scale_mode == PGC_SCALE_DIRECT) p.S = d.scale;
    else p.S = d.map == PGC_MAP_LOG ? d.scale / std::log(1.0 / std::tan(0.5 * a1))
                                    : d.scale * std::tan(a1);

    // sphere rule
    p.sigma.clear();
    p.sigma_w.clear();
    if (d.sphere == PGC_SPHERE_UNIFORM_2D) {
        if (p.dim != 2 || d.n_sigma < 2 || (d.n_sigma & 1)) return PGC_ERR_INVALID_ARG;
        for (int s = 0; s < d.n_sigma; ++s) {
            const double th = 2.0 * kPi * s / d.n_sigma;
            p.sigma.push_back(std::cos(th));
            p.sigma.push_back(std::sin(th));
            p.sigma_w.push_back(2.0 * kPi / d.n_sigma);
        }
    } else if (d.sphere == PGC_SPHERE_PRODUCT_3D) {
        if (p.dim != 3 || d.n_theta < 1 || d.n_phi < 2 || (d.n_phi & 1)) return PGC_ERR_INVALID_ARG;
        std::vector<double> x, w;
        gauss_legendre(d.n_theta, x, w);
        for (int a = 0; a < d.n_theta; ++a) {
            const double st = std::sqrt(std::max(0.0, 1.0 - x[a] * x[a]));
            for (int b = 0; b < d.n_phi; ++b) {
                const double ph = 2.0 * kPi * b / d.n_phi;
                p.sigma.push_back(st * std::cos(ph));
                p.sigma.push_back(st * std::sin(ph));
                p.sigma.push_back(x[a]);
                p.sigma_w.push_back(w[a] * 2.0 * kPi / d.n_phi);
            }
        }
    } else if (d.sphere == PGC_SPHERE_USER) {
        if (d.n_sigma < 1 || !d.user_sigma_host || !d.user_weights_host) return PGC_ERR_INVALID_ARG;
        for (int s = 0; s < d.n_sigma; ++s) {
            double nrm = 0.0;
            for (int l = 0; l < p.dim; ++l) {
                const double c = d.user_sigma_host[s * p.dim + l];
                nrm += c * c;
                p.sigma.push_back(c);
            }
            const double wt = d.user_weights_host[s];
            if (std::fabs(nrm - 1.0) > 1e-12 || !(wt > 0.0) || !std::isfinite(wt))
                return PGC_ERR_INVALID_ARG;
            p.sigma_w.push_back(wt);
        }
    } else {
        return PGC_ERR_INVALID_ARG;
    }
    p.n_sigma = (int)p.sigma_w.size();
    // antipodal symmetry: the discrete energy balance pairs (s, i, j) with
    // (-s, j, i), so every direction needs its opposite with the same weight
    for (int s = 0; s < p.n_sigma; ++s) {
        bool found = false;
        for (int t = 0; t < p.n_sigma && !found; ++t) {
            double dist = 0.0;
            for (int l = 0; l < p.dim; ++l) {
                const double e = p.sigma[s * p.dim + l] + p.sigma[t * p.dim + l];
                dist += e * e;
            }
            found = dist < 1e-20 && std::fabs(p.sigma_w[s] - p.sigma_w[t]) <= 1e-12 * p.sigma_w[s];
        }
        if (!found) return PGC_ERR_INVALID_ARG;
    }
    p.wsum = 0.0;
    for (double w : p.sigma_w) p.wsum += w;
    const double area = p.dim == 2 ? 2.0 * kPi : 4.0 * kPi;
    p.b0 = d.kernel_b0 > 0.0 ? d.kernel_b0 : 1.0 / area;

    // spreading kernel and fine grid
    // upsampling 3 trades a 1.5^d larger fine grid (cheap: one cosine transform per
    // evaluation) for a narrower kernel (W^d work per point): measured fastest
    p.upsample = d.upsample > 0.0 ? d.upsample : 3.0;
    p.tol = d.nufft_tol > 0.0 ? d.nufft_tol : (p.precision == PGC_PRECISION_FP64 ? 5e-13 : 1e-6);
    p.W = d.kernel_width > 0 ? d.kernel_width : width_for(p.tol, p.upsample);
    p.gain_mode = d.gain_mode == 1 ? kGainSlab : kGainBinned;
    // the binned scheme: kernels built for W <= 14, and point ids that hold the
    // first-dimension nodes in 8 bits, the direction in 10 and the pairs of the
    // other dimensions in 16 (n_i <= 256, n_sigma <= 1024)
    if (p.gain_mode == kGainBinned && (p.W > 14 || p.ni > kMaxBinnedNodes || p.n_sigma > kMaxBinnedDirections)) {
        if (d.gain_mode >= 2) return PGC_ERR_UNSUPPORTED;
        p.gain_mode = kGainSlab;
    }
    // the matrix-core binned gain: FP64 3D plans with W <= 12
    // an angle-dependent rate needs the per-direction orbit weights that only
    // the binned vector kernel forms (the slab scheme reads direction-free
    // orbit sums, the matrix-core variant has no such path)
    if (p.kernel == PGC_KERNEL_ANISO && (p.gain_mode != kGainBinned || d.gain_mode == 3))
        return PGC_ERR_UNSUPPORTED;
    p.mfma = d.gain_mode == 3;
    if (p.mfma && (p.precision != PGC_PRECISION_FP64 || p.dim != 3 || p.W < 4 || p.W > 12))
        return PGC_ERR_UNSUPPORTED;
    // the fixed-order gather reads the tiles of the binned vector kernel
    p.deterministic = d.deterministic == 1;
    if (p.deterministic && (p.gain_mode != kGainBinned || p.mfma)) return PGC_ERR_UNSUPPORTED;
    p.auto_gain = d.gain_mode == 0;
    p.terms = poly_terms(p.W);
    p.beta = beta_for(p.W, p.upsample);
    // n >= 2 sigma N, and n >= 4 W so that a footprint folds back at most once and
    // the kernel stays narrow against the period (small N only: a finer grid is
    // merely a larger upsampling factor)
    p.n = std::max(2 * (int)std::ceil(p.upsample * p.N), 4 * p.W);
    p.nh = p.n / 2;
    p.ng = p.nh + 1;
    p.h = 2.0 * kPi / p.n;

    auto ipow = [](int64_t b, int e) {
        int64_t r = 1;
        for (int i = 0; i < e; ++i) r *= b;
        return r;
    };
    p.nid = ipow(p.ni, p.dim);
    p.Nd = ipow(p.N, p.dim);
    p.ngd = ipow(p.ng, p.dim);
    p.np = p.ni * (p.ni + 1) / 2;
    p.n_triples = (int64_t)p.n_sigma * p.nid * p.nid;
    p.n_points = (int64_t)p.n_sigma * ipow(p.np, p.dim);
    // a budget below the whole index streams it in direction chunks (the
    // deterministic gather needs the whole index)
    p.index_budget = d.index_bytes;
    if (p.gain_mode == kGainBinned && p.index_budget > 0 && p.n_points * 8 > p.index_budget) {
        if (p.deterministic) return PGC_ERR_UNSUPPORTED;
        p.bins.dirs_per_chunk = stream_dirs(p, p.index_budget);
        if (p.bins.dirs_per_chunk < 0) return PGC_ERR_UNSUPPORTED;
    }
    // a unit is (a_1, s): the smaller first-dimension node of a pair and a direction
    p.n_units = (int64_t)p.n_sigma * p.ni;

    // LDS slabs along the first dimension
    const int64_t plane_bytes = ipow(p.ng, p.dim - 1) * (int64_t)sizeof(double);  // FP64 cells
    const int64_t max_planes = kLdsBudget / plane_bytes;
    if (max_planes < 1) return PGC_ERR_UNSUPPORTED;
    int planes = d.slab_planes > 0 ? d.slab_planes : (int)std::min<int64_t>(p.ng, max_planes);
    if (planes > max_planes) return PGC_ERR_UNSUPPORTED;
    planes = std::min(planes, p.ng);
    p.n_slabs = (p.ng + planes - 1) / planes;
    p.slab_planes = (p.ng + p.n_slabs - 1) / p.n_slabs;

    // chunks of collision units: enough workgroups to fill 256 CUs several times
    int64_t chunks = d.n_chunks > 0 ? d.n_chunks : std::max<int64_t>(1, 2048 / p.n_slabs);
    chunks = std::min<int64_t>(chunks, p.n_units);
    const int64_t cap = std::max<int64_t>(1, (int64_t)(1ll << 31) / (p.ngd * (int64_t)sizeof(double)));
    chunks = std::max<int64_t>(1, std::min(chunks, cap));
    p.units_per_chunk = (p.n_units + chunks - 1) / chunks;
    p.n_chunks = (int)((p.n_units + p.units_per_chunk - 1) / p.units_per_chunk);
    if ((int64_t)p.n_chunks > 2147483647ll) return PGC_ERR_UNSUPPORTED;
    const int max_threads = p.precision == PGC_PRECISION_FP64 ? 256 : 1024;
    if (d.block_threads > max_threads) return PGC_ERR_UNSUPPORTED;
    p.block_threads = d.block_threads > 0 ? d.block_threads : max_threads;
    return PGC_OK;
}

// ---------------------------------------------------------------- tables

// The footprint corner of a point in one dimension is ceil(z/h - W/2), the
// smallest k with z <= (k + W/2) h.  The transform angle z decreases with the
// velocity (r = 0: z = 2 atan(exp(-v/S)); r = 1: z = atan2(1, v/S)), so that
// is the smallest k with v >= V_k, V_k = -S ln tan(Z_k/2) (r = 0) or
// S cot Z_k (r = 1), Z_k = (k + W/2) h; +inf where Z_k <= 0, -inf where
// Z_k >= pi.  The table holds V_k for k = -off - 1 .. n_h + 2 - off (the bin
// coordinate k + off runs over -1 .. n_h + 2 before the clamp to the bins), in
// long double rounded once, so that binning needs no transcendental per point.
void build_bin_thresholds(Plan& p)
{
    const int nb = p.nh + 2, off = p.W / 2;
    const long double pi = acosl(-1.0L), h = pi / p.nh, hw = 0.5L * p.W;
    p.bin_vthr.assign((size_t)nb + 2, 0.0);
    for (int j = 0; j < nb + 2; ++j) {
        const int k = j - off - 1;
        const long double Z = (k + hw) * h;
        double V;
        if (Z <= 0.0L)
            V = HUGE_VAL;
        else if (Z >= pi)
            V = -HUGE_VAL;
        else if (p.map == PGC_MAP_LOG)
            V = (double)(-(long double)p.S * logl(tanl(0.5L * Z)));
        else
            V = (double)((long double)p.S * cosl(Z) / sinl(Z));
        p.bin_vthr[j] = V;
    }
}

// Monomial coefficients (in x) of the Chebyshev interpolant of degree
// deg <= kCellFitDeg of f on [-1, 1], at the Chebyshev points of the first
// kind, in long double; rounded to FP64 into out[0 .. deg].
template <typename F>
static void cheb_fit_monomials(const F& f, double* out, int deg = kCellFitDeg)
{
    const int n = deg + 1;
    const long double pi = acosl(-1.0L);
    long double fx[kCellFitDeg + 1], cc[kCellFitDeg + 1], tm[kCellFitDeg + 1], t[kCellFitDeg + 1],
        tn[kCellFitDeg + 1], mono[kCellFitDeg + 1];
    for (int j = 0; j < n; ++j) fx[j] = f(cosl(pi * (j + 0.5L) / n));
    for (int k = 0; k < n; ++k) {
        long double acc = 0.0L;
        for (int j = 0; j < n; ++j) acc += fx[j] * cosl(pi * k * (j + 0.5L) / n);
        cc[k] = (k == 0 ? 1.0L : 2.0L) * acc / n;
    }
    // sum_k cc_k T_k(x) -> monomials with T_{k+1} = 2 x T_k - T_{k-1}
    for (int e = 0; e < n; ++e) tm[e] = t[e] = mono[e] = 0.0L;
    tm[0] = 1.0L;
    t[1] = 1.0L;
    mono[0] = cc[0];
    mono[1] = cc[1];
    for (int k = 2; k < n; ++k) {
        for (int e = 0; e < n; ++e) tn[e] = -tm[e] + (e > 0 ? 2.0L * t[e - 1] : 0.0L);
        for (int e = 0; e < n; ++e) mono[e] += cc[k] * tn[e];
        for (int e = 0; e < n; ++e) {
            tm[e] = t[e];
            t[e] = tn[e];
        }
    }
    for (int k = 0; k < n; ++k) out[k] = (double)mono[k];
}

// The stored (rounded) polynomial c[0 .. deg] at x, in long double
static long double cheb_fit_eval(const double* c, long double x, int deg = kCellFitDeg)
{
    long double v = c[deg];
    for (int k = deg - 1; k >= 0; --k) v = v * x + c[k];
    return v;
}

// For every bin coordinate c of one dimension (footprint corner t0 = c - W/2,
// int division) the points of the cell have z in ((t0 - 1 + W/2) h, (t0 + W/2) h]
// and kernel offset s = 2 t0 + W - 1 - 2 z / h.  With z = pi/2 - 2 atan(w) the
// offset is a smooth function of w over the cell's w-interval [w_c - d, w_c + d];
// it is interpolated at the Chebyshev points of x = (w - w_c)/d in long double
// and stored as w_c, 1/d and the monomial coefficients in x.
//
// Every cell whose z-interval lies inside (0, pi) also gets a fit in the scaled
// velocity t = v/S itself, over the cell's t-interval [t_c - d, t_c + d]: the
// offset s(t) and the map factor m2(t) (cosh t for r = 0, 1 + t^2 for r = 1),
// each a polynomial of the same degree in x = (t - t_c)/d.  The functions are
// analytic within distance pi/2 (r = 0) or 1 (r = 1) of the real axis, so the
// interpolants converge on every cell whose t-interval is narrow against that;
// a cell keeps the velocity fit only where the stored polynomials are within
// 5e-16 of s and within 5e-16 relative of m2 (every cell but the one or few
// at each end of the grid), else 1/d = 0 marks it and its points take the map
// to w.  The velocity fit saves the exponential and reciprocals of the map.
// FP32 plans, whose kernel values are rounded to FP32, fit to degree 7 within
// 2e-10, which covers as many cells.
void build_cell_fits(Plan& p)
{
    constexpr int K = kCellFitDeg;
    const bool fp64 = p.precision == PGC_PRECISION_FP64;
    const int kv = fp64 ? kCellFitDeg : kCellFitDegV32;
    const long double kTol = fp64 ? 5e-16L : 2e-10L;
    const int nb = p.nh + 2, off = p.W / 2;
    const long double pi = acosl(-1.0L), h = pi / p.nh, hw = 0.5L * p.W;
    p.cellfit.assign((size_t)nb * kCellFitStride, 0.0);
    p.cellfit_v.assign((size_t)nb * kCellFitVStride, 0.0);
    p.cellfit_err = 0.0;
    p.cellfit_v_cells = 0;
    const bool log_map = p.map == PGC_MAP_LOG;
    for (int c = 0; c < nb; ++c) {
        const int t0 = c - off;
        const long double zlo = std::max(0.0L, (t0 - 1 + hw) * h);
        const long double zhi = std::min(pi, (t0 + hw) * h);
        double* out = p.cellfit.data() + (size_t)c * kCellFitStride;
        if (!(zhi > zlo)) continue;  // no point has this corner
        const long double wlo = tanl(0.25L * pi - 0.5L * zhi), whi = tanl(0.25L * pi - 0.5L * zlo);
        const long double wc = 0.5L * (wlo + whi), d = 0.5L * (whi - wlo);
        auto offset = [&](long double x) {
            const long double z = 0.5L * pi - 2.0L * atanl(wc + d * x);
            return (long double)(2 * t0 + p.W - 1) - 2.0L * z / h;
        };
        out[0] = (double)wc;
        out[1] = (double)(1.0L / d);
        cheb_fit_monomials(offset, out + 2);
        // deviation of the stored (rounded) fit from the exact offset
        for (int i = 0; i <= 64; ++i) {
            const long double x = -1.0L + i / 32.0L;
            p.cellfit_err = std::max(p.cellfit_err, (double)fabsl(cheb_fit_eval(out + 2, x) - offset(x)));
        }

        // the fit in the velocity
        if (!(zlo > 0.0L && zhi < pi)) continue;
        auto t_of_z = [&](long double z) { return log_map ? -logl(tanl(0.5L * z)) : cosl(z) / sinl(z); };
        const long double ta = t_of_z(zhi), tb = t_of_z(zlo);
        if (!(std::isfinite((double)ta) && std::isfinite((double)tb) && tb > ta)) continue;
        const long double tc = 0.5L * (ta + tb), dt = 0.5L * (tb - ta);
        auto offset_t = [&](long double x) {
            const long double t = tc + dt * x;
            const long double z = log_map ? 2.0L * atanl(expl(-t)) : 0.5L * pi - atanl(t);
            return (long double)(2 * t0 + p.W - 1) - 2.0L * z / h;
        };
        auto m2_t = [&](long double x) {
            const long double t = tc + dt * x;
            return log_map ? coshl(t) : 1.0L + t * t;
        };
        double fv[kCellFitVStride] = {};
        fv[0] = (double)tc;
        fv[1] = (double)(1.0L / dt);
        cheb_fit_monomials(offset_t, fv + 2, kv);
        cheb_fit_monomials(m2_t, fv + 3 + K, kv);
        bool good = true;
        for (int i = 0; i <= 256 && good; ++i) {
            const long double x = -1.0L + i / 128.0L;
            const long double es = fabsl(cheb_fit_eval(fv + 2, x, kv) - offset_t(x));
            const long double em = fabsl(cheb_fit_eval(fv + 3 + K, x, kv) / m2_t(x) - 1.0L);
            good = es <= kTol && em <= kTol;  // false for NaN too
        }
        if (!good) continue;
        std::copy(fv, fv + kCellFitVStride, p.cellfit_v.data() + (size_t)c * kCellFitVStride);
        ++p.cellfit_v_cells;
    }
}

void build_tables(Plan& p)
{
    const int m = p.m_v;
    p.xi_all.assign(m, 0.0);
    p.v_all.assign(m, 0.0);
    p.w_all.assign(m, 0.0);
    for (int j = 0; j < m; ++j) {
        // xi_j = -cos(theta_j) = cos(pi - theta_j), theta_j = pi j/(m-1)
        const double a = kPi * (m - 1 - j) / (m - 1);
        p.xi_all[j] = (j == 0) ? -1.0 : (j == m - 1 ? 1.0 : std::cos(a));
        const bool end = (j == 0 || j == m - 1);
        p.w_all[j] = end ? kPi / (2.0 * (m - 1)) : kPi / (m - 1);
        p.v_all[j] = end ? (j == 0 ? -HUGE_VAL : HUGE_VAL) : v_of_angle(p.map, p.S, a);
    }
    const int ni = p.ni, N = p.N;
    p.v1.assign(ni, 0.0);
    p.w1.assign(ni, 0.0);
    p.mu21.assign(ni, 0.0);
    p.C.assign((size_t)ni * N, 0.0);
    p.CT.assign((size_t)N * ni, 0.0);
    for (int i = 0; i < ni; ++i) {
        const int j = i + 1;
        const double a = kPi * (m - 1 - j) / (m - 1);
        const double sa = std::sin(a);  // sqrt(1 - xi^2)
        p.v1[i] = p.v_all[j];
        p.w1[i] = p.w_all[j];
        p.mu21[i] = (p.map == PGC_MAP_LOG ? sa : sa * sa) / p.S;
        for (int k = 0; k < N; ++k) {
            const double tk = std::cos(k * a) / cheb_norm_sqrt(k);  // T_k(cos a) = cos(k a)
            p.C[(size_t)i * N + k] = tk;
            p.CT[(size_t)k * ni + i] = tk;
        }
    }

    // kernel cells: g_a(s) = psi((a - W/2 + (s+1)/2) 2/W), s in [-1, 1]
    const int W = p.W, terms = p.terms;
    p.poly.assign((size_t)terms * W, 0.0);
    std::vector<double> mono(terms);
    for (int a = 0; a < W; ++a) {
        cheb_interp_monomial(
            [&](double s) { return es_kernel((a - 0.5 * W + 0.5 * (s + 1.0)) * 2.0 / W, p.beta); },
            terms, mono.data());
        for (int d = 0; d < terms; ++d) p.poly[(size_t)d * W + a] = mono[d];
    }

    // even and odd parts of the cells a < W/2 (cell W-1-a at s is cell a at -s)
    {
        const int H = (W + 1) / 2, HP = W / 2, NE = (terms + 1) / 2, NO = terms / 2;
        p.kpoly_eo.assign((size_t)NE * H + (size_t)NO * HP, 0.0);
        for (int j = 0; j < NE; ++j)
            for (int a = 0; a < H; ++a) p.kpoly_eo[(size_t)j * H + a] = p.poly[(size_t)(2 * j) * W + a];
        for (int j = 0; j < NO; ++j)
            for (int a = 0; a < HP; ++a)
                p.kpoly_eo[(size_t)NE * H + (size_t)j * HP + a] = p.poly[(size_t)(2 * j + 1) * W + a];
    }
    build_cell_fits(p);
    build_bin_thresholds(p);

    // Fourier transform of the kernel in z units, psi^(k) = int psi(x/alpha) cos(k x) dx,
    // alpha = W h / 2, by a 256-point Gauss-Legendre rule in x/alpha
    std::vector<double> gx, gw;
    gauss_legendre(256, gx, gw);
    const double alpha = 0.5 * W * p.h;
    std::vector<double> psihat(N);
    for (int k = 0; k < N; ++k) {
        double s = 0.0;
        for (size_t q = 0; q < gx.size(); ++q)
            s += gw[q] * es_kernel(gx[q], p.beta) * std::cos(k * alpha * gx[q]);
        psihat[k] = alpha * s;
    }
    // E[k][m] = cos(k m h) h / (psi^(k) sqrt(c_k)): cosine transform of the folded
    // grid, deconvolution and the Chebyshev normalisation in one matrix
    p.E.assign((size_t)N * p.ng, 0.0);
    for (int k = 0; k < N; ++k)
        for (int mm = 0; mm < p.ng; ++mm)
            p.E[(size_t)k * p.ng + mm] = std::cos((double)k * mm * p.h) * p.h /
                                         (psihat[k] * cheb_norm_sqrt(k));

    // v'_1 window of each slab: a point at grid coordinate x = z/h touches the
    // folded planes [p0, p1) iff x lies in [p0 - W/2, p1 - 1 + W/2] (reflections
    // at 0 and pi only add planes nearer the walls); one extra cell of margin.
    p.slab_vlo.assign(p.n_slabs, 0.0);
    p.slab_vhi.assign(p.n_slabs, 0.0);
    for (int b = 0; b < p.n_slabs; ++b) {
        const int p0 = b * p.slab_planes;
        const int p1 = std::min(p.ng, p0 + p.slab_planes);
        const double xlo = p0 - 0.5 * W - 1.0;
        const double xhi = (p1 - 1) + 0.5 * W + 1.0;
        const double zlo = xlo * p.h, zhi = xhi * p.h;
        // z = arccos(xi(v)) decreases in v
        p.slab_vhi[b] = zlo <= 0.0 ? HUGE_VAL : v_of_angle(p.map, p.S, zlo);
        p.slab_vlo[b] = zhi >= kPi ? -HUGE_VAL : v_of_angle(p.map, p.S, zhi);
    }

    // moment functionals m_p[k] = int v^p T~_k(v) dv, p = 0, 1, 2
    p.mom.assign(3 * (size_t)N, 0.0);
    const double S = p.S;
    if (p.map == PGC_MAP_ALGEBRAIC) {
        // xi = cos a: mu^4 dv = sin(a)^2/S da-type closed forms
        for (int k = 0; k < N; ++k) {
            const double sc = cheb_norm_sqrt(k);
            p.mom[k] = (k == 0 ? kPi / 2 : (k == 2 ? -kPi / 4 : 0.0)) / (S * sc);
            p.mom[2 * N + k] = S * (k == 0 ? kPi / 2 : (k == 2 ? kPi / 4 : 0.0)) / sc;
            // int_{-1}^{1} xi T_k(xi) dxi: nonzero for odd k
            double m1 = 0.0;
            if (k & 1) {
                auto int_t = [](int n) { return (n & 1) ? 0.0 : 2.0 / (1.0 - (double)n * n); };
                m1 = 0.5 * (int_t(k + 1) + int_t(k - 1));
            }
            p.mom[N + k] = m1 / sc;
        }
    } else {
        // r = 0: m_p[k] = S^p/(S sqrt c_k) int y^p T_k(tanh y) sech^2 y dy over R,
        // composite 16-point Gauss-Legendre on [-48, 48] in panels of width 1
        std::vector<double> px, pw;
        gauss_legendre(16, px, pw);
        std::vector<double> acc(3 * (size_t)N, 0.0);
        for (int panel = -48; panel < 48; ++panel) {
            for (int q = 0; q < 16; ++q) {
                const double y = panel + 0.5 + 0.5 * px[q];
                const double c = std::cosh(y);
                const double wgt = 0.5 * pw[q] / (c * c);
                const double ang = std::acos(std::tanh(y));
                for (int k = 0; k < N; ++k) {
                    const double t = std::cos(k * ang) * wgt;
                    acc[k] += t;
                    acc[N + k] += t * y;
                    acc[2 * N + k] += t * y * y;
                }
            }
        }
        for (int k = 0; k < N; ++k) {
            const double sc = cheb_norm_sqrt(k);
            p.mom[k] = acc[k] / (S * sc);
            p.mom[N + k] = acc[N + k] / sc;
            p.mom[2 * N + k] = S * acc[2 * N + k] / sc;
        }
    }
}

// ---------------------------------------------------------------- device memory

hipError_t dev_alloc(Plan& p, void** ptr, size_t bytes)
{
    *ptr = nullptr;
    if (bytes == 0) bytes = 16;
    p.allocations.push_back(nullptr);  // the slot first: a throwing push_back leaks no device memory
    hipError_t e = hipMalloc(&p.allocations.back(), bytes);
    if (e != hipSuccess) {
        p.allocations.pop_back();
        return e;
    }
    *ptr = p.allocations.back();
    p.workspace_bytes += (int64_t)bytes;
    return hipSuccess;
}

// FP64 tables (the dense transforms use them for both plan precisions)
hipError_t upload64(Plan& p, double** dst, const std::vector<double>& src, hipStream_t s)
{
    void* d = nullptr;
    hipError_t e = dev_alloc(p, &d, src.size() * sizeof(double));
    *dst = static_cast<double*>(d);
    if (e != hipSuccess || src.empty()) return e;
    return hipMemcpyAsync(d, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice, s);
}

// tables of the gain kernels, in the plan precision
hipError_t upload(Plan& p, void** dst, const std::vector<double>& src, hipStream_t s)
{
    hipError_t e = dev_alloc(p, dst, src.size() * p.elt);
    if (e != hipSuccess || src.empty()) return e;
    if (p.precision == PGC_PRECISION_FP64)
        return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice, s);
    std::vector<float> f(src.begin(), src.end());
    e = hipMemcpyAsync(*dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);  // f is about to go out of scope
}

void free_all(Plan& p)
{
    for (void* ptr : p.allocations) (void)hipFree(ptr);
    p.allocations.clear();
}

pgc_status from_hip(hipError_t e) { return status_of(e); }

// Sort the merged points by the base cell of their footprint: count per bin on
// the device, prefix sums and the work-item list on the host, then scatter the
// point ids.  Temporaries are freed before returning.
hipError_t build_stream(Plan& p, hipStream_t s);

hipError_t build_bins(Plan& p, hipStream_t s)
{
    BinIndex& B = p.bins;
    B.nb = p.nh + 2;
    B.off = p.W / 2;
    int64_t nbins = 1;
    for (int l = 0; l < p.dim; ++l) nbins *= B.nb;
    B.nbins = nbins;
    if (B.dirs_per_chunk > 0) return build_stream(p, s);
    unsigned int* count = nullptr;
    unsigned long long* cursor = nullptr;
    std::vector<unsigned int> hc(nbins);  // before the temporary, which nothing below may leak
    hipError_t e = hipMalloc(&count, nbins * sizeof(unsigned int));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(count, 0, nbins * sizeof(unsigned int), s);
    if (e == hipSuccess) e = launch_bin_build(p, count, nullptr, nullptr, nullptr, 0, 0, p.n_sigma, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), count, nbins * sizeof(unsigned int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(count);
    if (e != hipSuccess) return e;

    std::vector<unsigned long long> begin(nbins);
    unsigned long long total = 0;
    for (int64_t b = 0; b < nbins; ++b) {
        begin[b] = total;
        total += hc[b];
    }
    if ((int64_t)total != p.n_points) return hipErrorUnknown;  // every merged point has one bin

    struct Item {
        int bin;
        long long begin;
        int count;
    };
    std::vector<Item> items;
    for (int64_t b = 0; b < nbins; ++b)
        for (unsigned int o = 0; o < hc[b]; o += kBinChunk)
            items.push_back({(int)b, (long long)(begin[b] + o), (int)std::min<unsigned int>(kBinChunk, hc[b] - o)});
    std::vector<int> orig_bin, orig_count;  // the unsorted order (deterministic plans)
    if (p.deterministic) {
        orig_bin.resize(items.size());
        orig_count.resize(items.size());
        for (size_t k = 0; k < items.size(); ++k) {
            orig_bin[k] = items[k].bin;
            orig_count[k] = items[k].count;
        }
    }
    // full runs first: the long items start early and the short ones fill the tail
    std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.count > y.count; });
    B.n_items = (int64_t)items.size();
    std::vector<int> ib(items.size()), ic(items.size());
    std::vector<long long> ibeg(items.size());
    for (size_t k = 0; k < items.size(); ++k) {
        ib[k] = items[k].bin;
        ibeg[k] = items[k].begin;
        ic[k] = items[k].count;
    }
    void* d = nullptr;
    B.id_bytes = (int64_t)std::max<unsigned long long>(1, total) * 8;
    if ((e = dev_alloc(p, &d, (size_t)B.id_bytes)) != hipSuccess) return e;
    B.ids = static_cast<unsigned long long*>(d);
    if ((e = dev_alloc(p, &d, std::max<size_t>(1, ib.size()) * sizeof(int))) != hipSuccess) return e;
    B.item_bin = static_cast<int*>(d);
    if ((e = dev_alloc(p, &d, std::max<size_t>(1, ibeg.size()) * sizeof(long long))) != hipSuccess) return e;
    B.item_begin = static_cast<long long*>(d);
    if ((e = dev_alloc(p, &d, std::max<size_t>(1, ic.size()) * sizeof(int))) != hipSuccess) return e;
    B.item_count = static_cast<int*>(d);
    if (!items.empty()) {
        if ((e = hipMemcpyAsync(B.item_bin, ib.data(), ib.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(B.item_begin, ibeg.data(), ibeg.size() * sizeof(long long), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(B.item_count, ic.data(), ic.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    }
    if (p.deterministic) {
        // runs of every bin in run order: before the sort the items are grouped
        // by bin and ordered by run, so the sorted position of each original
        // item, taken in original order, is the CSR list
        std::vector<int> bptr(nbins + 1, 0), blist(items.size());
        std::vector<int> pos(items.size());
        {
            std::vector<int> idx(items.size());
            for (size_t k = 0; k < idx.size(); ++k) idx[k] = (int)k;
            // the same stable order as the sort above, on the original indices
            std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return orig_count[x] > orig_count[y]; });
            for (size_t k = 0; k < idx.size(); ++k) pos[idx[k]] = (int)k;
        }
        for (size_t k = 0; k < orig_bin.size(); ++k) {
            bptr[orig_bin[k] + 1] += 1;
            blist[k] = pos[k];
        }
        for (int64_t b = 0; b < nbins; ++b) bptr[b + 1] += bptr[b];
        int64_t cells = 1;
        for (int l = 0; l < p.dim; ++l) cells *= p.W;
        B.tile_bytes = (int64_t)items.size() * cells * (int64_t)sizeof(double);
        if ((e = dev_alloc(p, &d, bptr.size() * sizeof(int))) != hipSuccess) return e;
        B.bin_ptr = static_cast<int*>(d);
        if ((e = dev_alloc(p, &d, std::max<size_t>(1, blist.size()) * sizeof(int))) != hipSuccess) return e;
        B.bin_items = static_cast<int*>(d);
        if ((e = dev_alloc(p, &d, std::max<int64_t>(8, B.tile_bytes))) != hipSuccess) return e;
        B.tiles = static_cast<double*>(d);
        if ((e = hipMemcpyAsync(B.bin_ptr, bptr.data(), bptr.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        if (!blist.empty() &&
            (e = hipMemcpyAsync(B.bin_items, blist.data(), blist.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;  // the host vectors go out of scope
    }
    if ((e = hipMalloc(&cursor, nbins * sizeof(unsigned long long))) != hipSuccess) return e;
    e = hipMemcpyAsync(cursor, begin.data(), nbins * sizeof(unsigned long long), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_bin_build(p, nullptr, cursor, nullptr, B.ids, 1, 0, p.n_sigma, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(cursor);
    if (e == hipSuccess && p.deterministic) {
        // the scatter's order inside a bin varies between builds: sort it away
        // (58 id bits: b1 8, a1 8, s 10, p2 16, p3 16)
        begin.push_back(total);
        e = sort_bin_ids(B.ids, begin, 58, s);
    }
    B.n_chunks = 1;
    B.chunk_s0 = {0, p.n_sigma};
    B.chunk_item0 = {0, B.n_items};
    return e;
}

// The streamed index.  The point positions depend on the plan only, so the
// plan counts the points of every chunk per bin once and keeps each chunk's
// bin offsets and run list (runs of at most kBinChunk ids, the long ones
// first); an evaluation scatters one chunk's ids into the shared buffer and
// spreads them before the next chunk overwrites it.
hipError_t build_stream(Plan& p, hipStream_t s)
{
    BinIndex& B = p.bins;
    const int64_t nbins = B.nbins;
    const int dpc = B.dirs_per_chunk;
    const int D = (p.n_sigma + dpc - 1) / dpc;
    const int64_t per_dir = p.n_points / p.n_sigma;
    B.n_chunks = D;
    B.chunk_s0.assign(D + 1, p.n_sigma);
    for (int c = 0; c < D; ++c) B.chunk_s0[c] = c * dpc;

    std::vector<unsigned int> hc((size_t)D * nbins);  // before the temporary, which nothing below may leak
    unsigned int* count = nullptr;
    hipError_t e = hipMalloc(&count, hc.size() * sizeof(unsigned int));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(count, 0, hc.size() * sizeof(unsigned int), s);
    for (int c = 0; c < D && e == hipSuccess; ++c)
        e = launch_bin_build(p, count + (size_t)c * nbins, nullptr, nullptr, nullptr, 0, B.chunk_s0[c],
                             B.chunk_s0[c + 1] - B.chunk_s0[c], s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hc.data(), count, hc.size() * sizeof(unsigned int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(count);
    if (e != hipSuccess) return e;

    // per chunk: bin offsets in place of the counts, then the runs
    std::vector<int> ib;
    std::vector<long long> ibeg;
    std::vector<int> ic;
    B.chunk_item0.assign(D + 1, 0);
    int64_t max_ids = 1;
    struct Item {
        int bin;
        long long begin;
        int count;
    };
    std::vector<Item> items;
    for (int c = 0; c < D; ++c) {
        unsigned int* h = hc.data() + (size_t)c * nbins;
        items.clear();
        unsigned long long total = 0;
        for (int64_t b = 0; b < nbins; ++b) {
            const unsigned int n = h[b];
            for (unsigned int o = 0; o < n; o += kBinChunk)
                items.push_back({(int)b, (long long)(total + o), (int)std::min<unsigned int>(kBinChunk, n - o)});
            h[b] = (unsigned int)total;
            total += n;
        }
        if ((int64_t)total != per_dir * (B.chunk_s0[c + 1] - B.chunk_s0[c])) return hipErrorUnknown;
        max_ids = std::max<int64_t>(max_ids, (int64_t)total);
        std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.count > y.count; });
        B.chunk_item0[c] = (int64_t)ib.size();
        for (const Item& it : items) {
            ib.push_back(it.bin);
            ibeg.push_back(it.begin);
            ic.push_back(it.count);
        }
    }
    B.chunk_item0[D] = (int64_t)ib.size();
    B.n_items = (int64_t)ib.size();
    B.id_bytes = max_ids * 8;

    void* d = nullptr;
    if ((e = dev_alloc(p, &d, (size_t)B.id_bytes)) != hipSuccess) return e;
    B.ids = static_cast<unsigned long long*>(d);
    if ((e = dev_alloc(p, &d, hc.size() * sizeof(unsigned int))) != hipSuccess) return e;
    B.chunk_begin = static_cast<unsigned int*>(d);
    if ((e = dev_alloc(p, &d, nbins * sizeof(unsigned int))) != hipSuccess) return e;
    B.cursor = static_cast<unsigned int*>(d);
    if ((e = dev_alloc(p, &d, std::max<size_t>(1, ib.size()) * sizeof(int))) != hipSuccess) return e;
    B.item_bin = static_cast<int*>(d);
    if ((e = dev_alloc(p, &d, std::max<size_t>(1, ibeg.size()) * sizeof(long long))) != hipSuccess) return e;
    B.item_begin = static_cast<long long*>(d);
    if ((e = dev_alloc(p, &d, std::max<size_t>(1, ic.size()) * sizeof(int))) != hipSuccess) return e;
    B.item_count = static_cast<int*>(d);
    if ((e = hipMemcpyAsync(B.chunk_begin, hc.data(), hc.size() * sizeof(unsigned int), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return e;
    if (!ib.empty()) {
        if ((e = hipMemcpyAsync(B.item_bin, ib.data(), ib.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(B.item_begin, ibeg.data(), ibeg.size() * sizeof(long long), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(B.item_count, ic.data(), ic.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    }
    return hipStreamSynchronize(s);  // the host vectors go out of scope
}

hipError_t allocate(Plan& p, hipStream_t s)
{
    hipError_t e;
#define PGC_TRY(x)               \
    do {                         \
        e = (x);                 \
        if (e != hipSuccess) return e; \
    } while (0)
    // the FP64 double-HUGE_VAL windows become +-inf in float as well
    const bool fp64 = p.precision == PGC_PRECISION_FP64;
    PGC_TRY(upload(p, &p.dt.v1, p.v1, s));
    if (fp64)
        p.dt.v1d = static_cast<double*>(p.dt.v1);
    else
        PGC_TRY(upload64(p, &p.dt.v1d, p.v1, s));
    PGC_TRY(upload64(p, &p.dt.w1, p.w1, s));
    PGC_TRY(upload64(p, &p.dt.mu21, p.mu21, s));
    PGC_TRY(upload64(p, &p.dt.C, p.C, s));
    PGC_TRY(upload64(p, &p.dt.CT, p.CT, s));
    PGC_TRY(upload64(p, &p.dt.E, p.E, s));
    PGC_TRY(upload(p, &p.dt.poly, p.poly, s));
    if (fp64)
        p.dt.poly64 = static_cast<double*>(p.dt.poly);
    else
        PGC_TRY(upload64(p, &p.dt.poly64, p.poly, s));
    PGC_TRY(upload64(p, &p.dt.kpoly_eo, p.kpoly_eo, s));
    PGC_TRY(upload64(p, &p.dt.cellfit, p.cellfit, s));
    PGC_TRY(upload64(p, &p.dt.cellfit_v, p.cellfit_v, s));
    PGC_TRY(upload64(p, &p.dt.bin_vthr, p.bin_vthr, s));
    PGC_TRY(upload(p, &p.dt.sigma, p.sigma, s));
    {
        // W_s b0 S^d: the constant factors of every point's weight, one rounding in FP32
        p.wfac.resize(p.sigma_w.size());
        const double sd = std::pow(p.S, p.dim);
        for (size_t i = 0; i < p.wfac.size(); ++i) p.wfac[i] = p.sigma_w[i] * p.b0 * sd;
        PGC_TRY(upload(p, &p.dt.wfac, p.wfac, s));
    }
    PGC_TRY(upload(p, &p.dt.slab_vlo, p.slab_vlo, s));
    PGC_TRY(upload(p, &p.dt.slab_vhi, p.slab_vhi, s));

    const int64_t L = std::max<int64_t>(std::max(p.N, p.ni), p.ng);
    int64_t t = 1;
    for (int l = 0; l < p.dim; ++l) t *= L;
    p.tmp_elems = t;
    const size_t e8 = p.elt;
    auto alloc64 = [&p](double** dst, int64_t n) {
        void* d = nullptr;
        hipError_t r = dev_alloc(p, &d, (size_t)n * sizeof(double));
        *dst = static_cast<double*>(d);
        return r;
    };
    PGC_TRY(alloc64(&p.ws.P, p.nid));
    PGC_TRY(alloc64(&p.ws.G, p.nid));
    if (fp64)
        p.ws.Gg = p.ws.G;
    else
        PGC_TRY(dev_alloc(p, &p.ws.Gg, p.nid * e8));
    PGC_TRY(alloc64(&p.ws.H, p.nid));
    PGC_TRY(alloc64(&p.ws.cin, p.Nd));
    {
        int64_t nsym = 1;
        for (int l = 0; l < p.dim; ++l) nsym *= p.np;
        if (p.gain_mode == kGainSlab) PGC_TRY(dev_alloc(p, &p.ws.sym, nsym * e8));
        std::vector<int> pa(p.np), pb(p.np), base(p.ni);
        int q = 0;
        for (int a = 0; a < p.ni; ++a) {
            base[a] = q;
            for (int b = a; b < p.ni; ++b, ++q) {
                pa[q] = a;
                pb[q] = b;
            }
        }
        void* d = nullptr;
        PGC_TRY(dev_alloc(p, &d, pa.size() * sizeof(int)));
        p.dt.pair_a = static_cast<int*>(d);
        PGC_TRY(dev_alloc(p, &d, pb.size() * sizeof(int)));
        p.dt.pair_b = static_cast<int*>(d);
        PGC_TRY(dev_alloc(p, &d, base.size() * sizeof(int)));
        p.dt.pair_base = static_cast<int*>(d);
        PGC_TRY(hipMemcpyAsync(p.dt.pair_a, pa.data(), pa.size() * sizeof(int), hipMemcpyHostToDevice, s));
        PGC_TRY(hipMemcpyAsync(p.dt.pair_b, pb.data(), pb.size() * sizeof(int), hipMemcpyHostToDevice, s));
        PGC_TRY(hipMemcpyAsync(p.dt.pair_base, base.data(), base.size() * sizeof(int),
                               hipMemcpyHostToDevice, s));
        PGC_TRY(hipStreamSynchronize(s));
    }
    if (p.gain_mode == kGainSlab)
        PGC_TRY(dev_alloc(p, &p.ws.partial, (size_t)p.n_chunks * p.ngd * sizeof(double)));
    PGC_TRY(alloc64(&p.ws.grid, p.gain_mode == kGainSlab ? p.ngd : 1));
    PGC_TRY(alloc64(&p.ws.tmpA, t));
    PGC_TRY(alloc64(&p.ws.tmpB, t));
    PGC_TRY(alloc64(&p.ws.qminus, p.Nd));
    PGC_TRY(alloc64(&p.ws.qplus, p.Nd));
    PGC_TRY(dev_alloc(p, &p.ws.rk_y, p.Nd * e8));
    for (int r = 0; r < 4; ++r) PGC_TRY(dev_alloc(p, &p.ws.rk_k[r], p.Nd * e8));
    void* red = nullptr;
    PGC_TRY(dev_alloc(p, &red, 64 * sizeof(double)));
    p.ws.red = static_cast<double*>(red);
    void* mom = nullptr;
    PGC_TRY(dev_alloc(p, &mom, p.mom.size() * sizeof(double)));
    p.ws.mom = static_cast<double*>(mom);
    PGC_TRY(hipMemcpyAsync(mom, p.mom.data(), p.mom.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PGC_TRY(hipStreamSynchronize(s));
    if (p.gain_mode == kGainBinned) {
        void* g64 = nullptr;
        PGC_TRY(dev_alloc(p, &g64, p.ngd * sizeof(double)));
        p.ws.grid64 = static_cast<double*>(g64);
        if (p.index_budget == 0 && !p.deterministic) {
            // no budget given: the whole index when the device has room for it
            // (and its run list), else streamed within a quarter of the free memory
            size_t free_b = 0, total_b = 0;
            PGC_TRY(hipMemGetInfo(&free_b, &total_b));
            const int64_t whole = p.n_points * 8;
            if (whole + whole / 64 + (int64_t(1) << 30) > (int64_t)free_b) {
                const int dpc = stream_dirs(p, (int64_t)free_b / 4);
                if (dpc > 0) p.bins.dirs_per_chunk = dpc;
            }
        }
        e = build_bins(p, s);
        if (e == hipErrorOutOfMemory && p.auto_gain && p.kernel != PGC_KERNEL_ANISO && !p.deterministic) {
            // the bin index does not fit: fall back to LDS slabs
            (void)hipGetLastError();
            p.gain_mode = kGainSlab;
            p.bins = BinIndex();
            PGC_TRY(dev_alloc(p, &p.ws.partial, (size_t)p.n_chunks * p.ngd * sizeof(double)));
            PGC_TRY(alloc64(&p.ws.grid, p.ngd));
            int64_t nsym = 1;
            for (int l = 0; l < p.dim; ++l) nsym *= p.np;
            PGC_TRY(dev_alloc(p, &p.ws.sym, nsym * e8));
        } else if (e != hipSuccess) {
            return e;
        }
    }
#undef PGC_TRY
    return hipSuccess;
}

}  // namespace
}  // namespace pgc

// ==================================================================== C ABI

using pgc::Plan;

extern "C" {

const char* pgc_status_string(pgc_status s)
{
    switch (s) {
    case PGC_OK: return "ok";
    case PGC_ERR_INVALID_ARG: return "invalid argument";
    case PGC_ERR_UNSUPPORTED: return "unsupported configuration";
    case PGC_ERR_OUT_OF_MEMORY: return "out of device memory";
    case PGC_ERR_DEVICE: return "device error";
    case PGC_ERR_NUMERIC: return "non-finite result";
    case PGC_ERR_SCRATCH: return "the call needs more scratch memory than the static buffer holds";
    }
    return "unknown status";
}

pgc_status pgc_desc_init(pgc_plan_desc* d)
{
    if (!d) return PGC_ERR_INVALID_ARG;
    std::memset(d, 0, sizeof(*d));
    d->dim = 2;
    d->n_modes = 16;
    d->map = PGC_MAP_LOG;
    d->scale_mode = PGC_SCALE_DIRECT;
    d->scale = 4.0;
    d->kernel = PGC_KERNEL_MAXWELL;
    d->sphere = PGC_SPHERE_UNIFORM_2D;
    d->n_sigma = 16;
    d->precision = PGC_PRECISION_FP64;
    return PGC_OK;
}

pgc_status pgc_nufft_params(double tol, double upsample, int32_t* width, double* beta)
{
    if (!(tol > 0.0) || !(upsample >= 1.5 && upsample <= 4.0)) return PGC_ERR_INVALID_ARG;
    const int W = pgc::width_for(tol, upsample);
    if (width) *width = W;
    if (beta) *beta = pgc::beta_for(W, upsample);
    return PGC_OK;
}

pgc_status pgc_plan_create(const pgc_plan_desc* desc, void* stream, pgc_plan* plan_out)
{
    if (!desc || !plan_out) return PGC_ERR_INVALID_ARG;
    *plan_out = nullptr;
    pgc_plan_s* h = nullptr;
    try {
        h = new pgc_plan_s();
    } catch (const std::bad_alloc&) {
        return PGC_ERR_OUT_OF_MEMORY;
    }
    // host containers are the only thing here that throws (allocation failure)
    pgc_status st = PGC_OK;
    try {
        st = pgc::resolve(*desc, h->p);
        if (st == PGC_OK) st = pgc::from_hip(hipGetDevice(&h->p.device));
        if (st == PGC_OK) {
            pgc::build_tables(h->p);
            st = pgc::from_hip(pgc::allocate(h->p, static_cast<hipStream_t>(stream)));
        }
    } catch (...) {
        st = PGC_ERR_OUT_OF_MEMORY;
    }
    if (st != PGC_OK) {
        pgc::free_all(h->p);
        delete h;
        return st;
    }
    *plan_out = h;
    return PGC_OK;
}

pgc_status pgc_plan_destroy(pgc_plan plan)
{
    if (!plan) return PGC_OK;
    (void)pgc_set_profiling(plan, 0);
    (void)hipDeviceSynchronize();
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    pgc::free_all(plan->p);
    delete plan;
    return PGC_OK;
}

pgc_status pgc_plan_query(pgc_plan plan, pgc_plan_info* info)
{
    if (!plan || !info) return PGC_ERR_INVALID_ARG;
    const Plan& p = plan->p;
    std::memset(info, 0, sizeof(*info));
    info->dim = p.dim;
    info->n_modes = p.N;
    info->m_v = p.m_v;
    info->map = p.map;
    info->kernel = p.kernel;
    info->precision = p.precision;
    info->n_sigma = p.n_sigma;
    info->scale = p.S;
    info->grid_n = p.n;
    info->grid_folded = p.ng;
    info->kernel_width = p.W;
    info->kernel_beta = p.beta;
    info->upsample = p.upsample;
    info->slab_planes = p.slab_planes;
    info->n_slabs = p.n_slabs;
    info->n_chunks = p.n_chunks;
    info->block_threads = p.block_threads;
    info->n_triples = p.n_triples;
    info->n_points = p.n_points;
    info->gain_mode = p.mfma && p.gain_mode == pgc::kGainBinned ? 3 : p.gain_mode;
    info->n_bin_items = p.bins.n_items;
    info->offset_fit_err = p.cellfit_err;
    info->velocity_fit_cells = p.cellfit_v_cells;
    info->deterministic = p.deterministic ? 1 : 0;
    info->tile_bytes = p.bins.tile_bytes;
    if (p.gain_mode == pgc::kGainBinned) {
        info->index_chunks = p.bins.n_chunks;
        info->index_bytes = p.bins.id_bytes;
    }
    info->workspace_bytes = p.workspace_bytes;
    return PGC_OK;
}

pgc_status pgc_nodes(pgc_plan plan, double* xi, double* v, double* w)
{
    if (!plan) return PGC_ERR_INVALID_ARG;
    const Plan& p = plan->p;
    for (int j = 0; j < p.m_v; ++j) {
        if (xi) xi[j] = p.xi_all[j];
        if (v) v[j] = p.v_all[j];
        if (w) w[j] = p.w_all[j];
    }
    return PGC_OK;
}

pgc_status pgc_project(pgc_plan plan, const double* f_nodes, void* coeffs, void* stream)
{
    if (!plan || !f_nodes || !coeffs) return PGC_ERR_INVALID_ARG;
    return pgc::from_hip(pgc::launch_project(plan->p, f_nodes, coeffs, static_cast<hipStream_t>(stream)));
}

namespace {

// read back one recorded event set into the accumulators
hipError_t prof_collect(pgc::Profiler& pr, int set)
{
    hipError_t e = hipEventSynchronize(pr.ev[set][pgc::kStages]);
    if (e != hipSuccess) return e;
    for (int k = 0; k < pgc::kStages; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pr.ev[set][k], pr.ev[set][k + 1]) == hipSuccess) pr.ms[k] += ms;
    }
    pr.calls += 1;
    return hipSuccess;
}

}  // namespace

pgc_status pgc_coeffs_to_q(pgc_plan plan, const void* coeffs, void* q, void* qplus, void* stream)
{
    if (!plan || !coeffs || !q) return PGC_ERR_INVALID_ARG;
    Plan& p = plan->p;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p.prof) {
        pgc::Profiler& pr = *p.prof;
        if (pr.used == pgc::kProfRing) {  // ring full: fold in the oldest set first
            hipError_t e = prof_collect(pr, pr.head);
            if (e != hipSuccess) return pgc::from_hip(e);
            --pr.used;
        }
        p.prof_set = pr.head;
        pr.head = (pr.head + 1) % pgc::kProfRing;
        ++pr.used;
    }
    pgc::prof_mark(p, 0, s);
    hipError_t e = pgc::launch_synthesis(p, p.ws, coeffs, s);
    pgc::prof_mark(p, 1, s);
    if (e == hipSuccess) e = pgc::launch_loss(p, p.ws, s);
    if (e == hipSuccess) e = pgc::launch_gain(p, p.ws, q, qplus, s);
    pgc::prof_mark(p, 5, s);
    pgc::prof_mark(p, 6, s);  // the combination runs in the grid-to-modes stage
    p.prof_set = -1;
    return pgc::from_hip(e);
}

pgc_status pgc_set_profiling(pgc_plan plan, int32_t on)
{
    if (!plan) return PGC_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (on && !p.prof) {
        pgc::Profiler* pr = new (std::nothrow) pgc::Profiler();
        if (!pr) return PGC_ERR_OUT_OF_MEMORY;
        int made = 0;  // events created so far, destroyed again on failure
        hipError_t e = hipSuccess;
        for (int r = 0; r < pgc::kProfRing && e == hipSuccess; ++r)
            for (int k = 0; k <= pgc::kStages && e == hipSuccess; ++k)
                if ((e = hipEventCreate(&pr->ev[r][k])) == hipSuccess) ++made;
        if (e != hipSuccess) {
            for (int i = 0; i < made; ++i) (void)hipEventDestroy(pr->ev[i / (pgc::kStages + 1)][i % (pgc::kStages + 1)]);
            delete pr;
            return pgc::from_hip(e);
        }
        p.prof = pr;
    } else if (!on && p.prof) {
        (void)hipDeviceSynchronize();
        for (int r = 0; r < pgc::kProfRing; ++r)
            for (int k = 0; k <= pgc::kStages; ++k) (void)hipEventDestroy(p.prof->ev[r][k]);
        delete p.prof;
        p.prof = nullptr;
    }
    return PGC_OK;
}

pgc_status pgc_stage_times(pgc_plan plan, double* ms_out, int32_t n_stages, int64_t* calls_out)
{
    if (!plan || !ms_out || n_stages < 1 || n_stages > 8) return PGC_ERR_INVALID_ARG;
    Plan& p = plan->p;
    for (int k = 0; k < n_stages; ++k) ms_out[k] = 0.0;
    if (calls_out) *calls_out = 0;
    if (!p.prof) return PGC_OK;
    pgc::Profiler& pr = *p.prof;
    while (pr.used > 0) {
        const int set = (pr.head - pr.used + pgc::kProfRing) % pgc::kProfRing;
        hipError_t e = prof_collect(pr, set);
        if (e != hipSuccess) return pgc::from_hip(e);
        --pr.used;
    }
    for (int k = 0; k < n_stages && k < pgc::kStages; ++k) ms_out[k] = pr.ms[k];
    if (calls_out) *calls_out = pr.calls;
    for (int k = 0; k < pgc::kStages; ++k) pr.ms[k] = 0.0;
    pr.calls = 0;
    return PGC_OK;
}

pgc_status pgc_rk4(pgc_plan plan, double* coeffs, double dt, int32_t n_steps, void* stream)
{
    if (!plan || !coeffs || n_steps < 0 || !std::isfinite(dt)) return PGC_ERR_INVALID_ARG;
    const Plan& p = plan->p;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double a[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
    for (int st = 0; st < n_steps; ++st) {
        for (int r = 0; r < 4; ++r) {
            hipError_t e = pgc::launch_rk_stage(p, coeffs, r == 0 ? nullptr : p.ws.rk_k[r - 1], a[r],
                                                p.ws.rk_y, s);
            if (e != hipSuccess) return pgc::from_hip(e);
            pgc_status q = pgc_coeffs_to_q(plan, p.ws.rk_y, p.ws.rk_k[r], nullptr, stream);
            if (q != PGC_OK) return q;
        }
        hipError_t e = pgc::launch_rk_finish(p, coeffs, dt, s);
        if (e != hipSuccess) return pgc::from_hip(e);
    }
    return PGC_OK;
}

}  // extern "C"

namespace {

void drop_graph(pgc_plan plan)
{
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    plan->exec = nullptr;
    plan->graph = nullptr;
}

// records `body(stream)` into the plan's graph on a private stream, after the
// caller's stream has drained
template <typename F>
pgc_status capture_into(pgc_plan plan, hipStream_t user, F body)
{
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamSynchronize(user);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return pgc::from_hip(e);
    pgc_status st = PGC_OK;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = body(cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        plan->graph = g;
    }
    if (st == PGC_OK && e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (st == PGC_OK && e != hipSuccess) st = pgc::from_hip(e);
    if (st != PGC_OK) drop_graph(plan);
    return st;
}

}  // namespace

extern "C" {

pgc_status pgc_plan_capture(pgc_plan plan, const void* coeffs, void* q, void* qplus, void* stream)
{
    if (!plan || !coeffs || !q) return PGC_ERR_INVALID_ARG;
    if (plan->p.prof) return PGC_ERR_UNSUPPORTED;
    drop_graph(plan);
    pgc_status st = pgc_coeffs_to_q(plan, coeffs, q, qplus, stream);
    if (st != PGC_OK) return st;
    return capture_into(plan, static_cast<hipStream_t>(stream),
                        [&](hipStream_t cs) { return pgc_coeffs_to_q(plan, coeffs, q, qplus, cs); });
}

pgc_status pgc_plan_capture_rk4(pgc_plan plan, double* coeffs, double dt, int32_t n_steps, void* stream)
{
    if (!plan || !coeffs || n_steps < 1 || !std::isfinite(dt)) return PGC_ERR_INVALID_ARG;
    if (plan->p.prof) return PGC_ERR_UNSUPPORTED;
    drop_graph(plan);
    return capture_into(plan, static_cast<hipStream_t>(stream),
                        [&](hipStream_t cs) { return pgc_rk4(plan, coeffs, dt, n_steps, cs); });
}

pgc_status pgc_plan_graph_launch(pgc_plan plan, void* stream)
{
    if (!plan || !plan->exec) return PGC_ERR_INVALID_ARG;
    return pgc::from_hip(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
}

pgc_status pgc_moments(pgc_plan plan, const void* coeffs, double* out, void* stream)
{
    if (!plan || !coeffs || !out) return PGC_ERR_INVALID_ARG;
    return pgc::from_hip(pgc::launch_moments(plan->p, coeffs, out, static_cast<hipStream_t>(stream)));
}

pgc_status pgc_eval(pgc_plan plan, const void* coeffs, const double* v, int64_t n, double* out,
                    void* stream)
{
    if (!plan || n < 0 || (n > 0 && (!coeffs || !v || !out))) return PGC_ERR_INVALID_ARG;
    if (n > 2147483647ll) return PGC_ERR_UNSUPPORTED;
    return pgc::from_hip(pgc::launch_eval(plan->p, coeffs, v, n, out, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
