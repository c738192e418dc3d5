// Transport of the spatially inhomogeneous equation in coefficient space, and
// the split step that alternates it with collisions.
//
// The full Boltzmann equation adds the free-streaming term v . grad_x f to the
// spatially homogeneous equation whose collision operator the library
// evaluates; the two parts are treated separately by operator splitting
// (Sec. 1).  Along one periodic space dimension x (the direction of the first
// velocity component), testing f_t + v_1 f_x = 0 for f_N = sum_l f_l T~_l
// against T^_k (the Petrov-Galerkin step of Sec. 3, with the biorthogonality
// of eq. ortho) gives
//
//     d/dt f_k + sum_l V_kl d/dx f_l = 0,   V_kl = (v_1 T~_l, T^_k),
//
// acting on the first index of every coefficient tensor.  For the logarithmic
// map (Sec. 2.1) V is finite and has a closed form: with xi = cos t,
//     V_kl = S / sqrt(c_k c_l) int_0^pi ln cot(t/2) cos(kt) cos(lt) dt,
// and int_0^pi ln cot(t/2) cos(mt) dt = pi/|m| for odd m, 0 for even m (the
// cosine series of ln cot(t/2) has coefficients 2/n on odd n).  V is
// symmetric: V = R diag(lambda) R^T (Jacobi rotations at creation), so the
// characteristic variables w = R^T f each move at speed lambda_j.  In x the
// state is a trigonometric polynomial on n_x (odd) equispaced cells, and a
// shift by lambda_j dt is the circulant interpolation
//     w_j(x_c) <- sum_e D(x_c - x_e - lambda_j dt) w_j(x_e),
//     D(s) = (1 + 2 sum_{m=1}^{(n_x-1)/2} cos(2 pi m s / L)) / n_x,
// exact for every Fourier mode of the grid.  A step is three small kernels:
// to characteristics, the shifts, and back.
#include "pgc.h"
#include "pgc_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace pgc {
namespace {

constexpr double kPiT = 3.14159265358979323846264338327950288;

// Eigen-decomposition of a symmetric n x n matrix A (row-major) by cyclic
// Jacobi rotations: A = R diag(lam) R^T, R orthogonal (columns eigenvectors).
void jacobi_eigen(int n, std::vector<double> A, std::vector<double>& R, std::vector<double>& lam)
{
    R.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) R[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += a(i, i) * a(i, i);
            for (int j = i + 1; j < n; ++j) off += a(i, j) * a(i, j);
        }
        if (off <= 1e-34 * std::max(diag, 1e-300)) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a(p, q);
                if (apq == 0.0) continue;
                // rotation angle that zeroes a(p, q)
                const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    const double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * akq;
                    a(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    const double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * aqk;
                    a(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {  // R <- R J
                    const double rkp = R[(size_t)k * n + p], rkq = R[(size_t)k * n + q];
                    R[(size_t)k * n + p] = c * rkp - s * rkq;
                    R[(size_t)k * n + q] = s * rkp + c * rkq;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = a(i, i);
}

// out[x][j][r] = sum_k M[k][j] in[x][k][r] (trans = 1: M^T applied, to characteristics)
// or sum_k M[j][k] in[x][k][r] (trans = 0: back); N x N matrix M
__global__ void __launch_bounds__(256)
    first_index_product(const double* __restrict__ in, const double* __restrict__ M, int trans, int N,
                        int64_t rest, int64_t n_total, double* __restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const int64_t r = i % rest;
    const int64_t xj = i / rest;
    const int j = (int)(xj % N);
    const int64_t x = xj / N;
    const double* src = in + x * N * rest + r;
    double acc = 0.0;
    for (int k = 0; k < N; ++k) acc = fma(trans ? M[k * N + j] : M[j * N + k], src[k * rest], acc);
    out[i] = acc;
}

// out[x][j][r] = sum_e P[j][(x - e) mod n_x] in[e][j][r]
__global__ void __launch_bounds__(256)
    circulant_shift(const double* __restrict__ in, const double* __restrict__ P, int n_x, int N, int64_t rest,
                    int64_t n_total, double* __restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const int64_t r = i % rest;
    const int64_t xj = i / rest;
    const int j = (int)(xj % N);
    const int x = (int)(xj / N);
    const int64_t stride = (int64_t)N * rest;
    const double* row = P + (int64_t)j * n_x;
    const double* src = in + (int64_t)j * rest + r;
    double acc = 0.0;
    for (int e = 0; e < n_x; ++e) {
        int d = x - e;
        d += d < 0 ? n_x : 0;
        acc = fma(row[d], src[e * stride], acc);
    }
    out[i] = acc;
}

}  // namespace
}  // namespace pgc

struct pgc_transport_s {
    pgc_plan plan = nullptr;
    int n_x = 0, N = 0, dim = 0;
    int64_t rest = 0, n_total = 0;
    double length = 0.0, dt = 0.0;
    std::vector<double> lam;
    double* R = nullptr;   // N x N eigenvectors (columns)
    double* P = nullptr;   // N x n_x circulant rows of the shift by lambda_j dt
    double* w1 = nullptr;  // n_x x N^d each
    double* w2 = nullptr;
    int64_t bytes = 0;
    std::vector<void*> allocations;
};

namespace {

hipError_t t_alloc(pgc_transport_s& t, double** ptr, int64_t n)
{
    *ptr = nullptr;
    t.allocations.push_back(nullptr);
    hipError_t e = hipMalloc(&t.allocations.back(), (size_t)std::max<int64_t>(n, 2) * sizeof(double));
    if (e != hipSuccess) {
        t.allocations.pop_back();
        return e;
    }
    *ptr = static_cast<double*>(t.allocations.back());
    t.bytes += n * (int64_t)sizeof(double);
    return hipSuccess;
}

void t_free(pgc_transport_s* t)
{
    if (!t) return;
    (void)hipDeviceSynchronize();
    for (void* p : t->allocations) (void)hipFree(p);
    delete t;
}

}  // namespace

extern "C" {

pgc_status pgc_transport_create(pgc_plan plan, int32_t n_x, double length, double dt, void* stream,
                                pgc_transport* out)
{
    if (!plan || !out || n_x < 1 || n_x > 4095 || (n_x % 2) != 1 || !(length > 0.0) || !std::isfinite(length) ||
        !std::isfinite(dt))
        return PGC_ERR_INVALID_ARG;
    *out = nullptr;
    const pgc::Plan& p = plan->p;
    if (p.map != PGC_MAP_LOG) return PGC_ERR_UNSUPPORTED;  // V is infinite for the algebraic map
    pgc_transport_s* t = nullptr;
    hipError_t e = hipSuccess;
    pgc_status st = PGC_OK;
    try {
        t = new pgc_transport_s();
        t->plan = plan;
        t->n_x = n_x;
        t->N = p.N;
        t->dim = p.dim;
        t->length = length;
        t->dt = dt;
        t->rest = 1;
        for (int l = 1; l < p.dim; ++l) t->rest *= p.N;
        t->n_total = (int64_t)n_x * p.N * t->rest;
        const int N = p.N;
        std::vector<double> V((size_t)N * N), R, P((size_t)N * n_x);
        auto I = [](int m) { m = std::abs(m); return (m % 2 == 1) ? pgc::kPiT / m : 0.0; };
        for (int k = 0; k < N; ++k)
            for (int l = 0; l < N; ++l) {
                const double ck = k == 0 ? pgc::kPiT : 0.5 * pgc::kPiT, cl = l == 0 ? pgc::kPiT : 0.5 * pgc::kPiT;
                V[(size_t)k * N + l] = p.S / std::sqrt(ck * cl) * 0.5 * (I(k - l) + I(k + l));
            }
        pgc::jacobi_eigen(N, V, R, t->lam);
        const int M = (n_x - 1) / 2;
        for (int j = 0; j < N; ++j)
            for (int d = 0; d < n_x; ++d) {
                const double s = d * length / n_x - t->lam[j] * dt;
                double acc = 1.0;
                for (int m = 1; m <= M; ++m) acc += 2.0 * std::cos(2.0 * pgc::kPiT * m * s / length);
                P[(size_t)j * n_x + d] = acc / n_x;
            }
        if ((e = t_alloc(*t, &t->R, (int64_t)N * N)) == hipSuccess &&
            (e = t_alloc(*t, &t->P, (int64_t)N * n_x)) == hipSuccess &&
            (e = t_alloc(*t, &t->w1, t->n_total)) == hipSuccess && (e = t_alloc(*t, &t->w2, t->n_total)) == hipSuccess) {
            hipStream_t s = static_cast<hipStream_t>(stream);
            e = hipMemcpyAsync(t->R, R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(t->P, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
    } catch (...) {
        st = PGC_ERR_OUT_OF_MEMORY;
    }
    if (st == PGC_OK && e != hipSuccess) st = pgc::status_of(e);
    if (st != PGC_OK) {
        t_free(t);
        return st;
    }
    *out = t;
    return PGC_OK;
}

pgc_status pgc_transport_destroy(pgc_transport t)
{
    t_free(t);
    return PGC_OK;
}

pgc_status pgc_transport_query(pgc_transport t, pgc_transport_info* info, double* speeds_host)
{
    if (!t || (!info && !speeds_host)) return PGC_ERR_INVALID_ARG;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->n_x = t->n_x;
        info->dim = t->dim;
        info->n_modes = t->N;
        info->length = t->length;
        info->dt = t->dt;
        double mx = 0.0;
        for (double l : t->lam) mx = std::max(mx, std::fabs(l));
        info->max_speed = mx;
        info->workspace_bytes = t->bytes;
    }
    if (speeds_host)
        for (int j = 0; j < t->N; ++j) speeds_host[j] = t->lam[j];
    return PGC_OK;
}

pgc_status pgc_transport_step(pgc_transport t, double* coeffs_dev, void* stream)
{
    if (!t || !coeffs_dev) return PGC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned blocks = (unsigned)((t->n_total + 255) / 256);
    hipLaunchKernelGGL(pgc::first_index_product, dim3(blocks), dim3(256), 0, s, coeffs_dev, t->R, 1, t->N, t->rest,
                       t->n_total, t->w1);
    hipLaunchKernelGGL(pgc::circulant_shift, dim3(blocks), dim3(256), 0, s, t->w1, t->P, t->n_x, t->N, t->rest,
                       t->n_total, t->w2);
    hipLaunchKernelGGL(pgc::first_index_product, dim3(blocks), dim3(256), 0, s, t->w2, t->R, 0, t->N, t->rest,
                       t->n_total, coeffs_dev);
    return pgc::status_of(hipGetLastError());
}

pgc_status pgc_split_step(pgc_transport half, pgc_plan plan, pgc_direct direct, double* coeffs_dev, int32_t n_steps,
                          void* stream)
{
    if (!half || !coeffs_dev || n_steps < 0 || (!plan && !direct)) return PGC_ERR_INVALID_ARG;
    if (plan && plan != half->plan) return PGC_ERR_INVALID_ARG;
    const double dt = 2.0 * half->dt;
    const int64_t Nd = (int64_t)half->n_total / half->n_x;
    if (direct) {
        pgc_direct_info di;
        const pgc_status q = pgc_direct_query(direct, &di);
        if (q != PGC_OK) return q;
        if (di.n_modes_total != Nd) return PGC_ERR_INVALID_ARG;
    }
    for (int st = 0; st < n_steps; ++st) {
        pgc_status r = pgc_transport_step(half, coeffs_dev, stream);
        if (r != PGC_OK) return r;
        if (direct) {
            r = pgc_direct_rk4(direct, coeffs_dev, half->n_x, dt, 1, stream);
        } else {
            for (int c = 0; c < half->n_x && r == PGC_OK; ++c) r = pgc_rk4(plan, coeffs_dev + c * Nd, dt, 1, stream);
        }
        if (r != PGC_OK) return r;
        r = pgc_transport_step(half, coeffs_dev, stream);
        if (r != PGC_OK) return r;
    }
    return PGC_OK;
}

}  // extern "C"
