// The direct algorithm (Sec. 4.1): the discrete collision operator is a
// bilinear form whose tensor does not depend on f, so it is built once per
// plan, and Q of a batch of cells that share the plan is then one dense
// product on the FP64 matrix cores.
//
// The paper's tensors (eqs. tensor_I1, tensor_I2) pair Chebyshev modes and
// are contracted with the coefficients (eq. direct_online). Here the tensor
// pairs interior CGL nodes instead, and is contracted with the weighted nodal
// values G_a = w_a mu_a^2 P_a that the synthesis produces. Both orders of a
// pair give the same post-collision velocity, and cos theta = u.sigma/|u|
// only changes sign, so with a rate even in cos theta the two orders share
// one entry. For the unordered pair a <= b of flat node indices, with
// B = R(|u|) A(cos theta), R = b0 |u|^gamma (b0 for Maxwell) and
// A = 1 + beta cos^2 theta (1 for the angle-free rates):
//
//   K[p][k] = R * (2 gain_k - Lw (L_k(a) + L_k(b)))   (a < b)
//   K[p][k] = R * (gain_k - Lw L_k(a))                (a = b: u = 0, A = 1)
//   gain_k  = sum_s W_s A_s T^_k(v'_s),  v'_s = (v_a + v_b)/2 + |u| sigma_s / 2
//   Lw      = sum_s W_s A_s   (the loss's inner integral over sigma)
//   L_k(a)  = T^_k(v_a),  T^_k(v) = prod_l mu(xi(v_l))^-2 T_{k_l}(xi(v_l)) / sqrt(c_{k_l})
//
// and Q_k = sum_p G_a G_b K[p][k], which is the quadrature of eqs. Qplus and
// Qminus on the CGL nodes with the sphere rule, the same discrete sum the fast
// algorithm approximates, without its transform tolerance.
//
// The product Q[c][k] = sum_p X[c][p] K[p][k] (X the pair products of the
// cells) is a plain FP64 GEMM; it runs on a hand-written matrix-core kernel
// (dgemm_tile below) with a fixed summation order, so results repeat bit for
// bit.
#include "pgc.h"
#include "pgc_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace pgc {
namespace {

constexpr int kDirThreads = 256;
constexpr int kSigChunk = 32;      // directions staged in LDS at a time
constexpr int kMaxPerThread = 16;  // N^d <= 4096 outputs per pair
constexpr int64_t kMaxTensorBytes = 96ll << 30;

// zeta = xi(v) and mu(xi(v))^-2, both written in v (no cancellation near +-1)
__device__ __forceinline__ void dir_map(int map, double S, double v, double& zeta, double& m2)
{
    if (map == 0) {
        const double e = exp(v / S), ei = 1.0 / e;
        zeta = (e - ei) / (e + ei);
        m2 = 0.5 * S * (e + ei);
    } else {
        const double d = S * S + v * v;
        zeta = v / sqrt(d);
        m2 = d / S;
    }
}

// One workgroup per unordered node pair: the pair's N^d tensor entries.
template <int DIM>
__global__ void __launch_bounds__(kDirThreads)
    direct_tensor(const int* __restrict__ pa, const int* __restrict__ pb, int64_t n_pairs,
                  const double* __restrict__ v1, const double* __restrict__ ltab,
                  const double* __restrict__ sig, const double* __restrict__ sw, int n_sigma, int N,
                  int ni, int Nd, int map, double S, double b0, double gamma, int radial, double aniso,
                  double* __restrict__ K)
{
    extern __shared__ double vec[];  // [kSigChunk][DIM][N], then the chunk's W_s A_s
    double* lw = vec + kSigChunk * DIM * N;
    const int64_t p = blockIdx.x;
    if (p >= n_pairs) return;
    int a = pa[p], b = pb[p];
    const bool diag = a == b;
    int ia[DIM], ib[DIM];
#pragma unroll
    for (int l = DIM - 1; l >= 0; --l) {
        ia[l] = a % ni;
        a /= ni;
        ib[l] = b % ni;
        b /= ni;
    }
    double vm[DIM], ud[DIM], u2 = 0.0;
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
        const double x = v1[ia[l]], y = v1[ib[l]];
        vm[l] = 0.5 * (x + y);
        ud[l] = x - y;
        u2 += ud[l] * ud[l];
    }
    const double un = sqrt(u2);
    const double B = radial ? b0 * pow(un, gamma) : b0;
    double Lw = 0.0;
    const double r0 = 1.0 / sqrt(M_PI), r1 = sqrt(2.0 / M_PI);

    double gain[kMaxPerThread];
#pragma unroll
    for (int r = 0; r < kMaxPerThread; ++r) gain[r] = 0.0;

    for (int s0 = 0; s0 < n_sigma; s0 += kSigChunk) {
        const int ns = min(kSigChunk, n_sigma - s0);
        __syncthreads();  // the previous chunk's vectors are no longer read
        for (int row = threadIdx.x; row < ns * DIM; row += kDirThreads) {
            const int s = row / DIM, l = row % DIM;
            const double vp = vm[l] + 0.5 * un * sig[(int64_t)(s0 + s) * DIM + l];
            double zeta, m2;
            dir_map(map, S, vp, zeta, m2);
            double sc = m2;
            if (l == 0) {  // W_s A_s (twice off the diagonal) rides on the first dimension
                double c = 0.0;
                if (un > 0.0) {
#pragma unroll
                    for (int l2 = 0; l2 < DIM; ++l2) c += ud[l2] * sig[(int64_t)(s0 + s) * DIM + l2];
                    c /= un;
                }
                const double ws = sw[s0 + s] * (1.0 + aniso * c * c);
                lw[s] = ws;
                sc *= diag ? ws : 2.0 * ws;
            }
            double* out = vec + (s * DIM + l) * N;
            double tm = 1.0, t = zeta;
            out[0] = sc * r0;
            if (N > 1) out[1] = sc * r1 * zeta;
            for (int k = 2; k < N; ++k) {
                const double tn = 2.0 * zeta * t - tm;
                tm = t;
                t = tn;
                out[k] = sc * r1 * t;
            }
        }
        __syncthreads();
        for (int s = 0; s < ns; ++s) Lw += lw[s];
#pragma unroll
        for (int r = 0; r < kMaxPerThread; ++r) {
            const int k = threadIdx.x + r * kDirThreads;
            if (k >= Nd) break;
            int kk[DIM], f = k;
#pragma unroll
            for (int l = DIM - 1; l >= 0; --l) {
                kk[l] = f % N;
                f /= N;
            }
            double acc = 0.0;
            for (int s = 0; s < ns; ++s) {
                const double* vs = vec + s * DIM * N;
                double t = vs[kk[0]];
#pragma unroll
                for (int l = 1; l < DIM; ++l) t *= vs[l * N + kk[l]];
                acc += t;
            }
            gain[r] += acc;
        }
    }
#pragma unroll
    for (int r = 0; r < kMaxPerThread; ++r) {
        const int k = threadIdx.x + r * kDirThreads;
        if (k >= Nd) break;
        int kk[DIM], f = k;
#pragma unroll
        for (int l = DIM - 1; l >= 0; --l) {
            kk[l] = f % N;
            f /= N;
        }
        double la = 1.0, lb = 1.0;
#pragma unroll
        for (int l = 0; l < DIM; ++l) {
            la *= ltab[ia[l] * N + kk[l]];
            lb *= ltab[ib[l] * N + kk[l]];
        }
        K[p * Nd + k] = diag ? B * (gain[r] - Lw * la) : B * (gain[r] - Lw * (la + lb));
    }
}

// X[c][p] = G[c][a_p] G[c][b_p] for the cells of one chunk (row stride ldx,
// n_pairs rounded up to even).  A thread keeps two neighbouring pairs for
// kPairCells cells: the pair indices are read once, the cells' gathers are
// independent, and each cell's two products leave in one 16-byte store
// (HBM bound: the writes of X).
constexpr int kPairCells = 16;

__global__ void __launch_bounds__(256)
    pair_products(const double* __restrict__ G, const int* __restrict__ pa, const int* __restrict__ pb,
                  int64_t n_pairs, int64_t ldx, int64_t nid, int n_cells, double* __restrict__ X)
{
    const int64_t p = 2 * (blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
    if (p >= n_pairs) return;
    const bool two = p + 1 < n_pairs;
    const int a0 = pa[p], b0 = pb[p];
    const int a1 = two ? pa[p + 1] : a0, b1 = two ? pb[p + 1] : b0;
    const int c0 = blockIdx.y * kPairCells;
    const int nc = min(kPairCells, n_cells - c0);
    double2 v[kPairCells];
#pragma unroll
    for (int c = 0; c < kPairCells; ++c)
        if (c < nc) {
            const double* g = G + (int64_t)(c0 + c) * nid;
            v[c] = make_double2(g[a0] * g[b0], g[a1] * g[b1]);
        }
#pragma unroll
    for (int c = 0; c < kPairCells; ++c)
        if (c < nc) {
            double* x = X + (int64_t)(c0 + c) * ldx + p;
            if (two)
                *reinterpret_cast<double2*>(x) = v[c];
            else
                x[0] = v[c].x;
        }
}

// ----------------------------------------------------------------- FP64 GEMM
//
// C[m][n] = sum_k A[m][k] B[k][n] for row-major A (M x K, row stride lda),
// B (K x N, ldb) and C (M x N, ldc) on v_mfma_f64_16x16x4f64.  A workgroup of
// four waves owns a 128 x 128 tile of C (each wave a 64 x 64 quarter, 4 x 4
// instruction tiles of 16 x 16 held in 16 accumulators) and walks its share of
// K in chunks of 16: the chunk's 128 x 16 slice of A and 16 x 128 slice of B
// are staged in LDS (A transposed, so both operand fragments are 16
// consecutive doubles per k row), double buffered, the next chunk's global
// loads in flight while the matrix cores work on the current one.  Long K is
// split over `splits` workgroups per tile when the tiles alone do not fill the
// chip; each split writes its own partial tile and dgemm_reduce adds them in
// split order, so the sum order is fixed.  Workgroups are numbered so that the
// ones on one XCD (consecutive ids go round-robin over the 8 XCDs) share A row
// blocks, which then come from that XCD's L2.
constexpr int kGT = 128;          // tile rows and columns
constexpr int kGK = 16;           // K chunk
constexpr int kGS = kGT + 16;     // LDS row stride in doubles (shifts the four k rows of a fragment by 128 B)
constexpr int kGThreads = 256;

typedef double dvec4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
    const double* A;
    const double* B;
    double* C;        // splits == 1: the output; otherwise the partial tiles [split][M][N]
    int64_t lda, ldb, ldc;
    int M, N;
    int64_t K;
    int mt, nt, splits;
    int64_t kspan;    // K per split, a multiple of kGK
    int vec;          // rows of A and B 16-byte aligned: interior chunks load pairs of doubles
};

__device__ __forceinline__ void gemm_load(const GemmArgs& g, int m0, int n0, int64_t k0, int64_t k1, double ra[8],
                                          double rb[8])
{
    const int t = threadIdx.x;
    // interior chunks (the usual case) load without per-element guards, in
    // 16-byte pairs, so the loads carry no branches and schedule freely
    if (g.vec && m0 + kGT <= g.M && n0 + kGT <= g.N && k0 + kGK <= k1) {
        const double2* a = reinterpret_cast<const double2*>(g.A + (int64_t)(m0 + (t >> 1)) * g.lda + k0 + (t & 1) * 8);
        const double2* b = reinterpret_cast<const double2*>(g.B + (k0 + (t >> 4)) * g.ldb + n0 + (t & 15) * 8);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double2 x = a[j], y = b[j];
            ra[2 * j] = x.x;
            ra[2 * j + 1] = x.y;
            rb[2 * j] = y.x;
            rb[2 * j + 1] = y.y;
        }
        return;
    }
    // A: row t/2 of the tile, 8 consecutive k
    {
        const int m = m0 + (t >> 1);
        const int64_t kb = k0 + (t & 1) * 8;
        const double* src = g.A + (int64_t)m * g.lda + kb;
#pragma unroll
        for (int j = 0; j < 8; ++j) ra[j] = (m < g.M && kb + j < k1) ? src[j] : 0.0;
    }
    // B: k row t/16 of the chunk, 8 consecutive columns
    {
        const int64_t k = k0 + (t >> 4);
        const int n = n0 + (t & 15) * 8;
        const double* src = g.B + k * g.ldb + n;
#pragma unroll
        for (int j = 0; j < 8; ++j) rb[j] = (k < k1 && n + j < g.N) ? src[j] : 0.0;
    }
}

__device__ __forceinline__ void gemm_stage(double* As, double* Bs, const double ra[8], const double rb[8])
{
    const int t = threadIdx.x;
    const int m = t >> 1, kb = (t & 1) * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) As[(kb + j) * kGS + m] = ra[j];
    const int k = t >> 4, n = (t & 15) * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) Bs[k * kGS + n + j] = rb[j];
}

__global__ void __launch_bounds__(kGThreads, 2) dgemm_tile(GemmArgs g)
{
    __shared__ __align__(16) double As[2][kGK * kGS];
    __shared__ __align__(16) double Bs[2][kGK * kGS];

    // logical tile order: split, then tile row, then tile column (fastest);
    // XCD x takes the x-th contiguous eighth of it when the count allows
    const int total = g.mt * g.nt * g.splits;
    int L = blockIdx.x;
    if ((total & 7) == 0) L = (blockIdx.x & 7) * (total >> 3) + (blockIdx.x >> 3);
    const int ni = L % g.nt;
    const int mi = (L / g.nt) % g.mt;
    const int sp = L / (g.nt * g.mt);
    const int m0 = mi * kGT, n0 = ni * kGT;
    const int64_t kbeg = (int64_t)sp * g.kspan;
    const int64_t kend = min(g.K, kbeg + g.kspan);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int i16 = lane & 15, k4 = lane >> 4;

    dvec4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = dvec4{0.0, 0.0, 0.0, 0.0};

    double ra[8], rb[8];
    int cur = 0;
    if (kbeg < kend) {
        gemm_load(g, m0, n0, kbeg, kend, ra, rb);
        gemm_stage(As[0], Bs[0], ra, rb);
    }
    __syncthreads();
    for (int64_t k0 = kbeg; k0 < kend; k0 += kGK) {
        const bool more = k0 + kGK < kend;
        if (more) gemm_load(g, m0, n0, k0 + kGK, kend, ra, rb);
        const double* as = As[cur];
        const double* bs = Bs[cur];
#pragma unroll
        for (int ks = 0; ks < kGK / 4; ++ks) {
            const int kr = (4 * ks + k4) * kGS;
            double af[4], bf[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = as[kr + wm + 16 * i + i16];
#pragma unroll
            for (int j = 0; j < 4; ++j) bf[j] = bs[kr + wn + 16 * j + i16];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        if (more) gemm_stage(As[cur ^ 1], Bs[cur ^ 1], ra, rb);
        __syncthreads();
        cur ^= 1;
    }

    // lane l holds rows l/16 + 4 r of column l % 16 of each 16 x 16 tile
    double* out = g.C + (g.splits > 1 ? (int64_t)sp * g.M * (int64_t)g.N : 0);
    const int64_t ldo = g.splits > 1 ? (int64_t)g.N : g.ldc;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn + 16 * j + i16;
            if (n >= g.N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + k4 + 4 * r;
                if (m < g.M) out[(int64_t)m * ldo + n] = acc[i][j][r];
            }
        }
}

// C[m][n] = sum over splits, in split order, of the partial tiles
__global__ void dgemm_reduce(const double* __restrict__ part, int splits, int M, int N, double* __restrict__ C,
                             int64_t ldc)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t mn = (int64_t)M * N;
    if (i >= mn) return;
    double s = 0.0;
    for (int p = 0; p < splits; ++p) s += part[(int64_t)p * mn + i];
    C[(i / N) * ldc + i % N] = s;
}

// How many K splits a product of this shape takes: enough workgroups for two
// per CU on the 256 CUs, each split at least 16 chunks long.
int gemm_splits(int M, int N, int64_t K)
{
    const int64_t tiles = (int64_t)((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT);
    const int64_t chunks = (K + kGK - 1) / kGK;
    int64_t s = (512 + tiles - 1) / tiles;
    s = std::min<int64_t>(s, std::max<int64_t>(1, chunks / 16));
    return (int)std::max<int64_t>(1, std::min<int64_t>(s, 64));
}

// Elements of the partial-tile buffer a product of this shape needs (0 when unsplit).
int64_t gemm_partial_elems(int M, int N, int64_t K)
{
    const int s = gemm_splits(M, N, K);
    return s > 1 ? (int64_t)s * M * N : 0;
}

hipError_t gemm_launch(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, int M,
                       int N, int64_t K, double* partial, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    GemmArgs g;
    g.A = A;
    g.B = B;
    g.lda = lda;
    g.ldb = ldb;
    g.ldc = ldc;
    g.M = M;
    g.N = N;
    g.K = K;
    g.mt = (M + kGT - 1) / kGT;
    g.nt = (N + kGT - 1) / kGT;
    g.splits = gemm_splits(M, N, K);
    const int64_t chunks = (K + kGK - 1) / kGK;
    g.kspan = (chunks + g.splits - 1) / g.splits * kGK;
    g.C = g.splits > 1 ? partial : C;
    g.vec = (lda % 2 == 0 && ldb % 2 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
             (reinterpret_cast<uintptr_t>(B) & 15) == 0)
                ? 1
                : 0;
    const int64_t blocks = (int64_t)g.mt * g.nt * g.splits;
    hipLaunchKernelGGL(dgemm_tile, dim3((unsigned)blocks), dim3(kGThreads), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || g.splits == 1) return e;
    const int64_t mn = (int64_t)M * N;
    hipLaunchKernelGGL(dgemm_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, partial, g.splits, M, N,
                       C, ldc);
    return hipGetLastError();
}

// RK4 stages over the cells of one chunk: y = base + a k, and the final update
__global__ void rk_axpy(const double* __restrict__ base, const double* __restrict__ k, double a,
                        double* __restrict__ y, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = base[i] + a * k[i];
}

__global__ void rk_combine(double* __restrict__ base, const double* __restrict__ k1, const double* __restrict__ k2,
                           const double* __restrict__ k3, const double* __restrict__ k4, double h, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) base[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

}  // namespace
}  // namespace pgc

struct pgc_direct_s {
    pgc_plan plan = nullptr;
    int max_cells = 0;
    int64_t n_pairs = 0, nid = 0, Nd = 0;
    int64_t ldx = 0;          // row stride of X: n_pairs rounded up to even (16-byte rows)
    double* K = nullptr;      // n_pairs x N^d
    double* X = nullptr;      // max_cells x ldx
    int* pa = nullptr;
    int* pb = nullptr;
    pgc::DenseBufs bufs;      // synthesis of max_cells cells
    double* rk_y = nullptr;   // RK4 stage state and slopes, max_cells x N^d each
    double* rk_k[4] = {nullptr, nullptr, nullptr, nullptr};
    double* partial = nullptr;        // split-K partial tiles of the product
    hipGraph_t graph = nullptr;       // a captured evaluation (pgc_direct_capture)
    hipGraphExec_t exec = nullptr;
    double setup_ms = 0.0;
    int64_t bytes = 0;
    std::vector<void*> allocations;
};

namespace {

hipError_t d_alloc(pgc_direct_s& d, void** ptr, size_t bytes)
{
    *ptr = nullptr;
    d.allocations.push_back(nullptr);  // the slot first: a throwing push_back leaks no device memory
    hipError_t e = hipMalloc(&d.allocations.back(), std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
        d.allocations.pop_back();
        return e;
    }
    *ptr = d.allocations.back();
    d.bytes += (int64_t)bytes;
    return hipSuccess;
}

template <typename T>
hipError_t d_alloc_n(pgc_direct_s& d, T** ptr, int64_t n)
{
    void* v = nullptr;
    hipError_t e = d_alloc(d, &v, (size_t)n * sizeof(T));
    *ptr = static_cast<T*>(v);
    return e;
}

template <typename T>
hipError_t d_upload(pgc_direct_s& d, T** ptr, const std::vector<T>& src)
{
    hipError_t e = d_alloc_n(d, ptr, (int64_t)src.size());
    if (e == hipSuccess && !src.empty())
        e = hipMemcpy(*ptr, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

// Q of nc <= max_cells cells: synthesis, pair products, the FP64 product
pgc_status direct_chunk(pgc_direct_s& d, const double* c, int nc, double* q, hipStream_t s)
{
    const pgc::Plan& p = d.plan->p;
    hipError_t e = pgc::launch_dense_synthesis(p, c, nc, d.bufs, s);
    if (e != hipSuccess) return pgc::status_of(e);
    const int64_t n_threads = (d.n_pairs + 1) / 2;
    hipLaunchKernelGGL(pgc::pair_products, dim3((unsigned)((n_threads + 255) / 256),
                                                (unsigned)((nc + pgc::kPairCells - 1) / pgc::kPairCells)),
                       dim3(256), 0, s, d.bufs.G, d.pa, d.pb, d.n_pairs, d.ldx, d.nid, nc, d.X);
    if ((e = hipGetLastError()) != hipSuccess) return pgc::status_of(e);
    // Q (nc x N^d) = X (nc x n_pairs, row stride ldx) K (n_pairs x N^d)
    return pgc::status_of(pgc::gemm_launch(d.X, d.ldx, d.K, d.Nd, q, d.Nd, nc, (int)d.Nd, d.n_pairs, d.partial, s));
}

void d_free(pgc_direct_s* d)
{
    if (!d) return;
    (void)hipDeviceSynchronize();
    if (d->exec) (void)hipGraphExecDestroy(d->exec);
    if (d->graph) (void)hipGraphDestroy(d->graph);
    for (void* p : d->allocations) (void)hipFree(p);
    delete d;
}

}  // namespace

extern "C" {

pgc_status pgc_direct_create(pgc_plan plan, int32_t max_cells, void* stream, pgc_direct* out)
{
    if (!plan || !out || max_cells < 1 || max_cells > 65535) return PGC_ERR_INVALID_ARG;
    *out = nullptr;
    const pgc::Plan& p = plan->p;
    if (p.precision != PGC_PRECISION_FP64) return PGC_ERR_UNSUPPORTED;
    const int64_t nid = p.nid, Nd = p.Nd;
    const int64_t n_pairs = nid * (nid + 1) / 2;
    // one workgroup per pair: the grid's work-items must fit 32 bits
    if (Nd > (int64_t)pgc::kMaxPerThread * pgc::kDirThreads || n_pairs * pgc::kDirThreads > 4294967295ll ||
        n_pairs * Nd * (int64_t)sizeof(double) > pgc::kMaxTensorBytes)
        return PGC_ERR_UNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    pgc_direct_s* d = nullptr;
    pgc_status st = PGC_OK;
    hipError_t e = hipSuccess;
    try {  // host containers throw only on allocation failure
        d = new pgc_direct_s();
        d->plan = plan;
        d->max_cells = max_cells;
        d->n_pairs = n_pairs;
        d->ldx = (n_pairs + 1) / 2 * 2;
        d->nid = nid;
        d->Nd = Nd;
        // unordered pairs a <= b of flat interior-node indices, row by row
        std::vector<int> pa((size_t)n_pairs), pb((size_t)n_pairs);
        int64_t q = 0;
        for (int64_t a = 0; a < nid; ++a)
            for (int64_t b = a; b < nid; ++b) {
                pa[(size_t)q] = (int)a;
                pb[(size_t)q] = (int)b;
                ++q;
            }
        // per-dimension factor of T^_k at the nodes: T_k(xi_i) / sqrt(c_k) / mu_i^2
        std::vector<double> ltab((size_t)p.ni * p.N);
        for (int i = 0; i < p.ni; ++i)
            for (int k = 0; k < p.N; ++k) ltab[(size_t)i * p.N + k] = p.C[(size_t)i * p.N + k] / p.mu21[i];
        if ((e = d_upload(*d, &d->pa, pa)) == hipSuccess && (e = d_upload(*d, &d->pb, pb)) == hipSuccess) {
            double *v1 = nullptr, *lt = nullptr, *sig = nullptr, *sw = nullptr;
            const int64_t L = std::max(p.N, p.ni);
            int64_t t = 1;
            for (int l = 0; l < p.dim; ++l) t *= L;
            if ((e = d_upload(*d, &v1, p.v1)) == hipSuccess && (e = d_upload(*d, &lt, ltab)) == hipSuccess &&
                (e = d_upload(*d, &sig, p.sigma)) == hipSuccess && (e = d_upload(*d, &sw, p.sigma_w)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->K, n_pairs * Nd)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->X, (int64_t)max_cells * d->ldx)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->bufs.P, (int64_t)max_cells * nid)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->bufs.G, (int64_t)max_cells * nid)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->bufs.tmpA, (int64_t)max_cells * t)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->bufs.tmpB, (int64_t)max_cells * t)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->rk_y, (int64_t)max_cells * Nd)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->rk_k[0], (int64_t)max_cells * Nd)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->rk_k[1], (int64_t)max_cells * Nd)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->rk_k[2], (int64_t)max_cells * Nd)) == hipSuccess &&
                (e = d_alloc_n(*d, &d->rk_k[3], (int64_t)max_cells * Nd)) == hipSuccess) {
                hipEvent_t e0 = nullptr, e1 = nullptr;
                (void)hipEventCreate(&e0);
                (void)hipEventCreate(&e1);
                (void)hipEventRecord(e0, s);
                const size_t lds = sizeof(double) * pgc::kSigChunk * (p.dim * p.N + 1);
                const int radial = p.kernel == PGC_KERNEL_MAXWELL ? 0 : 1;
                if (p.dim == 2)
                    hipLaunchKernelGGL(pgc::direct_tensor<2>, dim3((unsigned)n_pairs), dim3(pgc::kDirThreads), lds, s,
                                       d->pa, d->pb, n_pairs, v1, lt, sig, sw, p.n_sigma, p.N, p.ni, (int)Nd, p.map,
                                       p.S, p.b0, p.gamma, radial, p.aniso, d->K);
                else
                    hipLaunchKernelGGL(pgc::direct_tensor<3>, dim3((unsigned)n_pairs), dim3(pgc::kDirThreads), lds, s,
                                       d->pa, d->pb, n_pairs, v1, lt, sig, sw, p.n_sigma, p.N, p.ni, (int)Nd, p.map,
                                       p.S, p.b0, p.gamma, radial, p.aniso, d->K);
                e = hipGetLastError();
                (void)hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                float ms = 0.0f;
                if (e == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) d->setup_ms = ms;
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
            }
        }
        if (e == hipSuccess) {
            // split-K partial tiles: the largest any chunk size up to max_cells needs
            int64_t part = 0;
            for (int nc = 1; nc <= max_cells; ++nc)
                part = std::max(part, pgc::gemm_partial_elems(nc, (int)Nd, n_pairs));
            if (part > 0) e = d_alloc_n(*d, &d->partial, part);
        }
    } catch (...) {
        st = PGC_ERR_OUT_OF_MEMORY;
    }
    if (st == PGC_OK && e != hipSuccess) st = pgc::status_of(e);
    if (st != PGC_OK) {
        d_free(d);
        return st;
    }
    *out = d;
    return PGC_OK;
}

pgc_status pgc_direct_destroy(pgc_direct d)
{
    d_free(d);
    return PGC_OK;
}

pgc_status pgc_direct_query(pgc_direct d, pgc_direct_info* info)
{
    if (!d || !info) return PGC_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    info->n_pairs = d->n_pairs;
    info->n_modes_total = d->Nd;
    info->max_cells = d->max_cells;
    info->tensor_bytes = d->n_pairs * d->Nd * (int64_t)sizeof(double);
    info->workspace_bytes = d->bytes;
    info->setup_ms = d->setup_ms;
    info->flops_per_cell = 2.0 * (double)d->n_pairs * (double)d->Nd;
    return PGC_OK;
}

pgc_status pgc_direct_coeffs_to_q(pgc_direct d, const double* coeffs_dev, int64_t n_cells, double* q_dev,
                                  void* stream)
{
    if (!d || n_cells < 0 || (n_cells > 0 && (!coeffs_dev || !q_dev))) return PGC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int64_t c0 = 0; c0 < n_cells; c0 += d->max_cells) {
        const int nc = (int)std::min<int64_t>(d->max_cells, n_cells - c0);
        const pgc_status st = direct_chunk(*d, coeffs_dev + c0 * d->Nd, nc, q_dev + c0 * d->Nd, s);
        if (st != PGC_OK) return st;
    }
    return PGC_OK;
}

pgc_status pgc_direct_capture(pgc_direct d, const double* coeffs_dev, int64_t n_cells, double* q_dev, void* stream)
{
    if (!d || n_cells < 1 || !coeffs_dev || !q_dev) return PGC_ERR_INVALID_ARG;
    if (d->exec) (void)hipGraphExecDestroy(d->exec);
    if (d->graph) (void)hipGraphDestroy(d->graph);
    d->exec = nullptr;
    d->graph = nullptr;
    // one eager evaluation first (it also writes q_dev)
    pgc_status st = pgc_direct_coeffs_to_q(d, coeffs_dev, n_cells, q_dev, stream);
    if (st != PGC_OK) return st;
    hipStream_t user = static_cast<hipStream_t>(stream);
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamSynchronize(user);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return pgc::status_of(e);
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = pgc_direct_coeffs_to_q(d, coeffs_dev, n_cells, q_dev, cs);
        e = hipStreamEndCapture(cs, &d->graph);
    }
    if (st == PGC_OK && e == hipSuccess) e = hipGraphInstantiate(&d->exec, d->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (st == PGC_OK && e != hipSuccess) st = pgc::status_of(e);
    if (st != PGC_OK) {
        if (d->exec) (void)hipGraphExecDestroy(d->exec);
        if (d->graph) (void)hipGraphDestroy(d->graph);
        d->exec = nullptr;
        d->graph = nullptr;
    }
    return st;
}

pgc_status pgc_direct_graph_launch(pgc_direct d, void* stream)
{
    if (!d || !d->exec) return PGC_ERR_INVALID_ARG;
    return pgc::status_of(hipGraphLaunch(d->exec, static_cast<hipStream_t>(stream)));
}

pgc_status pgc_direct_rk4(pgc_direct d, double* coeffs_dev, int64_t n_cells, double dt, int32_t n_steps,
                          void* stream)
{
    if (!d || n_cells < 0 || n_steps < 0 || !std::isfinite(dt) || (n_cells > 0 && !coeffs_dev))
        return PGC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double a[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
    // cells are independent: each chunk takes all its steps in turn
    for (int64_t c0 = 0; c0 < n_cells; c0 += d->max_cells) {
        const int nc = (int)std::min<int64_t>(d->max_cells, n_cells - c0);
        const int64_t n = (int64_t)nc * d->Nd;
        const unsigned blocks = (unsigned)((n + 255) / 256);
        double* base = coeffs_dev + c0 * d->Nd;
        for (int step = 0; step < n_steps; ++step) {
            for (int r = 0; r < 4; ++r) {
                const double* y = base;
                if (r > 0) {
                    hipLaunchKernelGGL(pgc::rk_axpy, dim3(blocks), dim3(256), 0, s, base, d->rk_k[r - 1], a[r],
                                       d->rk_y, n);
                    y = d->rk_y;
                }
                const pgc_status st = direct_chunk(*d, y, nc, d->rk_k[r], s);
                if (st != PGC_OK) return st;
            }
            hipLaunchKernelGGL(pgc::rk_combine, dim3(blocks), dim3(256), 0, s, base, d->rk_k[0], d->rk_k[1],
                               d->rk_k[2], d->rk_k[3], dt, n);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return pgc::status_of(e);
        }
    }
    return PGC_OK;
}

}  // extern "C"
