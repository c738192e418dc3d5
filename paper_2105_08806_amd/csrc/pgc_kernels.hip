// gfx950 kernels of the fast Petrov-Galerkin collision operator.
//
// Data flow of one evaluation Q = Q+ - Q- (Sec. 4.2 of arXiv 2105.08806):
//   synthesis   f_k -> P_i (interior CGL nodes), G_i = w_i mu_i^2 P_i
//   loss        A_i (inner sum of eq. Qminus), H_i = w_i A_i P_i, Q- = C^T H
//   gain        every collision triple (sigma_s, xi_i, eta_j) becomes one point
//               z = arccos(xi(v')) with weight q = W_s w_i g_i w_j g_j B mu(zeta)^-2
//               (eq. num_fast_k); all points of all units (s, i) are spread onto
//               ONE folded fine grid (the sums over s and i are linear, so the
//               paper's per-(sigma, xi) transforms of eq. (nufft) merge), then a
//               cosine transform with deconvolution gives Q+ directly (the
//               sign-pattern retrieval that follows eq. (nufft) is built into the
//               folded grid).
//   combine     Q = Q+ - Q-
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "pgc_device.h"
#include "pgc_internal.h"

namespace pgc {
namespace {

constexpr int kRedThreads = 1024;

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// ------------------------------------------------------------------ transforms

// out[a][k][b] = sum_l M[k][l] in[a][l][b]   (a < A, k < K, b < B)
template <typename T>
__global__ void __launch_bounds__(256) sep_apply(const T* __restrict__ in, T* __restrict__ out,
                                                 const T* __restrict__ M, int64_t A, int L,
                                                 int64_t B, int K)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t total = A * K * B;
    if (idx >= total) return;
    const int64_t b = idx % B;
    const int64_t t = idx / B;
    const int k = (int)(t % K);
    const int64_t a = t / K;
    const T* src = in + a * (int64_t)L * B + b;
    const T* m = M + (int64_t)k * L;
    T acc = 0;
    for (int l = 0; l < L; ++l) acc = fma(m[l], src[(int64_t)l * B], acc);
    out[idx] = acc;
}

// One pass of sep_apply for larger sizes: a workgroup computes 16 outputs k
// by 16 columns (a, b) from the tile's rows of M and columns of the input,
// staged in LDS, so the FMA chains read LDS instead of waiting on L2 at every
// step.  Each output is sep_apply's FMA chain in the same order.
constexpr int kSepTile = 16;
constexpr int kSepTiledMaxL = 256;  // 2 x 16 x L doubles of LDS

__global__ void __launch_bounds__(kSepTile * kSepTile) sep_tiled(const double* __restrict__ in,
                                                                double* __restrict__ out,
                                                                const double* __restrict__ M, int64_t A,
                                                                int L, int64_t B, int K)
{
    extern __shared__ double sep_tile[];
    double* sm = sep_tile;                  // sm[kk L + l]
    double* sx = sep_tile + kSepTile * L;   // sx[l 16 + cc]
    const int64_t c0 = blockIdx.x * (int64_t)kSepTile;
    const int k0 = blockIdx.y * kSepTile;
    const int64_t ncol = A * B;
    for (int i = threadIdx.x; i < kSepTile * L; i += kSepTile * kSepTile) {
        const int kk = i / L, l = i % L;
        sm[i] = (k0 + kk < K) ? M[(int64_t)(k0 + kk) * L + l] : 0.0;
    }
    for (int i = threadIdx.x; i < kSepTile * L; i += kSepTile * kSepTile) {
        const int l = i / kSepTile, cc = i % kSepTile;
        const int64_t c = c0 + cc;
        double v = 0.0;
        if (c < ncol) v = in[((c / B) * L + l) * B + c % B];
        sx[i] = v;
    }
    __syncthreads();
    const int cc = threadIdx.x % kSepTile, kk = threadIdx.x / kSepTile;
    const int64_t c = c0 + cc;
    const int k = k0 + kk;
    if (c >= ncol || k >= K) return;
    const double* m = sm + kk * L;
    double acc = 0;
    for (int l = 0; l < L; ++l) acc = fma(m[l], sx[l * kSepTile + cc], acc);
    out[((c / B) * K + k) * B + c % B] = acc;
}

// flat interior-node index -> product of per-dimension tables
template <typename T>
__device__ __forceinline__ void node_weights(int64_t f, int dim, int ni, const T* __restrict__ w1,
                                             const T* __restrict__ mu21, T& w, T& mu2)
{
    w = 1;
    mu2 = 1;
    for (int l = dim - 1; l >= 0; --l) {
        const int a = (int)(f % ni);
        f /= ni;
        w *= w1[a];
        mu2 *= mu21[a];
    }
}

// G_i = w_i mu_i^2 P_i  (the weighted f_N / mu^2 of the gain and loss integrals),
// in FP64 and, when Gg is given, rounded once to the precision of the gain
template <typename T>
__global__ void make_weighted(const double* __restrict__ P, double* __restrict__ G,
                              T* __restrict__ Gg, const double* __restrict__ w1,
                              const double* __restrict__ mu21, int dim, int ni, int64_t nid,
                              int64_t n_total)
{
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // over n_cells * nid
    if (f >= n_total) return;
    double w, mu2;
    node_weights(f % nid, dim, ni, w1, mu21, w, mu2);
    const double g = w * mu2 * P[f];
    G[f] = g;
    if (Gg) Gg[f] = (T)g;
}

template <typename T>
__global__ void widen(const T* __restrict__ x, double* __restrict__ y, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = (double)x[i];
}

template <typename T>
__global__ void narrow(const double* __restrict__ x, T* __restrict__ y, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = (T)x[i];
}

// ------------------------------------------------------------------ loss

// red[c] = sum_j G_j of cell c = blockIdx.x (Maxwell molecules: the inner
// integral of eq. Qminus is a single number; fixed order within one workgroup)
// the sum of g[0 .. n) over a workgroup of kRedThreads threads, in one fixed
// order; thread 0 receives it
__device__ __forceinline__ double block_sum(const double* __restrict__ g, int64_t n)
{
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    for (int64_t f = threadIdx.x; f < n; f += kRedThreads) acc += g[f];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedThreads / 64; ++w) t += sh[w];
    return t;
}

__global__ void __launch_bounds__(kRedThreads) sum_kernel(const double* __restrict__ G, int64_t n,
                                                          double* __restrict__ red)
{
    const double t = block_sum(G + blockIdx.x * n, n);
    if (threadIdx.x == 0) red[blockIdx.x] = t;
}

// H_i = w_i A P_i with A = (sum_s W_s) b0 sum_j G_j, over n_cells * nid nodes
__global__ void loss_h_maxwell(const double* __restrict__ P, double* __restrict__ H,
                               const double* __restrict__ w1, const double* __restrict__ mu21,
                               const double* __restrict__ red, double scale, int dim, int ni,
                               int64_t nid, int64_t n_total)
{
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= n_total) return;
    double w, mu2;
    node_weights(f % nid, dim, ni, w1, mu21, w, mu2);
    H[f] = w * (scale * red[f / nid]) * P[f];
}

// Q = Q+ - Q- formed in FP64, rounded once to the output precision (and Q+
// when qplus_out is given)
template <typename T>
__global__ void combine_kernel(const double* __restrict__ qp, const double* __restrict__ qm,
                               T* __restrict__ q, T* __restrict__ qplus_out, int64_t n)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double a = qp[k];
    q[k] = (T)(a - qm[k]);
    if (qplus_out) qplus_out[k] = (T)a;
}

// What a transform reads before its first pass and writes after its last
// besides its output, so that the elementwise stages around a small transform
// run inside it.  Where the transform is not fused, separable() launches the
// kernels of those stages around its passes instead; both forms compute the
// same values in the same order.
struct SepIO {
    // input: 0 = the input tensor; 1 = the Maxwell loss field of eq. Qminus,
    // H_i = w_i (scale sum_j G_j) P_i over the ni^dim interior nodes (the
    // unfused form writes it to H, with the sum in red)
    int pro = 0;
    const double* P = nullptr;
    const double* G = nullptr;
    double scale = 0.0;
    double* H = nullptr;
    double* red = nullptr;
    // after the last pass: 0 = nothing; 1 = G_i = w_i mu_i^2 out_i (Gout) and,
    // when Gg is given, G rounded once to the plan precision (FP32 if gg_f32)
    int epi = 0;
    double* Gout = nullptr;
    void* Gg = nullptr;
    int gg_f32 = 0;
    // 2 = Q = out - qm and Q+ = out rounded to the plan precision into q and,
    // when given, qp (FP32 if q_f32), as combine_kernel forms them
    const double* qm = nullptr;
    void* q = nullptr;
    void* qp = nullptr;
    int q_f32 = 0;
    // node tables of the prologue and epilogue (ni nodes per dimension)
    const double* w1 = nullptr;
    const double* mu21 = nullptr;
    int ni = 0;
};

// Every pass of separable() for one tensor per workgroup (small plans, where a
// pass is a few thousand outputs and passes launched one by one wait on one
// another's latency).  The tensor and the matrix are first copied to LDS by
// independent loads, then every pass reads and writes LDS only, except the
// last, which writes the output.  Each output is the FMA chain of sep_apply in
// the same order, so both forms agree bit for bit; the prologue's sum is
// block_sum over the same number of threads as sum_kernel.
constexpr int kSepFusedThreads = kRedThreads;
constexpr int64_t kSepFusedMaxFma = int64_t(1) << 18;  // per tensor, over all passes
constexpr int kSepFusedMaxLds = 64 * 1024;

// LDS layout, in doubles: M (K L), the input tensor (L^dim), then the
// intermediates of the passes before the last (two ping-pong buffers)
__global__ void __launch_bounds__(kSepFusedThreads) sep_fused(const double* __restrict__ in,
                                                              double* __restrict__ out,
                                                              const double* __restrict__ M, int dim,
                                                              int L, int K, int lds0, SepIO io)
{
    extern __shared__ double sep_lds[];
    int Ld = 1, Kd = 1;
    for (int l = 0; l < dim; ++l) {
        Ld *= L;
        Kd *= K;
    }
    double* sm = sep_lds;
    double* sx = sm + K * L;
    for (int i = threadIdx.x; i < K * L; i += kSepFusedThreads) sm[i] = M[i];
    const int64_t cell = blockIdx.x;
    if (io.pro == 1) {
        const double t = block_sum(io.G + cell * Ld, Ld);
        __shared__ double a_sh;
        if (threadIdx.x == 0) a_sh = io.scale * t;
        __syncthreads();
        const double A = a_sh;
        const double* P = io.P + cell * Ld;
        for (int i = threadIdx.x; i < Ld; i += kSepFusedThreads) {
            double w, mu2;
            node_weights(i, dim, io.ni, io.w1, io.mu21, w, mu2);
            sx[i] = w * A * P[i];
        }
    } else {
        const double* g = in + cell * Ld;
        for (int i = threadIdx.x; i < Ld; i += kSepFusedThreads) sx[i] = g[i];
    }
    __syncthreads();
    double* bufs[2] = {sx + Ld, sx + Ld + lds0};
    const double* src = sx;
    int dims[3] = {L, L, L};
    int pp = 0;
    for (int ax = dim - 1; ax >= 0; --ax) {
        const bool last = ax == 0;
        double* dst = last ? out + cell * Kd : bufs[pp];
        pp ^= 1;
        int A = 1, B = 1;
        for (int l = 0; l < ax; ++l) A *= dims[l];
        for (int l = ax + 1; l < dim; ++l) B *= dims[l];
        const int total = A * K * B;
        for (int idx = threadIdx.x; idx < total; idx += kSepFusedThreads) {
            const int b = idx % B;
            const int t = idx / B;
            const int k = t % K;
            const int a = t / K;
            const double* x = src + (a * L) * B + b;
            const double* m = sm + k * L;
            double acc = 0;
            for (int l = 0; l < L; ++l) acc = fma(m[l], x[l * B], acc);
            dst[idx] = acc;
            if (last && io.epi == 1) {
                double w, mu2;
                node_weights(idx, dim, io.ni, io.w1, io.mu21, w, mu2);
                const double g = w * mu2 * acc;
                io.Gout[cell * Kd + idx] = g;
                if (io.Gg) {
                    if (io.gg_f32) static_cast<float*>(io.Gg)[cell * Kd + idx] = (float)g;
                    else static_cast<double*>(io.Gg)[cell * Kd + idx] = g;
                }
            } else if (last && io.epi == 2) {
                const int64_t o = cell * Kd + idx;
                const double d = acc - io.qm[o];
                if (io.q_f32) {
                    static_cast<float*>(io.q)[o] = (float)d;
                    if (io.qp) static_cast<float*>(io.qp)[o] = (float)acc;
                } else {
                    static_cast<double*>(io.q)[o] = d;
                    if (io.qp) static_cast<double*>(io.qp)[o] = acc;
                }
            }
        }
        if (!last) __syncthreads();
        dims[ax] = K;
        src = dst;
    }
}

// apply the K x L matrix M along every axis of nb consecutive dim-dimensional
// L^dim tensors (FP64), with the input and output stages io; tmpA and tmpB
// hold nb * max(K, L)^dim values each
hipError_t separable(const Plan& p, const double* in, double* out, const double* M, int K, int L,
                     int nb, double* tmpA, double* tmpB, hipStream_t s, const SepIO& io = SepIO{})
{
    {
        // the fused form when every intermediate of one tensor fits in LDS and
        // the work per tensor is small; the choice depends on the sizes only
        int64_t fma_n = 0, lds[2] = {0, 0}, cur = 1;
        for (int l = 0; l < p.dim; ++l) cur *= L;
        const int64_t staged = (int64_t)K * L + cur;  // M and the input tensor
        for (int ax = p.dim - 1, pp = 0; ax >= 0; --ax, pp ^= 1) {
            cur = cur / L * K;
            fma_n += cur * L;
            if (ax > 0) lds[pp] = std::max(lds[pp], cur);
        }
        const int64_t lds_bytes = (staged + lds[0] + lds[1]) * (int64_t)sizeof(double);
        if (p.dim >= 2 && fma_n <= kSepFusedMaxFma && lds_bytes <= kSepFusedMaxLds) {
            hipLaunchKernelGGL(sep_fused, dim3(nb), dim3(kSepFusedThreads), (size_t)lds_bytes, s, in, out, M,
                               p.dim, L, K, (int)lds[0], io);
            return hipGetLastError();
        }
    }
    int64_t Ld = 1;
    for (int l = 0; l < p.dim; ++l) Ld *= L;
    if (io.pro == 1) {
        const int64_t n = (int64_t)nb * Ld;
        hipLaunchKernelGGL(sum_kernel, dim3(nb), dim3(kRedThreads), 0, s, io.G, Ld, io.red);
        hipLaunchKernelGGL(loss_h_maxwell, dim3(blocks_for(n, 256)), dim3(256), 0, s, io.P, io.H, io.w1,
                           io.mu21, io.red, io.scale, p.dim, io.ni, Ld, n);
        in = io.H;
    }
    int64_t dims[3] = {L, L, L};
    const double* src = in;
    double* bufs[2] = {tmpA, tmpB};
    int pp = 0;
    for (int ax = p.dim - 1; ax >= 0; --ax) {
        double* dst = (ax == 0) ? out : bufs[pp];
        pp ^= 1;
        int64_t A = nb, B = 1;
        for (int l = 0; l < ax; ++l) A *= dims[l];
        for (int l = ax + 1; l < p.dim; ++l) B *= dims[l];
        if (L <= kSepTiledMaxL) {
            const dim3 grid(blocks_for(A * B, kSepTile), blocks_for(K, kSepTile));
            const size_t lds = (size_t)2 * kSepTile * L * sizeof(double);
            hipLaunchKernelGGL(sep_tiled, grid, dim3(kSepTile * kSepTile), lds, s, src, dst, M, A, L, B, K);
        } else {
            const int64_t total = A * K * B;
            const int threads = 256;
            const int64_t blocks = (total + threads - 1) / threads;
            hipLaunchKernelGGL(sep_apply<double>, dim3((unsigned)blocks), dim3(threads), 0, s, src, dst, M,
                               A, L, B, K);
        }
        dims[ax] = K;
        src = dst;
    }
    int64_t Kd = 1;
    for (int l = 0; l < p.dim; ++l) Kd *= K;
    const int64_t n = (int64_t)nb * Kd;
    if (io.epi == 2) {
        if (io.q_f32)
            hipLaunchKernelGGL(combine_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, out, io.qm,
                               static_cast<float*>(io.q), static_cast<float*>(io.qp), n);
        else
            hipLaunchKernelGGL(combine_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, out, io.qm,
                               static_cast<double*>(io.q), static_cast<double*>(io.qp), n);
    }
    if (io.epi == 1) {
        if (io.gg_f32)
            hipLaunchKernelGGL(make_weighted<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, out, io.Gout,
                               static_cast<float*>(io.Gg), io.w1, io.mu21, p.dim, io.ni, Kd, n);
        else
            hipLaunchKernelGGL(make_weighted<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, out, io.Gout,
                               static_cast<double*>(io.Gg), io.w1, io.mu21, p.dim, io.ni, Kd, n);
    }
    return hipGetLastError();
}

// The angular factor of an angle-dependent rate in the loss.  With
// B = b0 |u|^gamma (1 + beta cos^2 theta) the inner integral over the sphere
// is sum_s W_s (1 + beta (u.sigma_s)^2 / |u|^2) = W (1 + u^T M u / |u|^2)
// with W = sum_s W_s and M = (beta / W) sum_s W_s sigma_s sigma_s^T (a d x d
// form, upper triangle m[0..5] = M11 M12 M13 M22 M23 M33; M22 = m[3] in 2D as
// well), so the loss stays one sum over node pairs.  on = 0: no factor.
struct AngleForm {
    double m[6];
    int on;
};

// VHS: A_i = (sum_s W_s) b0 sum_j G_j |v_i - v_j|^gamma (times the angular
// factor for an angle-dependent rate) over the nodes of cell blockIdx.y.  A
// workgroup takes kVhsI nodes i and splits the sweep over j into kVhsJ
// contiguous slices, one lane per (i, slice), then adds the slices of each i
// in slice order: one cell alone fills the chip, and the summation order
// depends on the sizes only.  The per-dimension node table (ni values) is in
// dynamic LDS.
constexpr int kVhsI = 8, kVhsJ = 32;
constexpr int kVhsMaxTableBytes = 60 * 1024;
template <int DIM>
__global__ void __launch_bounds__(kVhsI * kVhsJ) loss_h_vhs(const double* __restrict__ P,
                                                           const double* __restrict__ G,
                                                           double* __restrict__ H,
                                                           const double* __restrict__ v1,
                                                           const double* __restrict__ w1,
                                                           const double* __restrict__ mu21, double scale,
                                                           double gamma, int ni, int64_t nid, AngleForm af)
{
    extern __shared__ double sv[];
    __shared__ double part[kVhsJ][kVhsI];
    for (int a = threadIdx.x; a < ni; a += kVhsI * kVhsJ) sv[a] = v1[a];
    const int64_t cell = blockIdx.y;
    const double* Gc = G + cell * nid;
    const int ii = threadIdx.x % kVhsI, js = threadIdx.x / kVhsI;
    const int64_t f = blockIdx.x * (int64_t)kVhsI + ii;
    __syncthreads();
    double vi[DIM];
    {
        int64_t r = f < nid ? f : 0;
        for (int l = DIM - 1; l >= 0; --l) {
            vi[l] = sv[r % ni];
            r /= ni;
        }
    }
    // slice js: the nodes j in [j0, j1) of the flat order, walked by their
    // per-dimension indices (last dimension fastest)
    const int64_t span = (nid + kVhsJ - 1) / kVhsJ;
    const int64_t j0 = js * span < nid ? js * span : nid;
    const int64_t j1 = j0 + span < nid ? j0 + span : nid;
    int jd[DIM];
    {
        int64_t r = j0;
        for (int l = DIM - 1; l >= 0; --l) {
            jd[l] = (int)(r % ni);
            r /= ni;
        }
    }
    double acc = 0;
    for (int64_t j = j0; j < j1; ++j) {
        double u2 = 0, d[DIM];
        for (int l = 0; l < DIM; ++l) {
            d[l] = vi[l] - sv[jd[l]];
            u2 += d[l] * d[l];
        }
        double b;
        if (gamma == 1.0) b = sqrt(u2);
        else if (gamma == 0.0) b = 1;
        else b = u2 > 0 ? pow(u2, 0.5 * gamma) : 0.0;
        if (af.on && u2 > 0) {
            double quad;
            if constexpr (DIM == 2)
                quad = af.m[0] * d[0] * d[0] + 2.0 * af.m[1] * d[0] * d[1] + af.m[3] * d[1] * d[1];
            else
                quad = af.m[0] * d[0] * d[0] + af.m[3] * d[1] * d[1] + af.m[5] * d[2] * d[2] +
                       2.0 * (af.m[1] * d[0] * d[1] + af.m[2] * d[0] * d[2] + af.m[4] * d[1] * d[2]);
            b *= 1.0 + quad / u2;
        }
        acc = fma(Gc[j], b, acc);
        for (int l = DIM - 1; l >= 0; --l) {  // next j
            if (++jd[l] < ni) break;
            jd[l] = 0;
        }
    }
    part[js][ii] = acc;
    __syncthreads();
    if (js != 0 || f >= nid) return;
    double sum = 0;
    for (int k = 0; k < kVhsJ; ++k) sum += part[k][ii];
    double w, mu2;
    node_weights(f, DIM, ni, w1, mu21, w, mu2);
    H[cell * nid + f] = w * scale * sum * P[cell * nid + f];
}

// ------------------------------------------------------------------ gain

// Pair orbits.  v' = (v_i + v_j)/2 + |v_i - v_j| sigma/2 does not change when
// i_l and j_l are exchanged in any dimension l (each component of v_i + v_j
// and of (v_i - v_j)^2 is symmetric), so the 2^d triples (s, i, j) of one
// orbit share one point z.  The merged point carries the orbit sum
//   Sym(a, b) = sum over the distinct (i', j') of the orbit of G_i' G_j'
// for per-dimension unordered pairs a_l <= b_l.  Pairs are numbered
// p(a, b) = a n_i - a (a - 1)/2 + (b - a), so b runs contiguously for fixed a.
// Sym is stored [p_2][p_3][p_1] (3D) or [p_2][p_1] (2D): p_1 fastest.
template <typename T, int DIM>
__global__ void pair_orbit_sums(const T* __restrict__ G, T* __restrict__ sym,
                                const int* __restrict__ pair_a, const int* __restrict__ pair_b,
                                int ni, int np, int64_t n_total)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n_total) return;
    int pr[DIM];  // pair index per dimension, pr[0] = p_1
    {
        int64_t r = e;
        pr[0] = (int)(r % np);
        r /= np;
        for (int l = DIM - 1; l >= 1; --l) {
            pr[l] = (int)(r % np);
            r /= np;
        }
    }
    int a[DIM], b[DIM];
    double c = 1.0;
    for (int l = 0; l < DIM; ++l) {
        a[l] = pair_a[pr[l]];
        b[l] = pair_b[pr[l]];
        if (a[l] == b[l]) c *= 0.5;  // both orders of an equal pair are one triple
    }
    double acc = 0.0;
    for (int eps = 0; eps < (1 << DIM); ++eps) {
        int64_t x = 0, y = 0;
        for (int l = 0; l < DIM; ++l) {
            const bool sw = (eps >> l) & 1;
            x = x * ni + (sw ? b[l] : a[l]);
            y = y * ni + (sw ? a[l] : b[l]);
        }
        acc += (double)G[x] * (double)G[y];
    }
    sym[e] = (T)(c * acc);
}

// The fine grid accumulates in FP64 for both precisions: on gfx950 the LDS
// executes ds_add_f64 about 20x faster than ds_add_f32 (measured 7.4 vs 0.33
// lane-ops per clock per CU), and FP64 cells also remove the accumulation
// error of the FP32 path.
__device__ __forceinline__ void lds_add(double* addr, double v)
{
    __hip_atomic_fetch_add(addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// FP64 points need about 2x the registers of FP32 ones: 512 threads keep
// 256 VGPRs per lane available without spilling.
template <typename T>
constexpr int spread_max_threads() { return sizeof(T) == 8 ? 256 : 1024; }

// wave-uniform copy of lane p's value (p is uniform)
__device__ __forceinline__ int lane_get(int x, int p) { return __builtin_amdgcn_readlane(x, p); }
__device__ __forceinline__ float lane_get(float x, int p)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), p));
}
__device__ __forceinline__ double lane_get(double x, int p)
{
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), p);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), p);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T, int TERMS>
__device__ __forceinline__ T horner(const T* c, T s)
{
    T v = c[TERMS - 1];
#pragma unroll
    for (int d = TERMS - 2; d >= 0; --d) v = fma(v, s, c[d]);
    return v;
}

// One workgroup = (chunk of units, slab of fine-grid planes along the first
// dimension); the slab lives in LDS.  A unit is (a_1, s): the smaller node of
// the first-dimension pair and a direction.  A pencil fixes the pairs of the
// other dimensions; along it b_1 runs from a_1 to n_i - 1.  The first
// component of v' is non-decreasing in v_{b_1} (its derivative is
// (1 - sigma_1 cos)/2 >= 0), so the points reaching the slab form one
// contiguous b_1 range, found by a binary search against the slab window.
//
// Generation is per lane (each lane walks its own pencil); spreading is per
// wave: the lanes own the cells of one footprint -- (b, c) with a loop over
// the first-dimension offset a in 3D, (a, b) in 2D -- and the wave spreads the
// points of all its lanes one after the other.  Each lane evaluates the
// kernel cells it owns by Horner from the point's offsets; the point's data
// reaches the lanes through readlane.  The LDS atomics of one instruction then
// touch W consecutive cells per row, and the slab test on the first dimension
// is a scalar branch.
template <typename T, int DIM, int W>
__global__ void __launch_bounds__(spread_max_threads<T>()) gain_spread(GainParams<T> P)
{
    constexpr int TERMS = poly_terms(W);
    constexpr int NPASS = (W * W + 63) / 64;
    extern __shared__ unsigned char lds_raw[];
    double* slab = reinterpret_cast<double*>(lds_raw);

    const int blk = blockIdx.y;
    const int64_t c = blockIdx.x;
    const int p0 = blk * P.slab_planes;
    const int p1 = min(P.ng, p0 + P.slab_planes);
    const int plane = (DIM == 2) ? P.ng : P.ng * P.ng;
    const int slab_elems = (p1 - p0) * plane;
    for (int e = threadIdx.x; e < slab_elems; e += blockDim.x) slab[e] = 0;
    __syncthreads();

    const T vlo = P.slab_vlo[blk];
    const T vhi = P.slab_vhi[blk];
    const int ni = P.ni;
    const int np = P.np;
    const int npencil = (DIM == 2) ? np : np * np;
    const int64_t u0 = c * P.units_per_chunk;
    const int64_t u1 = min(P.n_units, u0 + P.units_per_chunk);
    const int64_t n_u = u1 - u0;
    const int64_t n_items = n_u * npencil;
    const T half = (T)0.5;
    const int lane = threadIdx.x & 63;

    // cells owned by this lane in each pass, and their kernel polynomials
    int own_x[NPASS], own_y[NPASS];
    bool own_ok[NPASS];
    T cx[NPASS][TERMS], cy[NPASS][TERMS];
#pragma unroll
    for (int r = 0; r < NPASS; ++r) {
        const int e = lane + 64 * r;
        own_ok[r] = e < W * W;
        own_x[r] = own_ok[r] ? e / W : 0;
        own_y[r] = own_ok[r] ? e % W : 0;
#pragma unroll
        for (int d = 0; d < TERMS; ++d) {
            cx[r][d] = P.poly[d * W + own_x[r]];
            cy[r][d] = P.poly[d * W + own_y[r]];
        }
    }

    // generation state of this lane
    int64_t item = threadIdx.x;
    bool have = false;
    int b1 = 0;
    T va1 = 0, r2 = 0, cs = 0;
    T sg[DIM], cen[DIM];
    const T* symrow = P.sym;

    while (true) {
        bool valid = false;
        T q = 0, sfr[DIM];
        int t0[DIM];
        for (int l = 0; l < DIM; ++l) {
            sfr[l] = 0;
            t0[l] = 0;
        }
        while (item < n_items) {
            if (!have) {
                const int64_t u = u0 + item % n_u;
                const int pencil = (int)(item / n_u);
                const int a1 = (int)(u / P.n_sigma);
                const int s = (int)(u % P.n_sigma);
                cs = P.wfac[s];
                for (int l = 0; l < DIM; ++l) sg[l] = P.sigma[s * DIM + l];
                va1 = P.v1[a1];
                const int pa = (DIM == 2) ? pencil : pencil / np;
                const T x = P.v1[P.pair_a[pa]], y = P.v1[P.pair_b[pa]];
                cen[1] = (x + y) * half;
                r2 = (x - y) * (x - y);
                if constexpr (DIM == 3) {
                    const int pb = pencil % np;
                    const T x2 = P.v1[P.pair_a[pb]], y2 = P.v1[P.pair_b[pb]];
                    cen[2] = (x2 + y2) * half;
                    r2 += (x2 - y2) * (x2 - y2);
                }
                symrow = P.sym + (int64_t)pencil * np + P.pair_base[a1] - a1;  // index by b_1
                int lo = a1, hi = ni;  // first b_1 whose v'_1 reaches the slab window
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const T vb = P.v1[mid];
                    const T d = va1 - vb;
                    const T v1p = (va1 + vb) * half + sqrt(d * d + r2) * sg[0] * half;
                    if (v1p < vlo) lo = mid + 1;
                    else hi = mid;
                }
                b1 = lo;
                have = true;
            }
            if (b1 >= ni) {
                have = false;
                item += blockDim.x;
                continue;
            }
            const T vb = P.v1[b1];
            const T d = va1 - vb;
            const T un = sqrt(d * d + r2);
            T vp[DIM];
            vp[0] = (va1 + vb) * half + un * sg[0] * half;
            if (vp[0] > vhi) {
                have = false;
                item += blockDim.x;
                continue;
            }
            const T sy = symrow[b1];
            ++b1;
            if (sy == (T)0) continue;
            q = cs * sy;
            if (P.vhs) q *= (P.gamma == (T)1) ? un : (un > (T)0 ? pow(un, P.gamma) : (T)(P.gamma == (T)0));
            for (int l = 1; l < DIM; ++l) vp[l] = cen[l] + un * sg[l] * half;
#pragma unroll
            for (int l = 0; l < DIM; ++l) {
                double z;
                T m2;
                map_point(vp[l], P, z, m2);
                q *= m2;
                const double xs = z * P.h_inv64 - 0.5 * W;
                const double tf = ceil(xs);
                t0[l] = (int)tf;
                sfr[l] = (T)(2.0 * (tf - xs) - 1.0);
            }
            valid = true;
            break;
        }

        const unsigned long long mask = __ballot(valid);
        if (mask == 0ull) break;

        // first-dimension kernel cells of this lane's point (3D: shared by the wave)
        T k1[W];
        if constexpr (DIM == 3) kernel_cells<T, W, TERMS>(P.poly, sfr[0], k1);

        unsigned long long rem = mask;
        while (rem) {
            const int p = __builtin_ctzll(rem);
            rem &= rem - 1ull;
            const T qp = lane_get(q, p);
            const int ta = lane_get(t0[0], p);
            const int tb = lane_get(t0[1], p);
            const T sa = lane_get(sfr[0], p);
            const T sb = lane_get(sfr[1], p);
            if constexpr (DIM == 2) {
#pragma unroll
                for (int r = 0; r < NPASS; ++r) {
                    const int m0 = fold_index(ta + own_x[r], P.nh);
                    if (own_ok[r] && m0 >= p0 && m0 < p1) {
                        const T val = qp * horner<T, TERMS>(cx[r], sa) * horner<T, TERMS>(cy[r], sb);
                        lds_add(slab + (m0 - p0) * plane + fold_index(tb + own_y[r], P.nh), (double)val);
                    }
                }
            } else {
                const int tc = lane_get(t0[2], p);
                const T sc = lane_get(sfr[2], p);
                T k1p[W];
#pragma unroll
                for (int a = 0; a < W; ++a) k1p[a] = lane_get(k1[a], p);
#pragma unroll
                for (int r = 0; r < NPASS; ++r) {
                    if (!own_ok[r]) continue;
                    const T val = qp * horner<T, TERMS>(cx[r], sb) * horner<T, TERMS>(cy[r], sc);
                    double* cell = slab + fold_index(tb + own_x[r], P.nh) * P.ng +
                                   fold_index(tc + own_y[r], P.nh) - (int64_t)p0 * plane;
#pragma unroll
                    for (int a = 0; a < W; ++a) {
                        const int m0 = fold_index(ta + a, P.nh);
                        if (m0 >= p0 && m0 < p1) lds_add(cell + m0 * plane, (double)(val * k1p[a]));
                    }
                }
            }
        }
    }
    __syncthreads();
    double* dst = P.partial + c * P.ngd + (int64_t)p0 * plane;
    for (int e = threadIdx.x; e < slab_elems; e += blockDim.x) dst[e] = slab[e];
}

// ------------------------------------------------------------------ binned gain
//
// The positions of the merged points depend on the plan only (not on f), so the
// plan sorts them once by the base cell of their spreading footprint (the
// corner t0 = ceil(z/h - W/2) in every dimension).  One evaluation then walks
// the bins: a wave regenerates 64 points of one bin, stages their kernel
// vectors in LDS and accumulates the bin's W^d footprint in registers, one
// lane per footprint column, before a single flush of W^d global FP64 atomics.

// Over the points of directions [s0, s0 + ns): MODE 0 counts the points of
// every bin, MODE 1 scatters their ids through 64-bit cursors (the whole
// index, plan time), MODE 2 through 32-bit ones (one chunk of a streamed index,
// every evaluation).
template <typename T, int DIM, int MODE>
__global__ void __launch_bounds__(256) bin_points(GainParams<T> P, BinGeo B,
                                                  unsigned int* __restrict__ count,
                                                  unsigned long long* __restrict__ cursor,
                                                  unsigned int* __restrict__ cursor32,
                                                  unsigned long long* __restrict__ ids)
{
    const int np = P.np;
    const int npencil = (DIM == 2) ? np : np * np;
    for (int64_t item = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; item < B.n_items;
         item += (int64_t)gridDim.x * blockDim.x) {
        const int pencil = (int)(item % npencil);
        const int64_t us = item / npencil;
        const int s = B.s0 + (int)(us % B.ns);
        const int a1 = (int)(us / B.ns);
        const int p2 = (DIM == 2) ? pencil : pencil / np;
        const int p3 = (DIM == 2) ? 0 : pencil % np;
        PairNodes<DIM> nd = pair_nodes<T, DIM>(P, a1, a1, p2, p3);
        for (int b1 = a1; b1 < P.ni; ++b1) {
            nd.b[0] = b1;
            T q, vp[DIM];
            point_velocity<T, DIM>(P, s, nd, q, vp);
            int64_t bin = 0;
#pragma unroll
            for (int l = 0; l < DIM; ++l) bin = bin * B.nb + bin_coord<T>((double)vp[l], P, B);
            if constexpr (MODE == 0) {
                atomicAdd(count + bin, 1u);
            } else if constexpr (MODE == 1) {
                const unsigned long long slot = atomicAdd(cursor + bin, 1ull);
                if (slot < B.id_cap) ids[slot] = pack_id<DIM>(s, nd);
            } else {
                const unsigned int slot = atomicAdd(cursor32 + bin, 1u);
                if (slot < B.id_cap) ids[slot] = pack_id<DIM>(s, nd);
            }
        }
    }
}

struct BinItems {
    int64_t n_items;             // work items of this launch
    const int* bin;              // bin of each work item
    const long long* begin;      // first id of the item
    const int* count;            // ids in the item (<= 64 * batches)
    const unsigned long long* ids;
    double* grid;                // n_g^d FP64 accumulation grid
    double* tiles;               // deterministic plans: one W^d tile per item (else nullptr)
    BinGeo geo;
};

// Lane layout of the binned gain.  A point's footprint has CELLS columns
// (3D: (b, c) pairs, 2D: b) of W cells each along the first dimension, which
// a lane keeps in registers.  LP lanes serve one point and G points are spread
// per step; a lane holds NPASS columns e = e0 + LP r.  Wide 3D footprints
// split the wave into G = 3 or 2 groups when the accumulators fit (ACC_MAX
// values per lane): every broadcast read of a first-dimension kernel vector
// then serves G points, which cuts the LDS traffic per point.  The FP64 bound
// gives three groups at W = 9 and two at W = 10 and 11: three at W = 11 (66
// accumulators) need more than 256 registers with the regeneration, and ran
// 1.1x slower at two waves per SIMD with spills, 1.6x slower at one.
template <typename T, int DIM, int W>
struct BinLayout {
    static constexpr int CELLS = (DIM == 2) ? W : W * W;
    static constexpr bool WIDE = CELLS > 64;
    static constexpr int ACC_MAX = sizeof(T) == 8 ? 48 : 96;
    static constexpr int VEC = 16 / (int)sizeof(T);
    // staged values per point, whole 16-byte vectors; a stride of a multiple
    // of 64 bytes would put every fourth lane's staging stores in the same
    // LDS banks, so such strides take one vector more
    static constexpr int STRIDE0 = (DIM * W + VEC - 1) / VEC * VEC;
    static constexpr int STRIDE = (STRIDE0 * (int)sizeof(T)) % 64 == 0 ? STRIDE0 + VEC : STRIDE0;
    static constexpr int STAGE_BYTES = 64 * STRIDE * (int)sizeof(T);
    // a wide layout with g groups fits when its accumulators do and one group's
    // FP64 partial tile fits in the stage buffer (groups are reduced one by one)
    static constexpr int lp_of(int g) { return 64 / g; }
    static constexpr int np_of(int g) { return (CELLS + lp_of(g) - 1) / lp_of(g); }
    static constexpr bool fits(int g) { return np_of(g) * W <= ACC_MAX && lp_of(g) * np_of(g) * W * 8 <= STAGE_BYTES; }
    static constexpr int G = !WIDE ? 64 / CELLS : (fits(3) ? 3 : (fits(2) ? 2 : 1));
    static constexpr int LP = !WIDE ? CELLS : lp_of(G);
    static constexpr int NPASS = (CELLS + LP - 1) / LP;
};

// One wave per work item (a run of ids of one bin), BinLayout lanes per point.
//
// Regeneration: a lane forms one point's velocity, then in every dimension the
// kernel offset and the map factor, from the fit of the bin's cell in v/S
// (cell_offset_v) or, in the few cells at the ends of the grid that have none,
// through w (map_w, cell_offset), and the W kernel values from the even and
// odd parts of the cells; the staged vectors are k_1, q k_2 (q the full weight
// with the orbit sum) and, in 3D, k_3.
template <typename T, int DIM, int W, bool ANISO>
__global__ void __launch_bounds__(64) gain_binned(GainParams<T> P, BinItems BI)
{
    using L = BinLayout<T, DIM, W>;
    constexpr int TERMS = poly_terms(W);
    constexpr int CELLS = L::CELLS, LP = L::LP, G = L::G, NPASS = L::NPASS;
    constexpr int STRIDE = L::STRIDE;
    // columns past the last one (partial last pass) read values of the same point
    static_assert(!L::WIDE || W + (LP * NPASS - 1) / W < STRIDE, "spare columns read out of the point");
    // the partial tile of one lane group is reduced through the stage buffer at a time
    static_assert(G == 1 || LP * NPASS * W * 8 <= L::STAGE_BYTES, "reduction buffer");
    __shared__ __align__(16) T stage[64 * STRIDE];

    const int lane = threadIdx.x;
    const int item = blockIdx.x;
    const int bin = BI.bin[item];
    const long long first = BI.begin[item];
    const int n = BI.count[item];

    // base cell of the bin and the offset fit of its cell in every dimension
    int t0[DIM];
    const double* fit[DIM];
    const double* fitv[DIM];
    {
        int r = bin;
        for (int l = DIM - 1; l >= 0; --l) {
            const int c = r % BI.geo.nb;
            t0[l] = c - BI.geo.off;
            fit[l] = P.cellfit + (int64_t)c * kCellFitStride;
            fitv[l] = P.cellfit_v + (int64_t)c * kCellFitVStride;
            r /= BI.geo.nb;
        }
    }
    const int g = lane / LP;
    const int e0 = lane % LP;
    const bool lane_on = g < G;

    // FP32 tiles are summed over one 64-point batch and then added into FP64;
    // FP64 tiles accumulate directly
    constexpr bool TWO_LEVEL = sizeof(T) < sizeof(double);
    double acc64[TWO_LEVEL ? NPASS : 1][TWO_LEVEL ? W : 1];
    T acc[NPASS][W];
#pragma unroll
    for (int r = 0; r < NPASS; ++r)
#pragma unroll
        for (int a = 0; a < W; ++a) {
            acc[r][a] = (T)0;
            if constexpr (TWO_LEVEL) acc64[r][a] = 0.0;
        }

    // the id of this lane's point in the next batch is loaded one batch ahead,
    // so its latency hides under the current batch's spreading
    unsigned long long id_next = lane < n ? BI.ids[first + lane] : 0ull;
    for (int base = 0; base < n; base += 64) {
        const int nv = min(64, n - base);
        const unsigned long long id = id_next;
        if (base + 64 + lane < n) id_next = BI.ids[first + base + 64 + lane];
        // regenerate one point per lane and stage its kernel vectors
        {
            T* st = stage + lane * STRIDE;
            if (lane < nv) {
                int s;
                const PairNodes<DIM> nd = unpack_id<DIM>(id, s);
                T q, vp[DIM];
                point_velocity<T, DIM>(P, s, nd, q, vp);
                if constexpr (ANISO) q *= orbit_sum_aniso<T, DIM>(P, s, nd);
                else q *= orbit_sum<T, DIM>(P, nd);
                double sv[DIM];
#pragma unroll
                for (int l = 0; l < DIM; ++l) {
                    // the bin's cell is the same on every lane: a uniform branch
                    T m2;
                    if (fitv[l][1] != 0.0) {
                        sv[l] = cell_offset_v(fitv[l], vp[l], P.inv_S64, m2);
                    } else {
                        const double w = map_w(vp[l], P, m2);
                        sv[l] = cell_offset(fit[l], w);
                    }
                    q *= m2;
                }
                // each kernel value is staged as soon as it is formed
                kernel_cells_eo_each<T, W, TERMS, DIM>(P.kpoly_eo, sv, [&](int l, int a, T v) {
                    st[l * W + a] = (l == 1) ? v * q : v;
                });
            } else {
#pragma unroll
                for (int a = 0; a < STRIDE; ++a) st[a] = (T)0;
            }
        }
        __syncthreads();
        if constexpr (TWO_LEVEL) {
#pragma unroll
            for (int r = 0; r < NPASS; ++r)
#pragma unroll
                for (int a = 0; a < W; ++a) acc[r][a] = (T)0;
        }
        // one staged point into the lane's columns.  Spare columns of a
        // partial last pass read values of the same point and accumulate
        // cells that are never flushed, so no pass carries a per-lane branch.
        auto spread_point = [&](int pnt) {
            const T* sp = stage + pnt * STRIDE;
            T k1[W];
#pragma unroll
            for (int a = 0; a < W; ++a) k1[a] = sp[a];
#pragma unroll
            for (int r = 0; r < NPASS; ++r) {
                const int e = e0 + LP * r;
                T t;
                if constexpr (DIM == 2) t = sp[W + e];
                else t = sp[W + e / W] * sp[2 * W + e % W];
#pragma unroll
                for (int a = 0; a < W; ++a) acc[r][a] = fma(t, k1[a], acc[r][a]);
            }
        };
        // full steps carry a point for every lane group (no per-lane guard, so
        // the LDS reads of the next step can be issued under this step's
        // arithmetic); a last partial step follows
        const int full = nv / G;
        if (lane_on) {
#pragma unroll 2
            for (int st_i = 0; st_i < full; ++st_i) spread_point(st_i * G + g);
            const int pnt = full * G + g;
            if (pnt < nv) spread_point(pnt);
        }
        if constexpr (TWO_LEVEL) {
#pragma unroll
            for (int r = 0; r < NPASS; ++r)
#pragma unroll
                for (int a = 0; a < W; ++a) acc64[r][a] += (double)acc[r][a];
        }
        __syncthreads();
    }
    double tot[NPASS][W];
#pragma unroll
    for (int r = 0; r < NPASS; ++r)
#pragma unroll
        for (int a = 0; a < W; ++a) {
            if constexpr (TWO_LEVEL) tot[r][a] = acc64[r][a];
            else tot[r][a] = (double)acc[r][a];
        }

    // groups of lanes that served different points hold partial sums of the
    // same cells: group 0 adds the others', one group at a time, through the
    // (now idle) stage buffer
    if constexpr (G > 1) {
        double* red = reinterpret_cast<double*>(stage);
        for (int gg = 1; gg < G; ++gg) {
            if (g == gg) {
#pragma unroll
                for (int r = 0; r < NPASS; ++r)
#pragma unroll
                    for (int a = 0; a < W; ++a) red[(e0 * NPASS + r) * W + a] = tot[r][a];
            }
            __syncthreads();
            if (g == 0) {
#pragma unroll
                for (int r = 0; r < NPASS; ++r)
#pragma unroll
                    for (int a = 0; a < W; ++a) tot[r][a] += red[(e0 * NPASS + r) * W + a];
            }
            __syncthreads();
        }
    }
    if (g != 0) return;
    if (BI.tiles) {
        // deterministic plans: the whole tile, [a][column], zeros included
        double* tile = BI.tiles + (int64_t)item * (W * CELLS);
#pragma unroll
        for (int r = 0; r < NPASS; ++r) {
            const int e = e0 + LP * r;
            if (e >= CELLS) continue;
#pragma unroll
            for (int a = 0; a < W; ++a) tile[a * CELLS + e] = tot[r][a];
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < NPASS; ++r) {
        const int e = e0 + LP * r;
        if (e >= CELLS) continue;
        int64_t rest;
        if constexpr (DIM == 2) rest = fold_index(t0[1] + e, P.nh);
        else rest = (int64_t)fold_index(t0[1] + e / W, P.nh) * P.ng + fold_index(t0[2] + e % W, P.nh);
        const int64_t plane = (DIM == 2) ? P.ng : (int64_t)P.ng * P.ng;
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const double v = tot[r][a];
            if (v != 0.0)
                __hip_atomic_fetch_add(BI.grid + fold_index(t0[0] + a, P.nh) * plane + rest, v,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Matrix-core variant of the binned gain for FP64 3D plans.  For one bin the
// footprint is tile[a][(b, c)] = sum_p kx_p[a] (q_p ky_p[b] kz_p[c]): a product
// of a W x P and a P x W^2 matrix over the P points of the bin.  Every staged
// batch of 64 points is contracted with v_mfma_f64_16x16x4f64 (rows a padded
// to 16, columns (b, c) in tiles of 16, four points per instruction), so the
// vector units only regenerate points and form the operands.
template <int W>
__global__ void __launch_bounds__(64) gain_binned_mfma(GainParams<double> P, BinItems BI)
{
    constexpr int TERMS = poly_terms(W);
    constexpr int CELLS = W * W;
    constexpr int NT = (CELLS + 15) / 16;
    constexpr int STRIDE = (3 * W + 1) / 2 * 2;  // kx[W], q ky[W], kz[W], padded to 16 bytes
    typedef double dvec4 __attribute__((ext_vector_type(4)));
    __shared__ __align__(16) double stage[64 * STRIDE];

    const int lane = threadIdx.x;
    const int item = blockIdx.x;
    const int bin = BI.bin[item];
    const long long first = BI.begin[item];
    const int n = BI.count[item];
    int t0[3];
    const double* fit[3];
    {
        int r = bin;
        for (int l = 2; l >= 0; --l) {
            const int c = r % BI.geo.nb;
            t0[l] = c - BI.geo.off;
            fit[l] = P.cellfit + (int64_t)c * kCellFitStride;
            r /= BI.geo.nb;
        }
    }
    // operand lanes: A[i][k] and B[k][j] come from lane i + 16 k (j = i), k < 4
    const int i16 = lane & 15, k4 = lane >> 4;
    dvec4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = dvec4{0.0, 0.0, 0.0, 0.0};

    for (int base = 0; base < n; base += 64) {
        const int nv = min(64, n - base);
        // regenerate one point per lane (as in gain_binned)
        {
            double* st = stage + lane * STRIDE;
            if (lane < nv) {
                const unsigned long long id = BI.ids[first + base + lane];
                int s;
                const PairNodes<3> nd = unpack_id<3>(id, s);
                double q, vp[3];
                point_velocity<double, 3>(P, s, nd, q, vp);
                q *= orbit_sum<double, 3>(P, nd);
                double sv[3];
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    double m2;
                    const double w = map_w(vp[l], P, m2);
                    q *= m2;
                    sv[l] = cell_offset(fit[l], w);
                }
                double k[3][W];
                kernel_cells_eo_dims<double, W, TERMS, 3>(P.kpoly_eo, sv, k);
#pragma unroll
                for (int l = 0; l < 3; ++l)
#pragma unroll
                    for (int a = 0; a < W; ++a) st[l * W + a] = (l == 1) ? k[l][a] * q : k[l][a];
            } else {
                for (int a = 0; a < STRIDE; ++a) st[a] = 0.0;
            }
        }
        __syncthreads();
        // lanes with i16 >= W (rows past the footprint) and columns past W^2
        // contribute zeros; their reads stay inside the point's staged values
        const int ksteps = (nv + 3) >> 2;
        for (int ks = 0; ks < ksteps; ++ks) {
            const double* sp = stage + (4 * ks + k4) * STRIDE;
            const double av = i16 < W ? sp[i16] : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int col = 16 * t + i16;
                const double bv = col < CELLS ? sp[W + col / W] * sp[2 * W + col % W] : 0.0;
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane l holds rows l / 16 + 4 r of column l % 16 of every tile (the FP64
    // 16 x 16 x 4 instruction interleaves rows over the lane groups)
    const int64_t plane = (int64_t)P.ng * P.ng;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = 16 * t + i16;
        if (col >= CELLS) continue;
        const int64_t rest = (int64_t)fold_index(t0[1] + col / W, P.nh) * P.ng + fold_index(t0[2] + col % W, P.nh);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = k4 + 4 * r;
            const double v = acc[t][r];
            if (a < W && v != 0.0)
                __hip_atomic_fetch_add(BI.grid + fold_index(t0[0] + a, P.nh) * plane + rest, v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Deterministic plans: grid[m] = the sum of every tile value that lands on the
// folded cell m, in a fixed order.  Cell m of one dimension receives the
// unfolded indices u = m, -m (m > 0) and 2 nh - m (m < nh); u lies in the
// footprint of the bins t0 = u - W + 1 .. u (offset u - t0), and each bin's
// runs are taken in run order.
template <int DIM>
__global__ void __launch_bounds__(256)
    gather_tiles(const double* __restrict__ tiles, const int* __restrict__ bin_ptr, const int* __restrict__ bin_items,
                 int nb, int off, int W, int nh, int ng, int64_t ngd, double* __restrict__ grid)
{
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= ngd) return;
    int m[DIM];
    {
        int64_t r = f;
#pragma unroll
        for (int l = DIM - 1; l >= 0; --l) {
            m[l] = (int)(r % ng);
            r /= ng;
        }
    }
    int cand[DIM][3], nc[DIM];
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
        nc[l] = 0;
        cand[l][nc[l]++] = m[l];
        if (m[l] > 0) cand[l][nc[l]++] = -m[l];
        if (m[l] < nh) cand[l][nc[l]++] = 2 * nh - m[l];
    }
    const int cells = (DIM == 2) ? W : W * W;  // columns of a tile
    const int64_t tile = (int64_t)W * cells;
    const int tlo = -off, thi = nb - 1 - off;
    double acc = 0.0;
    // one pass per combination of candidates, dimension 1 outermost
    int combos = 1;
#pragma unroll
    for (int l = 0; l < DIM; ++l) combos *= nc[l];
    for (int cb = 0; cb < combos; ++cb) {
        int u[DIM];
        {
            int r = cb;
#pragma unroll
            for (int l = DIM - 1; l >= 0; --l) {
                u[l] = cand[l][r % nc[l]];
                r /= nc[l];
            }
        }
        int lo[DIM], hi[DIM];
        bool empty = false;
#pragma unroll
        for (int l = 0; l < DIM; ++l) {
            lo[l] = max(u[l] - W + 1, tlo);
            hi[l] = min(u[l], thi);
            empty |= lo[l] > hi[l];
        }
        if (empty) continue;
        for (int t1 = lo[0]; t1 <= hi[0]; ++t1) {
            const int a = u[0] - t1;
            for (int t2 = lo[1]; t2 <= hi[1]; ++t2) {
                if constexpr (DIM == 2) {
                    const int bin = (t1 + off) * nb + (t2 + off);
                    const int idx = a * cells + (u[1] - t2);
                    for (int k = bin_ptr[bin]; k < bin_ptr[bin + 1]; ++k)
                        acc += tiles[(int64_t)bin_items[k] * tile + idx];
                } else {
                    for (int t3 = lo[2]; t3 <= hi[2]; ++t3) {
                        const int bin = ((t1 + off) * nb + (t2 + off)) * nb + (t3 + off);
                        const int idx = a * cells + (u[1] - t2) * W + (u[2] - t3);
                        for (int k = bin_ptr[bin]; k < bin_ptr[bin + 1]; ++k)
                            acc += tiles[(int64_t)bin_items[k] * tile + idx];
                    }
                }
            }
        }
    }
    grid[f] = acc;
}

__global__ void fill_zero(double* __restrict__ x, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

__global__ void copy_u32(const unsigned int* __restrict__ src, unsigned int* __restrict__ dst, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// grid[m] = sum_c partial[c][m], FP64 accumulation in chunk order
__global__ void reduce_partials(const double* __restrict__ partial, double* __restrict__ grid,
                                int64_t ngd, int n_chunks)
{
    const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (m >= ngd) return;
    double acc = 0.0;
    for (int c = 0; c < n_chunks; ++c) acc += partial[(int64_t)c * ngd + m];
    grid[m] = acc;
}


// ------------------------------------------------------------------ projection

// H_i = w_i mu_i^-4 f(v_i)  (eq. MultiD_spectral_coef on the interior CGL nodes)
__global__ void project_weight(const double* __restrict__ f, double* __restrict__ H,
                               const double* __restrict__ w1, const double* __restrict__ mu21,
                               int dim, int ni, int64_t nid)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nid) return;
    double w, mu2;
    node_weights(r, dim, ni, w1, mu21, w, mu2);
    H[r] = f[r] * w / (mu2 * mu2);
}

// ------------------------------------------------------------------ moments

// rho, rho u_l, E from 1D functionals m_p[k] = int v^p T~_k dv (FP64)
template <typename T>
__global__ void __launch_bounds__(kRedThreads) moments_kernel(const T* __restrict__ c,
                                                              const double* __restrict__ mom,
                                                              int dim, int N, int64_t Nd,
                                                              double* __restrict__ out)
{
    __shared__ double sh[5][kRedThreads / 64];
    double acc[5] = {0, 0, 0, 0, 0};
    const double* m0 = mom;
    const double* m1 = mom + N;
    const double* m2 = mom + 2 * N;
    for (int64_t f = threadIdx.x; f < Nd; f += blockDim.x) {
        int kk[3];
        int64_t r = f;
        for (int l = dim - 1; l >= 0; --l) {
            kk[l] = (int)(r % N);
            r /= N;
        }
        const double cv = (double)c[f];
        double p0 = cv;
        for (int l = 0; l < dim; ++l) p0 *= m0[kk[l]];
        acc[0] += p0;
        for (int l = 0; l < dim; ++l) {
            double a = cv, e = cv;
            for (int l2 = 0; l2 < dim; ++l2) {
                a *= (l2 == l) ? m1[kk[l2]] : m0[kk[l2]];
                e *= (l2 == l) ? m2[kk[l2]] : m0[kk[l2]];
            }
            acc[1 + l] += a;
            acc[1 + dim] += e;
        }
    }
    for (int q = 0; q < dim + 2; ++q) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)(dim + 2)) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[threadIdx.x][w];
        out[threadIdx.x] = t;
    }
}

// ------------------------------------------------------------------ evaluation

// out[r] = sum_k c_k prod_l T~_{k_l}(v_{r,l}); one workgroup per velocity.
template <typename T>
__global__ void __launch_bounds__(256) eval_kernel(const T* __restrict__ c,
                                                   const double* __restrict__ v, int dim, int N,
                                                   int64_t Nd, int map, double S,
                                                   double* __restrict__ out)
{
    extern __shared__ double tab[];  // dim x N
    __shared__ double sh[256 / 64];
    const int64_t r = blockIdx.x;
    if (threadIdx.x < (unsigned)dim) {
        const int l = threadIdx.x;
        const double x = v[r * dim + l];
        double xi, mu4;
        if (map == 0) {
            xi = tanh(x / S);
            const double ch = cosh(x / S);
            mu4 = 1.0 / (ch * ch * S * S);
        } else {
            const double d = S * S + x * x;
            xi = x / sqrt(d);
            mu4 = S * S / (d * d);
        }
        // T_k(xi)/sqrt(c_k) times mu^4
        double tkm = 1.0, tk = xi;
        const double r0 = 1.0 / sqrt(M_PI), r1 = sqrt(2.0 / M_PI);
        for (int k = 0; k < N; ++k) {
            double t;
            if (k == 0) t = 1.0;
            else if (k == 1) t = xi;
            else {
                t = 2.0 * xi * tk - tkm;
                tkm = tk;
                tk = t;
            }
            tab[l * N + k] = mu4 * t * (k == 0 ? r0 : r1);
        }
    }
    __syncthreads();
    double acc = 0.0;
    for (int64_t f = threadIdx.x; f < Nd; f += blockDim.x) {
        int64_t rr = f;
        double b = (double)c[f];
        for (int l = dim - 1; l >= 0; --l) {
            b *= tab[l * N + (int)(rr % N)];
            rr /= N;
        }
        acc += b;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
        out[r] = t;
    }
}

// ------------------------------------------------------------------ RK4 helpers

template <typename T>
__global__ void rk_stage_kernel(const double* __restrict__ base, const T* __restrict__ k, double a,
                                T* __restrict__ y, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = (T)(base[i] + (k ? a * (double)k[i] : 0.0));
}

template <typename T>
__global__ void rk_finish_kernel(double* __restrict__ base, const T* __restrict__ k1,
                                 const T* __restrict__ k2, const T* __restrict__ k3,
                                 const T* __restrict__ k4, double dt, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    base[i] += dt / 6.0 *
               ((double)k1[i] + 2.0 * (double)k2[i] + 2.0 * (double)k3[i] + (double)k4[i]);
}


DenseBufs plan_bufs(const Workspace& ws)
{
    DenseBufs b;
    b.P = ws.P;
    b.G = ws.G;
    b.Gg = ws.Gg;
    b.H = ws.H;
    b.qminus = ws.qminus;
    b.qplus = ws.qplus;
    b.tmpA = ws.tmpA;
    b.tmpB = ws.tmpB;
    b.red = ws.red;
    return b;
}

// ------------------------------------------------------------------ typed drivers

// a1 for nb cells: P = C^{(x)d} f and G = w mu^2 P in FP64 from FP64
// coefficients c64 (nb * N^d); Gg (plan precision) receives G rounded once
template <typename T>
hipError_t dense_synthesis_t(const Plan& p, const double* c64, int nb, const DenseBufs& b,
                             hipStream_t s)
{
    SepIO io;
    io.epi = 1;
    io.Gout = b.G;
    io.Gg = b.Gg;
    io.gg_f32 = sizeof(T) == sizeof(float);
    io.w1 = p.dt.w1;
    io.mu21 = p.dt.mu21;
    io.ni = p.ni;
    return separable(p, c64, b.P, p.dt.C, p.ni, p.N, nb, b.tmpA, b.tmpB, s, io);
}

template <typename T>
hipError_t synthesis_t(const Plan& p, const Workspace& ws, const void* coeffs, hipStream_t s)
{
    const double* c64 = static_cast<const double*>(coeffs);
    if (p.precision != PGC_PRECISION_FP64) {
        hipLaunchKernelGGL(widen<T>, dim3(blocks_for(p.Nd, 256)), dim3(256), 0, s,
                           static_cast<const T*>(coeffs), ws.cin, p.Nd);
        c64 = ws.cin;
    }
    DenseBufs b = plan_bufs(ws);
    if (p.precision == PGC_PRECISION_FP64) b.Gg = nullptr;  // G itself is read by the gain
    return dense_synthesis_t<T>(p, c64, 1, b, s);
}

// a2 + a3 for nb cells: the loss field and its projection Q- (FP64)
hipError_t dense_loss(const Plan& p, int nb, const DenseBufs& b, hipStream_t s)
{
    const double scale = p.wsum * p.b0;
    if (p.kernel == PGC_KERNEL_MAXWELL) {
        SepIO io;
        io.pro = 1;
        io.P = b.P;
        io.G = b.G;
        io.scale = scale;
        io.H = b.H;
        io.red = b.red;
        io.w1 = p.dt.w1;
        io.mu21 = p.dt.mu21;
        io.ni = p.ni;
        return separable(p, nullptr, b.qminus, p.dt.CT, p.N, p.ni, nb, b.tmpA, b.tmpB, s, io);
    } else {
        AngleForm af{};
        if (p.kernel == PGC_KERNEL_ANISO) {
            af.on = 1;
            const int D = p.dim;
            const int idx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
            for (int s2 = 0; s2 < p.n_sigma; ++s2)
                for (int a = 0; a < D; ++a)
                    for (int c = a; c < D; ++c)
                        af.m[idx[a][c]] += p.sigma_w[s2] * p.sigma[(size_t)s2 * D + a] * p.sigma[(size_t)s2 * D + c];
            for (double& x : af.m) x *= p.aniso / p.wsum;
        }
        const size_t table = (size_t)p.ni * sizeof(double);
        if (table > (size_t)kVhsMaxTableBytes) return hipErrorInvalidValue;
        const dim3 grid(blocks_for(p.nid, kVhsI), nb);
        if (p.dim == 2)
            hipLaunchKernelGGL(loss_h_vhs<2>, grid, dim3(kVhsI * kVhsJ), table, s, b.P, b.G, b.H, p.dt.v1d,
                               p.dt.w1, p.dt.mu21, scale, p.gamma, p.ni, p.nid, af);
        else
            hipLaunchKernelGGL(loss_h_vhs<3>, grid, dim3(kVhsI * kVhsJ), table, s, b.P, b.G, b.H, p.dt.v1d,
                               p.dt.w1, p.dt.mu21, scale, p.gamma, p.ni, p.nid, af);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return separable(p, b.H, b.qminus, p.dt.CT, p.N, p.ni, nb, b.tmpA, b.tmpB, s);
}

template <typename T, int DIM, int W>
hipError_t spread_launch(const Plan& p, const GainParams<T>& gp, hipStream_t s)
{
    const int plane = (DIM == 2) ? p.ng : p.ng * p.ng;
    const size_t lds = (size_t)p.slab_planes * plane * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&gain_spread<T, DIM, W>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((gain_spread<T, DIM, W>), dim3(p.n_chunks, p.n_slabs), dim3(p.block_threads),
                       lds, s, gp);
    return hipGetLastError();
}

template <typename T, int DIM>
hipError_t spread_dispatch(const Plan& p, const GainParams<T>& gp, hipStream_t s)
{
    switch (p.W) {
#define PGC_W_CASE(w) \
    case w: return spread_launch<T, DIM, w>(p, gp, s);
        PGC_W_CASE(4)
        PGC_W_CASE(5)
        PGC_W_CASE(6)
        PGC_W_CASE(7)
        PGC_W_CASE(8)
        PGC_W_CASE(9)
        PGC_W_CASE(10)
        PGC_W_CASE(11)
        PGC_W_CASE(12)
        PGC_W_CASE(13)
        PGC_W_CASE(14)
        PGC_W_CASE(15)
        PGC_W_CASE(16)
#undef PGC_W_CASE
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
GainParams<T> gain_params(const Plan& p, const Workspace& ws)
{
    GainParams<T> gp;
    gp.v1 = static_cast<const T*>(p.dt.v1);
    gp.G = static_cast<const T*>(ws.Gg);
    gp.sym = static_cast<const T*>(ws.sym);
    gp.pair_a = p.dt.pair_a;
    gp.pair_b = p.dt.pair_b;
    gp.pair_base = p.dt.pair_base;
    gp.sigma = static_cast<const T*>(p.dt.sigma);
    gp.wfac = static_cast<const T*>(p.dt.wfac);
    gp.poly = static_cast<const T*>(p.dt.poly);
    gp.slab_vlo = static_cast<const T*>(p.dt.slab_vlo);
    gp.slab_vhi = static_cast<const T*>(p.dt.slab_vhi);
    gp.partial = static_cast<double*>(ws.partial);
    gp.S = (T)p.S;
    gp.inv_S = (T)(1.0 / p.S);
    gp.inv_S64 = 1.0 / p.S;
    gp.h_inv = (T)(1.0 / p.h);
    gp.h_inv64 = 1.0 / p.h;
    gp.poly64 = p.dt.poly64;
    gp.kpoly_eo = p.dt.kpoly_eo;
    gp.cellfit = p.dt.cellfit;
    gp.cellfit_v = p.dt.cellfit_v;
    gp.b0 = (T)p.b0;
    gp.gamma = (T)p.gamma;
    gp.aniso = (T)p.aniso;
    gp.map = p.map;
    gp.vhs = p.kernel != PGC_KERNEL_MAXWELL;
    gp.ni = p.ni;
    gp.np = p.np;
    gp.ng = p.ng;
    gp.nh = p.nh;
    gp.slab_planes = p.slab_planes;
    gp.n_sigma = p.n_sigma;
    gp.ngd = p.ngd;
    gp.n_units = p.n_units;
    gp.units_per_chunk = p.units_per_chunk;
    return gp;
}

template <typename T, int DIM, int W>
hipError_t binned_launch(const Plan& p, const GainParams<T>& gp, const BinItems& bi, hipStream_t s)
{
    if (bi.n_items == 0) return hipSuccess;
    if (p.kernel == PGC_KERNEL_ANISO)
        hipLaunchKernelGGL((gain_binned<T, DIM, W, true>), dim3((unsigned)bi.n_items), dim3(64), 0, s, gp, bi);
    else
        hipLaunchKernelGGL((gain_binned<T, DIM, W, false>), dim3((unsigned)bi.n_items), dim3(64), 0, s, gp, bi);
    return hipGetLastError();
}

hipError_t mfma_dispatch(const Plan& p, const GainParams<double>& gp, const BinItems& bi, hipStream_t s)
{
    if (bi.n_items == 0) return hipSuccess;
    const dim3 grid((unsigned)bi.n_items);
    switch (p.W) {
#define PGC_M_CASE(w) \
    case w: hipLaunchKernelGGL(gain_binned_mfma<w>, grid, dim3(64), 0, s, gp, bi); break;
        PGC_M_CASE(4)
        PGC_M_CASE(5)
        PGC_M_CASE(6)
        PGC_M_CASE(7)
        PGC_M_CASE(8)
        PGC_M_CASE(9)
        PGC_M_CASE(10)
        PGC_M_CASE(11)
        PGC_M_CASE(12)
#undef PGC_M_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int DIM>
hipError_t binned_dispatch(const Plan& p, const GainParams<T>& gp, const BinItems& bi, hipStream_t s)
{
    switch (p.W) {
#define PGC_B_CASE(w) \
    case w: return binned_launch<T, DIM, w>(p, gp, bi, s);
        PGC_B_CASE(4)
        PGC_B_CASE(5)
        PGC_B_CASE(6)
        PGC_B_CASE(7)
        PGC_B_CASE(8)
        PGC_B_CASE(9)
        PGC_B_CASE(10)
        PGC_B_CASE(11)
        PGC_B_CASE(12)
        PGC_B_CASE(13)
        PGC_B_CASE(14)
#undef PGC_B_CASE
    default: return hipErrorInvalidValue;
    }
}

// count or scatter the merged points of directions [s0, s0 + ns) into their bins
template <typename T>
hipError_t bin_build_t(const Plan& p, unsigned int* count, unsigned long long* cursor, unsigned int* cursor32,
                       unsigned long long* ids, int mode, int s0, int ns, hipStream_t s)
{
    if (s0 < 0 || ns < 1 || s0 + ns > p.n_sigma || mode < 0 || mode > 2) return hipErrorInvalidValue;
    const GainParams<T> gp = gain_params<T>(p, p.ws);
    BinGeo bg;
    bg.nb = p.bins.nb;
    bg.off = p.bins.off;
    bg.W = p.W;
    bg.s0 = s0;
    bg.ns = ns;
    bg.id_cap = (unsigned long long)(p.bins.id_bytes / 8);
    bg.vthr = p.dt.bin_vthr;
    bg.h_inv = (float)(1.0 / p.h);
    bg.half_w = 0.5f * (float)p.W;
    const int64_t npencil = p.dim == 2 ? p.np : (int64_t)p.np * p.np;
    bg.n_items = (int64_t)ns * p.ni * npencil;
    const int64_t want = (bg.n_items + 255) / 256;
    const unsigned blocks = (unsigned)std::min<int64_t>(want, 65536);
#define PGC_BIN_LAUNCH(dim_, mode_)                                                                        \
    hipLaunchKernelGGL((bin_points<T, dim_, mode_>), dim3(blocks), dim3(256), 0, s, gp, bg, count, cursor, \
                       cursor32, ids)
    if (p.dim == 2) {
        if (mode == 0) PGC_BIN_LAUNCH(2, 0);
        else if (mode == 1) PGC_BIN_LAUNCH(2, 1);
        else PGC_BIN_LAUNCH(2, 2);
    } else {
        if (mode == 0) PGC_BIN_LAUNCH(3, 0);
        else if (mode == 1) PGC_BIN_LAUNCH(3, 1);
        else PGC_BIN_LAUNCH(3, 2);
    }
#undef PGC_BIN_LAUNCH
    return hipGetLastError();
}

template <typename T>
hipError_t gain_t(const Plan& p, const Workspace& ws, void* q, void* qplus, hipStream_t s)
{
    // the cosine transform of the grid ends with Q = Q+ - Q- into q (and Q+)
    SepIO io;
    io.epi = 2;
    io.qm = ws.qminus;
    io.q = q;
    io.qp = qplus;
    io.q_f32 = sizeof(T) == sizeof(float);
    prof_mark(p, 2, s);
    const int64_t n_sym = p.dim == 2 ? (int64_t)p.np * p.np : (int64_t)p.np * p.np * p.np;
    if (p.gain_mode == kGainBinned) {
        // the binned scheme forms each orbit sum from G where it is used
    } else if (p.dim == 2)
        hipLaunchKernelGGL((pair_orbit_sums<T, 2>), dim3(blocks_for(n_sym, 256)), dim3(256), 0, s,
                           static_cast<const T*>(ws.Gg), static_cast<T*>(ws.sym), p.dt.pair_a,
                           p.dt.pair_b, p.ni, p.np, n_sym);
    else
        hipLaunchKernelGGL((pair_orbit_sums<T, 3>), dim3(blocks_for(n_sym, 256)), dim3(256), 0, s,
                           static_cast<const T*>(ws.Gg), static_cast<T*>(ws.sym), p.dt.pair_a,
                           p.dt.pair_b, p.ni, p.np, n_sym);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    const GainParams<T> gp = gain_params<T>(p, ws);
    prof_mark(p, 3, s);
    if (p.gain_mode == kGainBinned) {
        if (!p.deterministic)
            hipLaunchKernelGGL(fill_zero, dim3(blocks_for(p.ngd, 256)), dim3(256), 0, s, ws.grid64, p.ngd);
        const BinIndex& B = p.bins;
        for (int c = 0; c < B.n_chunks; ++c) {
            if (B.dirs_per_chunk > 0) {
                // streamed index: sort this chunk's points into the id buffer
                hipLaunchKernelGGL(copy_u32, dim3(blocks_for(B.nbins, 256)), dim3(256), 0, s,
                                   B.chunk_begin + (int64_t)c * B.nbins, B.cursor, B.nbins);
                if ((e = hipGetLastError()) != hipSuccess) return e;
                e = launch_bin_build(p, nullptr, nullptr, B.cursor, B.ids, 2, B.chunk_s0[c],
                                     B.chunk_s0[c + 1] - B.chunk_s0[c], s);
                if (e != hipSuccess) return e;
            }
            const int64_t i0 = B.chunk_item0[c];
            BinItems bi;
            bi.n_items = B.chunk_item0[c + 1] - i0;
            bi.bin = B.item_bin + i0;
            bi.begin = B.item_begin + i0;
            bi.count = B.item_count + i0;
            bi.ids = B.ids;
            bi.grid = ws.grid64;
            bi.tiles = p.deterministic ? B.tiles : nullptr;
            bi.geo.nb = B.nb;
            bi.geo.off = B.off;
            bi.geo.W = p.W;
            bi.geo.n_items = 0;
            bi.geo.s0 = B.chunk_s0[c];
            bi.geo.ns = B.chunk_s0[c + 1] - B.chunk_s0[c];
            if constexpr (sizeof(T) == sizeof(double)) {
                if (p.mfma) e = mfma_dispatch(p, gp, bi, s);
                else e = (p.dim == 2) ? binned_dispatch<T, 2>(p, gp, bi, s) : binned_dispatch<T, 3>(p, gp, bi, s);
            } else {
                e = (p.dim == 2) ? binned_dispatch<T, 2>(p, gp, bi, s) : binned_dispatch<T, 3>(p, gp, bi, s);
            }
            if (e != hipSuccess) return e;
        }
        if (p.deterministic) {
            const dim3 g(blocks_for(p.ngd, 256));
            if (p.dim == 2)
                hipLaunchKernelGGL(gather_tiles<2>, g, dim3(256), 0, s, p.bins.tiles, p.bins.bin_ptr, p.bins.bin_items,
                                   p.bins.nb, p.bins.off, p.W, p.nh, p.ng, p.ngd, ws.grid64);
            else
                hipLaunchKernelGGL(gather_tiles<3>, g, dim3(256), 0, s, p.bins.tiles, p.bins.bin_ptr, p.bins.bin_items,
                                   p.bins.nb, p.bins.off, p.W, p.nh, p.ng, p.ngd, ws.grid64);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        prof_mark(p, 4, s);
        e = separable(p, ws.grid64, ws.qplus, p.dt.E, p.N, p.ng, 1, ws.tmpA, ws.tmpB, s, io);
    } else {
        e = (p.dim == 2) ? spread_dispatch<T, 2>(p, gp, s) : spread_dispatch<T, 3>(p, gp, s);
        if (e != hipSuccess) return e;
        prof_mark(p, 4, s);
        hipLaunchKernelGGL(reduce_partials, dim3(blocks_for(p.ngd, 256)), dim3(256), 0, s,
                           static_cast<const double*>(ws.partial), ws.grid, p.ngd, p.n_chunks);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = separable(p, ws.grid, ws.qplus, p.dt.E, p.N, p.ng, 1, ws.tmpA, ws.tmpB, s, io);
    }
    return e;
}

// the projection in FP64; FP32 plans round the coefficients once at the end
template <typename T>
hipError_t project_t(const Plan& p, const double* f, void* coeffs, hipStream_t s)
{
    hipLaunchKernelGGL(project_weight, dim3(blocks_for(p.nid, 256)), dim3(256), 0, s, f, p.ws.H,
                       p.dt.w1, p.dt.mu21, p.dim, p.ni, p.nid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (p.precision == PGC_PRECISION_FP64)
        return separable(p, p.ws.H, static_cast<double*>(coeffs), p.dt.CT, p.N, p.ni, 1, p.ws.tmpA,
                         p.ws.tmpB, s);
    e = separable(p, p.ws.H, p.ws.cin, p.dt.CT, p.N, p.ni, 1, p.ws.tmpA, p.ws.tmpB, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(narrow<T>, dim3(blocks_for(p.Nd, 256)), dim3(256), 0, s, p.ws.cin,
                       static_cast<T*>(coeffs), p.Nd);
    return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_synthesis(const Plan& p, const Workspace& ws, const void* coeffs, hipStream_t s)
{
    return p.precision == PGC_PRECISION_FP64 ? synthesis_t<double>(p, ws, coeffs, s)
                                             : synthesis_t<float>(p, ws, coeffs, s);
}

hipError_t launch_loss(const Plan& p, const Workspace& ws, hipStream_t s)
{
    return dense_loss(p, 1, plan_bufs(ws), s);
}

hipError_t launch_dense_synthesis(const Plan& p, const double* c64, int nb, const DenseBufs& b,
                                  hipStream_t s)
{
    return p.precision == PGC_PRECISION_FP64 ? dense_synthesis_t<double>(p, c64, nb, b, s)
                                             : dense_synthesis_t<float>(p, c64, nb, b, s);
}

hipError_t launch_dense_loss(const Plan& p, int nb, const DenseBufs& b, hipStream_t s)
{
    return dense_loss(p, nb, b, s);
}

hipError_t launch_dense_grid_to_modes(const Plan& p, const double* grid, int nb, const DenseBufs& b,
                                      hipStream_t s)
{
    return separable(p, grid, b.qplus, p.dt.E, p.N, p.ng, nb, b.tmpA, b.tmpB, s);
}

hipError_t launch_gain(const Plan& p, const Workspace& ws, void* q, void* qplus, hipStream_t s)
{
    return p.precision == PGC_PRECISION_FP64 ? gain_t<double>(p, ws, q, qplus, s)
                                             : gain_t<float>(p, ws, q, qplus, s);
}

hipError_t launch_bin_build(const Plan& p, unsigned int* count, unsigned long long* cursor,
                            unsigned int* cursor32, unsigned long long* ids, int mode, int s0, int ns,
                            hipStream_t s)
{
    return p.precision == PGC_PRECISION_FP64
               ? bin_build_t<double>(p, count, cursor, cursor32, ids, mode, s0, ns, s)
               : bin_build_t<float>(p, count, cursor, cursor32, ids, mode, s0, ns, s);
}

hipError_t launch_project(const Plan& p, const double* f_nodes, void* coeffs, hipStream_t s)
{
    return p.precision == PGC_PRECISION_FP64 ? project_t<double>(p, f_nodes, coeffs, s)
                                             : project_t<float>(p, f_nodes, coeffs, s);
}

hipError_t launch_moments(const Plan& p, const void* coeffs, double* out, hipStream_t s)
{
    if (p.precision == PGC_PRECISION_FP64)
        hipLaunchKernelGGL(moments_kernel<double>, dim3(1), dim3(kRedThreads), 0, s,
                           static_cast<const double*>(coeffs), p.ws.mom, p.dim, p.N, p.Nd, out);
    else
        hipLaunchKernelGGL(moments_kernel<float>, dim3(1), dim3(kRedThreads), 0, s,
                           static_cast<const float*>(coeffs), p.ws.mom, p.dim, p.N, p.Nd, out);
    return hipGetLastError();
}

hipError_t launch_eval(const Plan& p, const void* coeffs, const double* v, int64_t n, double* out,
                       hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t lds = sizeof(double) * p.dim * p.N;
    if (p.precision == PGC_PRECISION_FP64)
        hipLaunchKernelGGL(eval_kernel<double>, dim3((unsigned)n), dim3(256), lds, s,
                           static_cast<const double*>(coeffs), v, p.dim, p.N, p.Nd, p.map, p.S, out);
    else
        hipLaunchKernelGGL(eval_kernel<float>, dim3((unsigned)n), dim3(256), lds, s,
                           static_cast<const float*>(coeffs), v, p.dim, p.N, p.Nd, p.map, p.S, out);
    return hipGetLastError();
}

hipError_t launch_rk_stage(const Plan& p, const double* base, const void* k, double a, void* y,
                           hipStream_t s)
{
    if (p.precision == PGC_PRECISION_FP64)
        hipLaunchKernelGGL(rk_stage_kernel<double>, dim3(blocks_for(p.Nd, 256)), dim3(256), 0, s,
                           base, static_cast<const double*>(k), a, static_cast<double*>(y), p.Nd);
    else
        hipLaunchKernelGGL(rk_stage_kernel<float>, dim3(blocks_for(p.Nd, 256)), dim3(256), 0, s,
                           base, static_cast<const float*>(k), a, static_cast<float*>(y), p.Nd);
    return hipGetLastError();
}

hipError_t launch_copy_state(const Plan& p, const double* base, void* y, hipStream_t s)
{
    return launch_rk_stage(p, base, nullptr, 0.0, y, s);
}

hipError_t launch_rk_finish(const Plan& p, double* base, double dt, hipStream_t s)
{
    if (p.precision == PGC_PRECISION_FP64)
        hipLaunchKernelGGL(rk_finish_kernel<double>, dim3(blocks_for(p.Nd, 256)), dim3(256), 0, s,
                           base, static_cast<const double*>(p.ws.rk_k[0]),
                           static_cast<const double*>(p.ws.rk_k[1]),
                           static_cast<const double*>(p.ws.rk_k[2]),
                           static_cast<const double*>(p.ws.rk_k[3]), dt, p.Nd);
    else
        hipLaunchKernelGGL(rk_finish_kernel<float>, dim3(blocks_for(p.Nd, 256)), dim3(256), 0, s,
                           base, static_cast<const float*>(p.ws.rk_k[0]),
                           static_cast<const float*>(p.ws.rk_k[1]),
                           static_cast<const float*>(p.ws.rk_k[2]),
                           static_cast<const float*>(p.ws.rk_k[3]), dt, p.Nd);
    return hipGetLastError();
}

}  // namespace pgc
