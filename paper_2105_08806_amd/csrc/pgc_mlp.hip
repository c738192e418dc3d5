// Learned surrogate of the coefficients-to-Q map, with the fast method as its
// fallback and judge.
//
// The network is a multilayer perceptron on the N^d coefficients: per-feature
// normalisation, hidden layers y = silu(W x + b) of one width, a linear output
// layer, and de-normalisation.  Its output is projected onto the coefficient
// vectors with zero mass, momentum and energy (the invariants that the test
// space keeps, Sec. 3.2), so what it returns conserves them by construction.
//
// Every product runs on the matrix cores: BF16 operands, FP32 accumulation
// (v_mfma_f32_16x16x32_bf16).  Weights are kept in FP32 (Adam state too) and
// copied to BF16 after every step; activations are stored in BF16 for the
// products and in FP32 where the backward pass needs them.
//
// A call of the surrogate falls back to the plan's own evaluation for a
// sample when the mass or energy residual of the returned Q exceeds the gate,
// when the residual of the raw network output or the RMS z-score of the input
// is far outside what it was on the training set (an input unlike the
// training data), or, for the whole call,
// when the plain evaluation of every k-th sample (the judge) disagrees with
// the network by more than the judge tolerance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <random>
#include <vector>

#include "pgc_internal.h"

namespace pgc {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

__device__ __forceinline__ bf16 to_bf16(float f)
{
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (bf16)(u >> 16);
}

__device__ __forceinline__ float from_bf16(bf16 b) { return __uint_as_float((unsigned int)b << 16); }

constexpr int kBK = 64, kPad = 8;

// Column of element (r, k) of a staged 64 x 64 tile: the eight 8-element
// groups of a row are permuted by row bits 3..5 (an XOR swizzle).  Rows 16 B
// apart that sit eight apart map to the same LDS banks; the transposed stores
// write eight such rows at one k, which the swizzle spreads over eight banks.
// Every 8-element group stays contiguous, so the 16-byte accesses stay whole.
__device__ __forceinline__ int swz(int r, int k) { return k ^ (((r >> 3) & 7) << 3); }

// C[M x N] = op(A) op(B) (+ bias[n]), or C += ... when `accumulate`; A and B
// BF16, C FP32, all row-major:
//   op(A)[m][k] = TA ? A[k lda + m] : A[m lda + k]
//   op(B)[k][n] = TB ? B[n ldb + k] : B[k ldb + n]
// A workgroup of NW waves owns a BT x BT tile of C (BT = 64: four waves of
// 32 x 32; BT = 128: eight waves of 32 x 64), each wave a part of 16 x 16
// tiles; blockIdx.z takes the K range [z kc, (z+1) kc)
// and, when gridDim.z > 1, adds its partial tile into C atomically (C holds
// zeros or the values to accumulate onto).  Each 64-deep K slice is two
// v_mfma_f32_16x16x32_bf16 per 16 x 16 tile: lane l supplies row (column)
// l % 16 at k = 32 s + 8 (l / 16) .. + 7 and holds rows 4 (l / 16) + r, column
// l % 16 of the result.  With `vec` (16-byte aligned rows) the global loads
// of the slice after next are issued before the current slice's products.
template <bool TA, bool TB, int BT, int NW>
__global__ void __launch_bounds__(64 * NW) gemm_bf16(int M, int N, int K, int kc,
                                                 const bf16* __restrict__ A, int lda,
                                                 const bf16* __restrict__ B, int ldb,
                                                 float* __restrict__ C, int ldc,
                                                 const float* __restrict__ bias, int accumulate, int vec)
{
    typedef __bf16 bf16x8m __attribute__((ext_vector_type(8)));
    typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
    constexpr int NT = 64 * NW;                          // threads
    constexpr int WMS = BT / (NW / 2), WNS = BT / 2;     // a wave's part: NW/2 x 2 waves
    constexpr int NBM = WMS / 16, NBN = WNS / 16;        // its 16 x 16 tiles
    static_assert(NW % 2 == 0 && WMS % 16 == 0 && WNS % 16 == 0, "wave layout");
    __shared__ __attribute__((aligned(16))) bf16 sA[BT][kBK + kPad];
    __shared__ __attribute__((aligned(16))) bf16 sB[BT][kBK + kPad];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
    const int kbeg = blockIdx.z * kc;
    const int kend = min(K, kbeg + kc);
    const int wm = (wave >> 1) * WMS, wn = (wave & 1) * WNS;
    f32x4 acc[NBM][NBN];
#pragma unroll
    for (int i = 0; i < NBM; ++i)
#pragma unroll
        for (int j = 0; j < NBN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // 16 x 16 x 32 products of the wave's tiles over the staged slice
    auto compute = [&]() {
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 32) {
            const int kq = kk + 8 * (lane >> 4);
            bf16x8m a[NBM], b[NBN];
#pragma unroll
            for (int i = 0; i < NBM; ++i) {
                const int r = wm + i * 16 + (lane & 15);
                a[i] = __builtin_bit_cast(bf16x8m, *reinterpret_cast<const u16x8*>(&sA[r][swz(r, kq)]));
            }
#pragma unroll
            for (int j = 0; j < NBN; ++j) {
                const int r = wn + j * 16 + (lane & 15);
                b[j] = __builtin_bit_cast(bf16x8m, *reinterpret_cast<const u16x8*>(&sB[r][swz(r, kq)]));
            }
#pragma unroll
            for (int i = 0; i < NBM; ++i)
#pragma unroll
                for (int j = 0; j < NBN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };

    if (vec) {
        // every thread moves CH 16-byte runs of 8 elements of each operand along
        // its contiguous dimension (k, or m / n when the operand is transposed):
        // run c = tid + NT h covers, untransposed, row c / 8 at k = 8 (c % 8),
        // transposed, k = c / RM at rows 8 (c % RM) .. + 7
        constexpr int CH = BT * kBK / 8 / NT;
        constexpr int RM = BT / 8;  // 16-byte runs per k of an m- (n-) contiguous operand
        static_assert(BT * kBK == 8 * NT * CH && kBK == 64, "tile shape");
        auto gload = [&](int k0, u16x8* va, u16x8* vb) {
#pragma unroll
            for (int h = 0; h < CH; ++h) {
                const int c = tid + NT * h;
                va[h] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                vb[h] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                if (!TA) {
                    const int gm = m0 + (c >> 3), gk = k0 + (c & 7) * 8;
                    if (gm < M && gk + 8 <= kend) {
                        va[h] = *reinterpret_cast<const u16x8*>(A + (size_t)gm * lda + gk);
                    } else if (gm < M) {
                        for (int q = 0; q < 8; ++q)
                            if (gk + q < kend) va[h][q] = A[(size_t)gm * lda + gk + q];
                    }
                } else {
                    const int gk = k0 + c / RM, gm = m0 + (c % RM) * 8;
                    if (gk < kend && gm + 8 <= M) {
                        va[h] = *reinterpret_cast<const u16x8*>(A + (size_t)gk * lda + gm);
                    } else if (gk < kend) {
                        for (int q = 0; q < 8; ++q)
                            if (gm + q < M) va[h][q] = A[(size_t)gk * lda + gm + q];
                    }
                }
                if (TB) {
                    const int gn = n0 + (c >> 3), gk = k0 + (c & 7) * 8;
                    if (gn < N && gk + 8 <= kend) {
                        vb[h] = *reinterpret_cast<const u16x8*>(B + (size_t)gn * ldb + gk);
                    } else if (gn < N) {
                        for (int q = 0; q < 8; ++q)
                            if (gk + q < kend) vb[h][q] = B[(size_t)gn * ldb + gk + q];
                    }
                } else {
                    const int gk = k0 + c / RM, gn = n0 + (c % RM) * 8;
                    if (gk < kend && gn + 8 <= N) {
                        vb[h] = *reinterpret_cast<const u16x8*>(B + (size_t)gk * ldb + gn);
                    } else if (gk < kend) {
                        for (int q = 0; q < 8; ++q)
                            if (gn + q < N) vb[h][q] = B[(size_t)gk * ldb + gn + q];
                    }
                }
            }
        };
        // a slice inside the matrix on every side: unconditional 16-byte loads,
        // with no branch whose own waits would drain the loads in flight
        const bool inside_mn = m0 + BT <= M && n0 + BT <= N;
        auto gload_full = [&](int k0, u16x8* va, u16x8* vb) {
#pragma unroll
            for (int h = 0; h < CH; ++h) {
                const int c = tid + NT * h;
                va[h] = !TA ? *reinterpret_cast<const u16x8*>(A + (size_t)(m0 + (c >> 3)) * lda + k0 + (c & 7) * 8)
                            : *reinterpret_cast<const u16x8*>(A + (size_t)(k0 + c / RM) * lda + m0 + (c % RM) * 8);
                vb[h] = TB ? *reinterpret_cast<const u16x8*>(B + (size_t)(n0 + (c >> 3)) * ldb + k0 + (c & 7) * 8)
                           : *reinterpret_cast<const u16x8*>(B + (size_t)(k0 + c / RM) * ldb + n0 + (c % RM) * 8);
            }
        };
        auto sstore = [&](const u16x8* va, const u16x8* vb) {
#pragma unroll
            for (int h = 0; h < CH; ++h) {
                const int c = tid + NT * h;
                if (!TA) {
                    *reinterpret_cast<u16x8*>(&sA[c >> 3][swz(c >> 3, (c & 7) * 8)]) = va[h];
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q) sA[(c % RM) * 8 + q][swz((c % RM) * 8 + q, c / RM)] = va[h][q];
                }
                if (TB) {
                    *reinterpret_cast<u16x8*>(&sB[c >> 3][swz(c >> 3, (c & 7) * 8)]) = vb[h];
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q) sB[(c % RM) * 8 + q][swz((c % RM) * 8 + q, c / RM)] = vb[h][q];
                }
            }
        };
        const int nsl = (kend - kbeg) / kBK;
        if (inside_mn && nsl > 0 && kbeg + nsl * kBK == kend) {
            // whole slices inside the matrix: two register stages, so a slice's
            // loads are issued two slices before it is staged.  The loop body has
            // no branch around a load (the loads past the last slice reload it),
            // so the compiler waits for each stage's own loads only.
            const int klast = kend - kBK;
            u16x8 va0[CH], vb0[CH], va1[CH], vb1[CH];
            gload_full(kbeg, va0, vb0);
            gload_full(min(kbeg + kBK, klast), va1, vb1);
            for (int i = 0; i < nsl; i += 2) {
                const int k0 = kbeg + i * kBK;
                sstore(va0, vb0);
                __syncthreads();
                gload_full(min(k0 + 2 * kBK, klast), va0, vb0);
                compute();
                __syncthreads();
                sstore(va1, vb1);
                __syncthreads();
                gload_full(min(k0 + 3 * kBK, klast), va1, vb1);
                if (i + 1 < nsl) compute();  // uniform over the workgroup
                __syncthreads();
            }
        } else {
            u16x8 va[CH], vb[CH];
            gload(kbeg, va, vb);
            for (int k0 = kbeg; k0 < kend; k0 += kBK) {
                sstore(va, vb);
                __syncthreads();
                if (k0 + kBK < kend) gload(k0 + kBK, va, vb);
                compute();
                __syncthreads();
            }
        }
    } else {
        for (int k0 = kbeg; k0 < kend; k0 += kBK) {
            for (int e = tid; e < BT * kBK; e += NT) {
                int m, k;
                if (TA) {
                    m = e % BT;
                    k = e / BT;
                } else {
                    k = e % kBK;
                    m = e / kBK;
                }
                const int gm = m0 + m, gk = k0 + k;
                bf16 v = 0;
                if (gm < M && gk < kend) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
                sA[m][swz(m, k)] = v;
            }
            for (int e = tid; e < BT * kBK; e += NT) {
                int n, k;
                if (TB) {
                    k = e % kBK;
                    n = e / kBK;
                } else {
                    n = e % BT;
                    k = e / BT;
                }
                const int gn = n0 + n, gk = k0 + k;
                bf16 v = 0;
                if (gn < N && gk < kend) v = TB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
                sB[n][swz(n, k)] = v;
            }
            __syncthreads();
            compute();
            __syncthreads();
        }
    }
    const bool add = gridDim.z > 1;
#pragma unroll
    for (int i = 0; i < NBM; ++i)
#pragma unroll
        for (int j = 0; j < NBN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // lane l holds row 4 (l / 16) + r, column l % 16 of each 16 x 16 tile
                const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int gn = n0 + wn + j * 16 + (lane & 15);
                if (gm >= M || gn >= N) continue;
                float v = acc[i][j][r];
                if (bias && blockIdx.z == 0) v += bias[gn];
                float* c = C + (size_t)gm * ldc + gn;
                if (add)
                    atomicAdd(c, v);
                else if (accumulate)
                    *c += v;
                else
                    *c = v;
            }
}

__global__ void fill_f32(float* __restrict__ x, float v, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void zero_f64(double* __restrict__ x, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

// C[m][c] = 0 for m < M, c < N (row stride ldc)
__global__ void zero_rows(float* __restrict__ C, int ldc, int M, int N)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * N) return;
    C[(e / N) * ldc + e % N] = 0.f;
}

// the empty product (K = 0): C = bias (zero without one), or C += bias
__global__ void bias_rows(float* __restrict__ C, int ldc, int M, int N, const float* __restrict__ bias, int accumulate)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * N) return;
    float* c = C + (e / N) * ldc + e % N;
    const float v = bias ? bias[e % N] : 0.f;
    *c = accumulate ? *c + v : v;
}

__global__ void f32_to_bf16(const float* __restrict__ x, bf16* __restrict__ y, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

// rows of f picked by idx (or consecutive rows from `first`), normalised, in BF16
__global__ void normalise_in(const float* __restrict__ f, const int* __restrict__ idx, int64_t first,
                             int rows, int n, const float* __restrict__ mu, const float* __restrict__ sd,
                             bf16* __restrict__ x)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * n) return;
    const int r = (int)(e / n), c = (int)(e % n);
    const int64_t src = idx ? idx[r] : first + r;
    x[e] = to_bf16((f[src * n + c] - mu[c]) / sd[c]);
}

__device__ __forceinline__ float sigmoid(float z) { return 1.f / (1.f + expf(-z)); }

__global__ void silu_fwd(const float* __restrict__ z, bf16* __restrict__ h, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) h[i] = to_bf16(z[i] * sigmoid(z[i]));
}

// dz = dh silu'(z), silu'(z) = s (1 + z (1 - s)), s = sigmoid(z)
__global__ void silu_bwd(const float* __restrict__ dh, const float* __restrict__ z, bf16* __restrict__ dz,
                         float* __restrict__ dz32, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float s = sigmoid(z[i]);
    const float g = dh[i] * s * (1.f + z[i] * (1.f - s));
    dz32[i] = g;
    dz[i] = to_bf16(g);
}

// loss = mean over rows and features of (yhat - (q - mu)/sd)^2 and its gradient
// sq[r] = sum_c q[src_r][c]^2 (FP64), one block per row
__global__ void __launch_bounds__(256) row_sqnorm(const float* __restrict__ q, const int* __restrict__ idx,
                                                  int n, double* __restrict__ sq)
{
    __shared__ double sh[4];
    const int r = blockIdx.x;
    const int64_t src = idx ? idx[r] : r;
    double part = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const double v = q[src * n + c];
        part += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) sq[r] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Loss and its gradient with respect to the normalised outputs.  Without row
// norms: mean squared error of the normalised outputs.  With row norms rn (the
// squared L2 norms of the target rows): mean over rows of the squared relative
// error in the units of q, sum_c (sd_c d_rc)^2 / rn_r.
__global__ void __launch_bounds__(256) mse_grad(const float* __restrict__ yhat, const float* __restrict__ q,
                                                const int* __restrict__ idx, int rows, int n,
                                                const float* __restrict__ mu, const float* __restrict__ sd,
                                                const double* __restrict__ rn,
                                                float* __restrict__ dy32, bf16* __restrict__ dy,
                                                double* __restrict__ loss)
{
    __shared__ double sh[4];
    double part = 0.0;
    // grid-stride: a bounded grid keeps the atomic additions to the loss few
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)rows * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / n), c = (int)(e % n);
        const int64_t src = idx ? idx[r] : r;
        const float d = yhat[e] - (q[src * n + c] - mu[c]) / sd[c];
        // weight of d^2 in the loss
        const double wt = rn ? (double)sd[c] * (double)sd[c] / (rn[r] > 0.0 ? rn[r] : 1.0) / (double)rows
                             : 1.0 / ((double)rows * (double)n);
        const float g = (float)(2.0 * wt * (double)d);
        dy32[e] = g;
        dy[e] = to_bf16(g);
        part += wt * (double)d * (double)d;
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, sh[0] + sh[1] + sh[2] + sh[3]);
}

// db[c] = sum over rows of g[r][c]
__global__ void __launch_bounds__(256) col_sum(const float* __restrict__ g, int rows, int cols,
                                               float* __restrict__ db)
{
    // 16 columns per block, 16 row phases each (rows p, p + 16, ...), summed
    // in a fixed order, so the result does not depend on scheduling
    __shared__ float part[16][17];
    const int cx = threadIdx.x & 15, p = threadIdx.x >> 4;
    const int c = blockIdx.x * 16 + cx;
    float s = 0.f;
    if (c < cols)
        for (int r = p; r < rows; r += 16) s += g[(size_t)r * cols + c];
    part[p][cx] = s;
    __syncthreads();
    if (p == 0 && c < cols) {
        float t = 0.f;
        for (int q = 0; q < 16; ++q) t += part[q][cx];
        db[c] = t;
    }
}

// Adam (Kingma and Ba 2015) on FP32 master weights; refreshes the BF16 copy
__global__ void adam_step(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, bf16* __restrict__ wb, int64_t n, float lr, float b1,
                          float b2, float eps, float c1, float c2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = to_bf16(wi);
}

// per-feature mean and standard deviation over the rows of x (FP64 sums)
__global__ void feature_stats(const float* __restrict__ x, int64_t rows, int n, float* __restrict__ mu,
                              float* __restrict__ sd)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double s = 0.0, s2 = 0.0;
    for (int64_t r = 0; r < rows; ++r) {
        const double v = x[r * n + c];
        s += v;
        s2 += v * v;
    }
    const double m = s / (double)rows;
    mu[c] = (float)m;
    sd[c] = (float)std::sqrt(std::max(s2 / (double)rows - m * m, 0.0));
}

// keep standard deviations away from zero: sd = max(sd, floor)
__global__ void floor_sd(float* __restrict__ sd, int n, const float* __restrict__ sd_max, float rel)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) sd[c] = fmaxf(sd[c], rel * sd_max[0]);
}

__global__ void __launch_bounds__(1024) max_reduce(const float* __restrict__ x, int n, float* __restrict__ out)
{
    __shared__ float sh[16];
    float m = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, x[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = fmaxf(t, sh[w]);
        out[0] = t;
    }
}

// sums over the workgroup of nv values per thread (nv <= 8); result in out[0..nv)
// sums of nv <= 8 per-thread values over a workgroup of at most 1024 threads
__device__ void block_sums(double* vals, int nv, double* out)
{
    __shared__ double sh[8][16];
    for (int a = 0; a < nv; ++a)
        for (int off = 32; off > 0; off >>= 1) vals[a] += __shfl_down(vals[a], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < nv; ++a) sh[a][threadIdx.x >> 6] = vals[a];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int a = 0; a < nv; ++a) {
            double t = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[a][w];
            out[a] = t;
        }
    __syncthreads();
}

// Output stage, one 1024-thread workgroup per sample (nc <= 5 invariants):
// q = yhat sd + mu (FP64); the raw residual rho_raw = max_c |<C_c, q>| / (|C_c| |q|);
// the projection q -= C^T (C C^T)^{-1} C q onto the coefficient vectors that
// conserve every invariant; q stored in FP32; rho_out of the stored q.
constexpr int kOutThreads = 1024;  // threads per sample in output_stage

__global__ void __launch_bounds__(kOutThreads) output_stage(const float* __restrict__ yhat, int rows, int n,
                                                    const float* __restrict__ mu, const float* __restrict__ sd,
                                                    const double* __restrict__ cons, int nc,
                                                    const double* __restrict__ ginv,
                                                    const double* __restrict__ cnorm,
                                                    float* __restrict__ q, double* __restrict__ res_raw,
                                                    double* __restrict__ res_out)
{
    __shared__ double tot[8];
    __shared__ double coef[5];
    const int r = blockIdx.x;
    const float* y = yhat + (size_t)r * n;
    float* qo = q + (size_t)r * n;
    double vals[8];
    for (int pass = 0; pass < 2; ++pass) {
        for (int a = 0; a < 8; ++a) vals[a] = 0.0;
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            double v = (double)y[c] * (double)sd[c] + (double)mu[c];
            if (pass == 1) {
                for (int a = 0; a < nc; ++a) v -= coef[a] * cons[(size_t)a * n + c];
                const float vf = (float)v;
                qo[c] = vf;
                v = (double)vf;
            }
            for (int a = 0; a < nc; ++a) vals[a] += cons[(size_t)a * n + c] * v;
            vals[nc] += v * v;
        }
        block_sums(vals, nc + 1, tot);
        if (threadIdx.x == 0) {
            const double qn = fmax(sqrt(tot[nc]), 1e-300);
            double rho = 0.0;
            for (int a = 0; a < nc; ++a) rho = fmax(rho, fabs(tot[a]) / (cnorm[a] * qn));
            if (pass == 0) {
                res_raw[r] = rho;
                for (int a = 0; a < nc; ++a) {
                    double t = 0.0;
                    for (int b = 0; b < nc; ++b) t += ginv[a * nc + b] * tot[b];
                    coef[a] = t;
                }
            } else {
                res_out[r] = rho;
            }
        }
        __syncthreads();
    }
}

// RMS z-score of the rows first .. first + rows - 1 of f: sqrt(mean_c ((f - mu)/sd)^2)
__global__ void __launch_bounds__(256) row_zscore(const float* __restrict__ f, int64_t first, int n,
                                                  const float* __restrict__ mu, const float* __restrict__ sd,
                                                  double* __restrict__ out)
{
    __shared__ double sh[4];
    const int r = blockIdx.x;
    const float* x = f + (size_t)(first + r) * n;
    double s2 = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const double z = ((double)x[c] - (double)mu[c]) / (double)sd[c];
        s2 += z * z;
    }
    for (int off = 32; off > 0; off >>= 1) s2 += __shfl_down(s2, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s2;
    __syncthreads();
    if (threadIdx.x == 0) out[r] = sqrt((sh[0] + sh[1] + sh[2] + sh[3]) / (double)n);
}

// relative L2 distance of rows: err[r] = |a_r - b_r| / |b_r| (one workgroup per row)
__global__ void __launch_bounds__(256) row_rel_err(const float* __restrict__ a, const float* __restrict__ b,
                                                   int n, double* __restrict__ err)
{
    __shared__ double sh[2][4];
    const int r = blockIdx.x;
    double d2 = 0.0, b2 = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const double x = a[(size_t)r * n + c], y = b[(size_t)r * n + c];
        d2 += (x - y) * (x - y);
        b2 += y * y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        d2 += __shfl_down(d2, off, 64);
        b2 += __shfl_down(b2, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = d2;
        sh[1][threadIdx.x >> 6] = b2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double dd = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        const double bb = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
        err[r] = std::sqrt(dd / fmax(bb, 1e-300));
    }
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace
}  // namespace pgc

// ------------------------------------------------------------------ host side

namespace {

using pgc::bf16;

struct Layer {
    int in = 0, out = 0;
    float *W = nullptr, *b = nullptr, *gW = nullptr, *gb = nullptr;
    float *mW = nullptr, *vW = nullptr, *mb = nullptr, *vb = nullptr;
    bf16* Wb = nullptr;
    float* Z = nullptr;   // Bmax x out  pre-activation (FP32)
    bf16* H = nullptr;    // Bmax x out  activation (BF16), hidden layers
    float* dH = nullptr;  // Bmax x out
    float* dZ32 = nullptr;
    bf16* dZ = nullptr;
};

}  // namespace

struct pgc_surrogate_s {
    pgc_plan plan = nullptr;
    int n = 0, width = 0, n_layers = 0, bmax = 0;
    uint64_t seed = 0;
    double gate_residual = 1e-6, gate_raw_factor = 0.0, judge_tol = 0.0;
    float floor_in = 0.1f, floor_out = 1.0f;  // standard deviation floors, relative to the largest
    int judge_stride = 0;
    int loss_relative = 0;   // training loss: normalised MSE (0) or per-sample relative error (1)
    double* rownorm = nullptr;  // Bmax  squared norms of the target rows of a training batch
    double raw_calib = 0.0;  // largest raw residual seen on the training set
    double z_calib = 0.0;    // largest RMS z-score of a training input
    int64_t steps = 0;       // Adam steps taken
    std::vector<Layer> layers;
    float *mu_in = nullptr, *sd_in = nullptr, *mu_out = nullptr, *sd_out = nullptr;
    bf16* X = nullptr;         // Bmax x n
    float* dY32 = nullptr;     // Bmax x n
    bf16* dY = nullptr;
    float* qtmp = nullptr;     // Bmax x n  plain-path results of the judge
    float* scratch = nullptr;  // small FP32 scratch
    int* idx = nullptr;        // Bmax  row indices of a training batch
    double* loss = nullptr;    // 1
    double *res_raw = nullptr, *res_out = nullptr, *err = nullptr, *zs = nullptr;  // Bmax each
    int nc = 0;
    double *cons = nullptr, *ginv = nullptr, *cnorm = nullptr;
    std::vector<void*> allocations;
    int64_t bytes = 0;
};

namespace {

hipError_t s_alloc(pgc_surrogate_s& s, void** p, size_t bytes)
{
    *p = nullptr;
    s.allocations.push_back(nullptr);  // the slot first: a throwing push_back leaks no device memory
    hipError_t e = hipMalloc(&s.allocations.back(), std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
        s.allocations.pop_back();
        return e;
    }
    *p = s.allocations.back();
    s.bytes += (int64_t)bytes;
    return hipSuccess;
}

template <typename T>
hipError_t s_alloc_n(pgc_surrogate_s& s, T** p, int64_t n)
{
    void* v = nullptr;
    hipError_t e = s_alloc(s, &v, (size_t)n * sizeof(T));
    *p = static_cast<T*>(v);
    return e;
}

void s_free(pgc_surrogate_s* s)
{
    if (!s) return;
    (void)hipDeviceSynchronize();
    for (void* p : s->allocations) (void)hipFree(p);
    delete s;
}

hipError_t gemm(int M, int N, int K, const bf16* A, int lda, bool ta, const bf16* B, int ldb, bool tb, float* C,
                int ldc, const float* bias, bool accumulate, hipStream_t st)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K <= 0) {
        hipLaunchKernelGGL(pgc::bias_rows, dim3(pgc::nb((int64_t)M * N, 256)), dim3(256), 0, st, C, ldc, M, N, bias,
                           accumulate ? 1 : 0);
        return hipGetLastError();
    }
    // split K until the tiles cover the device twice over, while the atomic
    // traffic of the partial tiles (split x the bytes of C) stays below the
    // bytes of the operands: a product whose output is large next to its
    // operands (the 13824-wide layers) is bound by writing C, not by the
    // matrix cores, and runs unsplit
    const double operand_bytes = 2.0 * ((double)M * K + (double)N * K), c_bytes = 4.0 * (double)M * N;
    auto plan_split = [&](int bt, int& split, int& kc) {
        const int tiles = ((M + bt - 1) / bt) * ((N + bt - 1) / bt);
        split = 1;
        while (tiles * split < 512 && K / (split * 2) >= 256 && c_bytes * split * 2 <= operand_bytes) split *= 2;
        kc = ((K + split - 1) / split + pgc::kBK - 1) / pgc::kBK * pgc::kBK;
        split = (K + kc - 1) / kc;
        return tiles * split;
    };
    // 128 x 128 tiles (eight waves of 32 x 64) read half the operand bytes per
    // flop of 64 x 64 ones (four waves of 32 x 32).  Measured on the network's
    // products they pay only with many tiles (the weight gradients, 864 tiles:
    // 6-9% faster) and cost 40-80% on the 256-row products (216 or 256
    // workgroups), so they are taken from 512 workgroups on
    int split, kc, bt = 128;
    if (M < 128 || N < 128 || plan_split(128, split, kc) < 512) {
        bt = 64;
        plan_split(64, split, kc);
    }
    if (split > 1 && !accumulate)
        hipLaunchKernelGGL(pgc::zero_rows, dim3(pgc::nb((int64_t)M * N, 256)), dim3(256), 0, st, C, ldc, M, N);
    dim3 grid((N + bt - 1) / bt, (M + bt - 1) / bt, split);
    const int acc = accumulate ? 1 : 0;
    // 16-byte runs need 16-byte aligned rows: leading dimensions that are
    // multiples of 8 elements on 16-byte aligned bases (kc is a multiple of 32)
    const int vec = (lda % 8 == 0 && ldb % 8 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(B) & 15) == 0)
                        ? 1
                        : 0;
#define PGC_GEMM_LAUNCH(TA_, TB_)                                                                                    \
    do {                                                                                                             \
        if (bt == 128)                                                                                               \
            hipLaunchKernelGGL((pgc::gemm_bf16<TA_, TB_, 128, 8>), grid, dim3(512), 0, st, M, N, K, kc, A, lda, B,   \
                               ldb, C, ldc, bias, acc, vec);                                                         \
        else                                                                                                         \
            hipLaunchKernelGGL((pgc::gemm_bf16<TA_, TB_, 64, 4>), grid, dim3(256), 0, st, M, N, K, kc, A, lda, B,    \
                               ldb, C, ldc, bias, acc, vec);                                                         \
    } while (0)
    if (!ta && !tb)
        PGC_GEMM_LAUNCH(false, false);
    else if (!ta && tb)
        PGC_GEMM_LAUNCH(false, true);
    else if (ta && !tb)
        PGC_GEMM_LAUNCH(true, false);
    else
        PGC_GEMM_LAUNCH(true, true);
#undef PGC_GEMM_LAUNCH
    return hipGetLastError();
}

// forward pass of `rows` rows already normalised into s.X; the output layer's Z is yhat
hipError_t forward(pgc_surrogate_s& s, int rows, hipStream_t st)
{
    const bf16* x = s.X;
    int in = s.n;
    for (size_t l = 0; l < s.layers.size(); ++l) {
        Layer& L = s.layers[l];
        hipError_t e = gemm(rows, L.out, in, x, in, false, L.Wb, in, true, L.Z, L.out, L.b, false, st);
        if (e != hipSuccess) return e;
        if (l + 1 < s.layers.size()) {
            const int64_t m = (int64_t)rows * L.out;
            hipLaunchKernelGGL(pgc::silu_fwd, dim3(pgc::nb(m, 256)), dim3(256), 0, st, L.Z, L.H, m);
            x = L.H;
            in = L.out;
        }
    }
    return hipGetLastError();
}

// loss and gradients of the rows in s.X against targets q (rows idx, or 0..rows-1)
// gradients of one batch; the batch loss is added to s.loss[0], which is first
// cleared when zero_loss is set (training clears it once per epoch instead)
hipError_t backward(pgc_surrogate_s& s, int rows, const float* q, const int* idx, hipStream_t st,
                    bool zero_loss = true)
{
    const int n = s.n;
    Layer& out = s.layers.back();
    const int64_t m = (int64_t)rows * n;
    if (zero_loss) hipLaunchKernelGGL(pgc::zero_f64, dim3(1), dim3(64), 0, st, s.loss, 2);
    if (s.loss_relative)
        hipLaunchKernelGGL(pgc::row_sqnorm, dim3(rows), dim3(256), 0, st, q, idx, n, s.rownorm);
    hipLaunchKernelGGL(pgc::mse_grad, dim3(std::min<unsigned>(pgc::nb(m, 256), 1024u)), dim3(256), 0, st, out.Z, q,
                       idx, rows, n, s.mu_out,
                       s.sd_out, s.loss_relative ? s.rownorm : nullptr, s.dY32, s.dY, s.loss);
    const bf16* g = s.dY;
    const float* g32 = s.dY32;
    for (int l = (int)s.layers.size() - 1; l >= 0; --l) {
        Layer& L = s.layers[l];
        const bf16* hin = l > 0 ? s.layers[l - 1].H : s.X;
        // dW = g^T h_in  (out x in), db = column sums of g
        hipError_t e = gemm(L.out, L.in, rows, g, L.out, true, hin, L.in, false, L.gW, L.in, nullptr, false, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pgc::col_sum, dim3(pgc::nb(L.out, 16)), dim3(256), 0, st, g32, rows, L.out, L.gb);
        if (l == 0) break;
        Layer& P = s.layers[l - 1];
        // dh_in = g W (rows x in), then through the activation of layer l - 1
        e = gemm(rows, L.in, L.out, g, L.out, false, L.Wb, L.in, false, P.dH, L.in, nullptr, false, st);
        if (e != hipSuccess) return e;
        const int64_t mm = (int64_t)rows * P.out;
        hipLaunchKernelGGL(pgc::silu_bwd, dim3(pgc::nb(mm, 256)), dim3(256), 0, st, P.dH, P.Z, P.dZ, P.dZ32, mm);
        g = P.dZ;
        g32 = P.dZ32;
    }
    return hipGetLastError();
}

hipError_t adam_all(pgc_surrogate_s& s, double lr, hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    ++s.steps;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)s.steps));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)s.steps));
    for (Layer& L : s.layers) {
        const int64_t nw = (int64_t)L.in * L.out;
        hipLaunchKernelGGL(pgc::adam_step, dim3(pgc::nb(nw, 256)), dim3(256), 0, st, L.W, L.gW, L.mW, L.vW, L.Wb, nw,
                           (float)lr, b1, b2, eps, c1, c2);
        hipLaunchKernelGGL(pgc::adam_step, dim3(pgc::nb(L.out, 256)), dim3(256), 0, st, L.b, L.gb, L.mb, L.vb,
                           (bf16*)nullptr, (int64_t)L.out, (float)lr, b1, b2, eps, c1, c2);
    }
    return hipGetLastError();
}

hipError_t refresh_bf16(pgc_surrogate_s& s, hipStream_t st)
{
    for (Layer& L : s.layers) {
        const int64_t nw = (int64_t)L.in * L.out;
        hipLaunchKernelGGL(pgc::f32_to_bf16, dim3(pgc::nb(nw, 256)), dim3(256), 0, st, L.W, L.Wb, nw);
    }
    return hipGetLastError();
}

// the invariant functionals of the plan: mass, momentum (dim) and energy of
// sum_k c_k T~_k, as vectors over the N^d coefficients
void build_constraints(const pgc::Plan& p, std::vector<double>& cons, std::vector<double>& ginv,
                       std::vector<double>& cnorm, int& nc)
{
    const int N = p.N, d = p.dim;
    const int64_t n = p.Nd;
    nc = d + 2;
    cons.assign((size_t)nc * n, 0.0);
    const double* m0 = p.mom.data();
    const double* m1 = p.mom.data() + N;
    const double* m2 = p.mom.data() + 2 * N;
    for (int64_t f = 0; f < n; ++f) {
        int k[3] = {0, 0, 0};
        int64_t r = f;
        for (int l = d - 1; l >= 0; --l) {
            k[l] = (int)(r % N);
            r /= N;
        }
        double mass = 1.0;
        for (int l = 0; l < d; ++l) mass *= m0[k[l]];
        cons[f] = mass;
        double energy = 0.0;
        for (int l = 0; l < d; ++l) {
            double a = 1.0, e = 1.0;
            for (int j = 0; j < d; ++j) {
                a *= (j == l) ? m1[k[j]] : m0[k[j]];
                e *= (j == l) ? m2[k[j]] : m0[k[j]];
            }
            cons[(size_t)(1 + l) * n + f] = a;
            energy += e;
        }
        cons[(size_t)(1 + d) * n + f] = energy;
    }
    // Gram matrix and its inverse (Gauss-Jordan, small and well conditioned
    // after scaling each row to unit norm)
    cnorm.assign(nc, 0.0);
    for (int a = 0; a < nc; ++a) {
        double s = 0.0;
        for (int64_t f = 0; f < n; ++f) s += cons[(size_t)a * n + f] * cons[(size_t)a * n + f];
        cnorm[a] = std::sqrt(s);
    }
    std::vector<double> g((size_t)nc * nc), inv((size_t)nc * nc, 0.0);
    for (int a = 0; a < nc; ++a)
        for (int b = 0; b < nc; ++b) {
            double s = 0.0;
            for (int64_t f = 0; f < n; ++f) s += cons[(size_t)a * n + f] * cons[(size_t)b * n + f];
            g[a * nc + b] = s;
        }
    for (int a = 0; a < nc; ++a) inv[a * nc + a] = 1.0;
    for (int c = 0; c < nc; ++c) {
        int piv = c;
        for (int r = c + 1; r < nc; ++r)
            if (std::fabs(g[r * nc + c]) > std::fabs(g[piv * nc + c])) piv = r;
        for (int j = 0; j < nc; ++j) {
            std::swap(g[c * nc + j], g[piv * nc + j]);
            std::swap(inv[c * nc + j], inv[piv * nc + j]);
        }
        const double dpiv = g[c * nc + c];
        for (int j = 0; j < nc; ++j) {
            g[c * nc + j] /= dpiv;
            inv[c * nc + j] /= dpiv;
        }
        for (int r = 0; r < nc; ++r) {
            if (r == c) continue;
            const double f = g[r * nc + c];
            for (int j = 0; j < nc; ++j) {
                g[r * nc + j] -= f * g[c * nc + j];
                inv[r * nc + j] -= f * inv[c * nc + j];
            }
        }
    }
    ginv = inv;
}

hipError_t normalise_rows(pgc_surrogate_s& s, const float* f, const int* idx, int64_t first, int rows,
                          hipStream_t st)
{
    const int64_t m = (int64_t)rows * s.n;
    hipLaunchKernelGGL(pgc::normalise_in, dim3(pgc::nb(m, 256)), dim3(256), 0, st, f, idx, first, rows, s.n, s.mu_in,
                       s.sd_in, s.X);
    return hipGetLastError();
}

}  // namespace

extern "C" {

pgc_status pgc_surrogate_desc_init(pgc_surrogate_desc* d)
{
    if (!d) return PGC_ERR_INVALID_ARG;
    std::memset(d, 0, sizeof(*d));
    d->width = 1024;
    d->n_layers = 4;
    d->batch_max = 256;
    d->seed = 2024;
    d->gate_residual = 1e-6;
    d->gate_raw_factor = 4.0;
    d->judge_stride = 64;
    d->judge_tol = 5e-2;
    d->norm_floor_in = 0.1;
    d->norm_floor_out = 1.0;
    return PGC_OK;
}

pgc_status pgc_surrogate_create(pgc_plan plan, const pgc_surrogate_desc* d, void* stream, pgc_surrogate* out)
{
    if (!plan || !d || !out) return PGC_ERR_INVALID_ARG;
    *out = nullptr;
    const pgc::Plan& p = plan->p;
    // the plan's fast path is the fallback and the judge: FP32, rates of |u| alone
    if (p.precision != PGC_PRECISION_FP32) return PGC_ERR_UNSUPPORTED;
    if (d->width < 16 || d->width > 8192 || d->n_layers < 2 || d->n_layers > 16 || d->batch_max < 1 ||
        d->batch_max > 65536 || d->gate_residual < 0 || d->judge_stride < 0 || d->gate_raw_factor < 0 ||
        !(d->norm_floor_in > 0 && d->norm_floor_in <= 1) || !(d->norm_floor_out > 0 && d->norm_floor_out <= 1) ||
        (d->loss_relative != 0 && d->loss_relative != 1))
        return PGC_ERR_INVALID_ARG;
    if (p.Nd > (1 << 22)) return PGC_ERR_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    pgc_surrogate_s* s = nullptr;
    try {
        s = new pgc_surrogate_s();
    } catch (const std::bad_alloc&) {
        return PGC_ERR_OUT_OF_MEMORY;
    }
    s->plan = plan;
    s->n = (int)p.Nd;
    s->width = d->width;
    s->n_layers = d->n_layers;
    s->bmax = d->batch_max;
    s->seed = d->seed;
    s->gate_residual = d->gate_residual;
    s->gate_raw_factor = d->gate_raw_factor;
    s->judge_stride = d->judge_stride;
    s->judge_tol = d->judge_tol;
    s->floor_in = (float)d->norm_floor_in;
    s->floor_out = (float)d->norm_floor_out;
    s->loss_relative = d->loss_relative;
    hipError_t e = hipSuccess;
    std::vector<double> cons, ginv, cnorm;
    std::mt19937_64 rng(d->seed);
    std::vector<float> hostw;
    const int B = s->bmax;
    try {  // host containers throw only on allocation failure
        build_constraints(p, cons, ginv, cnorm, s->nc);
        for (int l = 0; l < d->n_layers && e == hipSuccess; ++l) {
            Layer L;
            L.in = l == 0 ? s->n : d->width;
            L.out = l + 1 == d->n_layers ? s->n : d->width;
            const int64_t nw = (int64_t)L.in * L.out;
            if ((e = s_alloc_n(*s, &L.W, nw)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.gW, nw)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.mW, nw)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.vW, nw)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.Wb, nw)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.b, L.out)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.gb, L.out)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.mb, L.out)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.vb, L.out)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.Z, (int64_t)B * L.out)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.H, (int64_t)B * L.out)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.dH, (int64_t)B * L.out)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.dZ32, (int64_t)B * L.out)) != hipSuccess) break;
            if ((e = s_alloc_n(*s, &L.dZ, (int64_t)B * L.out)) != hipSuccess) break;
            // He-style uniform initialisation, bound sqrt(6 / in) (SiLU ~ ReLU scale)
            hostw.resize((size_t)nw);
            const double bound = std::sqrt(6.0 / L.in) * (l + 1 == d->n_layers ? 0.1 : 1.0);
            std::uniform_real_distribution<double> U(-bound, bound);
            for (auto& w : hostw) w = (float)U(rng);
            if ((e = hipMemcpy(L.W, hostw.data(), nw * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) break;
            hipLaunchKernelGGL(pgc::fill_f32, dim3(pgc::nb(L.out, 256)), dim3(256), 0, st, L.b, 0.f, (int64_t)L.out);
            hipLaunchKernelGGL(pgc::fill_f32, dim3(pgc::nb(nw, 256)), dim3(256), 0, st, L.mW, 0.f, nw);
            hipLaunchKernelGGL(pgc::fill_f32, dim3(pgc::nb(nw, 256)), dim3(256), 0, st, L.vW, 0.f, nw);
            hipLaunchKernelGGL(pgc::fill_f32, dim3(pgc::nb(L.out, 256)), dim3(256), 0, st, L.mb, 0.f, (int64_t)L.out);
            hipLaunchKernelGGL(pgc::fill_f32, dim3(pgc::nb(L.out, 256)), dim3(256), 0, st, L.vb, 0.f, (int64_t)L.out);
            s->layers.push_back(L);
        }
    } catch (...) {
        s_free(s);
        return PGC_ERR_OUT_OF_MEMORY;
    }
    const int64_t n = s->n;
    if (e == hipSuccess) e = s_alloc_n(*s, &s->mu_in, n);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->sd_in, n);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->mu_out, n);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->sd_out, n);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->X, (int64_t)B * n);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->dY32, (int64_t)B * n);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->dY, (int64_t)B * n);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->qtmp, (int64_t)B * n);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->scratch, 64);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->idx, B);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->loss, 2);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->res_raw, B);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->rownorm, B);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->res_out, B);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->err, B);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->zs, B);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->cons, (int64_t)s->nc * n);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->ginv, (int64_t)s->nc * s->nc);
    if (e == hipSuccess) e = s_alloc_n(*s, &s->cnorm, s->nc);
    if (e == hipSuccess) e = hipMemcpy(s->cons, cons.data(), cons.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->ginv, ginv.data(), ginv.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->cnorm, cnorm.data(), cnorm.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pgc::fill_f32, dim3(pgc::nb(n, 256)), dim3(256), 0, st, s->mu_in, 0.f, n);
        hipLaunchKernelGGL(pgc::fill_f32, dim3(pgc::nb(n, 256)), dim3(256), 0, st, s->sd_in, 1.f, n);
        hipLaunchKernelGGL(pgc::fill_f32, dim3(pgc::nb(n, 256)), dim3(256), 0, st, s->mu_out, 0.f, n);
        hipLaunchKernelGGL(pgc::fill_f32, dim3(pgc::nb(n, 256)), dim3(256), 0, st, s->sd_out, 1.f, n);
        e = refresh_bf16(*s, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        s_free(s);
        return pgc::status_of(e);
    }
    *out = s;
    return PGC_OK;
}

pgc_status pgc_surrogate_destroy(pgc_surrogate s)
{
    s_free(s);
    return PGC_OK;
}

pgc_status pgc_surrogate_query(pgc_surrogate s, pgc_surrogate_info* info)
{
    if (!s || !info) return PGC_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    info->n_features = s->n;
    info->width = s->width;
    info->n_layers = s->n_layers;
    info->batch_max = s->bmax;
    int64_t np = 0;
    for (const Layer& L : s->layers) np += (int64_t)L.in * L.out + L.out;
    info->n_params = np;
    info->n_constraints = s->nc;
    info->steps = s->steps;
    info->raw_residual_calibrated = s->raw_calib;
    info->zscore_calibrated = s->z_calib;
    info->workspace_bytes = s->bytes;
    return PGC_OK;
}

pgc_status pgc_surrogate_set_normalization(pgc_surrogate s, const float* f_dev, const float* q_dev, int64_t n_samples,
                                           void* stream)
{
    if (!s || !f_dev || !q_dev || n_samples < 1) return PGC_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = s->n;
    hipLaunchKernelGGL(pgc::feature_stats, dim3(pgc::nb(n, 256)), dim3(256), 0, st, f_dev, n_samples, n, s->mu_in,
                       s->sd_in);
    hipLaunchKernelGGL(pgc::feature_stats, dim3(pgc::nb(n, 256)), dim3(256), 0, st, q_dev, n_samples, n, s->mu_out,
                       s->sd_out);
    // standard deviations are held at or above floor x the largest one: the
    // output floor 1 scales every output alike, so that the loss measures the
    // L2 error of Q itself rather than inflating its smallest modes
    hipLaunchKernelGGL(pgc::max_reduce, dim3(1), dim3(1024), 0, st, s->sd_in, n, s->scratch);
    hipLaunchKernelGGL(pgc::floor_sd, dim3(pgc::nb(n, 256)), dim3(256), 0, st, s->sd_in, n, s->scratch, s->floor_in);
    hipLaunchKernelGGL(pgc::max_reduce, dim3(1), dim3(1024), 0, st, s->sd_out, n, s->scratch + 1);
    hipLaunchKernelGGL(pgc::floor_sd, dim3(pgc::nb(n, 256)), dim3(256), 0, st, s->sd_out, n, s->scratch + 1,
                       s->floor_out);
    return pgc::status_of(hipGetLastError());
}

pgc_status pgc_surrogate_train(pgc_surrogate s, const float* f_dev, const float* q_dev, int64_t n_samples,
                               int32_t epochs, int32_t batch, double lr, uint64_t seed, double* loss_host,
                               void* stream)
{
    if (!s || !f_dev || !q_dev || n_samples < 1 || epochs < 0 || batch < 1 || batch > s->bmax || !(lr > 0))
        return PGC_ERR_INVALID_ARG;
    if (n_samples > 2147483647ll) return PGC_ERR_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::mt19937_64 rng(seed);
    std::vector<int> perm;
    std::vector<double> rr, zz;
    try {
        perm.resize((size_t)n_samples);
        rr.resize((size_t)s->bmax);
        zz.resize((size_t)s->bmax);
    } catch (...) {
        return PGC_ERR_OUT_OF_MEMORY;
    }
    // the epoch's sample order on the device: the steps of an epoch are queued
    // without host round trips, and the stream is synchronised once per epoch
    int* perm_dev = nullptr;
    hipError_t e = hipMalloc(&perm_dev, (size_t)n_samples * sizeof(int));
    if (e != hipSuccess) return pgc::status_of(e);
    bool diverged = false;  // an epoch's loss came back not finite: stop
    for (int ep = 0; ep < epochs && e == hipSuccess && !diverged; ++ep) {
        std::iota(perm.begin(), perm.end(), 0);
        std::shuffle(perm.begin(), perm.end(), rng);
        e = hipMemcpyAsync(perm_dev, perm.data(), (size_t)n_samples * sizeof(int), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(pgc::zero_f64, dim3(1), dim3(64), 0, st, s->loss, 2);
            e = hipGetLastError();
        }
        int64_t steps = 0;
        // cosine decay of the step size over the epochs
        const double lr_ep = lr * 0.5 * (1.0 + std::cos(3.141592653589793 * ep / std::max(1, epochs)));
        for (int64_t b0 = 0; b0 + batch <= n_samples && e == hipSuccess; b0 += batch) {
            const int* idx = perm_dev + b0;
            e = normalise_rows(*s, f_dev, idx, 0, batch, st);
            if (e == hipSuccess) e = forward(*s, batch, st);
            if (e == hipSuccess) e = backward(*s, batch, q_dev, idx, st, false);
            if (e == hipSuccess) e = adam_all(*s, lr_ep, st);
            ++steps;
        }
        // s->loss[0] holds the sum of the batch losses of the epoch; the
        // synchronisation also keeps perm until its copy has been read
        double l = 0.0;
        if (e == hipSuccess) e = hipMemcpyAsync(&l, s->loss, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (loss_host) loss_host[ep] = steps ? l / (double)steps : 0.0;
        if (e == hipSuccess && !std::isfinite(l)) diverged = true;
    }
    (void)hipFree(perm_dev);
    if (e != hipSuccess) return pgc::status_of(e);
    if (diverged) return PGC_ERR_NUMERIC;
    // calibrate the out-of-distribution gate: largest raw residual on the training set
    double worst = 0.0, worst_z = 0.0;
    for (int64_t b0 = 0; b0 < n_samples && e == hipSuccess; b0 += s->bmax) {
        const int rows = (int)std::min<int64_t>(s->bmax, n_samples - b0);
        e = normalise_rows(*s, f_dev, nullptr, b0, rows, st);
        if (e == hipSuccess) e = forward(*s, rows, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(pgc::output_stage, dim3(rows), dim3(pgc::kOutThreads), 0, st, s->layers.back().Z, rows, s->n,
                               s->mu_out, s->sd_out, s->cons, s->nc, s->ginv, s->cnorm, s->qtmp, s->res_raw,
                               s->res_out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(pgc::row_zscore, dim3(rows), dim3(256), 0, st, f_dev, b0, s->n, s->mu_in, s->sd_in,
                               s->zs);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(rr.data(), s->res_raw, rows * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(zz.data(), s->zs, rows * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        for (int r = 0; r < rows; ++r) {
            worst = std::max(worst, rr[r]);
            worst_z = std::max(worst_z, zz[r]);
        }
    }
    s->raw_calib = worst;
    s->z_calib = worst_z;
    return pgc::status_of(e);
}

pgc_status pgc_surrogate_coeffs_to_q(pgc_surrogate s, const float* f_dev, int64_t n_samples, float* q_dev,
                                     int32_t* fallback_host, int64_t* n_fallback, double* judge_err, void* stream)
{
    if (!s || n_samples < 0 || (n_samples > 0 && (!f_dev || !q_dev))) return PGC_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = s->n;
    hipError_t e = hipSuccess;
    int64_t nfb = 0;
    double worst_judge = 0.0;
    std::vector<double> rr, ro, er, zz;
    std::vector<int> fb, jrow;
    try {
        for (auto* v : {&rr, &ro, &er, &zz}) v->resize((size_t)s->bmax);
        fb.resize((size_t)s->bmax);
        jrow.resize((size_t)s->bmax);
    } catch (...) {
        return PGC_ERR_OUT_OF_MEMORY;
    }
    const bool ood_on = s->gate_raw_factor > 0 && s->raw_calib > 0;
    const double raw_gate = s->gate_raw_factor * s->raw_calib, z_gate = s->gate_raw_factor * s->z_calib;
    const int64_t stride = s->judge_stride;
    for (int64_t b0 = 0; b0 < n_samples && e == hipSuccess; b0 += s->bmax) {
        const int rows = (int)std::min<int64_t>(s->bmax, n_samples - b0);
        float* qo = q_dev + (size_t)b0 * n;
        e = normalise_rows(*s, f_dev, nullptr, b0, rows, st);
        if (e == hipSuccess) e = forward(*s, rows, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(pgc::output_stage, dim3(rows), dim3(pgc::kOutThreads), 0, st, s->layers.back().Z, rows, n, s->mu_out,
                               s->sd_out, s->cons, s->nc, s->ginv, s->cnorm, qo, s->res_raw, s->res_out);
            e = hipGetLastError();
        }
        if (e == hipSuccess && ood_on) {
            hipLaunchKernelGGL(pgc::row_zscore, dim3(rows), dim3(256), 0, st, f_dev, b0, n, s->mu_in, s->sd_in, s->zs);
            e = hipGetLastError();
        }
        // the judge: the plain evaluation of every judge_stride-th sample, compared
        // with the network's output; the sample then returns the plain value
        int nj = 0;
        if (e == hipSuccess && stride > 0) {
            for (int r = 0; r < rows; ++r) {
                if ((b0 + r) % stride != 0) continue;
                pgc_status ps = pgc_coeffs_to_q(s->plan, f_dev + (size_t)(b0 + r) * n, s->qtmp + (size_t)nj * n,
                                                nullptr, stream);
                if (ps != PGC_OK) return ps;
                hipLaunchKernelGGL(pgc::row_rel_err, dim3(1), dim3(256), 0, st, qo + (size_t)r * n,
                                   s->qtmp + (size_t)nj * n, n, s->err + nj);
                e = hipMemcpyAsync(qo + (size_t)r * n, s->qtmp + (size_t)nj * n, (size_t)n * sizeof(float),
                                   hipMemcpyDeviceToDevice, st);
                if (e != hipSuccess) break;
                jrow[nj++] = r;
            }
        }
        if (e == hipSuccess) e = hipMemcpyAsync(rr.data(), s->res_raw, rows * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(ro.data(), s->res_out, rows * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && ood_on)
            e = hipMemcpyAsync(zz.data(), s->zs, rows * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && nj > 0) e = hipMemcpyAsync(er.data(), s->err, nj * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        for (int r = 0; r < rows; ++r) {
            const bool bad = !(ro[r] <= s->gate_residual) ||
                             (ood_on && (!(rr[r] <= raw_gate) || !(zz[r] <= z_gate)));
            fb[r] = bad ? 1 : 0;
        }
        // a judged sample stands for the stride of samples that start with it:
        // when the network missed it, they fall back too
        for (int j = 0; j < nj; ++j) {
            worst_judge = std::max(worst_judge, er[j]);
            const int r0 = jrow[j];
            fb[r0] = 2;
            if (!(er[j] <= s->judge_tol))
                for (int r = r0 + 1; r < rows && r < r0 + stride; ++r) fb[r] = fb[r] ? fb[r] : 1;
        }
        for (int r = 0; r < rows && e == hipSuccess; ++r) {
            if (fb[r] != 1) continue;
            pgc_status ps = pgc_coeffs_to_q(s->plan, f_dev + (size_t)(b0 + r) * n, qo + (size_t)r * n, nullptr, stream);
            if (ps != PGC_OK) return ps;
            ++nfb;
        }
        if (fallback_host) std::copy(fb.begin(), fb.begin() + rows, fallback_host + b0);
    }
    if (n_fallback) *n_fallback = nfb;
    if (judge_err) *judge_err = worst_judge;
    return pgc::status_of(e);
}

pgc_status pgc_surrogate_loss_grad(pgc_surrogate s, const float* f_dev, const float* q_dev, int32_t n_samples,
                                   double* loss_host, float* grad_host, void* stream)
{
    if (!s || !f_dev || !q_dev || n_samples < 1 || n_samples > s->bmax) return PGC_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = normalise_rows(*s, f_dev, nullptr, 0, n_samples, st);
    if (e == hipSuccess) e = forward(*s, n_samples, st);
    if (e == hipSuccess) e = backward(*s, n_samples, q_dev, nullptr, st);
    double l = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&l, s->loss, sizeof(double), hipMemcpyDeviceToHost, st);
    size_t off = 0;
    for (const Layer& L : s->layers) {
        if (e != hipSuccess || !grad_host) break;
        const size_t nw = (size_t)L.in * L.out;
        e = hipMemcpyAsync(grad_host + off, L.gW, nw * sizeof(float), hipMemcpyDeviceToHost, st);
        off += nw;
        if (e == hipSuccess) e = hipMemcpyAsync(grad_host + off, L.gb, L.out * sizeof(float), hipMemcpyDeviceToHost, st);
        off += L.out;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (loss_host) *loss_host = l;
    return pgc::status_of(e);
}

// parameters, flattened layer by layer as W (out x in, row-major) then b,
// followed by the four normalisation vectors mu_in, sd_in, mu_out, sd_out
pgc_status pgc_surrogate_get_params(pgc_surrogate s, float* params_host, void* stream)
{
    if (!s || !params_host) return PGC_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    size_t off = 0;
    for (const Layer& L : s->layers) {
        const size_t nw = (size_t)L.in * L.out;
        if (e == hipSuccess) e = hipMemcpyAsync(params_host + off, L.W, nw * sizeof(float), hipMemcpyDeviceToHost, st);
        off += nw;
        if (e == hipSuccess) e = hipMemcpyAsync(params_host + off, L.b, L.out * sizeof(float), hipMemcpyDeviceToHost, st);
        off += L.out;
    }
    const float* nv[4] = {s->mu_in, s->sd_in, s->mu_out, s->sd_out};
    for (int k = 0; k < 4; ++k) {
        if (e == hipSuccess) e = hipMemcpyAsync(params_host + off, nv[k], s->n * sizeof(float), hipMemcpyDeviceToHost, st);
        off += s->n;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return pgc::status_of(e);
}

pgc_status pgc_surrogate_set_params(pgc_surrogate s, const float* params_host, void* stream)
{
    if (!s || !params_host) return PGC_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    size_t off = 0;
    for (Layer& L : s->layers) {
        const size_t nw = (size_t)L.in * L.out;
        if (e == hipSuccess) e = hipMemcpyAsync(L.W, params_host + off, nw * sizeof(float), hipMemcpyHostToDevice, st);
        off += nw;
        if (e == hipSuccess) e = hipMemcpyAsync(L.b, params_host + off, L.out * sizeof(float), hipMemcpyHostToDevice, st);
        off += L.out;
    }
    float* nv[4] = {s->mu_in, s->sd_in, s->mu_out, s->sd_out};
    for (int k = 0; k < 4; ++k) {
        if (e == hipSuccess) e = hipMemcpyAsync(nv[k], params_host + off, s->n * sizeof(float), hipMemcpyHostToDevice, st);
        off += s->n;
    }
    if (e == hipSuccess) e = refresh_bf16(*s, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return pgc::status_of(e);
}

pgc_status pgc_surrogate_save(pgc_surrogate s, const char* path, void* stream)
{
    if (!s || !path) return PGC_ERR_INVALID_ARG;
    pgc_surrogate_info info;
    pgc_surrogate_query(s, &info);
    const size_t total = (size_t)info.n_params + 4 * (size_t)s->n;
    std::vector<float> buf;
    try {
        buf.resize(total);
    } catch (const std::bad_alloc&) {
        return PGC_ERR_OUT_OF_MEMORY;
    }
    pgc_status ps = pgc_surrogate_get_params(s, buf.data(), stream);
    if (ps != PGC_OK) return ps;
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return PGC_ERR_INVALID_ARG;
    const int32_t hdr[4] = {0x50474353, s->n, s->width, s->n_layers};  // "PGCS"
    bool ok = std::fwrite(hdr, sizeof(hdr), 1, fp) == 1 && std::fwrite(&s->raw_calib, sizeof(double), 1, fp) == 1 &&
              std::fwrite(&s->z_calib, sizeof(double), 1, fp) == 1 &&
              std::fwrite(buf.data(), sizeof(float), total, fp) == total;
    ok = (std::fclose(fp) == 0) && ok;
    return ok ? PGC_OK : PGC_ERR_INVALID_ARG;
}

pgc_status pgc_surrogate_load(pgc_surrogate s, const char* path, void* stream)
{
    if (!s || !path) return PGC_ERR_INVALID_ARG;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return PGC_ERR_INVALID_ARG;
    int32_t hdr[4];
    double calib = 0.0, zcal = 0.0;
    bool ok = std::fread(hdr, sizeof(hdr), 1, fp) == 1 && std::fread(&calib, sizeof(double), 1, fp) == 1 &&
              std::fread(&zcal, sizeof(double), 1, fp) == 1;
    ok = ok && hdr[0] == 0x50474353 && hdr[1] == s->n && hdr[2] == s->width && hdr[3] == s->n_layers;
    pgc_surrogate_info info;
    pgc_surrogate_query(s, &info);
    const size_t total = (size_t)info.n_params + 4 * (size_t)s->n;
    std::vector<float> buf;
    if (ok) {
        try {
            buf.resize(total);
        } catch (const std::bad_alloc&) {
            std::fclose(fp);
            return PGC_ERR_OUT_OF_MEMORY;
        }
        ok = std::fread(buf.data(), sizeof(float), total, fp) == total;
    }
    std::fclose(fp);
    if (!ok) return PGC_ERR_INVALID_ARG;
    pgc_status ps = pgc_surrogate_set_params(s, buf.data(), stream);
    if (ps == PGC_OK) {
        s->raw_calib = calib;
        s->z_calib = zcal;
    }
    return ps;
}

// C = op(A) op(B) for BF16 host matrices (testing the matrix-core product)
pgc_status pgc_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* a_dev, int32_t lda, int32_t trans_a,
                         const uint16_t* b_dev, int32_t ldb, int32_t trans_b, float* c_dev, int32_t ldc,
                         const float* bias_dev, int32_t accumulate, void* stream)
{
    if (M < 0 || N < 0 || K < 0) return PGC_ERR_INVALID_ARG;
    if (M > 0 && N > 0) {
        // row strides cover the rows they step over
        if (!c_dev || ldc < N) return PGC_ERR_INVALID_ARG;
        if (K > 0 && (!a_dev || !b_dev || lda < (trans_a ? M : K) || ldb < (trans_b ? K : N)))
            return PGC_ERR_INVALID_ARG;
    }
    return pgc::status_of(gemm(M, N, K, a_dev, lda, trans_a != 0, b_dev, ldb, trans_b != 0, c_dev, ldc, bias_dev,
                               accumulate != 0, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
