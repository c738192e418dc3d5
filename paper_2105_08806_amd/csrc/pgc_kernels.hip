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

#include <cmath>
#include <cstdint>

#include "pgc_internal.h"

namespace pgc {
namespace {

constexpr int kRedThreads = 1024;

__device__ __forceinline__ int fold_index(int t, int nh)
{
    // reflection of an unfolded grid index into [0, nh]: the images -z and
    // 2 pi - z of a point z in [0, pi] land on -t and 2 nh - t.
    return t < 0 ? -t : (t > nh ? 2 * nh - t : t);
}

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

// apply the K x L matrix M along every axis of a dim-dimensional L^dim tensor
template <typename T>
hipError_t separable(const Plan& p, const T* in, T* out, const T* M, int K, int L, hipStream_t s)
{
    int64_t dims[3] = {L, L, L};
    const T* src = in;
    T* bufs[2] = {static_cast<T*>(p.ws.tmpA), static_cast<T*>(p.ws.tmpB)};
    int pp = 0;
    for (int ax = p.dim - 1; ax >= 0; --ax) {
        T* dst = (ax == 0) ? out : bufs[pp];
        pp ^= 1;
        int64_t A = 1, B = 1;
        for (int l = 0; l < ax; ++l) A *= dims[l];
        for (int l = ax + 1; l < p.dim; ++l) B *= dims[l];
        const int64_t total = A * K * B;
        const int threads = 256;
        const int64_t blocks = (total + threads - 1) / threads;
        hipLaunchKernelGGL(sep_apply<T>, dim3((unsigned)blocks), dim3(threads), 0, s, src, dst, M, A,
                           L, B, K);
        dims[ax] = K;
        src = dst;
    }
    return hipGetLastError();
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

// G_i = w_i mu_i^2 P_i  (the weighted f_N / mu^2 of the gain and loss integrals)
template <typename T>
__global__ void make_weighted(const T* __restrict__ P, T* __restrict__ G, const T* __restrict__ w1,
                              const T* __restrict__ mu21, int dim, int ni, int64_t nid)
{
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= nid) return;
    T w, mu2;
    node_weights(f, dim, ni, w1, mu21, w, mu2);
    G[f] = w * mu2 * P[f];
}

// ------------------------------------------------------------------ loss

// red[0] = sum_j G_j  (Maxwell molecules: the inner integral of eq. Qminus is
// a single number; FP64 accumulation, fixed order within one workgroup)
template <typename T>
__global__ void __launch_bounds__(kRedThreads) sum_kernel(const T* __restrict__ G, int64_t n,
                                                          double* __restrict__ red)
{
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    for (int64_t f = threadIdx.x; f < n; f += blockDim.x) acc += (double)G[f];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
        red[0] = t;
    }
}

// H_i = w_i A P_i with A = (sum_s W_s) b0 sum_j G_j
template <typename T>
__global__ void loss_h_maxwell(const T* __restrict__ P, T* __restrict__ H, const T* __restrict__ w1,
                               const T* __restrict__ mu21, const double* __restrict__ red,
                               double scale, int dim, int ni, int64_t nid)
{
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= nid) return;
    T w, mu2;
    node_weights(f, dim, ni, w1, mu21, w, mu2);
    const T A = (T)(scale * red[0]);
    H[f] = w * A * P[f];
}

// VHS: A_i = (sum_s W_s) b0 sum_j G_j |v_i - v_j|^gamma, one thread per node i,
// the j sweep staged through LDS in tiles.
template <typename T, int DIM>
__global__ void __launch_bounds__(256) loss_h_vhs(const T* __restrict__ P, const T* __restrict__ G,
                                                  T* __restrict__ H, const T* __restrict__ v1,
                                                  const T* __restrict__ w1,
                                                  const T* __restrict__ mu21, double scale,
                                                  T gamma, int ni, int64_t nid)
{
    constexpr int kTile = 256;
    __shared__ T sv[kTile][DIM];
    __shared__ T sg[kTile];
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    T vi[DIM];
    {
        int64_t r = f < nid ? f : 0;
        for (int l = DIM - 1; l >= 0; --l) {
            vi[l] = v1[r % ni];
            r /= ni;
        }
    }
    T acc = 0;
    for (int64_t j0 = 0; j0 < nid; j0 += kTile) {
        __syncthreads();
        const int64_t j = j0 + threadIdx.x;
        if (threadIdx.x < kTile) {
            if (j < nid) {
                int64_t r = j;
                for (int l = DIM - 1; l >= 0; --l) {
                    sv[threadIdx.x][l] = v1[r % ni];
                    r /= ni;
                }
                sg[threadIdx.x] = G[j];
            } else {
                for (int l = 0; l < DIM; ++l) sv[threadIdx.x][l] = 0;
                sg[threadIdx.x] = 0;
            }
        }
        __syncthreads();
        const int cnt = (int)((nid - j0) < kTile ? (nid - j0) : kTile);
        for (int t = 0; t < cnt; ++t) {
            T u2 = 0;
            for (int l = 0; l < DIM; ++l) {
                const T d = vi[l] - sv[t][l];
                u2 += d * d;
            }
            T b;
            if (gamma == (T)1) b = sqrt(u2);
            else if (gamma == (T)0) b = 1;
            else b = u2 > 0 ? pow(u2, (T)0.5 * gamma) : (T)0;
            acc = fma(sg[t], b, acc);
        }
    }
    if (f >= nid) return;
    T w, mu2;
    node_weights(f, DIM, ni, w1, mu21, w, mu2);
    H[f] = w * (T)scale * acc * P[f];
}

// ------------------------------------------------------------------ gain

template <typename T>
struct GainParams {
    const T* v1;        // n_i interior node velocities
    const T* G;         // n_i^d  w_j g_j
    const T* sigma;     // n_sigma x d
    const T* sigma_w;   // n_sigma
    const T* poly;      // terms x W
    const T* slab_vlo;  // n_slabs
    const T* slab_vhi;
    double* partial;    // n_chunks x n_g^d
    T S, inv_S, h_inv, b0, gamma;
    int map, vhs, ni, ng, nh, slab_planes;
    int64_t nid, ngd, n_units, units_per_chunk;
};

// post-collision coordinate in the transform variable and the factor mu^-2:
//   r = 0: zeta = tanh(v/S), z = arccos zeta = 2 atan(exp(-v/S)), mu^-2 = S cosh(v/S)
//   r = 1: zeta = v/sqrt(S^2+v^2), z = atan2(S, v),              mu^-2 = (S^2+v^2)/S
template <typename T>
__device__ __forceinline__ void map_point(T v, const GainParams<T>& P, T& z, T& m2)
{
    if (P.map == 0) {
        const T e = exp(-v * P.inv_S);
        z = (T)2 * atan(e);
        m2 = (T)0.5 * P.S * (e + (T)1 / e);
    } else {
        z = atan2(P.S, v);
        m2 = (P.S * P.S + v * v) * P.inv_S;
    }
}

// values of the W kernel cells at offset s in [-1, 1): Horner in s
template <typename T, int W, int TERMS>
__device__ __forceinline__ void kernel_cells(const T* __restrict__ poly, T s, T* out)
{
#pragma unroll
    for (int a = 0; a < W; ++a) out[a] = poly[(TERMS - 1) * W + a];
#pragma unroll
    for (int d = TERMS - 2; d >= 0; --d) {
#pragma unroll
        for (int a = 0; a < W; ++a) out[a] = fma(out[a], s, poly[d * W + a]);
    }
}

// The fine grid accumulates in FP64 for both precisions: on gfx950 the LDS
// executes ds_add_f64 about 20x faster than ds_add_f32 (measured 7.4 vs 0.33
// lane-ops per clock per CU), and FP64 cells also remove the accumulation
// error of the FP32 path.
__device__ __forceinline__ void lds_add(double* addr, double v)
{
    __hip_atomic_fetch_add(addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One workgroup = (chunk of collision units, slab of fine-grid planes along
// the first dimension).  The slab lives in LDS; every unit (s, i) of the chunk
// is split into pencils j = (j_1, j_rest) with j_1 running.  Along a pencil
// the first component of v' = (v_i + v_j)/2 + |v_i - v_j| sigma/2 is
// non-decreasing in v_{j,1} (its derivative is (1 - sigma_1 cos)/2 >= 0), so
// the points that reach the slab form one contiguous j_1 range, found by a
// binary search against the slab's v'-window.
// FP64 points need about 2x the registers of FP32 ones: 512 threads keep
// 256 VGPRs per lane available without spilling.
template <typename T>
constexpr int spread_max_threads() { return sizeof(T) == 8 ? 512 : 1024; }

template <typename T, int DIM, int W>
__global__ void __launch_bounds__(spread_max_threads<T>()) gain_spread(GainParams<T> P)
{
    constexpr int TERMS = W + 2;
    extern __shared__ unsigned char lds_raw[];
    double* slab = reinterpret_cast<double*>(lds_raw);

    const int b = blockIdx.y;
    const int64_t c = blockIdx.x;
    const int p0 = b * P.slab_planes;
    const int p1 = min(P.ng, p0 + P.slab_planes);
    const int plane = (DIM == 2) ? P.ng : P.ng * P.ng;
    const int slab_elems = (p1 - p0) * plane;
    for (int e = threadIdx.x; e < slab_elems; e += blockDim.x) slab[e] = 0;
    __syncthreads();

    const T vlo = P.slab_vlo[b];
    const T vhi = P.slab_vhi[b];
    const int ni = P.ni;
    const int npencil = (DIM == 2) ? ni : ni * ni;
    const int64_t u0 = c * P.units_per_chunk;
    const int64_t u1 = min(P.n_units, u0 + P.units_per_chunk);
    const int64_t n_items = (u1 - u0) * npencil;
    const T half = (T)0.5;

    // Lanes of a wave take consecutive units of the same pencil: their points
    // land far apart on the grid.  (Consecutive pencils of one unit can map
    // onto the same cells -- e.g. v'_2 = max(v_i2, v_j2) for sigma = e_2 --
    // and then every lane's LDS atomic hits one address.)
    const int64_t n_u = u1 - u0;
    for (int64_t item = threadIdx.x; item < n_items; item += blockDim.x) {
        const int64_t u = u0 + item % n_u;
        const int pencil = (int)(item / n_u);
        const int s = (int)(u / P.nid);
        const int64_t i = u % P.nid;
        const T cu = P.sigma_w[s] * P.G[i] * P.b0;
        if (cu == (T)0) continue;

        T vi[DIM], sg[DIM], vr[DIM];
        {
            int64_t r = i;
            for (int l = DIM - 1; l >= 0; --l) {
                vi[l] = P.v1[r % ni];
                r /= ni;
            }
        }
        for (int l = 0; l < DIM; ++l) sg[l] = P.sigma[s * DIM + l];
        T r2 = 0;
        if constexpr (DIM == 2) {
            vr[1] = P.v1[pencil];
            const T d = vi[1] - vr[1];
            r2 = d * d;
        } else {
            vr[1] = P.v1[pencil / ni];
            vr[2] = P.v1[pencil % ni];
            const T d1 = vi[1] - vr[1], d2 = vi[2] - vr[2];
            r2 = d1 * d1 + d2 * d2;
        }

        // first j_1 whose v'_1 reaches the slab window
        int lo = 0, hi = ni;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const T vj = P.v1[mid];
            const T d = vi[0] - vj;
            const T un = sqrt(d * d + r2);
            const T v1p = (vi[0] + vj) * half + un * sg[0] * half;
            if (v1p < vlo) lo = mid + 1;
            else hi = mid;
        }

        for (int j1 = lo; j1 < ni; ++j1) {
            const T vj = P.v1[j1];
            const T d = vi[0] - vj;
            const T un = sqrt(d * d + r2);
            T vp[DIM];
            vp[0] = (vi[0] + vj) * half + un * sg[0] * half;
            if (vp[0] > vhi) break;
            const int64_t j = (int64_t)j1 * npencil + pencil;
            const T gj = P.G[j];
            if (gj == (T)0) continue;
            T q = cu * gj;
            if (P.vhs) q *= (P.gamma == (T)1) ? un : (un > (T)0 ? pow(un, P.gamma) : (T)(P.gamma == (T)0));
            for (int l = 1; l < DIM; ++l) vp[l] = (vi[l] + vr[l]) * half + un * sg[l] * half;

            int t0[DIM];
            T ker[DIM][W];
#pragma unroll
            for (int l = 0; l < DIM; ++l) {
                T z, m2;
                map_point(vp[l], P, z, m2);
                q *= m2;
                const T xs = z * P.h_inv - (T)(0.5 * W);
                const T tf = ceil(xs);
                t0[l] = (int)tf;
                kernel_cells<T, W, TERMS>(P.poly, (T)2 * (tf - xs) - (T)1, ker[l]);
            }

            int idx1[W];
#pragma unroll
            for (int a = 0; a < W; ++a) idx1[a] = fold_index(t0[1] + a, P.nh);
            if constexpr (DIM == 2) {
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const int m0 = fold_index(t0[0] + a, P.nh);
                    if (m0 < p0 || m0 >= p1) continue;
                    const T qa = q * ker[0][a];
                    double* row = slab + (m0 - p0) * plane;
#pragma unroll
                    for (int bb = 0; bb < W; ++bb) lds_add(row + idx1[bb], (double)(qa * ker[1][bb]));
                }
            } else {
                int idx2[W];
#pragma unroll
                for (int a = 0; a < W; ++a) idx2[a] = fold_index(t0[DIM - 1] + a, P.nh);
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const int m0 = fold_index(t0[0] + a, P.nh);
                    if (m0 < p0 || m0 >= p1) continue;
                    const T qa = q * ker[0][a];
                    double* pl = slab + (m0 - p0) * plane;
#pragma unroll
                    for (int bb = 0; bb < W; ++bb) {
                        const T qab = qa * ker[1][bb];
                        double* row = pl + idx1[bb] * P.ng;
#pragma unroll
                        for (int cc = 0; cc < W; ++cc)
                            lds_add(row + idx2[cc], (double)(qab * ker[DIM - 1][cc]));
                    }
                }
            }
        }
    }
    __syncthreads();
    double* dst = P.partial + c * P.ngd + (int64_t)p0 * plane;
    for (int e = threadIdx.x; e < slab_elems; e += blockDim.x) dst[e] = slab[e];
}

// grid[m] = sum_c partial[c][m], FP64 accumulation in chunk order
template <typename T>
__global__ void reduce_partials(const double* __restrict__ partial, T* __restrict__ grid,
                                int64_t ngd, int n_chunks)
{
    const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (m >= ngd) return;
    double acc = 0.0;
    for (int c = 0; c < n_chunks; ++c) acc += (double)partial[(int64_t)c * ngd + m];
    grid[m] = (T)acc;
}

template <typename T>
__global__ void combine_kernel(const T* __restrict__ qp, const T* __restrict__ qm, T* __restrict__ q,
                               T* __restrict__ qplus_out, int64_t n)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const T a = qp[k];
    q[k] = a - qm[k];
    if (qplus_out) qplus_out[k] = a;
}

// ------------------------------------------------------------------ projection

// H_i = w_i mu_i^-4 f(v_i)  (eq. MultiD_spectral_coef on the interior CGL nodes)
template <typename T>
__global__ void project_weight(const double* __restrict__ f, T* __restrict__ H,
                               const T* __restrict__ w1, const T* __restrict__ mu21, int dim, int ni,
                               int64_t nid)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nid) return;
    T w, mu2;
    node_weights(r, dim, ni, w1, mu21, w, mu2);
    H[r] = (T)(f[r] * (double)w / ((double)mu2 * (double)mu2));
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

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// ------------------------------------------------------------------ typed drivers

template <typename T>
hipError_t synthesis_t(const Plan& p, const void* coeffs, hipStream_t s)
{
    hipError_t e = separable<T>(p, static_cast<const T*>(coeffs), static_cast<T*>(p.ws.P),
                                static_cast<const T*>(p.dt.C), p.ni, p.N, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(make_weighted<T>, dim3(blocks_for(p.nid, 256)), dim3(256), 0, s,
                       static_cast<const T*>(p.ws.P), static_cast<T*>(p.ws.G),
                       static_cast<const T*>(p.dt.w1), static_cast<const T*>(p.dt.mu21), p.dim, p.ni,
                       p.nid);
    return hipGetLastError();
}

template <typename T>
hipError_t loss_t(const Plan& p, hipStream_t s)
{
    const double scale = p.wsum * p.b0;
    if (p.kernel == PGC_KERNEL_MAXWELL) {
        hipLaunchKernelGGL(sum_kernel<T>, dim3(1), dim3(kRedThreads), 0, s,
                           static_cast<const T*>(p.ws.G), p.nid, p.ws.red);
        hipLaunchKernelGGL(loss_h_maxwell<T>, dim3(blocks_for(p.nid, 256)), dim3(256), 0, s,
                           static_cast<const T*>(p.ws.P), static_cast<T*>(p.ws.H),
                           static_cast<const T*>(p.dt.w1), static_cast<const T*>(p.dt.mu21),
                           p.ws.red, scale, p.dim, p.ni, p.nid);
    } else if (p.dim == 2) {
        hipLaunchKernelGGL((loss_h_vhs<T, 2>), dim3(blocks_for(p.nid, 256)), dim3(256), 0, s,
                           static_cast<const T*>(p.ws.P), static_cast<const T*>(p.ws.G),
                           static_cast<T*>(p.ws.H), static_cast<const T*>(p.dt.v1),
                           static_cast<const T*>(p.dt.w1), static_cast<const T*>(p.dt.mu21), scale,
                           (T)p.gamma, p.ni, p.nid);
    } else {
        hipLaunchKernelGGL((loss_h_vhs<T, 3>), dim3(blocks_for(p.nid, 256)), dim3(256), 0, s,
                           static_cast<const T*>(p.ws.P), static_cast<const T*>(p.ws.G),
                           static_cast<T*>(p.ws.H), static_cast<const T*>(p.dt.v1),
                           static_cast<const T*>(p.dt.w1), static_cast<const T*>(p.dt.mu21), scale,
                           (T)p.gamma, p.ni, p.nid);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return separable<T>(p, static_cast<const T*>(p.ws.H), static_cast<T*>(p.ws.qminus),
                        static_cast<const T*>(p.dt.CT), p.N, p.ni, s);
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
hipError_t gain_t(const Plan& p, hipStream_t s)
{
    GainParams<T> gp;
    gp.v1 = static_cast<const T*>(p.dt.v1);
    gp.G = static_cast<const T*>(p.ws.G);
    gp.sigma = static_cast<const T*>(p.dt.sigma);
    gp.sigma_w = static_cast<const T*>(p.dt.sigma_w);
    gp.poly = static_cast<const T*>(p.dt.poly);
    gp.slab_vlo = static_cast<const T*>(p.dt.slab_vlo);
    gp.slab_vhi = static_cast<const T*>(p.dt.slab_vhi);
    gp.partial = static_cast<double*>(p.ws.partial);
    gp.S = (T)p.S;
    gp.inv_S = (T)(1.0 / p.S);
    gp.h_inv = (T)(1.0 / p.h);
    gp.b0 = (T)p.b0;
    gp.gamma = (T)p.gamma;
    gp.map = p.map;
    gp.vhs = p.kernel == PGC_KERNEL_VHS;
    gp.ni = p.ni;
    gp.ng = p.ng;
    gp.nh = p.nh;
    gp.slab_planes = p.slab_planes;
    gp.nid = p.nid;
    gp.ngd = p.ngd;
    gp.n_units = p.n_units;
    gp.units_per_chunk = p.units_per_chunk;
    hipError_t e = (p.dim == 2) ? spread_dispatch<T, 2>(p, gp, s) : spread_dispatch<T, 3>(p, gp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_partials<T>, dim3(blocks_for(p.ngd, 256)), dim3(256), 0, s,
                       static_cast<const double*>(p.ws.partial), static_cast<T*>(p.ws.grid), p.ngd,
                       p.n_chunks);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return separable<T>(p, static_cast<const T*>(p.ws.grid), static_cast<T*>(p.ws.qplus),
                        static_cast<const T*>(p.dt.E), p.N, p.ng, s);
}

template <typename T>
hipError_t combine_t(const Plan& p, void* q, void* qplus, hipStream_t s)
{
    hipLaunchKernelGGL(combine_kernel<T>, dim3(blocks_for(p.Nd, 256)), dim3(256), 0, s,
                       static_cast<const T*>(p.ws.qplus), static_cast<const T*>(p.ws.qminus),
                       static_cast<T*>(q), static_cast<T*>(qplus), p.Nd);
    return hipGetLastError();
}

template <typename T>
hipError_t project_t(const Plan& p, const double* f, void* coeffs, hipStream_t s)
{
    hipLaunchKernelGGL(project_weight<T>, dim3(blocks_for(p.nid, 256)), dim3(256), 0, s, f,
                       static_cast<T*>(p.ws.H), static_cast<const T*>(p.dt.w1),
                       static_cast<const T*>(p.dt.mu21), p.dim, p.ni, p.nid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return separable<T>(p, static_cast<const T*>(p.ws.H), static_cast<T*>(coeffs),
                        static_cast<const T*>(p.dt.CT), p.N, p.ni, s);
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_synthesis(const Plan& p, const void* coeffs, hipStream_t s)
{
    return p.precision == PGC_PRECISION_FP64 ? synthesis_t<double>(p, coeffs, s)
                                             : synthesis_t<float>(p, coeffs, s);
}

hipError_t launch_loss(const Plan& p, hipStream_t s)
{
    return p.precision == PGC_PRECISION_FP64 ? loss_t<double>(p, s) : loss_t<float>(p, s);
}

hipError_t launch_gain(const Plan& p, hipStream_t s)
{
    return p.precision == PGC_PRECISION_FP64 ? gain_t<double>(p, s) : gain_t<float>(p, s);
}

hipError_t launch_combine(const Plan& p, void* q, void* qplus, hipStream_t s)
{
    return p.precision == PGC_PRECISION_FP64 ? combine_t<double>(p, q, qplus, s)
                                             : combine_t<float>(p, q, qplus, s);
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
