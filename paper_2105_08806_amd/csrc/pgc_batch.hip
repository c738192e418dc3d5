// Batched evaluation of Q for many velocity cells with mixed N (2D, FP32 gain).
//
// A kinetic solver calls the collision operator once per spatial cell; the
// cells of one batch may use different numbers of modes.  The positions of the
// merged transform points (and so their bins, kernel values and fine-grid
// footprints) depend only on the discretisation of a cell, not on its f, so
// every cell with the same N shares one plan: its node tables, its sphere rule
// and its plan-time bin index.  Only the orbit-sum weight of a point differs
// between cells.  One work unit of the gain is (bin run, group of C cells of
// one N).  Two schemes: register tiles (each lane regenerates points of the
// run, forms C orbit sums and accumulates C private W x W footprint tiles), and
// lane per cell (the wave stages the geometry of 64 points in LDS once and
// each lane accumulates the tile of its own cell over every staged point,
// reading its cell's G from a cell-minor copy, so 64 cells share one
// geometry).  A single persistent launch pulls the units of every N group from
// one counter, the longest runs first; the autotuner picks the scheme and C.  The dense stages (synthesis, loss, grid to modes) are
// batched contractions over the cells of each group, in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "pgc_device.h"
#include "pgc_internal.h"

namespace pgc {
namespace {

constexpr int kMaxGroups = 8;

// per-N group, as the persistent gain kernel reads it
struct GroupDev {
    GainParams<float> gp;
    const int* item_bin;
    const long long* item_begin;
    const int* item_count;
    const unsigned long long* ids;
    const float* Gg;     // n_cells x nid, G of every cell rounded to FP32
    const float* Gt;     // nid x ldg, the same with the cell index fastest
    const int* order;    // bin runs in processing order (NULL: the plan's longest-first order)
    double* grid;        // n_cells x ngd FP64 fine grids
    int nb, off, n_cells, ncg;  // ncg = cell groups of C cells
    int ldg;             // row length of Gt (n_cells rounded up to 64)
    int group_major;     // units run through every bin run of one cell group before the next
    int64_t nid, ngd, unit_begin, n_items;
};

// bin run and first cell of unit `local` of a group
__device__ __forceinline__ void unit_of(const GroupDev& D, long long local, int C, int& item, int& c0)
{
    long long run, cg;
    if (D.group_major) {
        run = local % D.n_items;
        cg = local / D.n_items;
    } else {
        run = local / D.ncg;
        cg = local % D.ncg;
    }
    item = D.order ? D.order[run] : (int)run;
    c0 = (int)cg * C;
}

__device__ __forceinline__ unsigned long long lane0(unsigned long long x)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(x & 0xffffffffull), 0);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), 0);
    return ((unsigned long long)hi << 32) | lo;
}

// Persistent gain over every group: one 64-lane wave per workgroup takes units
// u = atomicAdd(counter) until the counter passes n_units (every wave reaches
// that exit).  Unit u of group g covers one bin run and C cells of the group:
// bin run (u - begin_g) / ncg_g and cells C ((u - begin_g) % ncg_g) .. + C - 1
// (bin-run major), or with the roles swapped (cell-group major: the waves
// that run at the same time read the G rows of one cell group, which stay in L2).
template <int W, int C>
__global__ void __launch_bounds__(64) gain_batched(const GroupDev* __restrict__ groups, int n_groups,
                                                   unsigned long long n_units,
                                                   unsigned long long* __restrict__ counter)
{
    constexpr int TERMS = poly_terms(W);
    constexpr int CELLS = W * W;
    constexpr int NOUT = C * CELLS;
    constexpr int RS = 65;  // row stride of the reduction buffer (no bank conflicts)
    __shared__ float red[NOUT * RS];
    const int lane = threadIdx.x;
    const double halfW = 0.5 * W;

    for (;;) {
        unsigned long long u = 0;
        if (lane == 0) u = atomicAdd(counter, 1ull);
        u = lane0(u);
        if (u >= n_units) break;
        int g = 0;
        while (g + 1 < n_groups && (long long)u >= groups[g + 1].unit_begin) ++g;
        const GroupDev& D = groups[g];
        const long long local = (long long)u - D.unit_begin;
        int item, c0;
        unit_of(D, local, C, item, c0);
        const int nc = min(C, D.n_cells - c0);
        const int bin = D.item_bin[item];
        const long long first = D.item_begin[item];
        const int n = D.item_count[item];
        const int t0x = bin / D.nb - D.off;
        const int t0y = bin % D.nb - D.off;

        float acc[C][CELLS];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int e = 0; e < CELLS; ++e) acc[c][e] = 0.f;

        for (int i = lane; i < n; i += 64) {
            const unsigned long long id = D.ids[first + i];
            int s;
            const PairNodes<2> nd = unpack_id<2>(id, s);
            float q;
            double xs[2];
            point_geometry<float, 2>(D.gp, s, nd, halfW, q, xs);
            float kx[W], ky[W];
            kernel_cells64<float, W, TERMS>(D.gp.poly64, 2.0 * ((double)t0x - xs[0]) - 1.0, kx);
            kernel_cells64<float, W, TERMS>(D.gp.poly64, 2.0 * ((double)t0y - xs[1]) - 1.0, ky);
            int ix[2], iy[2];
            q *= orbit_terms<float, 2>(D.gp, nd, ix, iy);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float w = 0.f;
                if (c < nc) {
                    const float* Gc = D.Gg + (int64_t)(c0 + c) * D.nid;
                    w = q * fmaf(Gc[ix[0]], Gc[iy[0]], Gc[ix[1]] * Gc[iy[1]]);
                }
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const float t = w * kx[a];
#pragma unroll
                    for (int b = 0; b < W; ++b) acc[c][a * W + b] = fmaf(t, ky[b], acc[c][a * W + b]);
                }
            }
        }

        // sum the 64 private tiles (FP64) and flush one atomic per footprint cell
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int e = 0; e < CELLS; ++e) red[(c * CELLS + e) * RS + lane] = acc[c][e];
        __syncthreads();
        for (int o = lane; o < nc * CELLS; o += 64) {
            const float* r = red + o * RS;
            double v = 0.0;
            for (int l = 0; l < 64; ++l) v += (double)r[l];
            if (v != 0.0) {
                const int c = o / CELLS, e = o % CELLS;
                double* grid = D.grid + (int64_t)(c0 + c) * D.ngd;
                const int64_t cell = (int64_t)fold_index(t0x + e / W, D.gp.nh) * D.gp.ng +
                                     fold_index(t0y + e % W, D.gp.nh);
                __hip_atomic_fetch_add(grid + cell, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

// Lane-per-cell scheme: CW cells per wave, NS = 64 / CW point streams.  Lane
// l serves cell c = C0 + l % CW and the staged points j = l / CW (mod NS).
// The geometry of each 64-point batch is generated once (lane = point) and
// read from LDS by every cell; a batch is summed in registers and the batch
// sums in LDS (FP32, at most 64 and 128 terms; the running tile stays out of
// the registers that point regeneration needs), the streams and the grid in FP64.
template <int W, int CW>
__global__ void __launch_bounds__(64) gain_batched_lanes(const GroupDev* __restrict__ groups, int n_groups,
                                                         unsigned long long n_units,
                                                         unsigned long long* __restrict__ counter)
{
    constexpr int TERMS = poly_terms(W);
    constexpr int CELLS = W * W;
    constexpr int NS = 64 / CW;
    constexpr int PB = 8;  // points whose G rows are gathered together
    // the staged points of a batch, with PAD zero-weight entries past the last
    // lane, so a gather of PB points past the batch's end reads weight 0
    // (offsets 0: row 0 of G) and needs no clamp per point
    constexpr int PAD = PB * NS;
    __shared__ float sq[64 + PAD];
    __shared__ float sk[64 + PAD][2 * W];
    __shared__ unsigned int sx[64 + PAD][4];  // byte offsets of the four G rows of each point
    __shared__ double red[(NS > 1) ? (NS - 1) * CW * CELLS : 1];
    // the kernel cells depend on W and the upsampling only, the same for every
    // group: read from LDS they are not hoisted into registers
    constexpr int EO = ((TERMS + 1) / 2) * ((W + 1) / 2) + (TERMS / 2) * (W / 2);
    __shared__ double seo[EO];
    __shared__ float sacc[CELLS * 64];  // running tile of every lane, lane fastest
    const int lane = threadIdx.x;
    // one stream (CW = 64): the point index is the same for every lane, and the
    // compiler knows it
    const int cl = lane % CW, stream = (NS == 1) ? 0 : lane / CW;
    for (int i = lane; i < EO; i += 64) seo[i] = groups[0].gp.kpoly_eo[i];
    for (int i = 64 + lane; i < 64 + PAD; i += 64) {
        sq[i] = 0.f;
        for (int m = 0; m < 4; ++m) sx[i][m] = 0u;
        for (int a = 0; a < 2 * W; ++a) sk[i][a] = 0.f;
    }
    __syncthreads();

    for (;;) {
        unsigned long long u = 0;
        if (lane == 0) u = atomicAdd(counter, 1ull);
        u = lane0(u);
        if (u >= n_units) break;
        int g = 0;
        while (g + 1 < n_groups && (long long)u >= groups[g + 1].unit_begin) ++g;
        const GroupDev& D = groups[g];
        const long long local = (long long)u - D.unit_begin;
        int item, c0;
        unit_of(D, local, CW, item, c0);
        const int c = c0 + cl;
        const bool valid = c < D.n_cells;
        // the unit is the same for the whole wave: keep its run in scalar registers
        item = __builtin_amdgcn_readfirstlane(item);
        const int bin = __builtin_amdgcn_readfirstlane(D.item_bin[item]);
        const long long first = lane0((unsigned long long)D.item_begin[item]);
        const int n = __builtin_amdgcn_readfirstlane(D.item_count[item]);
        const int t0x = bin / D.nb - D.off;
        const int t0y = bin % D.nb - D.off;
        // the cell-minor G copy is device memory: global loads, not flat ones
        // (which would also count against the LDS wait counter)
        const __attribute__((address_space(1))) float* Gt =
            (const __attribute__((address_space(1))) float*)D.Gt;
        const int ldg = D.ldg;

#pragma unroll
        for (int e = 0; e < CELLS; ++e) sacc[e * 64 + lane] = 0.f;

        for (int base = 0; base < n; base += 64) {
            const int nv = min(64, n - base);
            if (lane < nv) {
                // the regeneration of gain_binned: w per dimension, the offset
                // from the cell fit, the mirrored kernel cells
                const unsigned long long id = D.ids[first + base + lane];
                int s;
                const PairNodes<2> nd = unpack_id<2>(id, s);
                float q, vp[2];
                point_velocity<float, 2>(D.gp, s, nd, q, vp);
                double sv[2];
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    float m2;
                    const double w = map_w(vp[l], D.gp, m2);
                    q *= m2;
                    sv[l] = cell_offset(D.gp.cellfit + (int64_t)((l == 0 ? t0x : t0y) + D.off) * kCellFitStride, w);
                }
                float k[2][W];
                kernel_cells_eo_dims<float, W, TERMS, 2>(seo, sv, k);
                int ix[2], iy[2];
                sq[lane] = q * orbit_terms<float, 2>(D.gp, nd, ix, iy);
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    sk[lane][a] = k[0][a];
                    sk[lane][W + a] = k[1][a];
                }
                sx[lane][0] = (unsigned)(ix[0] * ldg) * 4u;
                sx[lane][1] = (unsigned)(iy[0] * ldg) * 4u;
                sx[lane][2] = (unsigned)(ix[1] * ldg) * 4u;
                sx[lane][3] = (unsigned)(iy[1] * ldg) * 4u;
            } else {
                sq[lane] = 0.f;
                for (int m = 0; m < 4; ++m) sx[lane][m] = 0u;
                for (int a = 0; a < 2 * W; ++a) sk[lane][a] = 0.f;
            }
            __syncthreads();
            if (valid) {
                float ab[CELLS];
#pragma unroll
                for (int e = 0; e < CELLS; ++e) ab[e] = 0.f;
                // The G rows of PB points are gathered together (4 PB loads in
                // flight) before their arithmetic, so the memory latency is
                // paid once per PB points.  Points past the batch are the
                // zero-weight entries.
                // 32-bit byte offsets from the uniform base: the loads take the
                // scalar-base form, with no 64-bit address arithmetic per load
                const unsigned c4 = (unsigned)c * 4u;
                const __attribute__((address_space(1))) char* Gb =
                    (const __attribute__((address_space(1))) char*)Gt;
                for (int j0 = stream; j0 < nv; j0 += PB * NS) {
                    float gv[PB][4];
#pragma unroll
                    for (int k = 0; k < PB; ++k) {
                        const int j = j0 + k * NS;
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            gv[k][m] = *(const __attribute__((address_space(1))) float*)(Gb + (sx[j][m] + c4));
                    }
#pragma unroll
                    for (int k = 0; k < PB; ++k) {
                        const int j = j0 + k * NS;
                        const float w = sq[j] * fmaf(gv[k][0], gv[k][1], gv[k][2] * gv[k][3]);
#pragma unroll
                        for (int a = 0; a < W; ++a) {
                            const float t = w * sk[j][a];
#pragma unroll
                            for (int b = 0; b < W; ++b) ab[a * W + b] = fmaf(t, sk[j][W + b], ab[a * W + b]);
                        }
                    }
                }
#pragma unroll
                for (int e = 0; e < CELLS; ++e) sacc[e * 64 + lane] += ab[e];
            }
            __syncthreads();
        }

        if constexpr (NS > 1) {
            if (stream > 0) {
#pragma unroll
                for (int e = 0; e < CELLS; ++e) red[((stream - 1) * CW + cl) * CELLS + e] = (double)sacc[e * 64 + lane];
            }
            __syncthreads();
        }
        if (stream == 0 && valid) {
            double* grid = D.grid + (int64_t)c * D.ngd;
            for (int e = 0; e < CELLS; ++e) {
                double v = (double)sacc[e * 64 + lane];
                for (int r = 1; r < NS; ++r) v += red[((r - 1) * CW + cl) * CELLS + e];
                if (v != 0.0) {
                    const int64_t cell = (int64_t)fold_index(t0x + e / W, D.gp.nh) * D.gp.ng +
                                         fold_index(t0y + e % W, D.gp.nh);
                    __hip_atomic_fetch_add(grid + cell, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        if constexpr (NS > 1) __syncthreads();
    }
}

// Gt[node][c] = Gg[c][node] for the cell-minor copy read by the lane-per-cell scheme
__global__ void transpose_g(const float* __restrict__ Gg, float* __restrict__ Gt, int n_cells, int64_t nid,
                            int ldg)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nid * ldg) return;
    const int c = (int)(e % ldg);
    const int64_t node = e / ldg;
    Gt[e] = c < n_cells ? Gg[(int64_t)c * nid + node] : 0.f;
}

__global__ void reset_counter(unsigned long long* __restrict__ counter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0ull;
}

__global__ void fill_zero64(double* __restrict__ x, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

__global__ void fill_one32(float* __restrict__ x, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = 1.f;
}

// cin[c][k] = packed[offsets[cells[c]] + k] (widened to FP64)
__global__ void batch_gather(const float* __restrict__ packed, const int64_t* __restrict__ offsets,
                             const int* __restrict__ cells, int64_t Nd, int64_t n_total,
                             double* __restrict__ cin)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const int64_t c = i / Nd;
    cin[i] = (double)packed[offsets[cells[c]] + (i - c * Nd)];
}

// packed_q[offsets[cells[c]] + k] = Q+ - Q- (FP64, rounded once)
__global__ void batch_scatter(const double* __restrict__ qp, const double* __restrict__ qm,
                              const int64_t* __restrict__ offsets, const int* __restrict__ cells,
                              int64_t Nd, int64_t n_total, float* __restrict__ packed_q)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const int64_t c = i / Nd;
    packed_q[offsets[cells[c]] + (i - c * Nd)] = (float)(qp[i] - qm[i]);
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// the cells-per-wave values the gain kernels are built for, by kernel width:
// C = 1, 2, 4, 8 register tiles (C W^2 <= 200), C = 16, 32, 64 lane per cell
bool tile_supported(int W, int C)
{
    if (W < 4 || W > 8) return false;
    if (C == 16 || C == 32 || C == 64) return true;
    if (C != 1 && C != 2 && C != 4 && C != 8) return false;
    return C * W * W <= 200;
}

template <int W, int C>
hipError_t gain_launch_wc(const GroupDev* groups, int n_groups, unsigned long long n_units,
                          unsigned long long* counter, int waves, hipStream_t s)
{
    if constexpr (C * W * W <= 200) {
        hipLaunchKernelGGL((gain_batched<W, C>), dim3(waves), dim3(64), 0, s, groups, n_groups, n_units,
                           counter);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <int W, int CW>
hipError_t lanes_launch(const GroupDev* groups, int n_groups, unsigned long long n_units,
                        unsigned long long* counter, int waves, hipStream_t s)
{
    hipLaunchKernelGGL((gain_batched_lanes<W, CW>), dim3(waves), dim3(64), 0, s, groups, n_groups, n_units,
                       counter);
    return hipGetLastError();
}

template <int W>
hipError_t gain_launch_w(int C, const GroupDev* groups, int n_groups, unsigned long long n_units,
                         unsigned long long* counter, int waves, hipStream_t s)
{
    switch (C) {
    case 16: return lanes_launch<W, 16>(groups, n_groups, n_units, counter, waves, s);
    case 32: return lanes_launch<W, 32>(groups, n_groups, n_units, counter, waves, s);
    case 64: return lanes_launch<W, 64>(groups, n_groups, n_units, counter, waves, s);
    case 1: return gain_launch_wc<W, 1>(groups, n_groups, n_units, counter, waves, s);
    case 2: return gain_launch_wc<W, 2>(groups, n_groups, n_units, counter, waves, s);
    case 4: return gain_launch_wc<W, 4>(groups, n_groups, n_units, counter, waves, s);
    case 8: return gain_launch_wc<W, 8>(groups, n_groups, n_units, counter, waves, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gain_launch(int W, int C, const GroupDev* groups, int n_groups, unsigned long long n_units,
                       unsigned long long* counter, int waves, hipStream_t s)
{
    switch (W) {
    case 4: return gain_launch_w<4>(C, groups, n_groups, n_units, counter, waves, s);
    case 5: return gain_launch_w<5>(C, groups, n_groups, n_units, counter, waves, s);
    case 6: return gain_launch_w<6>(C, groups, n_groups, n_units, counter, waves, s);
    case 7: return gain_launch_w<7>(C, groups, n_groups, n_units, counter, waves, s);
    case 8: return gain_launch_w<8>(C, groups, n_groups, n_units, counter, waves, s);
    default: return hipErrorInvalidValue;
    }
}

// resident 64-lane workgroups of the gain kernel on the whole device
template <int W, int C>
int resident_waves_wc()
{
    if constexpr (C * W * W <= 200) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gain_batched<W, C>, 64, 0) != hipSuccess)
            return 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        return std::max(1, per_cu) * std::max(1, cus);
    } else {
        return 0;
    }
}

template <int W, int CW>
int resident_waves_lanes()
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gain_batched_lanes<W, CW>, 64, 0) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return std::max(1, per_cu) * std::max(1, cus);
}

template <int W>
int resident_waves_w(int C)
{
    switch (C) {
    case 16: return resident_waves_lanes<W, 16>();
    case 32: return resident_waves_lanes<W, 32>();
    case 64: return resident_waves_lanes<W, 64>();
    case 1: return resident_waves_wc<W, 1>();
    case 2: return resident_waves_wc<W, 2>();
    case 4: return resident_waves_wc<W, 4>();
    case 8: return resident_waves_wc<W, 8>();
    default: return 0;
    }
}

int resident_waves(int W, int C)
{
    switch (W) {
    case 4: return resident_waves_w<4>(C);
    case 5: return resident_waves_w<5>(C);
    case 6: return resident_waves_w<6>(C);
    case 7: return resident_waves_w<7>(C);
    case 8: return resident_waves_w<8>(C);
    default: return 0;
    }
}

GainParams<float> group_gain_params(const Plan& p)
{
    GainParams<float> gp;
    std::memset(&gp, 0, sizeof(gp));
    gp.v1 = static_cast<const float*>(p.dt.v1);
    gp.pair_a = p.dt.pair_a;
    gp.pair_b = p.dt.pair_b;
    gp.pair_base = p.dt.pair_base;
    gp.sigma = static_cast<const float*>(p.dt.sigma);
    gp.wfac = static_cast<const float*>(p.dt.wfac);
    gp.poly = static_cast<const float*>(p.dt.poly);
    gp.S = (float)p.S;
    gp.inv_S = (float)(1.0 / p.S);
    gp.inv_S64 = 1.0 / p.S;
    gp.h_inv = (float)(1.0 / p.h);
    gp.h_inv64 = 1.0 / p.h;
    gp.poly64 = p.dt.poly64;
    gp.kpoly_eo = p.dt.kpoly_eo;
    gp.cellfit = p.dt.cellfit;
    gp.cellfit_v = p.dt.cellfit_v;
    gp.b0 = (float)p.b0;
    gp.gamma = (float)p.gamma;
    gp.map = p.map;
    gp.vhs = p.kernel == PGC_KERNEL_VHS;
    gp.ni = p.ni;
    gp.np = p.np;
    gp.ng = p.ng;
    gp.nh = p.nh;
    gp.n_sigma = p.n_sigma;
    gp.ngd = p.ngd;
    return gp;
}

}  // namespace
}  // namespace pgc

using pgc::Plan;

struct BatchGroup {
    pgc_plan plan = nullptr;  // the shared discretisation of every cell with this N
    int N = 0;
    std::vector<int> cells;   // batch indices of the group's cells
    int* cells_dev = nullptr;
    double* cin = nullptr;    // n_cells x N^d FP64 coefficients
    double* grid = nullptr;   // n_cells x n_g^d
    float* Gt = nullptr;      // n_i^d x ldg, cell-minor G (lane-per-cell scheme)
    int ldg = 0;
    int* order = nullptr;     // the plan's bin runs in raster order of their bins
    pgc::DenseBufs b;
};

struct pgc_batch_s {
    int n_cells = 0, W = 0;
    std::vector<int> cell_modes;
    std::vector<int64_t> offsets;  // dense packing, cell order
    int64_t total = 0;
    int64_t* offsets_dev = nullptr;
    std::vector<BatchGroup> groups;
    pgc::GroupDev* groups_dev = nullptr;
    unsigned long long* counter = nullptr;
    int C = 0, waves = 0;
    int spatial = 1;          // process bin runs in raster order (else longest first)
    double order_ms[2] = {0, 0};  // autotuner: best C in longest-first / raster order
    int group_major = 0;      // units cell-group major (else bin-run major)
    double major_ms[2] = {0, 0};  // autotuner: bin-run major / cell-group major at the chosen C and order
    unsigned long long n_units = 0;
    int64_t n_points = 0;
    double tuned_ms[7] = {0, 0, 0, 0, 0, 0, 0};  // C = 1, 2, 4, 8, 16, 32, 64
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> allocations;
    int64_t workspace_bytes = 0;
    bool deterministic = false;  // every cell through its group's deterministic plan
};

namespace {

hipError_t batch_alloc(pgc_batch_s& b, void** ptr, size_t bytes)
{
    *ptr = nullptr;
    b.allocations.push_back(nullptr);  // the slot first: a throwing push_back leaks no device memory
    hipError_t e = hipMalloc(&b.allocations.back(), std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
        b.allocations.pop_back();
        return e;
    }
    *ptr = b.allocations.back();
    b.workspace_bytes += (int64_t)bytes;
    return hipSuccess;
}

template <typename T>
hipError_t batch_alloc_n(pgc_batch_s& b, T** ptr, int64_t n)
{
    void* v = nullptr;
    hipError_t e = batch_alloc(b, &v, (size_t)n * sizeof(T));
    *ptr = static_cast<T*>(v);
    return e;
}

void batch_free(pgc_batch_s* b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void* p : b->allocations) (void)hipFree(p);
    for (BatchGroup& g : b->groups) (void)pgc_plan_destroy(g.plan);
    delete b;
}

void drop_graph(pgc_batch_s& b)
{
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
}

// lay out the work units for C cells per wave and upload the group table
hipError_t set_units(pgc_batch_s& b, int C, hipStream_t s)
{
    std::vector<pgc::GroupDev> gd;
    try {
        gd.resize(b.groups.size());
    } catch (...) {
        return hipErrorOutOfMemory;
    }
    unsigned long long begin = 0;
    for (size_t g = 0; g < b.groups.size(); ++g) {
        const BatchGroup& G = b.groups[g];
        const Plan& p = G.plan->p;
        pgc::GroupDev& d = gd[g];
        std::memset(&d, 0, sizeof(d));
        d.gp = pgc::group_gain_params(p);
        d.item_bin = p.bins.item_bin;
        d.item_begin = p.bins.item_begin;
        d.item_count = p.bins.item_count;
        d.ids = p.bins.ids;
        d.Gg = static_cast<const float*>(G.b.Gg);
        d.Gt = G.Gt;
        d.ldg = G.ldg;
        d.order = b.spatial ? G.order : nullptr;
        d.grid = G.grid;
        d.nb = p.bins.nb;
        d.off = p.bins.off;
        d.n_cells = (int)G.cells.size();
        d.ncg = (d.n_cells + C - 1) / C;
        d.group_major = b.group_major;
        d.n_items = p.bins.n_items;
        d.nid = p.nid;
        d.ngd = p.ngd;
        d.unit_begin = (int64_t)begin;
        begin += (unsigned long long)p.bins.n_items * (unsigned long long)d.ncg;
    }
    hipError_t e = hipMemcpyAsync(b.groups_dev, gd.data(), gd.size() * sizeof(pgc::GroupDev),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    b.C = C;
    b.n_units = begin;
    b.waves = pgc::resident_waves(b.W, C);
    return b.waves > 0 ? hipSuccess : hipErrorInvalidValue;
}

hipError_t enqueue_gain(const pgc_batch_s& b, hipStream_t s)
{
    for (const BatchGroup& G : b.groups) {
        const Plan& p = G.plan->p;
        const int64_t n = (int64_t)G.cells.size() * p.ngd;
        hipLaunchKernelGGL(pgc::fill_zero64, dim3(pgc::nblocks(n, 256)), dim3(256), 0, s, G.grid, n);
        if (b.C >= 16) {
            const int64_t nt = p.nid * G.ldg;
            hipLaunchKernelGGL(pgc::transpose_g, dim3(pgc::nblocks(nt, 256)), dim3(256), 0, s,
                               static_cast<const float*>(G.b.Gg), G.Gt, (int)G.cells.size(), p.nid, G.ldg);
        }
    }
    hipLaunchKernelGGL(pgc::reset_counter, dim3(1), dim3(64), 0, s, b.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return pgc::gain_launch(b.W, b.C, b.groups_dev, (int)b.groups.size(), b.n_units, b.counter, b.waves, s);
}

// every stage of one batched evaluation, stream-ordered, no allocation
hipError_t enqueue_all(const pgc_batch_s& b, const float* packed, const int64_t* offsets, float* packed_q,
                       hipStream_t s)
{
    hipError_t e;
    for (const BatchGroup& G : b.groups) {
        const Plan& p = G.plan->p;
        const int nb = (int)G.cells.size();
        const int64_t n = (int64_t)nb * p.Nd;
        hipLaunchKernelGGL(pgc::batch_gather, dim3(pgc::nblocks(n, 256)), dim3(256), 0, s, packed, offsets,
                           G.cells_dev, p.Nd, n, G.cin);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = pgc::launch_dense_synthesis(p, G.cin, nb, G.b, s)) != hipSuccess) return e;
        if ((e = pgc::launch_dense_loss(p, nb, G.b, s)) != hipSuccess) return e;
    }
    if ((e = enqueue_gain(b, s)) != hipSuccess) return e;
    for (const BatchGroup& G : b.groups) {
        const Plan& p = G.plan->p;
        const int nb = (int)G.cells.size();
        const int64_t n = (int64_t)nb * p.Nd;
        if ((e = pgc::launch_dense_grid_to_modes(p, G.grid, nb, G.b, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(pgc::batch_scatter, dim3(pgc::nblocks(n, 256)), dim3(256), 0, s, G.b.qplus,
                           G.b.qminus, offsets, G.cells_dev, p.Nd, n, packed_q);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Deterministic batches: every cell through its group's plan (created with
// deterministic = 1), whose gain adds footprint tiles in a fixed order and
// whose bins hold their ids sorted, so each cell's Q equals an unbatched
// evaluation by a plan of the same descriptor bit for bit.
pgc_status enqueue_cells(const pgc_batch_s& b, const float* packed, float* packed_q, hipStream_t s)
{
    for (const BatchGroup& G : b.groups)
        for (int c : G.cells) {
            const pgc_status st = pgc_coeffs_to_q(G.plan, packed + b.offsets[c], packed_q + b.offsets[c], nullptr, s);
            if (st != PGC_OK) return st;
        }
    return PGC_OK;
}

// the lane-per-cell scheme addresses the cell-minor G with 32-bit byte offsets
bool lanes_fit(const pgc_batch_s& b)
{
    for (const BatchGroup& G : b.groups)
        if (G.plan->p.nid * (int64_t)G.ldg * 4 >= 4294967295ll) return false;
    return true;
}

bool tile_ok(const pgc_batch_s& b, int C)
{
    return pgc::tile_supported(b.W, C) && (C < 16 || lanes_fit(b));
}

// time the gain for every supported C on G = 1 and keep the fastest
hipError_t autotune(pgc_batch_s& b, hipStream_t s)
{
    for (const BatchGroup& G : b.groups) {
        const int64_t n = (int64_t)G.cells.size() * G.plan->p.nid;
        hipLaunchKernelGGL(pgc::fill_one32, dim3(pgc::nblocks(n, 256)), dim3(256), 0, s,
                           static_cast<float*>(G.b.Gg), n);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipEvent_t t0, t1;
    if ((e = hipEventCreate(&t0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&t1)) != hipSuccess) {
        (void)hipEventDestroy(t0);
        return e;
    }
    // widest tiles first; a candidate more than 1.5x slower than the best so
    // far on its first run is not timed again (its first run stands)
    const int cands[7] = {1, 2, 4, 8, 16, 32, 64};
    int best = 0;
    double best_ms = 0.0;
    for (int k = 6; k >= 0 && e == hipSuccess; --k) {
        b.tuned_ms[k] = 0.0;
        if (!tile_ok(b, cands[k])) continue;
        if ((e = set_units(b, cands[k], s)) != hipSuccess) break;
        double ms_k = 0.0;
        for (int run = 0; run < 2 && e == hipSuccess; ++run) {
            if ((e = hipEventRecord(t0, s)) != hipSuccess) break;
            if ((e = enqueue_gain(b, s)) != hipSuccess) break;
            if ((e = hipEventRecord(t1, s)) != hipSuccess) break;
            if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
            ms_k = run == 0 ? ms : std::min(ms_k, (double)ms);
            if (run == 0 && best != 0 && ms > 1.5 * best_ms) break;
        }
        if (e != hipSuccess) break;
        b.tuned_ms[k] = ms_k;
        if (best == 0 || ms_k < best_ms) {
            best = cands[k];
            best_ms = ms_k;
        }
    }
    if (e == hipSuccess && best != 0) {
        // the other processing order at the best C
        const int keep = b.spatial;
        b.order_ms[keep] = best_ms;
        b.spatial = 1 - keep;
        float ms = 0.f;
        if ((e = set_units(b, best, s)) == hipSuccess && (e = enqueue_gain(b, s)) == hipSuccess &&
            (e = hipEventRecord(t0, s)) == hipSuccess && (e = enqueue_gain(b, s)) == hipSuccess &&
            (e = hipEventRecord(t1, s)) == hipSuccess && (e = hipEventSynchronize(t1)) == hipSuccess &&
            (e = hipEventElapsedTime(&ms, t0, t1)) == hipSuccess) {
            // switch only for a clear gain: the orders are often within noise
            b.order_ms[b.spatial] = ms;
            if (!(ms < 0.97 * best_ms)) b.spatial = keep;
            else best_ms = ms;
        }
    }
    if (e == hipSuccess && best != 0) {
        // the other unit order at the best C and bin-run order
        const int keep = b.group_major;
        b.major_ms[keep] = best_ms;
        b.group_major = 1 - keep;
        float ms = 0.f;
        if ((e = set_units(b, best, s)) == hipSuccess && (e = enqueue_gain(b, s)) == hipSuccess &&
            (e = hipEventRecord(t0, s)) == hipSuccess && (e = enqueue_gain(b, s)) == hipSuccess &&
            (e = hipEventRecord(t1, s)) == hipSuccess && (e = hipEventSynchronize(t1)) == hipSuccess &&
            (e = hipEventElapsedTime(&ms, t0, t1)) == hipSuccess) {
            b.major_ms[b.group_major] = ms;
            if (!(ms < 0.97 * best_ms)) b.group_major = keep;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return e;
    if (best == 0) return hipErrorInvalidValue;
    return set_units(b, best, s);
}

}  // namespace

extern "C" {

pgc_status pgc_batch_create(const pgc_plan_desc* base, int32_t n_cells, const int32_t* n_modes_host,
                            int32_t autotune_on, void* stream, pgc_batch* out)
{
    if (!base || !n_modes_host || !out || n_cells <= 0) return PGC_ERR_INVALID_ARG;
    *out = nullptr;
    if (base->dim != 2 || base->precision != PGC_PRECISION_FP32 || base->kernel == PGC_KERNEL_ANISO)
        return PGC_ERR_UNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    pgc_batch_s* b = nullptr;
    try {
        b = new pgc_batch_s();
        b->n_cells = n_cells;
        b->deterministic = base->deterministic == 1;
        b->cell_modes.assign(n_modes_host, n_modes_host + n_cells);
        std::map<int, std::vector<int>, std::greater<int>> by_n;  // largest N first
        for (int c = 0; c < n_cells; ++c) {
            const int N = n_modes_host[c];
            if (N < 3 || N > 255) {
                delete b;
                return PGC_ERR_INVALID_ARG;
            }
            by_n[N].push_back(c);
            b->offsets.push_back(b->total);
            b->total += (int64_t)N * N;
        }
        if (by_n.size() > (size_t)pgc::kMaxGroups) {
            delete b;
            return PGC_ERR_UNSUPPORTED;
        }
        for (auto& kv : by_n) {
            BatchGroup g;
            g.N = kv.first;
            g.cells = kv.second;
            b->groups.push_back(g);
        }
    } catch (const std::bad_alloc&) {
        delete b;
        return PGC_ERR_OUT_OF_MEMORY;
    }

    pgc_status st = PGC_OK;
    hipError_t e = hipSuccess;
    try {  // host containers below throw only on allocation failure
        for (BatchGroup& g : b->groups) {
            pgc_plan_desc d = *base;
            d.n_modes = g.N;
            d.m_v = 0;
            d.gain_mode = pgc::kGainBinned;
            d.index_bytes = 0;
            st = pgc_plan_create(&d, stream, &g.plan);
            if (st != PGC_OK) break;
            const Plan& p = g.plan->p;
            if (b->W == 0) b->W = p.W;
            // the lane kernel walks every cell group over the whole point index
            if (p.W != b->W || !pgc::tile_supported(p.W, 1) || p.gain_mode != pgc::kGainBinned ||
                p.bins.n_chunks != 1) {
                st = PGC_ERR_UNSUPPORTED;
                break;
            }
            b->n_points += p.n_points * (int64_t)g.cells.size();
            const int64_t nb = (int64_t)g.cells.size();
            const int64_t L = std::max<int64_t>(std::max(p.N, p.ni), p.ng);
            const int64_t t = L * L;
            if ((e = batch_alloc_n(*b, &g.cells_dev, nb)) != hipSuccess) break;
            if ((e = batch_alloc_n(*b, &g.cin, nb * p.Nd)) != hipSuccess) break;
            if ((e = batch_alloc_n(*b, &g.b.P, nb * p.nid)) != hipSuccess) break;
            if ((e = batch_alloc_n(*b, &g.b.G, nb * p.nid)) != hipSuccess) break;
            float* gg = nullptr;
            if ((e = batch_alloc_n(*b, &gg, nb * p.nid)) != hipSuccess) break;
            g.b.Gg = gg;
            if ((e = batch_alloc_n(*b, &g.b.H, nb * p.nid)) != hipSuccess) break;
            if ((e = batch_alloc_n(*b, &g.b.qminus, nb * p.Nd)) != hipSuccess) break;
            if ((e = batch_alloc_n(*b, &g.b.qplus, nb * p.Nd)) != hipSuccess) break;
            if ((e = batch_alloc_n(*b, &g.b.tmpA, nb * t)) != hipSuccess) break;
            if ((e = batch_alloc_n(*b, &g.b.tmpB, nb * t)) != hipSuccess) break;
            if ((e = batch_alloc_n(*b, &g.b.red, nb)) != hipSuccess) break;
            if ((e = batch_alloc_n(*b, &g.grid, nb * p.ngd)) != hipSuccess) break;
            g.ldg = (int)((nb + 63) / 64 * 64);
            if ((e = batch_alloc_n(*b, &g.Gt, p.nid * g.ldg)) != hipSuccess) break;
            {
                // raster order of the bins: consecutive runs flush into overlapping grid lines
                std::vector<int> bins((size_t)p.bins.n_items), ord((size_t)p.bins.n_items);
                if (p.bins.n_items > 0 &&
                    (e = hipMemcpy(bins.data(), p.bins.item_bin, bins.size() * sizeof(int), hipMemcpyDeviceToHost)) !=
                        hipSuccess)
                    break;
                for (size_t k = 0; k < ord.size(); ++k) ord[k] = (int)k;
                std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return bins[x] < bins[y]; });
                if ((e = batch_alloc_n(*b, &g.order, std::max<int64_t>(1, p.bins.n_items))) != hipSuccess) break;
                if (!ord.empty() &&
                    (e = hipMemcpy(g.order, ord.data(), ord.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
                    break;
            }
            if ((e = hipMemcpyAsync(g.cells_dev, g.cells.data(), nb * sizeof(int), hipMemcpyHostToDevice, s)) !=
                hipSuccess)
                break;
        }
        if (st == PGC_OK && e == hipSuccess) {
            if ((e = batch_alloc_n(*b, &b->offsets_dev, b->n_cells)) == hipSuccess &&
                (e = hipMemcpyAsync(b->offsets_dev, b->offsets.data(), b->n_cells * sizeof(int64_t),
                                    hipMemcpyHostToDevice, s)) == hipSuccess &&
                (e = batch_alloc_n(*b, &b->groups_dev, (int64_t)b->groups.size())) == hipSuccess &&
                (e = batch_alloc_n(*b, &b->counter, 1)) == hipSuccess) {
                // a deterministic batch never runs the batched gain: nothing to tune
                e = autotune_on && !b->deterministic ? autotune(*b, s) : set_units(*b, 1, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
            }
        }
    } catch (...) {
        st = PGC_ERR_OUT_OF_MEMORY;
    }
    if (st == PGC_OK && e != hipSuccess) st = pgc::status_of(e);
    if (st != PGC_OK) {
        batch_free(b);
        return st;
    }
    *out = b;
    return PGC_OK;
}

pgc_status pgc_batch_destroy(pgc_batch batch)
{
    batch_free(batch);
    return PGC_OK;
}

pgc_status pgc_batch_query(pgc_batch b, pgc_batch_info* info)
{
    if (!b || !info) return PGC_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    info->n_cells = b->n_cells;
    info->n_groups = (int32_t)b->groups.size();
    for (size_t g = 0; g < b->groups.size(); ++g) {
        info->group_n_modes[g] = b->groups[g].N;
        info->group_cells[g] = (int32_t)b->groups[g].cells.size();
    }
    info->coeffs_total = b->total;
    info->kernel_width = b->W;
    info->cells_per_wave = b->C;
    info->waves = b->waves;
    info->n_units = (int64_t)b->n_units;
    info->n_points = b->n_points;
    info->workspace_bytes = b->workspace_bytes;
    for (const BatchGroup& g : b->groups) info->workspace_bytes += g.plan->p.workspace_bytes;
    for (int k = 0; k < 7; ++k) info->tuned_ms[k] = b->tuned_ms[k];
    info->scheme = b->C >= 16 ? 1 : 0;
    info->spatial_order = b->spatial;
    info->order_ms[0] = b->order_ms[0];
    info->order_ms[1] = b->order_ms[1];
    info->group_major = b->group_major;
    info->major_ms[0] = b->major_ms[0];
    info->major_ms[1] = b->major_ms[1];
    info->has_graph = b->exec != nullptr;
    info->deterministic = b->deterministic ? 1 : 0;
    return PGC_OK;
}

pgc_status pgc_batch_offsets(pgc_batch b, int64_t* offsets_host)
{
    if (!b || !offsets_host) return PGC_ERR_INVALID_ARG;
    std::copy(b->offsets.begin(), b->offsets.end(), offsets_host);
    return PGC_OK;
}

pgc_status pgc_batch_set_tile(pgc_batch b, int32_t cells_per_wave, void* stream)
{
    if (!b) return PGC_ERR_INVALID_ARG;
    if (!tile_ok(*b, cells_per_wave)) return PGC_ERR_UNSUPPORTED;
    drop_graph(*b);
    return pgc::status_of(set_units(*b, cells_per_wave, static_cast<hipStream_t>(stream)));
}

pgc_status pgc_batch_set_order(pgc_batch b, int32_t raster, int32_t group_major, void* stream)
{
    if (!b || (raster != 0 && raster != 1) || (group_major != 0 && group_major != 1)) return PGC_ERR_INVALID_ARG;
    drop_graph(*b);
    b->spatial = raster;
    b->group_major = group_major;
    return pgc::status_of(set_units(*b, b->C, static_cast<hipStream_t>(stream)));
}

pgc_status pgc_batch_autotune(pgc_batch b, void* stream)
{
    if (!b) return PGC_ERR_INVALID_ARG;
    drop_graph(*b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = autotune(*b, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return pgc::status_of(e);
}

pgc_status pgc_batch_coeffs_to_q(pgc_batch b, const void* packed_coeffs_dev, const int64_t* offsets_dev,
                                 void* packed_q_dev, void* stream)
{
    if (!b || !packed_coeffs_dev || !packed_q_dev) return PGC_ERR_INVALID_ARG;
    if (b->deterministic) {
        if (offsets_dev) return PGC_ERR_UNSUPPORTED;  // the cells are enqueued from host offsets
        return enqueue_cells(*b, static_cast<const float*>(packed_coeffs_dev), static_cast<float*>(packed_q_dev),
                             static_cast<hipStream_t>(stream));
    }
    const int64_t* off = offsets_dev ? offsets_dev : b->offsets_dev;
    return pgc::status_of(enqueue_all(*b, static_cast<const float*>(packed_coeffs_dev), off,
                                      static_cast<float*>(packed_q_dev), static_cast<hipStream_t>(stream)));
}

pgc_status pgc_batch_capture(pgc_batch b, const void* packed_coeffs_dev, const int64_t* offsets_dev,
                             void* packed_q_dev, void* stream)
{
    if (!b || !packed_coeffs_dev || !packed_q_dev) return PGC_ERR_INVALID_ARG;
    if (b->deterministic) return PGC_ERR_UNSUPPORTED;
    const int64_t* off = offsets_dev ? offsets_dev : b->offsets_dev;
    drop_graph(*b);
    hipStream_t user = static_cast<hipStream_t>(stream);
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamSynchronize(user);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return pgc::status_of(e);
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t ee = enqueue_all(*b, static_cast<const float*>(packed_coeffs_dev), off,
                                    static_cast<float*>(packed_q_dev), cs);
        e = hipStreamEndCapture(cs, &b->graph);
        if (ee != hipSuccess) e = ee;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        drop_graph(*b);
        return pgc::status_of(e);
    }
    return PGC_OK;
}

pgc_status pgc_batch_graph_launch(pgc_batch b, void* stream)
{
    if (!b || !b->exec) return PGC_ERR_INVALID_ARG;
    return pgc::status_of(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
