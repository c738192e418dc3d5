// Internal declarations shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "pgc.h"

namespace pgc {

constexpr int kMaxWidth = 16;         // largest spreading kernel width W

// Horner terms of the kernel polynomial of one cell (degree + 1).  Beyond
// W + 1 terms the interpolation error of the cells stops falling (it is set by
// the kernel's value at the edge of its support, exp(-beta)); narrow kernels
// keep one more term.
constexpr int poly_terms(int w) { return w >= 10 ? w + 1 : w + 2; }
constexpr int kMaxPolyTerms = 18;     // Horner terms per kernel cell (degree + 1)
// Degree of the per-cell polynomial that gives the kernel offset from w: a
// Chebyshev interpolant of degree 12 over one grid cell is within 5e-16 of the
// exact offset on every grid with at least 8 cells per half period.
constexpr int kCellFitDeg = 12;
constexpr int kCellFitStride = kCellFitDeg + 3;  // w_c, 1/delta, c_0 .. c_12
// t_c, 1/delta (0: no fit), offset c_0 .. c_12, map factor c_0 .. c_12
constexpr int kCellFitVStride = 2 * kCellFitDeg + 4;
// FP32 plans fit the offset and map factor in v/S to degree 7 (within 2e-10,
// far below the FP32 rounding of the kernel values), in the same slots
constexpr int kCellFitDegV32 = 7;
constexpr int kMaxLdsBytes = 160 * 1024;
constexpr int kLdsBudget = 155 * 1024;  // slab bytes per workgroup

// Device tables.  The dense transforms (synthesis, loss, grid -> modes,
// projection) run in FP64 for both plan precisions, so their tables are FP64;
// the tables read by point generation and spreading are in the plan precision
// (T = float or double).
struct DeviceTables {
    void* v1 = nullptr;       // n_i      interior node velocities (plan precision)
    double* v1d = nullptr;    // n_i      the same in FP64 (aliases v1 for FP64 plans)
    double* w1 = nullptr;     // n_i      CGL weights
    double* mu21 = nullptr;   // n_i      mu(xi)^2
    double* C = nullptr;      // n_i x N  T_k(xi_i)/sqrt(c_k)
    double* CT = nullptr;     // N x n_i  transpose of C
    double* E = nullptr;      // N x n_g  cos(k m h) h / (psi^(k) sqrt(c_k))
    void* poly = nullptr;     // terms x W Horner coefficients of the kernel cells
    double* poly64 = nullptr; // the same in FP64 (aliases poly for FP64 plans)
    double* kpoly_eo = nullptr;  // even/odd parts of the cells a < W/2 (FP64)
    double* cellfit = nullptr;   // (n_h + 2) x (deg + 3) kernel-offset fits per grid cell (FP64)
    double* cellfit_v = nullptr; // (n_h + 2) x (2 deg + 4) offset and map-factor fits in v/S (FP64)
    double* bin_vthr = nullptr;  // n_h + 4 velocity thresholds of the footprint corners (FP64)
    void* sigma = nullptr;    // n_sigma x dim
    void* wfac = nullptr;     // n_sigma  W_s b0 S^d (direction weight, kernel constant, map scale)
    void* slab_vlo = nullptr; // n_slabs  v'_1 window of each slab
    void* slab_vhi = nullptr; // n_slabs
    int* pair_a = nullptr;    // np  unordered node pairs (a <= b) per dimension
    int* pair_b = nullptr;    // np
    int* pair_base = nullptr; // n_i  index of the pair (a, a)
};

constexpr int kGainSlab = 1;    // LDS slabs, per-point atomics
constexpr int kGainBinned = 2;  // plan-time bins by base cell, register accumulation

// Merged points sorted by the base cell of their footprint (built at plan time).
struct BinIndex {
    int nb = 0;                 // bins per dimension
    int off = 0;                // bin index = t0 + off
    int64_t n_items = 0;        // work items (runs of at most kBinChunk ids of one bin)
    int* item_bin = nullptr;
    long long* item_begin = nullptr;
    int* item_count = nullptr;
    unsigned long long* ids = nullptr;  // n_points packed point ids, grouped by bin
    // deterministic plans: the runs of every bin in run order (CSR), and one
    // W^d footprint tile per run
    int* bin_ptr = nullptr;     // nbins + 1
    int* bin_items = nullptr;   // n_items
    double* tiles = nullptr;    // n_items x W^d
    int64_t tile_bytes = 0;
    // streamed index: direction chunks [chunk_s0[c], chunk_s0[c + 1]) whose ids
    // are sorted into `ids` again at every evaluation; the chunk's runs are the
    // items [chunk_item0[c], chunk_item0[c + 1]) (begin relative to the chunk)
    int n_chunks = 1;
    int dirs_per_chunk = 0;      // 0: the whole index
    std::vector<int> chunk_s0;
    std::vector<int64_t> chunk_item0;
    unsigned int* chunk_begin = nullptr;  // n_chunks x nbins  first slot of every bin in its chunk
    unsigned int* cursor = nullptr;       // nbins  scatter cursors of the chunk being sorted
    int64_t nbins = 0;
    int64_t id_bytes = 0;        // bytes of `ids`
};
constexpr int kBinChunk = 8192;
constexpr int kMaxBinnedNodes = 256;        // n_i: 8-bit node fields of a point id
constexpr int kMaxBinnedDirections = 1024;  // n_sigma: 10-bit direction field

// Buffers marked FP64 are FP64 for both plan precisions.
struct Workspace {
    double* cin = nullptr;    // N^d    FP64 copy of FP32 input coefficients
    double* P = nullptr;      // n_i^d  polynomial part at the interior nodes (FP64)
    double* G = nullptr;      // n_i^d  w_i g_i = w_i mu_i^2 P_i (FP64)
    void* Gg = nullptr;       // n_i^d  G in the plan precision, read by the gain (aliases G for FP64)
    void* sym = nullptr;      // np^d   orbit sums of G_i G_j over exchanged node pairs
    double* H = nullptr;      // n_i^d  w_i A_i P_i (loss integrand) / projection input (FP64)
    void* partial = nullptr;  // n_chunks x n_g^d  per-chunk fine grids (FP64 cells)
    double* grid = nullptr;   // n_g^d  reduced fine grid of the slab scheme (FP64)
    double* tmpA = nullptr;   // separable-transform ping-pong buffers (FP64)
    double* tmpB = nullptr;
    double* qminus = nullptr; // N^d (FP64)
    double* qplus = nullptr;  // N^d (FP64)
    void* rk_y = nullptr;     // N^d  stage input (plan precision)
    void* rk_k[4] = {nullptr, nullptr, nullptr, nullptr};
    double* red = nullptr;    // small FP64 scratch (reductions)
    double* grid64 = nullptr; // n_g^d FP64 grid of the binned gain
    double* mom = nullptr;    // 3 x N  moment functionals m_0, m_1, m_2 (FP64)
};

constexpr int kStages = 6;     // synthesis, loss, orbit sums, spreading, grid->modes, combine
constexpr int kProfRing = 32;  // event sets recorded before the oldest must be read back

struct Profiler {
    hipEvent_t ev[kProfRing][kStages + 1];
    int used = 0;          // recorded sets not yet read back
    int head = 0;          // next set to record
    double ms[kStages] = {0, 0, 0, 0, 0, 0};
    int64_t calls = 0;
};

struct Plan {
    // resolved description
    int dim = 2, N = 0, m_v = 0, ni = 0, map = 0, kernel = 0, precision = 0;
    double S = 0.0, b0 = 0.0, gamma = 0.0, wsum = 0.0, aniso = 0.0;
    int n_sigma = 0;
    std::vector<double> sigma, sigma_w, wfac;

    // fine grid and spreading kernel
    double upsample = 2.0, beta = 0.0, h = 0.0, tol = 0.0;
    int W = 0, terms = 0, n = 0, nh = 0, ng = 0;

    // gain decomposition
    int slab_planes = 0, n_slabs = 0, n_chunks = 0, block_threads = 0;
    int np = 0;  // unordered node pairs per dimension, n_i (n_i + 1) / 2
    int64_t nid = 0, Nd = 0, ngd = 0, n_units = 0, units_per_chunk = 0, n_triples = 0;
    int64_t n_points = 0;  // merged points per evaluation, n_sigma * np^d
    int64_t index_budget = 0;  // bytes for the binned gain's point ids (0: whole index if it fits)
    int64_t tmp_elems = 0;

    // host tables (FP64)
    std::vector<double> xi_all, v_all, w_all;
    std::vector<double> v1, w1, mu21, C, CT, E, poly, slab_vlo, slab_vhi, mom;
    std::vector<double> kpoly_eo, cellfit, cellfit_v, bin_vthr;
    double cellfit_err = 0.0;  // largest deviation of a cell fit from the exact offset
    int cellfit_v_cells = 0;   // cells with a fit in the velocity

    size_t elt = 8;
    int gain_mode = kGainBinned;
    bool mfma = false;         // binned gain on the FP64 matrix cores (FP64 3D plans)
    bool deterministic = false;  // fixed-order tile gather instead of grid atomics
    bool auto_gain = true;
    Profiler* prof = nullptr;  // stage timing, off unless requested
    int prof_set = -1;         // event set of the call being recorded
    BinIndex bins;
    DeviceTables dt;
    Workspace ws;
    int64_t workspace_bytes = 0;
    std::vector<void*> allocations;
    int device = -1;           // HIP device current when the plan was created
};

// Buffers of the dense (FP64) stages for nb cells, each nb times the size of
// the corresponding single-cell Workspace buffer.
struct DenseBufs {
    double* P = nullptr;
    double* G = nullptr;
    void* Gg = nullptr;       // plan precision; NULL when the gain reads G itself (FP64)
    double* H = nullptr;
    double* qminus = nullptr;
    double* qplus = nullptr;
    double* tmpA = nullptr;   // nb * max(N, n_i, n_g)^d each
    double* tmpB = nullptr;
    double* red = nullptr;    // nb
};

// record the event that closes stage `stage - 1` / opens `stage` (no-op when off)
inline void prof_mark(const Plan& p, int stage, hipStream_t s)
{
    if (p.prof && p.prof_set >= 0) (void)hipEventRecord(p.prof->ev[p.prof_set][stage], s);
}

// ----- launchers (pgc_kernels.hip); all enqueue on `s` and return the launch status
// The four stages of one evaluation read and write the buffers of `ws`: the
// plan's own Workspace, or one carved from the library's static scratch array.
hipError_t launch_synthesis(const Plan& p, const Workspace& ws, const void* coeffs, hipStream_t s);
hipError_t launch_loss(const Plan& p, const Workspace& ws, hipStream_t s);
// the gain and its cosine transform, ending with Q = Q+ - Q- into q (and Q+
// into qplus when it is given) in the plan precision
hipError_t launch_gain(const Plan& p, const Workspace& ws, void* q, void* qplus, hipStream_t s);
// the dense stages for nb cells of one plan's size (batches)
hipError_t launch_dense_synthesis(const Plan& p, const double* c64, int nb, const DenseBufs& b,
                                  hipStream_t s);
hipError_t launch_dense_loss(const Plan& p, int nb, const DenseBufs& b, hipStream_t s);
hipError_t launch_dense_grid_to_modes(const Plan& p, const double* grid, int nb, const DenseBufs& b,
                                      hipStream_t s);
// mode 0 counts the points of directions [s0, s0 + ns) per bin into `count`;
// mode 1 scatters their ids through 64-bit per-bin cursors (the whole index,
// plan time), mode 2 through 32-bit ones (a chunk of a streamed index)
hipError_t launch_bin_build(const Plan& p, unsigned int* count, unsigned long long* cursor,
                            unsigned int* cursor32, unsigned long long* ids, int mode, int s0, int ns,
                            hipStream_t s);
// deterministic plans: sort the point ids inside every bin by value (begin:
// nbins + 1 offsets into ids; the ids use bits [0, end_bit))
hipError_t sort_bin_ids(unsigned long long* ids, const std::vector<unsigned long long>& begin, int end_bit,
                        hipStream_t s);
hipError_t launch_project(const Plan& p, const double* f_nodes, void* coeffs, hipStream_t s);
hipError_t launch_moments(const Plan& p, const void* coeffs, double* out, hipStream_t s);
hipError_t launch_eval(const Plan& p, const void* coeffs, const double* v, int64_t n, double* out,
                       hipStream_t s);
// y = base + a * k (stage input, plan precision); base is FP64
hipError_t launch_rk_stage(const Plan& p, const double* base, const void* k, double a, void* y,
                           hipStream_t s);
// base += dt/6 (k1 + 2 k2 + 2 k3 + k4)
hipError_t launch_rk_finish(const Plan& p, double* base, double dt, hipStream_t s);
hipError_t launch_copy_state(const Plan& p, const double* base, void* y, hipStream_t s);

// status of a HIP error code
inline pgc_status status_of(hipError_t e)
{
    if (e == hipSuccess) return PGC_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return PGC_ERR_OUT_OF_MEMORY;
    return PGC_ERR_DEVICE;
}

}  // namespace pgc

// the opaque plan handle of the C ABI
struct pgc_plan_s {
    pgc::Plan p;
    hipGraph_t graph = nullptr;  // a captured evaluation or RK4 run (pgc_plan_capture*)
    hipGraphExec_t exec = nullptr;
};
