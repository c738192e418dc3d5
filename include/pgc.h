/*
 * pgc.h -- C ABI of the MI355X (gfx950) library for the fast Petrov-Galerkin
 * mapped-Chebyshev collision operator of Hu, Huang, Shen and Yang,
 * "A fast Petrov-Galerkin spectral method for the multi-dimensional Boltzmann
 * equation using mapped Chebyshev functions" (arXiv 2105.08806).
 *
 * What the library computes
 * -------------------------
 * For f_N = sum_k f_k T~_k (eq. fN_Expansion, Sec. 3) the Galerkin
 * coefficients of the collision operator (eq. Qk_component, Sec. 3)
 *     Q_k = (Q(f_N, f_N), T^_k) = Q+_k - Q-_k            (eqs. Qplus, Qminus)
 * discretised with Chebyshev-Gauss-Lobatto rules in xi and eta and a rule on
 * the unit sphere (Sec. 4.1), and evaluated with the fast algorithm of
 * Sec. 4.2: the gain through a type-1 non-uniform cosine transform
 * (eqs. num_fast_k, nufft) -- here one merged transform per evaluation -- and
 * the loss through its inner kernel sum plus a Chebyshev transform.
 *
 * Conventions
 * -----------
 *  - N = n_modes is the number of modes per dimension, k_l = 0..N-1 (the
 *    paper's degree is N-1).  Coefficient tensors are dense, row-major,
 *    last index fastest: index (k_1*N + k_2)*N + k_3 in 3D.
 *  - m_v Chebyshev-Gauss-Lobatto nodes per dimension, xi_j = -cos(pi j/(m_v-1)),
 *    both endpoints included; every velocity sum runs over the m_v - 2
 *    interior nodes (f_N vanishes at xi = +-1, i.e. v = +-infinity).
 *    Nodal arrays are n_i^dim, n_i = m_v - 2, row-major.
 *  - Maps (Sec. 2.1): LOG is r = 0, v = S atanh(xi); ALGEBRAIC is r = 1,
 *    v = S xi / sqrt(1 - xi^2).
 *  - Kernels: MAXWELL, B = b0; VHS, B = b0 |v - v_*|^gamma (0 <= gamma <= 1).
 *
 * Memory, streams, errors
 * -----------------------
 *  - Every array argument named *_dev is a caller-owned DEVICE pointer on the
 *    current HIP device; *_host arguments are host pointers.
 *  - Coefficient and Q arrays have the plan's precision: double for
 *    PGC_PRECISION_FP64, float for PGC_PRECISION_FP32.  State, nodal input
 *    and moment arrays are always double.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls only
 *    enqueue work on it and return; no call synchronises the host unless its
 *    comment says so.  A plan owns all its workspace (allocated in
 *    pgc_plan_create, freed in pgc_plan_destroy); the calls that enqueue
 *    work on a plan (pgc_project, pgc_coeffs_to_q, pgc_rk4, pgc_moments,
 *    pgc_eval) allocate nothing.
 *  - A plan must not be used by two calls that can run concurrently.
 *  - By default the fast path's gain accumulates with FP64 atomics whose
 *    order varies, so repeated evaluations agree to rounding, not bit for bit;
 *    a plan created with deterministic = 1, a batch created from such a
 *    descriptor, and the direct algorithm (pgc_direct_*), repeat bit for bit.
 *  - Every call returns a pgc_status.  On an error return the outputs are
 *    untouched (for argument errors) or unspecified (device errors).  No C++
 *    exception crosses this interface.  PGC_ERR_NUMERIC needs a result on the
 *    host, so only calls that read one back return it (pgc_surrogate_train,
 *    when an epoch's loss is not finite); asynchronous calls never do.
 */
#ifndef PGC_H
#define PGC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pgc_status {
    PGC_OK = 0,
    PGC_ERR_INVALID_ARG = 1,
    PGC_ERR_UNSUPPORTED = 2,
    PGC_ERR_OUT_OF_MEMORY = 3,
    PGC_ERR_DEVICE = 4,
    PGC_ERR_NUMERIC = 5,
    PGC_ERR_SCRATCH = 6     /* pgc_coeffs_to_q_static: the plan needs more than
                               PGC_STATIC_SCRATCH_BYTES of scratch */
} pgc_status;

enum { PGC_MAP_LOG = 0, PGC_MAP_ALGEBRAIC = 1 };
enum { PGC_SCALE_DIRECT = 0, PGC_SCALE_FROM_DOMAIN = 1 };
enum { PGC_KERNEL_MAXWELL = 0, PGC_KERNEL_VHS = 1, PGC_KERNEL_ANISO = 2 };
enum { PGC_SPHERE_UNIFORM_2D = 0, PGC_SPHERE_PRODUCT_3D = 1, PGC_SPHERE_USER = 2 };
enum { PGC_PRECISION_FP64 = 0, PGC_PRECISION_FP32 = 1 };

/* Description of one discretised operator.  Fill with pgc_desc_init, then
 * set what differs.  Tuning fields left at 0 are chosen by the library. */
typedef struct pgc_plan_desc {
    int32_t dim;          /* 2 or 3 */
    int32_t n_modes;      /* N >= 3 (degree >= 2 keeps 1 and |v|^2 in the test space, Sec. 3.2) */
    int32_t m_v;          /* CGL nodes per dimension incl. endpoints; 0 = n_modes + 1 */
    int32_t map;          /* PGC_MAP_LOG or PGC_MAP_ALGEBRAIC */
    int32_t scale_mode;   /* PGC_SCALE_DIRECT: S = scale.  PGC_SCALE_FROM_DOMAIN: S such that
                             the second and second-to-last nodes map to -scale and +scale
                             (the adaptive choice of Sec. 5) */
    double scale;         /* > 0 */
    int32_t kernel;       /* PGC_KERNEL_MAXWELL (B = b0), PGC_KERNEL_VHS (B = b0 |u|^gamma) or
                             PGC_KERNEL_ANISO (B = b0 |u|^gamma (1 + kernel_aniso cos^2 theta),
                             cos theta = u.sigma/|u|: an angle-dependent rate, the general
                             B(|u|, cos theta) of Sec. 4.2).  ANISO runs on the binned fast path
                             (gain_mode 0 or 2: each merged point weighs its orbit's triples by their
                             own angle; the loss's inner integral over sigma is a quadratic form in u)
                             and on the direct algorithm; gain_mode 1 and 3, and batches, return
                             UNSUPPORTED for it */
    double kernel_b0;     /* kernel constant; 0 = 1/|S^{d-1}| (so that int B dsigma = 1 for Maxwell) */
    double kernel_gamma;  /* exponent of |u| in [0, 1] (VHS and ANISO) */
    int32_t sphere;       /* PGC_SPHERE_UNIFORM_2D (theta_s = 2 pi s/n_sigma, W_s = 2 pi/n_sigma),
                             PGC_SPHERE_PRODUCT_3D (n_theta Gauss-Legendre nodes in cos(theta)
                             x n_phi uniform phi), or PGC_SPHERE_USER */
    int32_t n_sigma;      /* UNIFORM_2D and USER: number of directions (even for UNIFORM_2D) */
    int32_t n_theta;      /* PRODUCT_3D */
    int32_t n_phi;        /* PRODUCT_3D, even */
    const double* user_sigma_host;   /* USER: n_sigma x dim unit vectors (copied) */
    const double* user_weights_host; /* USER: n_sigma positive weights (copied) */
    int32_t precision;    /* PGC_PRECISION_FP64 or PGC_PRECISION_FP32 */
    double nufft_tol;     /* requested accuracy of the cosine transform relative to sum |q|;
                             0 = 5e-13 (FP64) or 1e-6 (FP32) */
    double upsample;      /* fine-grid upsampling factor sigma_up in [1.5, 4]; 0 = 3 */
    int32_t kernel_width; /* spreading kernel width W in grid cells (2..16); 0 = from nufft_tol */
    int32_t slab_planes;  /* fine-grid planes held in LDS per workgroup; 0 = as many as fit */
    int32_t n_chunks;     /* collision-unit chunks (partial grids); 0 = automatic */
    int32_t block_threads;/* threads per spreading workgroup (256, 512 or 1024); 0 = automatic */
    int32_t gain_mode;    /* spreading scheme: 0 = automatic (binned, falling back to slabs when the
                             bin index does not fit in device memory or the plan is outside the
                             binned limits), 1 = LDS slabs with one atomic per contribution,
                             2 = plan-time bins by footprint corner with register accumulation (the
                             index holds 8 bytes per merged point; W <= 14, at most 256 interior
                             nodes per dimension and 1024 directions, UNSUPPORTED otherwise), 3 = the
                             same bins contracted on the FP64 matrix cores (FP64 3D plans with
                             W <= 12 only, UNSUPPORTED otherwise) */
    double kernel_aniso;  /* ANISO: beta in [-1, 10] (B >= 0); Q(f, f) sees only the part of B
                             even in cos theta, so an even polynomial is the general smooth
                             low-order angular law */
    int32_t deterministic;/* 0: the binned gain adds each bin run's footprint tile into the fine
                             grid with FP64 atomics (fastest; repeated evaluations agree to
                             rounding).  1: every run writes its tile to plan workspace
                             (n_bin_items x W^d doubles) and a gather adds the tiles of every grid
                             cell in a fixed order, and the plan sorts the point ids inside every
                             bin once after building the index, so the evaluations of every plan
                             of the same descriptor are bit-identical (on one device type).
                             Needs the binned vector gain (gain_mode 0 or 2; UNSUPPORTED with 1
                             or 3) and the whole point index (UNSUPPORTED when index_bytes
                             streams it) */
    int64_t index_bytes;  /* device memory for the point ids of the binned gain (the sort of the
                             merged points by footprint corner that Sec. 4.3's on-the-fly evaluation
                             leaves to each evaluation).  0: the plan builds the whole index once
                             (8 bytes per merged point) when the device has room for it, and
                             streams it within a quarter of the free memory otherwise.  > 0: when
                             the whole index needs more than index_bytes, the directions are split
                             into chunks whose ids fit in index_bytes (at least one direction per
                             chunk) and every evaluation sorts each chunk's points into bins again
                             (one more pass that regenerates every point) before spreading them.
                             The plan keeps per chunk only the point count of every bin.  Negative:
                             PGC_ERR_INVALID_ARG */
} pgc_plan_desc;

typedef struct pgc_plan_s* pgc_plan;

typedef struct pgc_plan_info {
    int32_t dim, n_modes, m_v, map, kernel, precision;
    int32_t n_sigma;        /* directions actually used */
    double scale;           /* the S actually used */
    int32_t grid_n;         /* periodic fine-grid size n (cells over [0, 2 pi)) */
    int32_t grid_folded;    /* n/2 + 1 points per dimension over [0, pi] */
    int32_t kernel_width;   /* W */
    double kernel_beta;     /* ES shape parameter */
    double upsample;
    int32_t slab_planes, n_slabs, n_chunks, block_threads;
    int64_t n_triples;      /* collision triples per evaluation, n_sigma * n_i^(2 dim) */
    int64_t n_points;       /* distinct transform points after merging the triples that share
                               v' (exchanging i_l and j_l in any dimension): n_sigma * (n_i (n_i+1)/2)^dim */
    int64_t workspace_bytes;/* device memory owned by the plan */
    int32_t gain_mode;      /* 1 = slabs, 2 = bins, 3 = bins on the FP64 matrix cores */
    int64_t n_bin_items;    /* binned mode: work items (runs of one bin) per evaluation */
    double offset_fit_err;  /* largest deviation, over every grid cell, of the stored per-cell
                               polynomial that gives a point's kernel offset from w (binned
                               gain) from the exact offset, in units of the offset's range [-1, 1] */
    int32_t deterministic;  /* 1: fixed-order tile gather (bit-identical repeats) */
    int64_t tile_bytes;     /* deterministic plans: workspace of the per-run footprint tiles */
    int32_t index_chunks;   /* binned gain: 1 = the whole point index, built at plan time; > 1 =
                               direction chunks sorted again at every evaluation */
    int64_t index_bytes;    /* binned gain: bytes of the point-id buffer (the largest chunk) */
    int32_t velocity_fit_cells; /* grid cells (of grid_folded + 1 bin coordinates) whose points take
                               their kernel offset and map factor from a per-cell polynomial in
                               v/S, within 5e-16 of the exact values; the points of the other cells
                               (one or a few at each end of the grid) go through the map to w */
} pgc_plan_info;

/* Human-readable text of a status code (static storage, never NULL). */
const char* pgc_status_string(pgc_status s);

/* Fill *desc with defaults: 2D, N = 16, LOG map, S = 4, Maxwell, 16 directions,
 * FP64.  Returns PGC_ERR_INVALID_ARG for NULL. */
pgc_status pgc_desc_init(pgc_plan_desc* desc);

/* Kernel width W and shape beta that the library would use for a cosine
 * transform of accuracy tol at upsampling factor upsample (host only, no GPU).
 * The "exponential of semicircle" kernel exp(beta (sqrt(1 - y^2) - 1)) is the
 * one of the NUFFT library the paper uses for eq. (nufft). */
pgc_status pgc_nufft_params(double tol, double upsample, int32_t* width, double* beta);

/* Validate *desc, build every table (nodes, maps, sphere rule, Chebyshev and
 * cosine-transform matrices, kernel polynomials, moment functionals) in FP64
 * on the host, upload them and allocate all workspace on the current device.
 * `stream` orders the uploads; the call synchronises it before returning.
 * Errors: INVALID_ARG (bad descriptor, odd or non-antipodal sphere rule),
 * UNSUPPORTED (sizes beyond the kernels' limits), OUT_OF_MEMORY, DEVICE. */
pgc_status pgc_plan_create(const pgc_plan_desc* desc, void* stream, pgc_plan* plan_out);

/* Free the plan and its workspace (NULL is a no-op).  Synchronises the device. */
pgc_status pgc_plan_destroy(pgc_plan plan);

/* Copy the plan's resolved parameters into *info (host only). */
pgc_status pgc_plan_query(pgc_plan plan, pgc_plan_info* info);

/* Host copies of the m_v CGL nodes xi_j, mapped velocities v_j (endpoints
 * -/+HUGE_VAL) and weights w_j.  Any pointer may be NULL. */
pgc_status pgc_nodes(pgc_plan plan, double* xi_host, double* v_host, double* w_host);

/* Coefficients of the initial data, eq. (MultiD_spectral_coef) by the
 * interior CGL rule: f_k = sum_i w_i mu_i^-4 f(v_i) T_k(xi_i)/sqrt(c_k).
 * f_nodes_dev: n_i^dim doubles (f at the interior nodes); coeffs_dev: N^dim
 * in the plan's precision. */
pgc_status pgc_project(pgc_plan plan, const double* f_nodes_dev, void* coeffs_dev, void* stream);

/* The hot path: Q = Q+ - Q- for the coefficients coeffs_dev (N^dim, plan
 * precision).  q_dev receives Q (N^dim); qplus_dev, if not NULL, receives Q+.
 * Steps: Chebyshev synthesis of f_N at the nodes (Sec. 4.2), loss field and
 * loss projection (eq. Qminus), generation of every collision triple and
 * spreading of its weight onto the folded fine grid (eqs. num_fast_k, nufft),
 * cosine transform, deconvolution and the final combination. */
pgc_status pgc_coeffs_to_q(pgc_plan plan, const void* coeffs_dev, void* q_dev, void* qplus_dev,
                           void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as pgc_coeffs_to_q, with the same arguments, results and stream
 * ordering, but every per-call buffer (nodal values, loss field, fine grid,
 * transform buffers, partial sums: about 23 MB for the 3D 32-mode FP64
 * workload) is carved from one static device array of
 * PGC_STATIC_SCRATCH_BYTES held by the library on each device it runs on
 * until the process ends.  The call allocates nothing; its first call on a
 * device looks the array's address up once.  The plan's own tables (and its
 * bin index) are still read.  Every call on a device shares that device's
 * array, so calls that can overlap on one device -- on two streams, or from
 * two threads -- race and must be serialised by the caller.  The array keeps
 * the last call's contents; the call clears what must start at zero itself.
 * Errors: INVALID_ARG (NULL arguments, or the current device is not the one
 * the plan was created on), SCRATCH (the plan needs more than the array
 * holds), DEVICE. */
#define PGC_STATIC_SCRATCH_BYTES (32u * 1024u * 1024u)
pgc_status pgc_coeffs_to_q_static(pgc_plan plan, const void* coeffs_dev, void* q_dev, void* qplus_dev,
                                  void* stream);

/* n_steps classical fourth-order Runge-Kutta steps of size dt on
 * d f_k/dt = Q_k (eq. spectral_ODE), in place on coeffs_dev (N^dim doubles,
 * whatever the plan precision; FP32 plans round each stage input to float). */
pgc_status pgc_rk4(pgc_plan plan, double* coeffs_dev, double dt, int32_t n_steps, void* stream);

/* HIP graphs of a plan's launch sequences, for callers that evaluate the same
 * buffers many times (a small plan's evaluation is a dozen short launches;
 * a replay issues them as one).  Each capture replaces the plan's earlier
 * graph.  pgc_plan_capture records pgc_coeffs_to_q for these pointers: one
 * eager evaluation runs first on `stream` (it writes q_dev and qplus_dev), then
 * the capture, on a private stream.  pgc_plan_capture_rk4 records
 * pgc_rk4(coeffs_dev, dt, n_steps) (n_steps >= 1), in place on coeffs_dev:
 * `stream` is synchronised first and nothing runs.  pgc_plan_graph_launch
 * replays the graph on `stream`.  A graph reads and writes the pointers it was
 * captured with (refill the same input buffer between replays) and uses the
 * plan's workspace, which eager calls share in stream order.  Errors:
 * INVALID_ARG (NULL plan or buffers, n_steps < 1, non-finite dt, a launch
 * with no graph), UNSUPPORTED (profiling is on: its events stay out of
 * graphs), DEVICE. */
pgc_status pgc_plan_capture(pgc_plan plan, const void* coeffs_dev, void* q_dev, void* qplus_dev, void* stream);
pgc_status pgc_plan_capture_rk4(pgc_plan plan, double* coeffs_dev, double dt, int32_t n_steps, void* stream);
pgc_status pgc_plan_graph_launch(pgc_plan plan, void* stream);

/* Mass, momentum (dim values) and energy int |v|^2 f_N dv of the expansion
 * with coefficients coeffs_dev (plan precision), eq. (def_mom), computed in
 * FP64 from 1D moment functionals: out_dev receives dim + 2 doubles. */
pgc_status pgc_moments(pgc_plan plan, const void* coeffs_dev, double* out_dev, void* stream);

/* out_dev[r] = sum_k c_k T~_k(v_r) for n velocities v_dev (n x dim doubles);
 * coeffs_dev in the plan's precision, evaluation in FP64.  Evaluates f_N and
 * Q_N = sum_k Q_k T~_k (the equivalent form, eq. P_G_method) off the hot path. */
pgc_status pgc_eval(pgc_plan plan, const void* coeffs_dev, const double* v_dev, int64_t n,
                    double* out_dev, void* stream);

/* Stage timing.  With profiling on, every pgc_coeffs_to_q records HIP events
 * on its stream between its stages (no host synchronisation); pgc_stage_times
 * waits for the recorded events and returns, per stage, the accumulated
 * milliseconds (ms_out) and the number of timed calls (calls_out may be NULL),
 * then resets the accumulators.  Stages: 0 synthesis, 1 loss field and loss
 * projection, 2 pair-orbit sums, 3 spreading (the dominant kernel), 4 grid to
 * modes (conversion, cosine transform and the combination Q = Q+ - Q-), 5
 * empty (the combination, which stage 4 now ends with).  n_stages <= 8.
 * pgc_set_profiling(plan, 0) stops recording. */
pgc_status pgc_set_profiling(pgc_plan plan, int32_t on);
pgc_status pgc_stage_times(pgc_plan plan, double* ms_out, int32_t n_stages, int64_t* calls_out);

/* ------------------------------------------------------------------------
 * Batches: one evaluation of Q for each of many velocity cells (for example
 * the spatial cells of a kinetic solver), with mixed N.  Every cell applies
 * the discretisation of `base` with its own n_modes.  The cells that share an
 * N share one internal plan (tables and plan-time bin index); the gain of all
 * cells runs as one persistent launch over (bin run, group of cells) work
 * units, so the geometry of a merged point is generated once for every group
 * of cells that reads it.  Supported: dim = 2, precision FP32 (the gain in
 * FP32 with FP64 fine grids, the dense stages in FP64, as for FP32 plans),
 * at most 8 distinct N, 3 <= N <= 255, kernel widths 4..8.
 *
 * Packed layout: the coefficients of cell c are the dense N_c^2 block that
 * starts at element offsets[c] of the packed array (float).  The packed Q
 * array uses the same offsets.  Passing offsets_dev = NULL selects the dense
 * packing in cell order (offsets[c] = sum of N_b^2 over b < c, returned by
 * pgc_batch_offsets).  offsets_dev is a device array of n_cells int64.
 * ------------------------------------------------------------------------ */
typedef struct pgc_batch_s* pgc_batch;

typedef struct pgc_batch_info {
    int32_t n_cells;
    int32_t n_groups;           /* distinct N */
    int32_t group_n_modes[8];   /* N of each group, descending */
    int32_t group_cells[8];     /* cells in each group */
    int64_t coeffs_total;       /* length of the dense packing, sum of N_c^2 */
    int32_t kernel_width;       /* W of the spreading kernel (the same for every N) */
    int32_t cells_per_wave;     /* C: cells a gain work unit serves: 1, 2, 4, 8 (register tiles,
                                   each lane generates points for its C cells) or 16, 32, 64
                                   (lane per cell, 64 / C point streams per wave) */
    int32_t waves;              /* persistent 64-lane workgroups of the gain launch */
    int64_t n_units;            /* gain work units per evaluation */
    int64_t n_points;           /* merged transform points over all cells */
    int64_t workspace_bytes;    /* device memory owned by the batch and its plans */
    double tuned_ms[7];         /* autotuner: gain time for C = 1, 2, 4, 8, 16, 32, 64 (0 = not tried) */
    int32_t has_graph;          /* a captured graph is ready for pgc_batch_graph_launch */
    int32_t scheme;             /* 0 register tiles, 1 lane per cell */
    int32_t spatial_order;      /* 1: bin runs in raster order of their bins, 0: longest first */
    double order_ms[2];         /* autotuner: gain time at the chosen C, longest-first / raster order */
    int32_t group_major;        /* 1: work units run through all bin runs of one cell group before the
                                   next group (the G rows in use stay in L2); 0: bin-run major */
    double major_ms[2];         /* autotuner: gain time at the chosen C and order, bin-run / cell-group major */
    int32_t deterministic;      /* 1: every cell through its group's deterministic plan */
} pgc_batch_info;

/* Build a batch of n_cells cells; n_modes_host[c] is the N of cell c.
 * With autotune != 0 the call times the gain for every supported C on the
 * device (the best of two evaluations; one when the first is over 1.5x the
 * best so far) and keeps the fastest, then times the other bin-run order and
 * the other unit order at that C and keeps each only when it is over 3%
 * faster; otherwise C = 1, raster order, bin-run major.  `stream` orders the set-up work, which the call synchronises.
 * With base->deterministic = 1 the batch evaluates every cell through its
 * group's plan (created with deterministic = 1) instead of the batched gain:
 * each cell's Q is then bit-identical to pgc_coeffs_to_q on a plan created
 * from the same descriptor with that cell's N (gain_mode 0 or 2), at the
 * speed of one plan evaluation per cell.  Such a batch takes no offsets_dev
 * (UNSUPPORTED) and cannot be captured (UNSUPPORTED); the tile and order
 * settings have no effect on it.
 * Errors: INVALID_ARG, UNSUPPORTED (dim != 2, precision != FP32, more than 8
 * distinct N, a kernel width outside 4..8), OUT_OF_MEMORY, DEVICE. */
pgc_status pgc_batch_create(const pgc_plan_desc* base, int32_t n_cells, const int32_t* n_modes_host,
                            int32_t autotune, void* stream, pgc_batch* batch_out);
/* Free the batch (NULL is a no-op).  Synchronises the device. */
pgc_status pgc_batch_destroy(pgc_batch batch);
pgc_status pgc_batch_query(pgc_batch batch, pgc_batch_info* info);
/* The n_cells offsets of the dense packing (host array). */
pgc_status pgc_batch_offsets(pgc_batch batch, int64_t* offsets_host);
/* Force C cells per work unit (1, 2, 4 or 8 with C W^2 <= 200, or 16, 32, 64), or re-run
 * the autotuner.  Both drop a captured graph and synchronise `stream`. */
pgc_status pgc_batch_set_tile(pgc_batch batch, int32_t cells_per_wave, void* stream);
pgc_status pgc_batch_autotune(pgc_batch batch, void* stream);
/* Force the order of the gain's work units at the current C: raster = 1 takes
 * the bin runs in raster order of their bins (0: longest first); group_major = 1
 * runs through all bin runs of one cell group before the next (0: all cell
 * groups of one bin run first).  The result does not depend on the order up to
 * FP64 summation order.  Drops a captured graph and synchronises `stream`.
 * Errors: INVALID_ARG (a flag other than 0 or 1), DEVICE. */
pgc_status pgc_batch_set_order(pgc_batch batch, int32_t raster, int32_t group_major, void* stream);
/* Q of every cell: packed_q_dev receives Q_c at offsets[c] (float).  Stream
 * ordered, allocates nothing.  The input and output ranges must not overlap. */
pgc_status pgc_batch_coeffs_to_q(pgc_batch batch, const void* packed_coeffs_dev, const int64_t* offsets_dev,
                                 void* packed_q_dev, void* stream);
/* Record the same evaluation, for these three device pointers, into a HIP
 * graph owned by the batch (replacing any earlier one); `stream` is
 * synchronised first and nothing runs.  pgc_batch_graph_launch replays it on
 * `stream` (INVALID_ARG when no graph is ready).  The graph reads the pointers
 * captured, so the caller refills the same input buffer between replays. */
pgc_status pgc_batch_capture(pgc_batch batch, const void* packed_coeffs_dev, const int64_t* offsets_dev,
                             void* packed_q_dev, void* stream);
pgc_status pgc_batch_graph_launch(pgc_batch batch, void* stream);

/* ------------------------------------------------------------------------
 * Learned surrogate of the coefficients-to-Q map of one FP32 plan.
 *
 * A multilayer perceptron on the N^d coefficients (per-feature normalisation,
 * n_layers - 1 hidden layers of `width` units with SiLU, a linear output
 * layer), trained by the library's own forward and backward kernels on pairs
 * (f, Q) that the plan itself produced.  Products run on the matrix cores in
 * BF16 with FP32 accumulation; master weights and Adam state are FP32.  The
 * network output is projected onto the coefficient vectors whose mass,
 * momentum and energy vanish (the invariants of the test space, Sec. 3.2),
 * which is exact for the algebraic map and the quadrature rule of the plan.
 *
 * The plan is the fallback and the judge.  A sample falls back to
 * pgc_coeffs_to_q of the plan when (a) the relative mass/momentum/energy
 * residual of the returned Q exceeds gate_residual, or (b) the residual of the
 * raw network output, or the RMS z-score of the normalised input, exceeds
 * gate_raw_factor times the largest one seen on the training set (an input
 * unlike the training data; 0 disables).  Every
 * judge_stride-th sample of a call is also evaluated by the plan and returns
 * the plan's value; if the network's output for it differs from the plan's by
 * more than judge_tol (relative L2), the judge_stride - 1 samples that follow
 * it (its window, within the batch_max rows of one pass) fall back as well
 * (0 disables the judge).  Fallback flags: 0 network, 1 plan (a gate or the
 * judge's window), 2 judged (the plan's value, computed for the judge).
 *
 * Arrays: f and q are n_samples x N^d float rows (device).  The plan must
 * outlive the surrogate and must not be used concurrently with it.
 * ------------------------------------------------------------------------ */
typedef struct pgc_surrogate_s* pgc_surrogate;

typedef struct pgc_surrogate_desc {
    int32_t width;           /* hidden width; default 1024 */
    int32_t n_layers;        /* linear layers (>= 2); default 4 */
    int32_t batch_max;       /* rows per forward/backward pass; default 256 */
    uint64_t seed;           /* weight initialisation */
    double gate_residual;    /* default 1e-6 */
    double gate_raw_factor;  /* default 4 */
    int32_t judge_stride;    /* default 64 */
    double judge_tol;        /* default 5e-2 */
    double norm_floor_in;    /* per-feature standard deviations of the inputs are held at or
                                above this fraction of the largest; default 0.1 */
    double norm_floor_out;   /* the same for the outputs; default 1 (one common scale) */
    int32_t loss_relative;   /* training loss: 0 (default) the mean squared error of the
                                normalised outputs, (1 / (B n)) sum_r sum_c d_rc^2 with
                                d = yhat - (q - mu_out) / sd_out; 1 the mean squared relative
                                error of every sample in the units of q,
                                (1 / B) sum_r sum_c (sd_out_c d_rc)^2 / sum_c q_rc^2, which
                                weights every sample by its own scale as the judge does */
} pgc_surrogate_desc;

typedef struct pgc_surrogate_info {
    int32_t n_features;      /* N^d */
    int32_t width, n_layers, batch_max;
    int64_t n_params;        /* weights and biases */
    int32_t n_constraints;   /* d + 2 invariants */
    int64_t steps;           /* optimiser steps taken */
    double raw_residual_calibrated;
    int64_t workspace_bytes;
    double zscore_calibrated;   /* largest RMS z-score of a training input */
} pgc_surrogate_info;

pgc_status pgc_surrogate_desc_init(pgc_surrogate_desc* desc);
/* Allocate and initialise the network for `plan` (FP32 plans only:
 * UNSUPPORTED otherwise).  Synchronises `stream`. */
pgc_status pgc_surrogate_create(pgc_plan plan, const pgc_surrogate_desc* desc, void* stream, pgc_surrogate* out);
pgc_status pgc_surrogate_destroy(pgc_surrogate s);
pgc_status pgc_surrogate_query(pgc_surrogate s, pgc_surrogate_info* info);
/* Per-feature mean and standard deviation of inputs and targets over the
 * n_samples rows of f_dev and q_dev (call before training). */
pgc_status pgc_surrogate_set_normalization(pgc_surrogate s, const float* f_dev, const float* q_dev,
                                           int64_t n_samples, void* stream);
/* `epochs` passes of mini-batch Adam (batch <= batch_max rows, step size lr
 * with cosine decay over the epochs) on the loss chosen by desc.loss_relative;
 * loss_host (may be NULL) receives the mean batch loss of each epoch.  Then
 * calibrates the raw-residual gate on the training set.  NUMERIC (training
 * stops) when an epoch's loss is not finite, e.g. for a step size that
 * diverges; the parameters are then unspecified.  Allocates a device
 * copy of each epoch's sample order (n_samples ints, freed before returning)
 * and synchronises `stream` once per epoch. */
pgc_status pgc_surrogate_train(pgc_surrogate s, const float* f_dev, const float* q_dev, int64_t n_samples,
                               int32_t epochs, int32_t batch, double lr, uint64_t seed, double* loss_host,
                               void* stream);
/* Q of n_samples rows: q_dev receives the surrogate's Q, or the plan's for
 * the samples that fall back or are judged.  fallback_host (may be NULL)
 * receives one flag per sample (0, 1 or 2 as above), n_fallback the count of
 * flag-1 samples, judge_err the largest relative error the judge saw.  The
 * gates are read on the host: the call synchronises `stream` once per pass of
 * batch_max rows, then enqueues the fallbacks' plan evaluations. */
pgc_status pgc_surrogate_coeffs_to_q(pgc_surrogate s, const float* f_dev, int64_t n_samples, float* q_dev,
                                     int32_t* fallback_host, int64_t* n_fallback, double* judge_err, void* stream);
/* Loss and gradient (all parameters, in the get_params order without the
 * normalisation vectors) of the first n_samples <= batch_max rows. */
pgc_status pgc_surrogate_loss_grad(pgc_surrogate s, const float* f_dev, const float* q_dev, int32_t n_samples,
                                   double* loss_host, float* grad_host, void* stream);
/* Parameters flattened layer by layer, W (out x in, row-major) then b, then
 * mu_in, sd_in, mu_out, sd_out (N^d each): n_params + 4 N^d floats. */
pgc_status pgc_surrogate_get_params(pgc_surrogate s, float* params_host, void* stream);
pgc_status pgc_surrogate_set_params(pgc_surrogate s, const float* params_host, void* stream);
/* Binary file of the parameters and the gate calibration; load checks the shape. */
pgc_status pgc_surrogate_save(pgc_surrogate s, const char* path, void* stream);
pgc_status pgc_surrogate_load(pgc_surrogate s, const char* path, void* stream);

/* The matrix-core product the surrogate is built on, exposed for testing:
 * C (M x N, FP32, row stride ldc) = op(A) op(B) + bias (or C += ... when
 * accumulate != 0), A and B BF16 device matrices given as uint16 bit
 * patterns, op(A)[m][k] = trans_a ? A[k lda + m] : A[m lda + k], likewise B.
 * INVALID_ARG for negative sizes, missing pointers, or a row stride shorter
 * than its row (lda < K, or < M when transposed; ldb likewise; ldc < N).
 * K = 0 gives C = bias (zero without one), or C += bias. */
pgc_status pgc_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* a_dev, int32_t lda, int32_t trans_a,
                         const uint16_t* b_dev, int32_t ldb, int32_t trans_b, float* c_dev, int32_t ldc,
                         const float* bias_dev, int32_t accumulate, void* stream);

/* ---------------------------------------------------------------------------
 * The direct algorithm (Sec. 4.1, eqs. direct_online, tensor_I1, tensor_I2)
 * for many cells that share one FP64 plan.  The discrete Q is a bilinear form
 * in the weighted nodal values G_a = w_a mu_a^2 P_a, with a tensor that does
 * not depend on f; it is built once, over unordered pairs a <= b of interior
 * nodes (n_pairs = n_i^d (n_i^d + 1) / 2 rows of N^d entries), and each call
 * forms the pair products G_a G_b of its cells and multiplies them by the
 * tensor on the FP64 matrix cores.  The result is the same discrete sum the
 * plan's fast path approximates, with no transform tolerance.
 * ------------------------------------------------------------------------- */
typedef struct pgc_direct_s* pgc_direct;

typedef struct pgc_direct_info {
    int64_t n_pairs;          /* tensor rows */
    int64_t n_modes_total;    /* N^d, tensor columns */
    int32_t max_cells;        /* cells per product (the chunk of a call) */
    int64_t tensor_bytes;
    int64_t workspace_bytes;  /* tensor, pair products of max_cells cells, synthesis buffers */
    double setup_ms;          /* device time of the tensor build */
    double flops_per_cell;    /* 2 n_pairs N^d: the product's share of one cell */
} pgc_direct_info;

/* Build the tensor of `plan` (FP64 plans only) and the workspace for
 * max_cells (1..65535) cells per product; synchronises `stream`.  The plan
 * must outlive the object.  Calls on one object share its workspace and must
 * not overlap; separate objects are independent.  UNSUPPORTED for FP32
 * plans, N^d > 4096, or a tensor above 96 GiB (2D N <= 55, 3D N <= 15 fit). */
pgc_status pgc_direct_create(pgc_plan plan, int32_t max_cells, void* stream, pgc_direct* out);
pgc_status pgc_direct_destroy(pgc_direct d);
pgc_status pgc_direct_query(pgc_direct d, pgc_direct_info* info);
/* q_dev[c][k] = Q_k of the coefficients coeffs_dev[c][k] (FP64, row-major
 * k_d fastest, n_cells x N^d each), max_cells at a time; stream-ordered.
 * The library allocates nothing here: the product is the library's own FP64
 * matrix-core kernel, whose split-K partial tiles live in the object's
 * workspace (sized at creation for every chunk up to max_cells); its
 * summation order is fixed, so a result repeats bit for bit. */
pgc_status pgc_direct_coeffs_to_q(pgc_direct d, const double* coeffs_dev, int64_t n_cells, double* q_dev,
                                  void* stream);
/* Record pgc_direct_coeffs_to_q for these pointers and n_cells into a HIP
 * graph owned by the object (replacing any earlier one).  One eager
 * evaluation runs first on `stream` (it writes q_dev), then the capture, on a
 * private stream.  Eager calls of any size may run between replays: the graph
 * and they share only the object's fixed workspace, used in stream order.
 * pgc_direct_graph_launch replays it on `stream` (INVALID_ARG without a
 * graph).  The graph reads the captured pointers: refill the same input
 * buffer between replays. */
pgc_status pgc_direct_capture(pgc_direct d, const double* coeffs_dev, int64_t n_cells, double* q_dev, void* stream);
pgc_status pgc_direct_graph_launch(pgc_direct d, void* stream);
/* n_steps classical RK4 steps (eq. spectral_ODE) of dc/dt = Q(c) for every
 * cell, in place on coeffs_dev (FP64, n_cells x N^d), max_cells at a time,
 * each chunk taking all its steps in turn; the stage state lives in the
 * object.  Stream-ordered, like pgc_direct_coeffs_to_q. */
pgc_status pgc_direct_rk4(pgc_direct d, double* coeffs_dev, int64_t n_cells, double dt, int32_t n_steps,
                          void* stream);

/* ---------------------------------------------------------------------------
 * Spatial transport and the split step (Sec. 1: the full equation adds the
 * free-streaming term v . grad_x f, and splitting treats transport and
 * collisions separately).  One periodic space dimension x along the first
 * velocity component, n_x (odd) equispaced cells on [0, length), every cell
 * holding the N^d coefficients of one plan (FP64, cell-major:
 * coeffs_dev[c * N^d + k]).  Testing f_t + v_1 f_x = 0 against T^_k gives
 * d/dt f_k + sum_l V_kl d/dx f_l = 0 on the first coefficient index, with
 * V_kl = (v_1 T~_l, T^_k), finite for the logarithmic map only: for the
 * closed form and the method see the comment of pgc_transport.hip.  Each
 * step moves the characteristic variables of V exactly over dt on the
 * trigonometric interpolant of the cells.
 * ------------------------------------------------------------------------- */
typedef struct pgc_transport_s* pgc_transport;

typedef struct pgc_transport_info {
    int32_t n_x, dim, n_modes;
    double length, dt;
    double max_speed;         /* largest |eigenvalue| of V (the fastest characteristic) */
    int64_t workspace_bytes;
} pgc_transport_info;

/* Build the transport over dt for the cells of `plan` (LOG map only:
 * UNSUPPORTED otherwise); synchronises `stream`.  INVALID_ARG for n_x even or
 * outside 1..4095, length <= 0, a non-finite dt.  The plan must outlive the
 * object. */
pgc_status pgc_transport_create(pgc_plan plan, int32_t n_x, double length, double dt, void* stream,
                                pgc_transport* out);
pgc_status pgc_transport_destroy(pgc_transport t);
/* Resolved parameters; speeds_host (may be NULL) receives the N
 * characteristic speeds (eigenvalues of V). */
pgc_status pgc_transport_query(pgc_transport t, pgc_transport_info* info, double* speeds_host);
/* One transport step over dt, in place on coeffs_dev (n_x x N^d FP64);
 * stream-ordered, allocates nothing. */
pgc_status pgc_transport_step(pgc_transport t, double* coeffs_dev, void* stream);
/* n_steps Strang steps of the full equation: transport over dt/2, one
 * classical RK4 step of d f/dt = Q(f) in every cell over dt, transport over
 * dt/2, where `half` is a transport built with dt/2.  The collisions run
 * through `direct` (all cells in one product per stage) when it is not NULL,
 * else cell by cell through pgc_rk4 of `plan` (which must be half's plan).
 * Stream-ordered; INVALID_ARG for mismatched objects. */
pgc_status pgc_split_step(pgc_transport half, pgc_plan plan, pgc_direct direct, double* coeffs_dev,
                          int32_t n_steps, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PGC_H */
