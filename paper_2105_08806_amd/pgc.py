"""Thin Python binding of the C ABI in include/pgc.h.

Argument marshalling only: every step of the collision path runs in the HIP
kernels of ``libpgc.so``.  torch tensors supply device memory and the current
stream; nothing here computes.  If the library is missing the import of this
module fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpgc.so")

MAP_LOG, MAP_ALGEBRAIC = 0, 1
SCALE_DIRECT, SCALE_FROM_DOMAIN = 0, 1
KERNEL_MAXWELL, KERNEL_VHS, KERNEL_ANISO = 0, 1, 2
SPHERE_UNIFORM_2D, SPHERE_PRODUCT_3D, SPHERE_USER = 0, 1, 2
FP64, FP32 = 0, 1
GAIN_AUTO, GAIN_SLAB, GAIN_BINNED, GAIN_MFMA = 0, 1, 2, 3

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported configuration", 3: "out of device memory",
          4: "device error", 5: "non-finite result",
          6: "the call needs more scratch memory than the static buffer holds"}


class PgcError(RuntimeError):
    def __init__(self, what, code):
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(code, "?"), code))
        self.code = code


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n_modes", ctypes.c_int32), ("m_v", ctypes.c_int32),
        ("map", ctypes.c_int32), ("scale_mode", ctypes.c_int32), ("scale", ctypes.c_double),
        ("kernel", ctypes.c_int32), ("kernel_b0", ctypes.c_double), ("kernel_gamma", ctypes.c_double),
        ("sphere", ctypes.c_int32), ("n_sigma", ctypes.c_int32), ("n_theta", ctypes.c_int32),
        ("n_phi", ctypes.c_int32),
        ("user_sigma_host", ctypes.POINTER(ctypes.c_double)),
        ("user_weights_host", ctypes.POINTER(ctypes.c_double)),
        ("precision", ctypes.c_int32), ("nufft_tol", ctypes.c_double), ("upsample", ctypes.c_double),
        ("kernel_width", ctypes.c_int32), ("slab_planes", ctypes.c_int32),
        ("n_chunks", ctypes.c_int32), ("block_threads", ctypes.c_int32),
        ("gain_mode", ctypes.c_int32),
        ("kernel_aniso", ctypes.c_double),
        ("deterministic", ctypes.c_int32),
        ("index_bytes", ctypes.c_int64),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n_modes", ctypes.c_int32), ("m_v", ctypes.c_int32),
        ("map", ctypes.c_int32), ("kernel", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n_sigma", ctypes.c_int32), ("scale", ctypes.c_double), ("grid_n", ctypes.c_int32),
        ("grid_folded", ctypes.c_int32), ("kernel_width", ctypes.c_int32),
        ("kernel_beta", ctypes.c_double), ("upsample", ctypes.c_double),
        ("slab_planes", ctypes.c_int32), ("n_slabs", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
        ("block_threads", ctypes.c_int32), ("n_triples", ctypes.c_int64),
        ("n_points", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
        ("gain_mode", ctypes.c_int32), ("n_bin_items", ctypes.c_int64),
        ("offset_fit_err", ctypes.c_double), ("deterministic", ctypes.c_int32),
        ("tile_bytes", ctypes.c_int64),
        ("index_chunks", ctypes.c_int32), ("index_bytes", ctypes.c_int64),
        ("velocity_fit_cells", ctypes.c_int32),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int32), ("n_groups", ctypes.c_int32),
        ("group_n_modes", ctypes.c_int32 * 8), ("group_cells", ctypes.c_int32 * 8),
        ("coeffs_total", ctypes.c_int64), ("kernel_width", ctypes.c_int32),
        ("cells_per_wave", ctypes.c_int32), ("waves", ctypes.c_int32), ("n_units", ctypes.c_int64),
        ("n_points", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
        ("tuned_ms", ctypes.c_double * 7), ("has_graph", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("spatial_order", ctypes.c_int32), ("order_ms", ctypes.c_double * 2),
        ("group_major", ctypes.c_int32), ("major_ms", ctypes.c_double * 2),
        ("deterministic", ctypes.c_int32),
    ]


class DirectInfo(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_int64), ("n_modes_total", ctypes.c_int64), ("max_cells", ctypes.c_int32),
        ("tensor_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64), ("setup_ms", ctypes.c_double),
        ("flops_per_cell", ctypes.c_double),
    ]


class TransportInfo(ctypes.Structure):
    _fields_ = [
        ("n_x", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_modes", ctypes.c_int32),
        ("length", ctypes.c_double), ("dt", ctypes.c_double), ("max_speed", ctypes.c_double),
        ("workspace_bytes", ctypes.c_int64),
    ]


class SurrogateDesc(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("n_layers", ctypes.c_int32), ("batch_max", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("gate_residual", ctypes.c_double), ("gate_raw_factor", ctypes.c_double),
        ("judge_stride", ctypes.c_int32), ("judge_tol", ctypes.c_double),
        ("norm_floor_in", ctypes.c_double), ("norm_floor_out", ctypes.c_double),
        ("loss_relative", ctypes.c_int32),
    ]


class SurrogateInfo(ctypes.Structure):
    _fields_ = [
        ("n_features", ctypes.c_int32), ("width", ctypes.c_int32), ("n_layers", ctypes.c_int32),
        ("batch_max", ctypes.c_int32), ("n_params", ctypes.c_int64), ("n_constraints", ctypes.c_int32),
        ("steps", ctypes.c_int64), ("raw_residual_calibrated", ctypes.c_double),
        ("workspace_bytes", ctypes.c_int64), ("zscore_calibrated", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load libpgc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpgc.so is not built: run python -m paper_2105_08806_amd.build "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        L.pgc_status_string.restype = ctypes.c_char_p
        L.pgc_status_string.argtypes = [ctypes.c_int]
        L.pgc_desc_init.argtypes = [ctypes.POINTER(PlanDesc)]
        L.pgc_nufft_params.argtypes = [dbl, dbl, ctypes.POINTER(i32), dp]
        L.pgc_plan_create.argtypes = [ctypes.POINTER(PlanDesc), vp, ctypes.POINTER(vp)]
        L.pgc_plan_destroy.argtypes = [vp]
        L.pgc_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.pgc_nodes.argtypes = [vp, dp, dp, dp]
        L.pgc_project.argtypes = [vp, vp, vp, vp]
        L.pgc_coeffs_to_q.argtypes = [vp, vp, vp, vp, vp]
        L.pgc_coeffs_to_q_static.argtypes = [vp, vp, vp, vp, vp]
        L.pgc_rk4.argtypes = [vp, vp, dbl, i32, vp]
        L.pgc_plan_capture.argtypes = [vp, vp, vp, vp, vp]
        L.pgc_plan_capture_rk4.argtypes = [vp, vp, dbl, i32, vp]
        L.pgc_plan_graph_launch.argtypes = [vp, vp]
        L.pgc_moments.argtypes = [vp, vp, vp, vp]
        L.pgc_eval.argtypes = [vp, vp, vp, i64, vp, vp]
        L.pgc_set_profiling.argtypes = [vp, i32]
        L.pgc_stage_times.argtypes = [vp, dp, i32, ctypes.POINTER(i64)]
        L.pgc_batch_create.argtypes = [ctypes.POINTER(PlanDesc), i32, ctypes.POINTER(i32), i32, vp,
                                       ctypes.POINTER(vp)]
        L.pgc_batch_destroy.argtypes = [vp]
        L.pgc_batch_query.argtypes = [vp, ctypes.POINTER(BatchInfo)]
        L.pgc_batch_offsets.argtypes = [vp, ctypes.POINTER(i64)]
        L.pgc_batch_set_tile.argtypes = [vp, i32, vp]
        L.pgc_batch_autotune.argtypes = [vp, vp]
        L.pgc_batch_set_order.argtypes = [vp, i32, i32, vp]
        L.pgc_batch_coeffs_to_q.argtypes = [vp, vp, vp, vp, vp]
        L.pgc_batch_capture.argtypes = [vp, vp, vp, vp, vp]
        L.pgc_batch_graph_launch.argtypes = [vp, vp]
        u64 = ctypes.c_uint64
        L.pgc_surrogate_desc_init.argtypes = [ctypes.POINTER(SurrogateDesc)]
        L.pgc_surrogate_create.argtypes = [vp, ctypes.POINTER(SurrogateDesc), vp, ctypes.POINTER(vp)]
        L.pgc_surrogate_destroy.argtypes = [vp]
        L.pgc_surrogate_query.argtypes = [vp, ctypes.POINTER(SurrogateInfo)]
        L.pgc_surrogate_set_normalization.argtypes = [vp, vp, vp, i64, vp]
        L.pgc_surrogate_train.argtypes = [vp, vp, vp, i64, i32, i32, dbl, u64, dp, vp]
        L.pgc_surrogate_coeffs_to_q.argtypes = [vp, vp, i64, vp, ctypes.POINTER(i32), ctypes.POINTER(i64), dp, vp]
        L.pgc_surrogate_loss_grad.argtypes = [vp, vp, vp, i32, dp, ctypes.POINTER(ctypes.c_float), vp]
        L.pgc_surrogate_get_params.argtypes = [vp, ctypes.POINTER(ctypes.c_float), vp]
        L.pgc_surrogate_set_params.argtypes = [vp, ctypes.POINTER(ctypes.c_float), vp]
        L.pgc_surrogate_save.argtypes = [vp, ctypes.c_char_p, vp]
        L.pgc_surrogate_load.argtypes = [vp, ctypes.c_char_p, vp]
        L.pgc_gemm_bf16.argtypes = [i32, i32, i32, vp, i32, i32, vp, i32, i32, vp, i32, vp, i32, vp]
        L.pgc_direct_create.argtypes = [vp, i32, vp, ctypes.POINTER(vp)]
        L.pgc_direct_destroy.argtypes = [vp]
        L.pgc_direct_query.argtypes = [vp, ctypes.POINTER(DirectInfo)]
        L.pgc_direct_coeffs_to_q.argtypes = [vp, vp, i64, vp, vp]
        L.pgc_direct_rk4.argtypes = [vp, vp, i64, dbl, i32, vp]
        L.pgc_direct_capture.argtypes = [vp, vp, i64, vp, vp]
        L.pgc_direct_graph_launch.argtypes = [vp, vp]
        L.pgc_transport_create.argtypes = [vp, i32, dbl, dbl, vp, ctypes.POINTER(vp)]
        L.pgc_transport_destroy.argtypes = [vp]
        L.pgc_transport_query.argtypes = [vp, ctypes.POINTER(TransportInfo), dp]
        L.pgc_transport_step.argtypes = [vp, vp, vp]
        L.pgc_split_step.argtypes = [vp, vp, vp, vp, i32, vp]
        for name in ("pgc_transport_create", "pgc_transport_destroy", "pgc_transport_query",
                     "pgc_transport_step", "pgc_split_step"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("pgc_direct_create", "pgc_direct_destroy", "pgc_direct_query", "pgc_direct_coeffs_to_q",
                     "pgc_direct_rk4", "pgc_direct_capture", "pgc_direct_graph_launch"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("pgc_surrogate_desc_init", "pgc_surrogate_create", "pgc_surrogate_destroy",
                     "pgc_surrogate_query", "pgc_surrogate_set_normalization", "pgc_surrogate_train",
                     "pgc_surrogate_coeffs_to_q", "pgc_surrogate_loss_grad", "pgc_surrogate_get_params",
                     "pgc_surrogate_set_params", "pgc_surrogate_save", "pgc_surrogate_load", "pgc_gemm_bf16"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("pgc_desc_init", "pgc_nufft_params", "pgc_plan_create", "pgc_plan_destroy",
                     "pgc_plan_query", "pgc_nodes", "pgc_project", "pgc_coeffs_to_q",
                     "pgc_coeffs_to_q_static", "pgc_rk4",
                     "pgc_moments", "pgc_eval", "pgc_set_profiling", "pgc_stage_times",
                     "pgc_batch_create", "pgc_batch_destroy", "pgc_batch_query", "pgc_batch_offsets",
                     "pgc_batch_set_tile", "pgc_batch_set_order", "pgc_batch_autotune", "pgc_batch_coeffs_to_q",
                     "pgc_batch_capture", "pgc_batch_graph_launch"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code, what):
    if code != 0:
        raise PgcError(what, code)


def nufft_params(tol, upsample=2.0):
    w = ctypes.c_int32(0)
    b = ctypes.c_double(0.0)
    _check(lib().pgc_nufft_params(tol, upsample, ctypes.byref(w), ctypes.byref(b)), "pgc_nufft_params")
    return w.value, b.value


def default_desc() -> PlanDesc:
    d = PlanDesc()
    _check(lib().pgc_desc_init(ctypes.byref(d)), "pgc_desc_init")
    return d


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _desc_from(fields, sigma=None, sigma_w=None, keep=None):
    d = default_desc()
    for k, v in fields.items():
        if not hasattr(d, k):
            raise TypeError("unknown plan field %r" % k)
        setattr(d, k, v)
    if sigma is not None:
        s = np.ascontiguousarray(sigma, dtype=np.float64)
        w = np.ascontiguousarray(sigma_w, dtype=np.float64)
        keep += [s, w]
        d.sphere = SPHERE_USER
        d.n_sigma = int(w.size)
        d.user_sigma_host = s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.user_weights_host = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d


class Plan:
    """One collision operator on the current GPU.

    Keyword arguments are pgc_plan_desc fields (dim, n_modes, scale, map, kernel,
    kernel_b0, kernel_gamma, sphere, n_sigma, n_theta, n_phi, precision, ...);
    ``sigma``/``sigma_w`` give a user sphere rule.
    """

    def __init__(self, sigma=None, sigma_w=None, **fields):
        import torch
        self._torch = torch
        self._keep = []
        d = _desc_from(fields, sigma, sigma_w, self._keep)
        self.desc = d
        h = ctypes.c_void_p()
        _check(lib().pgc_plan_create(ctypes.byref(d), _stream(), ctypes.byref(h)), "pgc_plan_create")
        self._h = h
        self.info = PlanInfo()
        _check(lib().pgc_plan_query(self._h, ctypes.byref(self.info)), "pgc_plan_query")
        self.dim = self.info.dim
        self.n_modes = self.info.n_modes
        self.n_int = self.info.m_v - 2
        self.dtype = torch.float64 if self.info.precision == FP64 else torch.float32

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pgc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- shapes
    def shape(self):
        return (self.n_modes,) * self.dim

    def node_shape(self):
        return (self.n_int,) * self.dim

    def _coeffs(self, c):
        torch = self._torch
        if not (c.is_cuda and c.dtype == self.dtype and c.is_contiguous() and tuple(c.shape) == self.shape()):
            raise ValueError("coefficients must be a contiguous %s CUDA tensor of shape %s"
                             % (self.dtype, self.shape()))
        return c

    # ---------------------------------------------------------------- calls
    def nodes(self):
        m = self.info.m_v
        xi, v, w = (np.zeros(m) for _ in range(3))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().pgc_nodes(self._h, xi.ctypes.data_as(dp), v.ctypes.data_as(dp), w.ctypes.data_as(dp)),
               "pgc_nodes")
        return xi, v, w

    def interior_velocities(self):
        _, v, _ = self.nodes()
        vi = v[1:-1]
        g = np.meshgrid(*([vi] * self.dim), indexing="ij")
        return np.stack([a.ravel() for a in g], axis=1)

    def project(self, f_nodes):
        torch = self._torch
        f = torch.as_tensor(f_nodes, dtype=torch.float64).reshape(self.node_shape()).contiguous().cuda()
        out = torch.empty(self.shape(), dtype=self.dtype, device=f.device)
        _check(lib().pgc_project(self._h, _ptr(f), _ptr(out), _stream()), "pgc_project")
        return out

    def coeffs_to_q(self, coeffs, q=None, qplus=None, want_qplus=False):
        torch = self._torch
        c = self._coeffs(coeffs)
        if q is None:
            q = torch.empty_like(c)
        if want_qplus and qplus is None:
            qplus = torch.empty_like(c)
        _check(lib().pgc_coeffs_to_q(self._h, _ptr(c), _ptr(q), _ptr(qplus) if qplus is not None else None,
                                     _stream()), "pgc_coeffs_to_q")
        return (q, qplus) if want_qplus else q

    def coeffs_to_q_static(self, coeffs, q=None, qplus=None, want_qplus=False):
        """pgc_coeffs_to_q_static: the same evaluation with the library's static
        scratch array in place of the plan's per-call buffers."""
        torch = self._torch
        c = self._coeffs(coeffs)
        if q is None:
            q = torch.empty_like(c)
        if want_qplus and qplus is None:
            qplus = torch.empty_like(c)
        _check(lib().pgc_coeffs_to_q_static(self._h, _ptr(c), _ptr(q),
                                            _ptr(qplus) if qplus is not None else None, _stream()),
               "pgc_coeffs_to_q_static")
        return (q, qplus) if want_qplus else q

    def rk4(self, coeffs, dt, n_steps):
        """In place on a float64 CUDA tensor of shape N^dim."""
        torch = self._torch
        if not (coeffs.is_cuda and coeffs.dtype == torch.float64 and coeffs.is_contiguous()):
            raise ValueError("rk4 state must be a contiguous float64 CUDA tensor")
        _check(lib().pgc_rk4(self._h, _ptr(coeffs), float(dt), int(n_steps), _stream()), "pgc_rk4")
        return coeffs

    def capture(self, coeffs, q=None, qplus=None, want_qplus=False):
        """pgc_plan_capture: one evaluation of these buffers, then its HIP graph,
        which graph_launch replays.  The graph reads coeffs and writes q (and
        qplus) in place: refill coeffs between replays."""
        torch = self._torch
        c = self._coeffs(coeffs)
        if q is None:
            q = torch.empty_like(c)
        if want_qplus and qplus is None:
            qplus = torch.empty_like(c)
        _check(lib().pgc_plan_capture(self._h, _ptr(c), _ptr(q), _ptr(qplus) if qplus is not None else None,
                                      _stream()), "pgc_plan_capture")
        self._graph_io = (c, q, qplus)  # the graph reads and writes these buffers
        return (q, qplus) if want_qplus else q

    def capture_rk4(self, coeffs, dt, n_steps):
        """pgc_plan_capture_rk4: the graph of n_steps RK4 steps in place on a
        float64 CUDA tensor of shape N^dim (nothing runs until graph_launch)."""
        torch = self._torch
        if not (coeffs.is_cuda and coeffs.dtype == torch.float64 and coeffs.is_contiguous()):
            raise ValueError("rk4 state must be a contiguous float64 CUDA tensor")
        _check(lib().pgc_plan_capture_rk4(self._h, _ptr(coeffs), float(dt), int(n_steps), _stream()),
               "pgc_plan_capture_rk4")
        self._graph_io = (coeffs,)

    def graph_launch(self):
        _check(lib().pgc_plan_graph_launch(self._h, _stream()), "pgc_plan_graph_launch")

    def moments(self, coeffs):
        torch = self._torch
        c = self._coeffs(coeffs)
        out = torch.empty(self.dim + 2, dtype=torch.float64, device=c.device)
        _check(lib().pgc_moments(self._h, _ptr(c), _ptr(out), _stream()), "pgc_moments")
        return out

    STAGES = ("synthesis", "loss", "orbit_sums", "spread", "grid_to_modes", "combine")

    def set_profiling(self, on=True):
        _check(lib().pgc_set_profiling(self._h, 1 if on else 0), "pgc_set_profiling")

    def stage_times(self):
        """Accumulated ms per stage since the last call, and the number of timed calls."""
        ms = np.zeros(len(self.STAGES))
        calls = ctypes.c_int64(0)
        _check(lib().pgc_stage_times(self._h, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     len(self.STAGES), ctypes.byref(calls)), "pgc_stage_times")
        return dict(zip(self.STAGES, ms.tolist())), int(calls.value)

    def eval(self, coeffs, v):
        torch = self._torch
        c = self._coeffs(coeffs)
        vv = torch.as_tensor(v, dtype=torch.float64).reshape(-1, self.dim).contiguous().to(c.device)
        out = torch.empty(vv.shape[0], dtype=torch.float64, device=c.device)
        _check(lib().pgc_eval(self._h, _ptr(c), _ptr(vv), int(vv.shape[0]), _ptr(out), _stream()),
               "pgc_eval")
        return out


class Batch:
    """Q for many 2D velocity cells with mixed N in one batched evaluation (FP32).

    ``n_modes`` lists the N of every cell; keyword arguments are the shared
    pgc_plan_desc fields (precision defaults to FP32, the only one supported).
    Packed arrays hold the cells' N^2 coefficient blocks at ``offsets``.
    """

    def __init__(self, n_modes, autotune=True, sigma=None, sigma_w=None, **fields):
        import torch
        self._torch = torch
        fields.setdefault("dim", 2)
        fields.setdefault("precision", FP32)
        self._keep = []
        d = _desc_from(fields, sigma, sigma_w, self._keep)
        self.desc = d
        nm = np.ascontiguousarray(n_modes, dtype=np.int32)
        self.n_modes = nm.copy()
        h = ctypes.c_void_p()
        _check(lib().pgc_batch_create(ctypes.byref(d), int(nm.size),
                                      nm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      1 if autotune else 0, _stream(), ctypes.byref(h)), "pgc_batch_create")
        self._h = h
        self.refresh_info()
        off = np.zeros(nm.size, dtype=np.int64)
        _check(lib().pgc_batch_offsets(self._h, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
               "pgc_batch_offsets")
        self.offsets = off
        self.total = int(self.info.coeffs_total)

    def refresh_info(self):
        self.info = BatchInfo()
        _check(lib().pgc_batch_query(self._h, ctypes.byref(self.info)), "pgc_batch_query")
        return self.info

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pgc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _packed(self, x, name):
        torch = self._torch
        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 1):
            raise ValueError("%s must be a contiguous 1-D float32 CUDA tensor" % name)
        return x

    def pack(self, blocks):
        """Dense packing of a list of per-cell N^2 arrays (host) into one CUDA tensor."""
        torch = self._torch
        flat = np.concatenate([np.asarray(b, dtype=np.float32).reshape(-1) for b in blocks])
        if flat.size != self.total:
            raise ValueError("blocks hold %d values, the batch packs %d" % (flat.size, self.total))
        return torch.tensor(flat, device="cuda")

    def unpack(self, packed):
        """Per-cell N x N float64 host arrays of a dense packed tensor."""
        x = packed.double().cpu().numpy()
        return [x[o:o + n * n].reshape(n, n) for o, n in zip(self.offsets, self.n_modes)]

    def set_tile(self, cells_per_wave):
        _check(lib().pgc_batch_set_tile(self._h, int(cells_per_wave), _stream()), "pgc_batch_set_tile")
        self.refresh_info()

    def set_order(self, raster, group_major):
        _check(lib().pgc_batch_set_order(self._h, int(raster), int(group_major), _stream()), "pgc_batch_set_order")
        self.refresh_info()

    def autotune(self):
        _check(lib().pgc_batch_autotune(self._h, _stream()), "pgc_batch_autotune")
        self.refresh_info()

    def coeffs_to_q(self, packed, q=None, offsets=None):
        torch = self._torch
        c = self._packed(packed, "packed coefficients")
        if q is None:
            q = torch.empty_like(c)
        self._packed(q, "packed q")
        _check(lib().pgc_batch_coeffs_to_q(self._h, _ptr(c), _ptr(offsets) if offsets is not None else None,
                                           _ptr(q), _stream()), "pgc_batch_coeffs_to_q")
        return q

    def capture(self, packed, q, offsets=None):
        self._packed(packed, "packed coefficients")
        self._packed(q, "packed q")
        _check(lib().pgc_batch_capture(self._h, _ptr(packed), _ptr(offsets) if offsets is not None else None,
                                       _ptr(q), _stream()), "pgc_batch_capture")
        self._graph_io = (packed, q, offsets)  # the graph reads these buffers
        self.refresh_info()

    def graph_launch(self):
        _check(lib().pgc_batch_graph_launch(self._h, _stream()), "pgc_batch_graph_launch")


def gemm_bf16(a, b, trans_a=False, trans_b=False, bias=None, out=None, accumulate=False):
    """C = op(a) op(b) (+ bias) on the matrix cores; a, b are torch.bfloat16 CUDA matrices."""
    import torch
    if a.dtype != torch.bfloat16 or b.dtype != torch.bfloat16:
        raise ValueError("a and b must be bfloat16")
    a, b = a.contiguous(), b.contiguous()
    M = a.shape[1] if trans_a else a.shape[0]
    K = a.shape[0] if trans_a else a.shape[1]
    N = b.shape[0] if trans_b else b.shape[1]
    Kb = b.shape[1] if trans_b else b.shape[0]
    if K != Kb:
        raise ValueError("inner dimensions differ")
    if out is None:
        out = torch.zeros(M, N, dtype=torch.float32, device=a.device)
    if tuple(out.shape) != (M, N) or out.dtype != torch.float32 or (N > 1 and out.stride(1) != 1):
        raise ValueError("out must be a float32 (M, N) matrix with unit column stride")
    if bias is not None and (tuple(bias.shape) != (N,) or bias.dtype != torch.float32 or not bias.is_contiguous()):
        raise ValueError("bias must be a contiguous float32 vector of length N")
    _check(lib().pgc_gemm_bf16(M, N, K, _ptr(a), a.shape[1], int(trans_a), _ptr(b), b.shape[1], int(trans_b),
                               _ptr(out), max(out.stride(0), N), _ptr(bias) if bias is not None else None,
                               int(accumulate), _stream()), "pgc_gemm_bf16")
    return out


class Direct:
    """The direct algorithm for many cells that share one FP64 plan: the
    plan's bilinear tensor is built once, then Q of a batch of cells is one
    FP64 matrix product (``max_cells`` cells per product)."""

    def __init__(self, plan, max_cells=256):
        import torch
        self._torch = torch
        self.plan = plan  # the tensor reads the plan's tables: keep it alive
        h = ctypes.c_void_p()
        _check(lib().pgc_direct_create(plan._h, int(max_cells), _stream(), ctypes.byref(h)), "pgc_direct_create")
        self._h = h
        self.info = DirectInfo()
        _check(lib().pgc_direct_query(self._h, ctypes.byref(self.info)), "pgc_direct_query")
        self.nd = int(self.info.n_modes_total)

    def coeffs_to_q(self, coeffs, q=None):
        """coeffs: float64 CUDA tensor (n_cells, N^d) or (n_cells, N, ..., N)."""
        torch = self._torch
        if not (coeffs.is_cuda and coeffs.dtype == torch.float64 and coeffs.is_contiguous()):
            raise ValueError("coefficients must be a contiguous float64 CUDA tensor")
        if coeffs.numel() % self.nd:
            raise ValueError("coefficients must hold whole cells of N^d values")
        n = coeffs.numel() // self.nd
        if q is None:
            q = torch.empty_like(coeffs)
        elif not (q.is_cuda and q.dtype == torch.float64 and q.is_contiguous() and q.numel() == coeffs.numel()):
            raise ValueError("q must be a contiguous float64 CUDA tensor of the coefficients' size")
        _check(lib().pgc_direct_coeffs_to_q(self._h, _ptr(coeffs), n, _ptr(q), _stream()), "pgc_direct_coeffs_to_q")
        return q

    def capture(self, coeffs, q):
        """Record Q of these cells into a HIP graph (runs one eager evaluation first)."""
        torch = self._torch
        for t in (coeffs, q):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("coefficients and q must be contiguous float64 CUDA tensors")
        if coeffs.numel() % self.nd or q.numel() != coeffs.numel():
            raise ValueError("coefficients and q must hold the same whole cells")
        _check(lib().pgc_direct_capture(self._h, _ptr(coeffs), coeffs.numel() // self.nd, _ptr(q), _stream()),
               "pgc_direct_capture")
        self._graph_io = (coeffs, q)  # the graph reads these buffers

    def graph_launch(self):
        _check(lib().pgc_direct_graph_launch(self._h, _stream()), "pgc_direct_graph_launch")

    def rk4(self, coeffs, dt, n_steps):
        """In place on a contiguous float64 CUDA tensor of whole cells."""
        torch = self._torch
        if not (coeffs.is_cuda and coeffs.dtype == torch.float64 and coeffs.is_contiguous()):
            raise ValueError("coefficients must be a contiguous float64 CUDA tensor")
        if coeffs.numel() % self.nd:
            raise ValueError("coefficients must hold whole cells of N^d values")
        _check(lib().pgc_direct_rk4(self._h, _ptr(coeffs), coeffs.numel() // self.nd, float(dt), int(n_steps),
                                    _stream()), "pgc_direct_rk4")
        return coeffs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pgc_direct_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Transport:
    """Free streaming along x over dt for n_x (odd) periodic cells of one
    plan's coefficients (pgc_transport_*), and the Strang split step."""

    def __init__(self, plan, n_x, length, dt):
        import torch
        self._torch = torch
        self.plan = plan
        h = ctypes.c_void_p()
        _check(lib().pgc_transport_create(plan._h, int(n_x), float(length), float(dt), _stream(), ctypes.byref(h)),
               "pgc_transport_create")
        self._h = h
        self.info = TransportInfo()
        _check(lib().pgc_transport_query(self._h, ctypes.byref(self.info), None), "pgc_transport_query")

    def speeds(self):
        out = np.zeros(self.info.n_modes)
        _check(lib().pgc_transport_query(self._h, None, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "pgc_transport_query")
        return out

    def _state(self, coeffs):
        torch = self._torch
        if not (coeffs.is_cuda and coeffs.dtype == torch.float64 and coeffs.is_contiguous()):
            raise ValueError("the state must be a contiguous float64 CUDA tensor")
        if coeffs.numel() != self.info.n_x * self.info.n_modes ** self.info.dim:
            raise ValueError("the state must hold n_x cells of N^d coefficients")

    def step(self, coeffs):
        """One transport step, in place."""
        self._state(coeffs)
        _check(lib().pgc_transport_step(self._h, _ptr(coeffs), _stream()), "pgc_transport_step")
        return coeffs

    def split_step(self, coeffs, n_steps=1, direct=None):
        """Strang steps over 2 dt (this object is the half-step transport):
        collisions cell by cell through the plan, or through ``direct``."""
        self._state(coeffs)
        _check(lib().pgc_split_step(self._h, None if direct is not None else self.plan._h,
                                    direct._h if direct is not None else None, _ptr(coeffs), int(n_steps),
                                    _stream()), "pgc_split_step")
        return coeffs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pgc_transport_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """Learned coefficients-to-Q map of an FP32 plan, with the plan as fallback and judge."""

    def __init__(self, plan, **fields):
        import torch
        self._torch = torch
        if plan.info.precision != FP32:
            raise ValueError("the surrogate needs an FP32 plan")
        self.plan = plan  # kept alive: the surrogate falls back to it
        d = SurrogateDesc()
        _check(lib().pgc_surrogate_desc_init(ctypes.byref(d)), "pgc_surrogate_desc_init")
        for k, v in fields.items():
            if not hasattr(d, k):
                raise TypeError("unknown surrogate field %r" % k)
            setattr(d, k, v)
        self.desc = d
        h = ctypes.c_void_p()
        _check(lib().pgc_surrogate_create(plan._h, ctypes.byref(d), _stream(), ctypes.byref(h)),
               "pgc_surrogate_create")
        self._h = h
        self.refresh_info()
        self.n = self.info.n_features

    def refresh_info(self):
        self.info = SurrogateInfo()
        _check(lib().pgc_surrogate_query(self._h, ctypes.byref(self.info)), "pgc_surrogate_query")
        return self.info

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pgc_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rows(self, x, name):
        torch = self._torch
        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 2
                and x.shape[1] == self.n):
            raise ValueError("%s must be a contiguous float32 CUDA tensor of shape (rows, %d)" % (name, self.n))
        return x

    def set_normalization(self, f, q):
        self._rows(f, "f")
        self._rows(q, "q")
        _check(lib().pgc_surrogate_set_normalization(self._h, _ptr(f), _ptr(q), f.shape[0], _stream()),
               "pgc_surrogate_set_normalization")

    def train(self, f, q, epochs, batch=None, lr=1e-3, seed=0):
        self._rows(f, "f")
        self._rows(q, "q")
        batch = batch or self.info.batch_max
        losses = np.zeros(max(1, epochs))
        _check(lib().pgc_surrogate_train(self._h, _ptr(f), _ptr(q), f.shape[0], int(epochs), int(batch),
                                         float(lr), int(seed),
                                         losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()),
               "pgc_surrogate_train")
        self.refresh_info()
        return losses[:epochs]

    def coeffs_to_q(self, f, q=None):
        """(q, fallback flags, number of fallbacks, largest judge error)."""
        torch = self._torch
        self._rows(f, "f")
        if q is None:
            q = torch.empty_like(f)
        flags = np.zeros(f.shape[0], dtype=np.int32)
        nfb = ctypes.c_int64(0)
        jerr = ctypes.c_double(0.0)
        _check(lib().pgc_surrogate_coeffs_to_q(self._h, _ptr(f), f.shape[0], _ptr(q),
                                               flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                               ctypes.byref(nfb), ctypes.byref(jerr), _stream()),
               "pgc_surrogate_coeffs_to_q")
        return q, flags, int(nfb.value), float(jerr.value)

    def loss_grad(self, f, q):
        self._rows(f, "f")
        self._rows(q, "q")
        g = np.zeros(self.info.n_params, dtype=np.float32)
        loss = ctypes.c_double(0.0)
        _check(lib().pgc_surrogate_loss_grad(self._h, _ptr(f), _ptr(q), f.shape[0], ctypes.byref(loss),
                                             g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream()),
               "pgc_surrogate_loss_grad")
        return loss.value, g

    def get_params(self):
        p = np.zeros(self.info.n_params + 4 * self.n, dtype=np.float32)
        _check(lib().pgc_surrogate_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream()),
               "pgc_surrogate_get_params")
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.info.n_params + 4 * self.n:
            raise ValueError("expected %d values" % (self.info.n_params + 4 * self.n))
        _check(lib().pgc_surrogate_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream()),
               "pgc_surrogate_set_params")

    def layer_dims(self):
        w, L, n = self.info.width, self.info.n_layers, self.n
        return [n] + [w] * (L - 1) + [n]

    def unflatten(self, p):
        """[(W, b), ...] and (mu_in, sd_in, mu_out, sd_out) from a flat parameter vector."""
        dims = self.layer_dims()
        out, off = [], 0
        for i, o in zip(dims[:-1], dims[1:]):
            W = p[off:off + i * o].reshape(o, i)
            off += i * o
            b = p[off:off + o]
            off += o
            out.append((W, b))
        norms = tuple(p[off + k * self.n: off + (k + 1) * self.n] for k in range(4))
        return out, norms

    def save(self, path):
        _check(lib().pgc_surrogate_save(self._h, str(path).encode(), _stream()), "pgc_surrogate_save")

    def load(self, path):
        _check(lib().pgc_surrogate_load(self._h, str(path).encode(), _stream()), "pgc_surrogate_load")
        self.refresh_info()
