"""The C-ABI library loads and exports every entry point include/pgc.h declares.

CPU only: no call here touches a GPU (only host-only entry points are called).
"""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "pgc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pgc_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pgc_plan_create", "pgc_plan_destroy", "pgc_coeffs_to_q", "pgc_rk4", "pgc_project",
                 "pgc_moments", "pgc_eval", "pgc_nodes", "pgc_plan_query", "pgc_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2105_08806_amd import pgc
    L = pgc.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_entry_points():
    from paper_2105_08806_amd import pgc
    L = pgc.lib()
    assert L.pgc_status_string(0) == b"ok"
    assert L.pgc_status_string(1) == b"invalid argument"
    d = pgc.default_desc()
    assert d.dim == 2 and d.n_modes == 16 and d.n_sigma == 16 and d.precision == pgc.FP64
    assert L.pgc_desc_init(None) == 1
    w64, b64 = pgc.nufft_params(1e-12)
    w32, b32 = pgc.nufft_params(1e-6)
    assert 10 <= w64 <= 14 and 5 <= w32 <= 7
    assert abs(b64 - 0.98 * 3.141592653589793 * w64 * 0.75) < 1e-12
    with pytest.raises(pgc.PgcError):
        pgc.nufft_params(-1.0)
    with pytest.raises(pgc.PgcError):
        pgc.nufft_params(1e-6, upsample=8.0)
    # larger upsampling never needs a wider kernel
    assert pgc.nufft_params(1e-10, 3.0)[0] <= pgc.nufft_params(1e-10, 2.0)[0] + 1


def test_null_plan_is_rejected_without_a_device():
    from paper_2105_08806_amd import pgc
    L = pgc.lib()
    assert L.pgc_plan_destroy(None) == 0
    assert L.pgc_plan_query(None, None) == 1
    assert L.pgc_coeffs_to_q(None, None, None, None, None) == 1
    assert L.pgc_coeffs_to_q_static(None, None, None, None, None) == 1
    assert L.pgc_status_string(6).startswith(b"the call needs more scratch")
    assert L.pgc_rk4(None, None, 0.1, 1, None) == 1
    assert L.pgc_plan_capture(None, None, None, None, None) == 1
    assert L.pgc_plan_capture_rk4(None, None, 0.1, 1, None) == 1
    assert L.pgc_plan_graph_launch(None, None) == 1
    out = ctypes.c_void_p()
    assert L.pgc_plan_create(None, None, ctypes.byref(out)) == 1


def test_oracle_and_library_share_no_code():
    """The oracle sources never include or load the GPU library and vice versa."""
    osrc = open(os.path.join(ROOT, "oracle", "pgc_oracle.c")).read()
    opy = open(os.path.join(ROOT, "oracle", "__init__.py")).read()
    assert "pgc.h" not in osrc and "paper_2105_08806_amd" not in opy
    csrc = os.path.join(ROOT, "paper_2105_08806_amd", "csrc")
    for f in os.listdir(csrc):
        assert "oracle" not in open(os.path.join(csrc, f)).read().lower()
    for f in ("pgc.py", "build.py", "inputs.py", "__init__.py"):
        src = open(os.path.join(ROOT, "paper_2105_08806_amd", f)).read()
        assert "import oracle" not in src and "from oracle" not in src


def test_batch_argument_errors_without_a_device():
    """Batch entry points reject bad arguments before any device work."""
    from paper_2105_08806_amd import pgc
    L = pgc.lib()
    assert L.pgc_batch_destroy(None) == 0
    info = pgc.BatchInfo()
    assert L.pgc_batch_query(None, ctypes.byref(info)) == 1
    assert L.pgc_batch_graph_launch(None, None) == 1
    assert L.pgc_batch_coeffs_to_q(None, None, None, None, None) == 1
    d = pgc.default_desc()
    d.precision = pgc.FP32
    modes = (ctypes.c_int32 * 3)(8, 8, 10)
    h = ctypes.c_void_p()
    assert L.pgc_batch_create(ctypes.byref(d), 0, modes, 0, None, ctypes.byref(h)) == 1
    assert L.pgc_batch_create(ctypes.byref(d), 3, None, 0, None, ctypes.byref(h)) == 1
    d3 = pgc.default_desc()
    d3.dim, d3.precision = 3, pgc.FP32
    assert L.pgc_batch_create(ctypes.byref(d3), 3, modes, 0, None, ctypes.byref(h)) == 2
    d64 = pgc.default_desc()   # FP64 batches are not built
    assert L.pgc_batch_create(ctypes.byref(d64), 3, modes, 0, None, ctypes.byref(h)) == 2
    assert not h.value


def _create_status(pgc, L, **fields):
    d = pgc.default_desc()
    for k, v in fields.items():
        setattr(d, k, v)
    h = ctypes.c_void_p()
    st = L.pgc_plan_create(ctypes.byref(d), None, ctypes.byref(h))
    assert not h.value  # a rejected descriptor leaves no plan behind
    return st


def test_plan_descriptor_rejections_without_a_device():
    """Descriptor validation runs on the host before any device call: every
    out-of-range field is an argument error, and the combinations the kernels
    do not cover are unsupported."""
    from paper_2105_08806_amd import pgc
    L = pgc.lib()
    bad = [dict(dim=1), dict(dim=4), dict(n_modes=2), dict(m_v=2), dict(map=7), dict(scale=0.0),
           dict(scale=float("inf")), dict(scale=float("nan")), dict(scale_mode=5), dict(kernel=9),
           dict(kernel=pgc.KERNEL_VHS, kernel_gamma=1.5), dict(kernel=pgc.KERNEL_VHS, kernel_gamma=-0.1),
           dict(kernel_b0=-1.0), dict(precision=3),
           dict(kernel=pgc.KERNEL_ANISO, kernel_aniso=-1.5), dict(kernel=pgc.KERNEL_ANISO, kernel_aniso=11.0),
           dict(kernel=pgc.KERNEL_ANISO, kernel_gamma=2.0), dict(kernel=3), dict(nufft_tol=-1e-6), dict(upsample=1.2),
           dict(upsample=5.0), dict(kernel_width=3), dict(kernel_width=99), dict(slab_planes=-1),
           dict(n_chunks=-2), dict(block_threads=300), dict(gain_mode=4), dict(gain_mode=-1),
           dict(deterministic=2), dict(deterministic=-1), dict(index_bytes=-1),
           dict(n_sigma=7),                                  # a circle rule needs antipodal pairs
           dict(n_sigma=0), dict(sphere=9),
           dict(dim=3),                                      # the circle rule is a 2D rule
           dict(dim=3, sphere=pgc.SPHERE_PRODUCT_3D, n_theta=4, n_phi=5),
           dict(dim=3, sphere=pgc.SPHERE_PRODUCT_3D, n_theta=0, n_phi=8),
           dict(sphere=pgc.SPHERE_USER, n_sigma=4)]          # user rule without its arrays
    for fields in bad:
        assert _create_status(pgc, L, **fields) == 1, fields
    # user rules: unit vectors with positive weights in antipodal pairs
    def user(sig, wts):
        s = np.ascontiguousarray(sig, dtype=np.float64)
        w = np.ascontiguousarray(wts, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        return _create_status(pgc, L, sphere=pgc.SPHERE_USER, n_sigma=len(w),
                              user_sigma_host=s.ctypes.data_as(dp), user_weights_host=w.ctypes.data_as(dp))
    assert user([[1, 0], [0, 1]], [1.0, 1.0]) == 1                   # not antipodal
    assert user([[1, 0], [-1, 0]], [1.0, 2.0]) == 1                  # opposite weights differ
    assert user([[2, 0], [-2, 0]], [1.0, 1.0]) == 1                  # not unit vectors
    assert user([[1, 0], [-1, 0]], [1.0, 0.0]) == 1                  # zero weight
    assert user([[np.nan, 0], [-1, 0]], [1.0, 1.0]) == 1             # not finite
    # the matrix-core gain covers FP64 3D plans only; an explicit binned mode
    # beyond the binned scheme's node limit is refused rather than replaced
    assert _create_status(pgc, L, gain_mode=3) == 2
    assert _create_status(pgc, L, gain_mode=2, n_modes=300) == 2
    # the fixed-order tile gather and an angle-dependent rate need the binned
    # vector gain: refused with the slab and matrix-core schemes
    assert _create_status(pgc, L, deterministic=1, gain_mode=1) == 2
    assert _create_status(pgc, L, deterministic=1, gain_mode=3, dim=3, sphere=pgc.SPHERE_PRODUCT_3D,
                          n_theta=2, n_phi=4) == 2
    assert _create_status(pgc, L, kernel=pgc.KERNEL_ANISO, kernel_aniso=0.5, gain_mode=1) == 2
    # the fixed-order gather needs the whole point index, not a streamed one
    assert _create_status(pgc, L, deterministic=1, index_bytes=1) == 2


def test_gemm_argument_errors_without_a_device():
    """The BF16 product rejects negative sizes, missing operands and row
    strides shorter than their rows before it launches anything (the pointers
    here are never dereferenced)."""
    from paper_2105_08806_amd import pgc
    L = pgc.lib()
    fake = ctypes.c_void_p(0x1000)

    def call(M, N, K, lda, ta, ldb, tb, ldc, a=fake, b=fake, c=fake):
        return L.pgc_gemm_bf16(M, N, K, a, lda, ta, b, ldb, tb, c, ldc, None, 0, None)
    assert call(-1, 4, 4, 4, 0, 4, 0, 4) == 1
    assert call(4, 4, -1, 4, 0, 4, 0, 4) == 1
    assert call(8, 6, 5, 4, 0, 6, 0, 6) == 1       # lda < K
    assert call(8, 6, 5, 5, 1, 6, 0, 6) == 1       # transposed A: lda < M
    assert call(8, 6, 5, 5, 0, 5, 0, 6) == 1       # ldb < N
    assert call(8, 6, 5, 5, 0, 4, 1, 6) == 1       # transposed B: ldb < K
    assert call(8, 6, 5, 5, 0, 6, 0, 5) == 1       # ldc < N
    assert call(8, 6, 5, 5, 0, 6, 0, 6, a=None) == 1
    assert call(8, 6, 5, 5, 0, 6, 0, 6, c=None) == 1
    # empty outputs need no operands at all
    assert call(0, 6, 5, 0, 0, 0, 0, 0, a=None, b=None, c=None) == 0


def test_direct_argument_errors_without_a_device():
    from paper_2105_08806_amd import pgc
    L = pgc.lib()
    h = ctypes.c_void_p()
    assert L.pgc_direct_create(None, 4, None, ctypes.byref(h)) == 1
    assert not h.value
    assert L.pgc_direct_destroy(None) == 0
    info = pgc.DirectInfo()
    assert L.pgc_direct_query(None, ctypes.byref(info)) == 1
    assert L.pgc_direct_coeffs_to_q(None, None, 0, None, None) == 1
    assert L.pgc_direct_rk4(None, None, 0, 0.1, 1, None) == 1
    assert L.pgc_direct_capture(None, None, 1, None, None) == 1
    assert L.pgc_direct_graph_launch(None, None) == 1
