"""The streamed point index (plan descriptor `index_bytes`).  When the whole
index of the binned gain (8 bytes per merged point) needs more than the budget,
the plan splits the directions into chunks whose ids fit it, keeps per chunk
only the point count of every bin, and every evaluation sorts each chunk's
points into bins again before spreading them (the on-the-fly evaluation of
Sec. 4.3 with a bounded buffer).  Parity against the oracle at the FP64 and
FP32 bars, agreement with the whole index, RK4, the angle-dependent rate, the
allocation-free entry point, and the 3D N = 32 workload within 8 GB.
"""
import math
import sys
import time

import numpy as np
import pytest

from paper_2105_08806_amd import inputs as I
from test_gpu_parity import FP32_TOL, FP64_TOL, make_pair, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def mixture_coeffs(plan, dim):
    comps = ([(0.55, (0.7, -0.4), 0.6), (0.45, (-0.9, 0.5), 1.2)] if dim == 2 else
             [(0.55, (0.5, -0.3, 0.2), 0.6), (0.45, (-0.7, 0.5, -0.1), 1.1)])
    return plan.project(I.mixture(plan.interior_velocities(), comps))


def q_of(torch, plan, c):
    q, qp = plan.coeffs_to_q(c, want_qplus=True)
    torch.cuda.synchronize()
    return q.double().cpu().numpy(), qp.double().cpu().numpy()


def streamed_twin(pair_args, dirs, **kw):
    """The oracle, a whole-index plan and a plan of the same descriptor whose
    budget holds `dirs` directions of ids."""
    ora, whole = make_pair(*pair_args, **kw)
    per_dir = whole.info.n_points // whole.info.n_sigma
    _, streamed = make_pair(*pair_args, index_bytes=8 * per_dir * dirs, **kw)
    return ora, whole, streamed, per_dir


# (dim, N, S, map, kernel, gamma), rule and options, directions per chunk,
# precision.  FP32 plans ask for a 1e-8 transform: Q of these near-equilibrium
# mixtures is a small difference of Q+ and Q-, which the default 1e-6 relative
# to sum |q| leaves above the 1e-5 bar (the whole index alike)
STREAM_CASES = [
    ((2, 12, 3.0, 0, "maxwell", 0.0), dict(n_sigma=16), 3, 0),
    ((2, 10, 2.5, 1, "vhs", 1.0), dict(n_sigma=12), 5, 0),
    ((3, 8, 3.0, 0, "maxwell", 0.0), dict(n_theta=4, n_phi=8), 7, 0),
    ((3, 7, 2.5, 1, "vhs", 0.5), dict(n_theta=2, n_phi=4), 1, 0),
    ((2, 9, 3.0, 0, "maxwell", 0.0), dict(n_sigma=8, nufft_tol=1e-8), 2, 1),
    ((3, 6, 2.5, 0, "vhs", 1.0), dict(n_theta=2, n_phi=6, nufft_tol=1e-8), 4, 1),
]


@pytest.mark.parametrize("case", range(len(STREAM_CASES)))
def test_streamed_index_vs_oracle_and_whole(torch_cuda, case):
    torch = torch_cuda
    (dim, N, S, map_, kernel, gamma), rule, dirs, prec = STREAM_CASES[case]
    args = (dim, N, S, map_, kernel, gamma)
    ora, whole, streamed, per_dir = streamed_twin(args, dirs, prec=prec, **rule)
    n_sigma = whole.info.n_sigma
    chunks = math.ceil(n_sigma / dirs)
    say("case: streamed index dim=%d N=%d prec=%d %s, %d directions, budget %d -> %d chunks, ids %d B" % (
        dim, N, prec, kernel, n_sigma, dirs, streamed.info.index_chunks, streamed.info.index_bytes))
    assert whole.info.index_chunks == 1 and whole.info.index_bytes == 8 * whole.info.n_points
    assert streamed.info.gain_mode == 2
    assert streamed.info.index_chunks == chunks
    # the chunks are spread evenly, so the largest holds at most `dirs` directions
    assert streamed.info.index_bytes == 8 * per_dir * math.ceil(n_sigma / chunks)
    assert streamed.info.index_bytes <= 8 * per_dir * dirs
    ct = mixture_coeffs(whole, dim)
    tol = FP64_TOL if prec == 0 else FP32_TOL
    qs, qps = q_of(torch, streamed, ct)
    qw, qpw = q_of(torch, whole, ct)
    q_ref, qp_ref, _ = ora.collision(ct.double().cpu().numpy())
    r, rp = rel_l2(qs, q_ref), rel_l2(qps, qp_ref)
    agree = rel_l2(qps, qpw)
    say("  vs oracle Q %.3e Q+ %.3e; Q+ vs whole index %.3e" % (r, rp, agree))
    assert r <= tol and rp <= tol
    # the same points spread in another grouping: FP64 atomics in another order
    # (FP64 plans); FP32 plans also sum each 64-point batch in FP32 first
    assert agree <= (1e-13 if prec == 0 else 1e-6)
    # a second evaluation re-sorts the chunks and agrees to rounding again
    qs2, _ = q_of(torch, streamed, ct)
    assert rel_l2(qs2, qs) <= (1e-13 if prec == 0 else 1e-6)
    whole.close()
    streamed.close()


def test_streamed_index_one_direction_per_chunk(torch_cuda):
    """A budget below one direction's ids still streams, one direction per chunk."""
    torch = torch_cuda
    ora, plan = make_pair(2, 8, 3.0, n_sigma=10, index_bytes=1)
    per_dir = plan.info.n_points // plan.info.n_sigma
    say("case: index_bytes = 1:", plan.info.index_chunks, "chunks")
    assert plan.info.index_chunks == 10 and plan.info.index_bytes == 8 * per_dir
    c = mixture_coeffs(plan, 2)
    q, qp = q_of(torch, plan, c)
    q_ref, qp_ref, _ = ora.collision(c.cpu().numpy())
    assert rel_l2(q, q_ref) <= FP64_TOL and rel_l2(qp, qp_ref) <= FP64_TOL
    plan.close()


def test_streamed_index_angle_dependent_rate(torch_cuda):
    torch = torch_cuda
    from test_gpu_direct import make_aniso
    for dim, N, S, map_, beta, gamma, n_sigma in ((2, 8, 3.0, 0, 1.2, 0.5, 12), (3, 6, 2.5, 1, -0.5, 1.0, 0)):
        ora, whole = make_aniso(dim, N, S, map_, beta, gamma, n_sigma=n_sigma)
        per_dir = whole.info.n_points // whole.info.n_sigma
        _, plan = make_aniso(dim, N, S, map_, beta, gamma, n_sigma=n_sigma, index_bytes=8 * per_dir * 3)
        say("case: streamed ANISO dim=%d N=%d: %d chunks" % (dim, N, plan.info.index_chunks))
        assert plan.info.index_chunks == math.ceil(whole.info.n_sigma / 3)
        c = mixture_coeffs(plan, dim)
        q, qp = q_of(torch, plan, c)
        q_ref, qp_ref, _ = ora.collision(c.cpu().numpy())
        r, rp = rel_l2(q, q_ref), rel_l2(qp, qp_ref)
        say("  vs oracle Q %.3e Q+ %.3e" % (r, rp))
        assert r <= FP64_TOL and rp <= FP64_TOL
        whole.close()
        plan.close()


def test_streamed_index_rk4_and_static_entry(torch_cuda):
    """RK4 over a streamed plan matches the whole index; the allocation-free
    entry point evaluates a streamed plan like the plan's own workspace."""
    torch = torch_cuda
    _, whole, plan, _ = streamed_twin((3, 8, 3.0, 1, "vhs", 1.0), 5, n_theta=4, n_phi=4)
    assert plan.info.index_chunks == 4
    c = mixture_coeffs(whole, 3)
    yw = whole.rk4(c.clone(), 0.05, 3)
    ys = plan.rk4(c.clone(), 0.05, 3)
    torch.cuda.synchronize()
    r = rel_l2(ys.cpu().numpy(), yw.cpu().numpy())
    say("case: streamed RK4, 3 steps vs whole index %.3e" % r)
    assert r <= 1e-13
    q_ref, qp_ref = plan.coeffs_to_q(c, want_qplus=True)
    q_st, qp_st = plan.coeffs_to_q_static(c, want_qplus=True)
    torch.cuda.synchronize()
    r_q = rel_l2(q_st.cpu().numpy(), q_ref.cpu().numpy())
    r_qp = rel_l2(qp_st.cpu().numpy(), qp_ref.cpu().numpy())
    say("  static entry vs plan workspace Q %.3e Q+ %.3e" % (r_q, r_qp))
    assert r_q <= 1e-13 and r_qp <= 1e-13
    whole.close()
    plan.close()


def test_streamed_index_option_checks(torch_cuda):
    from paper_2105_08806_amd import pgc
    # the deterministic gather needs the whole index
    with pytest.raises(pgc.PgcError) as err:
        make_pair(2, 8, 3.0, n_sigma=8, index_bytes=1, deterministic=1)
    assert err.value.code == 2
    # a budget the whole index fits in keeps it whole
    _, plan = make_pair(2, 8, 3.0, n_sigma=8, index_bytes=1 << 30)
    assert plan.info.index_chunks == 1
    plan.close()
    # batches keep the whole index whatever the budget
    b = pgc.Batch([8, 8, 10], scale=3.0, n_sigma=8, index_bytes=1, autotune=False)
    q = b.unpack(b.coeffs_to_q(b.pack([np.zeros((n, n), np.float32) for n in (8, 8, 10)])))
    assert all(np.all(x == 0.0) for x in q)
    b.close()


def test_streamed_index_3d_n32_workload(torch_cuda):
    """The 3D N = 32 workload (BKW at t = 6.5, S = 5, Maxwell, 8 x 8 product
    rule, FP64) with the point ids in 8 GB instead of 62.5 GB: against the
    whole index, and the time of both."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    budget = 8 * 10 ** 9
    plans = {}
    for name, extra in (("whole", {}), ("streamed", dict(index_bytes=budget))):
        t = time.time()
        plans[name] = pgc.Plan(dim=3, n_modes=32, scale=5.0, map=pgc.MAP_LOG, kernel=pgc.KERNEL_MAXWELL,
                               sphere=pgc.SPHERE_PRODUCT_3D, n_theta=8, n_phi=8, precision=pgc.FP64, **extra)
        info = plans[name].info
        say("3D N=32 %s: plan %.1f s, %d chunks, ids %.2f GB, workspace %.2f GB" % (
            name, time.time() - t, info.index_chunks, info.index_bytes / 1e9, info.workspace_bytes / 1e9))
    s = plans["streamed"].info
    assert s.index_chunks == 8 and s.index_bytes <= budget
    assert s.workspace_bytes <= 10 * 10 ** 9
    w = plans["whole"]
    c = w.project(I.bkw_f(6.5, w.interior_velocities()))
    out = {}
    for name, plan in plans.items():
        plan.coeffs_to_q(c)
        torch.cuda.synchronize()
        t = time.time()
        for _ in range(2):
            q, qp = plan.coeffs_to_q(c, want_qplus=True)
        torch.cuda.synchronize()
        say("  %s: %.3f s per evaluation" % (name, (time.time() - t) / 2))
        out[name] = qp.cpu().numpy()
    r = rel_l2(out["streamed"], out["whole"])
    say("  Q+ streamed vs whole index %.3e" % r)
    assert r <= 1e-13
    for p in plans.values():
        p.close()
