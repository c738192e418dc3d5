"""HIP graphs of a plan's launch sequences (pgc_plan_capture,
pgc_plan_capture_rk4, pgc_plan_graph_launch).  Every replay runs after eager
work of other inputs on the same plan, with the caller's buffers refilled
in place, and is checked against the eager result: bit for bit for
deterministic plans (fixed summation order), to rounding otherwise.
"""
import sys

import numpy as np
import pytest

from paper_2105_08806_amd import inputs as I
from test_gpu_parity import FP32_TOL, rel_l2

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


def coeff_set(torch, plan, seeds):
    shape = plan.shape()
    return [torch.as_tensor(I.random_coeffs(shape, seed=s), dtype=plan.dtype, device="cuda") for s in seeds]


def test_evaluation_graph_replays_bit_for_bit(torch_cuda):
    """A deterministic FP64 plan: the captured evaluation, replayed on refilled
    input between eager evaluations of other inputs, equals the eager result
    bit for bit every time."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    for dim, N, rule in ((2, 12, dict(n_sigma=12)), (3, 6, dict(sphere=pgc.SPHERE_PRODUCT_3D, n_theta=2, n_phi=4))):
        plan = pgc.Plan(dim=dim, n_modes=N, scale=3.0, precision=pgc.FP64, deterministic=1, **rule)
        ca, cb, cc, cx = coeff_set(torch, plan, (1, 2, 3, 4))
        buf = ca.clone()
        q, qp = plan.capture(buf, want_qplus=True)
        ref_q, ref_qp = plan.coeffs_to_q(ca, want_qplus=True)
        torch.cuda.synchronize()
        say("case: evaluation graph dim=%d N=%d" % (dim, N))
        assert torch.equal(q, ref_q) and torch.equal(qp, ref_qp)
        for c in (cb, cc, ca, cb):
            plan.coeffs_to_q(cx)  # eager work of another input on the same workspace
            torch.cuda.synchronize()
            buf.copy_(c)
            plan.graph_launch()
            e_q, e_qp = plan.coeffs_to_q(c, want_qplus=True)
            torch.cuda.synchronize()
            assert torch.equal(q, e_q) and torch.equal(qp, e_qp)
        plan.close()


@pytest.mark.parametrize("kind", ["fp32", "streamed"])
def test_evaluation_graph_replays_to_rounding(torch_cuda, kind):
    """Plans that flush with atomics (FP32; a streamed index) replay within
    rounding of the eager result."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    if kind == "fp32":
        plan = pgc.Plan(dim=3, n_modes=8, scale=3.0, map=pgc.MAP_ALGEBRAIC, kernel=pgc.KERNEL_VHS, kernel_gamma=1.0,
                        sphere=pgc.SPHERE_PRODUCT_3D, n_theta=4, n_phi=4, precision=pgc.FP32)
        tol = FP32_TOL
    else:
        probe = pgc.Plan(dim=2, n_modes=10, scale=3.0, n_sigma=12, precision=pgc.FP64)
        per_dir = probe.info.n_points // probe.info.n_sigma
        probe.close()
        plan = pgc.Plan(dim=2, n_modes=10, scale=3.0, n_sigma=12, precision=pgc.FP64, index_bytes=8 * per_dir * 5)
        assert plan.info.index_chunks == 3
        tol = 1e-13
    ca, cb, cx = coeff_set(torch, plan, (5, 6, 7))
    buf = ca.clone()
    q = plan.capture(buf)
    for c in (ca, cb, ca):
        plan.coeffs_to_q(cx)
        torch.cuda.synchronize()
        buf.copy_(c)
        plan.graph_launch()
        e = plan.coeffs_to_q(c)
        torch.cuda.synchronize()
        r = rel_l2(q.double().cpu().numpy(), e.double().cpu().numpy())
        say("case: %s evaluation graph replay vs eager %.2e" % (kind, r))
        assert r <= tol
    plan.close()


def test_rk4_graph_replays_bit_for_bit(torch_cuda):
    """The captured RK4 steps run nothing at capture, then each replay advances
    the state exactly as the eager steps do (deterministic plan)."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    plan = pgc.Plan(dim=2, n_modes=12, scale=3.0, n_sigma=12, precision=pgc.FP64, deterministic=1)
    y0 = plan.project(I.bkw_f(0.0, plan.interior_velocities())).double()
    dt, steps = 0.05, 3
    y = y0.clone()
    plan.capture_rk4(y, dt, steps)
    torch.cuda.synchronize()
    assert torch.equal(y, y0)
    ref = y0.clone()
    for rep in range(3):
        plan.rk4(ref, dt, steps)
        plan.coeffs_to_q(coeff_set(torch, plan, (9,))[0])  # eager work between replays
        torch.cuda.synchronize()
        plan.graph_launch()
        torch.cuda.synchronize()
        say("case: RK4 graph replay %d, max |diff| %.1e" % (rep, float((y - ref).abs().max())))
        assert torch.equal(y, ref)
    plan.close()


def test_graph_call_errors(torch_cuda):
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    plan = pgc.Plan(dim=2, n_modes=8, scale=3.0, n_sigma=8, precision=pgc.FP64)
    c = coeff_set(torch, plan, (3,))[0]
    with pytest.raises(pgc.PgcError) as err:
        plan.graph_launch()  # nothing captured
    assert err.value.code == 1
    y = c.clone()
    with pytest.raises(pgc.PgcError) as err:
        plan.capture_rk4(y, 0.1, 0)
    assert err.value.code == 1
    plan.set_profiling(True)
    with pytest.raises(pgc.PgcError) as err:
        plan.capture(c)
    assert err.value.code == 2
    plan.set_profiling(False)
    q = plan.capture(c)
    plan.graph_launch()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(q.cpu().numpy()))
    plan.close()
