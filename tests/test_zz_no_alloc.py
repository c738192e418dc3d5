"""pgc_coeffs_to_q_static (the entry point for callers that cannot allocate)
against pgc_coeffs_to_q on the same plans and inputs, through the C ABI.

Two calls in a row on different plans, the second smaller, so a call that
read what the previous one left in the shared static array would show.
Bars: relative L2 1e-11 (FP64 plans) and 1e-5 (FP32 plans); the two paths
run the same kernels, and differ only in the order of the gain's FP64
atomic additions.
"""
import sys

import numpy as np
import pytest

from paper_2105_08806_amd import inputs as I

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make_plan(pgc, dim, N, prec, scale=3.0, **kw):
    if dim == 3:
        kw.setdefault("sphere", pgc.SPHERE_PRODUCT_3D)
        kw.setdefault("n_theta", 4)
        kw.setdefault("n_phi", 8)
    else:
        kw.setdefault("n_sigma", 16)
    return pgc.Plan(dim=dim, n_modes=N, scale=scale, precision=prec, **kw)


def both(torch, plan, c):
    q_ref, qp_ref = plan.coeffs_to_q(c, want_qplus=True)
    q_st, qp_st = plan.coeffs_to_q_static(c, want_qplus=True)
    torch.cuda.synchronize()
    return ([x.double().cpu().numpy() for x in (q_st, qp_st)],
            [x.double().cpu().numpy() for x in (q_ref, qp_ref)])


@pytest.mark.parametrize("prec,first,second", [
    (0, (3, 32, dict(n_theta=8, n_phi=8, scale=5.0)), (2, 12, {})),
    (0, (3, 16, {}), (2, 10, dict(kernel=1, kernel_gamma=1.0))),
    (1, (2, 48, dict(kernel=1, kernel_gamma=1.0)), (2, 9, {})),
    (1, (3, 12, dict(gain_mode=1, n_chunks=8)), (2, 8, dict(gain_mode=1, n_chunks=4))),
])
def test_static_scratch_matches_plan_workspace(torch_cuda, prec, first, second):
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    bar = 1e-11 if prec == 0 else 1e-5
    for dim, N, kw in (first, second):
        plan = make_plan(pgc, dim, N, prec, **kw)
        comps = ([(0.6, (0.8, -0.4), 0.7), (0.4, (-1.0, 0.6), 1.3)] if dim == 2 else
                 [(0.6, (0.5, -0.3, 0.1), 0.7), (0.4, (-0.8, 0.6, 0.2), 1.2)])
        c = plan.project(I.mixture(plan.interior_velocities(), comps))
        say("static scratch: dim=%d N=%d prec=%d gain_mode=%d" % (dim, N, prec, plan.info.gain_mode))
        (q_st, qp_st), (q_ref, qp_ref) = both(torch, plan, c)
        r_q, r_qp = rel(q_st, q_ref), rel(qp_st, qp_ref)
        say("  rel-L2 Q %.3e  Q+ %.3e" % (r_q, r_qp))
        assert r_q <= bar and r_qp <= bar
        plan.close()


def test_static_scratch_rejects_plans_that_do_not_fit(torch_cuda):
    """A 3D 40-mode plan needs three fine-grid-sized buffers of 14 MB and more:
    beyond the 32 MiB static array, so the call returns PGC_ERR_SCRATCH and
    leaves its output untouched (two antipodal directions keep the plan small)."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    sigma = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    plan = pgc.Plan(dim=3, n_modes=40, scale=3.0, precision=0, sigma=sigma,
                    sigma_w=np.array([2 * np.pi, 2 * np.pi]))
    say("static scratch: 3D N=40 plan, grid %d^3, gain_mode %d" % (plan.info.grid_folded, plan.info.gain_mode))
    assert 3 * plan.info.grid_folded ** 3 * 8 > 32 * 1024 * 1024
    c = torch.zeros(plan.shape(), dtype=torch.float64, device="cuda")
    q = torch.full(plan.shape(), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(pgc.PgcError) as err:
        plan.coeffs_to_q_static(c, q=q)
    assert err.value.code == 6
    torch.cuda.synchronize()
    assert bool(torch.all(q == 7.0))
    plan.close()
