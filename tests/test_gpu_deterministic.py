"""Plans created with deterministic = 1: the binned gain writes one footprint
tile per bin run and a gather adds the tiles of every fine-grid cell in a
fixed order, so repeated evaluations of one plan are bit-identical (two plans
of one descriptor agree to rounding: the order of the points inside a bin
comes from the plan-time scatter).  Parity against the
oracle at the FP64 and FP32 bars, bit-for-bit repeats, agreement with the
atomic flush, and the full-size 3D workload.
"""
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    return torch


CASES = [
    (2, 12, 3.0, 0, "maxwell", 0.0, 0),
    (2, 10, 2.5, 1, "vhs", 1.0, 0),
    (3, 7, 3.0, 0, "vhs", 0.5, 0),
    (3, 6, 2.5, 1, "maxwell", 0.0, 1),
    (2, 9, 3.0, 0, "maxwell", 0.0, 1),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dd-N%d-r%d-%s-p%d" % (c[0], c[1], c[3], c[4], c[6]))
def test_deterministic_plan_vs_oracle_and_repeats(torch_cuda, case):
    torch = torch_cuda
    dim, N, S, map_, kernel, gamma, prec = case
    # FP32: transform tolerance 1e-8 (W = 7); the default 1e-6 is relative to
    # sum |q|, which these random coefficients inflate by cancellation
    tol = dict(nufft_tol=1e-8) if prec else {}
    ora, plan = make_pair(dim, N, S, map_, kernel, gamma, prec=prec, n_sigma=8, deterministic=1, **tol)
    _, atomic = make_pair(dim, N, S, map_, kernel, gamma, prec=prec, n_sigma=8, **tol)
    assert plan.info.deterministic == 1 and plan.info.tile_bytes > 0
    say("case: deterministic", case, "tiles %d bytes" % plan.info.tile_bytes)
    coeffs = I.random_coeffs((N,) * dim, seed=77)
    cin = coeffs.astype(np.float32).astype(np.float64) if prec else coeffs
    c = torch.tensor(cin, dtype=plan.dtype, device="cuda")
    q1, qp1 = plan.coeffs_to_q(c, want_qplus=True)
    q1, qp1 = q1.clone(), qp1.clone()
    q2, qp2 = plan.coeffs_to_q(c, want_qplus=True)
    qa = atomic.coeffs_to_q(c)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2) and torch.equal(qp1, qp2)
    q_ref, qp_ref, _ = ora.collision(cin)
    r = rel_l2(q1.double().cpu().numpy(), q_ref)
    ra = rel_l2(q1.double().cpu().numpy(), qa.double().cpu().numpy())
    say("  rel-L2 vs oracle %.3e; vs the atomic flush %.3e" % (r, ra))
    assert r <= (FP64_TOL if prec == 0 else FP32_TOL)
    # two plans: the plan-time scatter fills every bin in an order set by
    # atomics, which FP32 point batches see as a reordered sum (FP64 tiles only
    # as rounding of FP64 additions)
    assert ra <= (1e-13 if prec == 0 else 1e-7)
    plan.close()
    atomic.close()


def test_deterministic_option_checks(torch_cuda):
    from paper_2105_08806_amd import pgc
    say("case: deterministic option checks")
    for mode in (pgc.GAIN_SLAB, pgc.GAIN_MFMA):
        with pytest.raises(pgc.PgcError):
            pgc.Plan(dim=3, n_modes=6, scale=3.0, sphere=pgc.SPHERE_PRODUCT_3D, n_theta=2, n_phi=4,
                     deterministic=1, gain_mode=mode)
    with pytest.raises(pgc.PgcError):
        pgc.Plan(dim=2, n_modes=6, scale=3.0, n_sigma=8, deterministic=2)


def test_deterministic_3d_n32_workload(torch_cuda):
    """The 3D BKW workload (32 modes, S = 5, the 64-direction product rule,
    FP64): two evaluations are bit-identical, they agree with the atomic
    flush to rounding, and the cost of the gather is timed."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    out, ms = {}, {}
    for det in (0, 1):
        plan = pgc.Plan(dim=3, n_modes=32, scale=5.0, sphere=pgc.SPHERE_PRODUCT_3D, n_theta=8, n_phi=8,
                        precision=0, deterministic=det)
        c = plan.project(I.bkw_f(6.5, plan.interior_velocities()))
        say("3D N=32 deterministic=%d: items %d, tiles %.2f GB" % (det, plan.info.n_bin_items,
                                                                   plan.info.tile_bytes / 1e9))
        a = plan.coeffs_to_q(c).clone()
        torch.cuda.synchronize()
        t = time.time()
        b = plan.coeffs_to_q(c).clone()
        torch.cuda.synchronize()
        ms[det] = (time.time() - t) * 1e3
        out[det] = (a, b)
        plan.close()
    a1, b1 = out[1]
    assert torch.equal(a1, b1)
    r = float(torch.linalg.norm(a1 - out[0][0]) / torch.linalg.norm(out[0][0]))
    say("  deterministic vs atomic rel-L2 %.3e; %.1f ms vs %.1f ms per evaluation" % (r, ms[1], ms[0]))
    assert r <= 1e-13
