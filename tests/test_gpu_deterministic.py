"""Plans created with deterministic = 1: the binned gain writes one footprint
tile per bin run and a gather adds the tiles of every fine-grid cell in a
fixed order, and the plan sorts the point ids inside every bin after the
plan-time scatter, so every plan of one descriptor evaluates bit for bit
alike.  Parity against the oracle at the FP64 and FP32 bars, bit-for-bit
repeats within and across plans, agreement with the atomic flush, batches
that equal unbatched plans bit for bit, and the full-size 3D workload.
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
    _, twin = make_pair(dim, N, S, map_, kernel, gamma, prec=prec, n_sigma=8, deterministic=1, **tol)
    _, atomic = make_pair(dim, N, S, map_, kernel, gamma, prec=prec, n_sigma=8, **tol)
    assert plan.info.deterministic == 1 and plan.info.tile_bytes > 0
    say("case: deterministic", case, "tiles %d bytes" % plan.info.tile_bytes)
    coeffs = I.random_coeffs((N,) * dim, seed=77)
    cin = coeffs.astype(np.float32).astype(np.float64) if prec else coeffs
    c = torch.tensor(cin, dtype=plan.dtype, device="cuda")
    q1, qp1 = plan.coeffs_to_q(c, want_qplus=True)
    q1, qp1 = q1.clone(), qp1.clone()
    q2, qp2 = plan.coeffs_to_q(c, want_qplus=True)
    qt, qpt = twin.coeffs_to_q(c, want_qplus=True)
    qa = atomic.coeffs_to_q(c)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2) and torch.equal(qp1, qp2)
    # another plan of the same descriptor: the same sorted bins, the same sums
    assert torch.equal(q1, qt) and torch.equal(qp1, qpt)
    q_ref, qp_ref, _ = ora.collision(cin)
    r = rel_l2(q1.double().cpu().numpy(), q_ref)
    ra = rel_l2(q1.double().cpu().numpy(), qa.double().cpu().numpy())
    say("  rel-L2 vs oracle %.3e; vs the atomic flush %.3e" % (r, ra))
    assert r <= (FP64_TOL if prec == 0 else FP32_TOL)
    # the atomic plan spreads the unsorted bins: FP32 point batches see a
    # reordered sum (FP64 tiles only the rounding of FP64 additions)
    assert ra <= (1e-13 if prec == 0 else 1e-7)
    plan.close()
    twin.close()
    atomic.close()


def test_deterministic_plans_with_sliced_sorts(torch_cuda):
    """A 3D plan whose 4.4e8 ids are sorted in four slices: two plans of the
    descriptor agree bit for bit and with the atomic flush to rounding."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    kw = dict(dim=3, n_modes=20, scale=4.0, sphere=pgc.SPHERE_PRODUCT_3D, n_theta=8, n_phi=8, precision=0)
    plans = [pgc.Plan(deterministic=1, **kw) for _ in range(2)]
    atomic = pgc.Plan(**kw)
    info = plans[0].info
    say("case: 3D N=20, %d points in %d runs" % (info.n_points, info.n_bin_items))
    assert info.n_points * 8 > 3 * 2 ** 30  # more than three 1 GiB sorting slices
    c = plans[0].project(I.bkw_f(6.5, plans[0].interior_velocities()))
    qs = [p.coeffs_to_q(c).clone() for p in plans]
    qa = atomic.coeffs_to_q(c)
    torch.cuda.synchronize()
    assert torch.equal(qs[0], qs[1])
    r = float(torch.linalg.norm(qs[0] - qa) / torch.linalg.norm(qa))
    say("  deterministic vs atomic rel-L2 %.3e" % r)
    assert r <= 1e-13
    for p in plans + [atomic]:
        p.close()


def test_deterministic_batch_equals_unbatched_plans(torch_cuda):
    """A batch of mixed-N 2D cells created from a deterministic descriptor:
    every cell's Q equals, bit for bit, the evaluation of that cell by a
    separately created plan of the same descriptor, and two batched
    evaluations are bit-identical."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    fields = dict(scale=4.0, n_sigma=16, nufft_tol=1e-8, deterministic=1)
    modes = [12, 8, 16, 12, 8, 16, 16, 12, 10]
    b = pgc.Batch(modes, **fields)
    assert b.info.deterministic == 1
    cells = [I.random_coeffs((n, n), seed=400 + i) for i, n in enumerate(modes)]
    packed = b.pack(cells)
    q1 = b.coeffs_to_q(packed).clone()
    q2 = b.coeffs_to_q(packed)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2)
    got = b.unpack(q1)
    plans = {n: pgc.Plan(dim=2, n_modes=n, precision=pgc.FP32, **fields) for n in sorted(set(modes))}
    say("case: deterministic batch of %d cells, N in %s" % (len(modes), sorted(plans)))
    for i, n in enumerate(modes):
        c = torch.tensor(cells[i].astype(np.float32), device="cuda")
        ref = plans[n].coeffs_to_q(c).double().cpu().numpy()
        assert np.array_equal(got[i], ref), (i, n, float(np.max(np.abs(got[i] - ref))))
    # custom offsets and graph capture are refused in this mode
    with pytest.raises(pgc.PgcError) as err:
        b.coeffs_to_q(packed, offsets=torch.tensor(b.offsets, device="cuda"))
    assert err.value.code == 2
    with pytest.raises(pgc.PgcError) as err:
        b.capture(packed, torch.empty_like(packed))
    assert err.value.code == 2
    b.close()
    for p in plans.values():
        p.close()


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
    FP64): two evaluations are bit-identical, so is a second deterministic
    plan (its bins hold up to several runs each), they agree with the atomic
    flush to rounding, and the cost of the gather is timed."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    out, ms = {}, {}
    for det in (0, 1, 2):
        t = time.time()
        plan = pgc.Plan(dim=3, n_modes=32, scale=5.0, sphere=pgc.SPHERE_PRODUCT_3D, n_theta=8, n_phi=8,
                        precision=0, deterministic=min(det, 1))
        say("3D N=32 plan %d built in %.1f s" % (det, time.time() - t))
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
    assert torch.equal(a1, out[2][0])
    r = float(torch.linalg.norm(a1 - out[0][0]) / torch.linalg.norm(out[0][0]))
    say("  deterministic vs atomic rel-L2 %.3e; %.1f ms vs %.1f ms per evaluation" % (r, ms[1], ms[0]))
    assert r <= 1e-13
