"""GPU parity of the direct algorithm (Sec. 4.1): the node-pair tensor built
on the device and its FP64 matrix product, cell by cell against the FP64 CPU
oracle, and at the batched workload's N = 32 against the plan's fast path.

The direct path evaluates the same discrete sum as the oracle with no
transform tolerance, so the oracle bar is the FP64 one, 1e-11 in rel-L2 of Q.
Against the fast path the difference is the fast path's own transform error,
which scales with Q+ rather than with Q; near equilibrium Q is a few percent
of Q+, so that comparison is normalised by |Q+| (the near-equilibrium
reading of the parity metric), with the same 1e-11 bar.
"""
import hashlib
import os
import sys

import numpy as np
import pytest

from paper_2105_08806_amd import inputs as I
from test_gpu_parity import FP64_TOL, make_pair, rel_l2

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


def direct_q(torch, plan, cells, max_cells):
    from paper_2105_08806_amd import pgc
    d = pgc.Direct(plan, max_cells=max_cells)
    c = torch.tensor(np.stack(cells), dtype=torch.float64, device="cuda")
    q = d.coeffs_to_q(c)
    torch.cuda.synchronize()
    out, info = q.cpu().numpy(), d.info
    d.close()
    return out, info


# dim, N, S, map, kernel, gamma, directions (2D)
CASES = [
    (2, 7, 3.0, 0, "maxwell", 0.0, 8),
    (2, 6, 2.5, 1, "vhs", 1.0, 6),
    (2, 8, 4.0, 0, "vhs", 0.5, 10),
    (3, 4, 2.0, 1, "maxwell", 0.0, 0),
    (3, 5, 3.0, 0, "vhs", 1.0, 0),
    (2, 5, 3.0, 0, "vhs", 1.0, 40),     # two direction chunks (32 + 8)
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dd-N%d-r%d-%s" % (c[0], c[1], c[3], c[4]))
def test_direct_vs_oracle(torch_cuda, case):
    dim, N, S, map_, kernel, gamma, n_sigma = case
    ora, plan = make_pair(dim, N, S, map_, kernel, gamma, n_sigma=n_sigma or 8)
    cells = [I.random_coeffs((N,) * dim, seed=300 + c) for c in range(5)]
    say("case: direct", case, "5 cells in products of 2")
    q, info = direct_q(torch_cuda, plan, cells, max_cells=2)  # products of 2, 2 and 1 cells
    nid = (N - 1) ** dim
    assert info.n_pairs == nid * (nid + 1) // 2 and info.n_modes_total == N ** dim
    assert info.tensor_bytes == info.n_pairs * N ** dim * 8
    for c in range(5):
        q_ref, _, _ = ora.collision(cells[c])
        r = rel_l2(q[c].reshape(q_ref.shape), q_ref)
        say("  cell %d rel-L2 Q = %.3e" % (c, r))
        assert r <= FP64_TOL, (case, c, r)
    plan.close()


def make_aniso(dim, N, S, map_, beta, gamma, n_sigma=8, prec=0, sigma=None, sigma_w=None, **tune):
    """Oracle and plan with B = b0 |u|^gamma (1 + beta cos^2 theta)."""
    import oracle as O
    from paper_2105_08806_amd import pgc
    if sigma is not None:
        sg, sw = sigma, sigma_w
        sph = dict(sigma=sg, sigma_w=sw)
    elif dim == 2:
        sg, sw = O.circle_rule(n_sigma)
        sph = dict(sphere=pgc.SPHERE_UNIFORM_2D, n_sigma=n_sigma)
    else:
        sg, sw = O.sphere_product_rule(2, 4)
        sph = dict(sphere=pgc.SPHERE_PRODUCT_3D, n_theta=2, n_phi=4)
    ora = O.Problem(dim, N, S, map_, kernel="aniso", aniso=beta, gamma=gamma, sphere=sg, sphere_w=sw)
    plan = pgc.Plan(dim=dim, n_modes=N, scale=S, map=map_, kernel=pgc.KERNEL_ANISO, kernel_gamma=gamma,
                    kernel_aniso=beta, precision=prec, **sph, **tune)
    return ora, plan


# dim, N, S, map, beta, gamma, directions (2D)
ANISO_CASES = [
    (2, 7, 3.0, 0, 0.8, 0.5, 8),
    (2, 6, 2.5, 1, 3.0, 1.0, 10),
    (3, 4, 2.0, 1, -0.6, 0.0, 0),
    (3, 5, 3.0, 0, 1.5, 0.5, 0),
    (2, 5, 2.0, 1, 1.5, 0.0, 48),       # two direction chunks (32 + 16)
]


@pytest.mark.parametrize("case", ANISO_CASES, ids=lambda c: "%dd-N%d-r%d-beta%g" % (c[0], c[1], c[3], c[4]))
def test_direct_angle_dependent_rate_vs_oracle(torch_cuda, case):
    """The direct algorithm with B = b0 |u|^gamma (1 + beta cos^2 theta): the
    gain weights and the loss's inner integral over sigma both carry the angle."""
    dim, N, S, map_, beta, gamma, n_sigma = case
    ora, plan = make_aniso(dim, N, S, map_, beta, gamma, n_sigma or 8)
    cells = [I.random_coeffs((N,) * dim, seed=500 + c) for c in range(3)]
    say("case: direct, angle-dependent rate", case)
    q, _ = direct_q(torch_cuda, plan, cells, max_cells=2)
    for c in range(3):
        q_ref, _, _ = ora.collision(cells[c])
        r = rel_l2(q[c].reshape(q_ref.shape), q_ref)
        say("  cell %d rel-L2 Q = %.3e" % (c, r))
        assert r <= FP64_TOL, (case, c, r)
    plan.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", ANISO_CASES, ids=lambda c: "%dd-N%d-r%d-beta%g" % (c[0], c[1], c[3], c[4]))
def test_fast_path_angle_dependent_rate_vs_oracle(torch_cuda, case, prec):
    """The fast path with B = b0 |u|^gamma (1 + beta cos^2 theta): every merged
    point weighs the terms of its orbit with their own cos theta, and the
    loss's inner integral over sigma is a quadratic form in u.  Every
    coefficient against the oracle's triple-by-triple sum (kernel 2).  FP32
    plans run at transform tolerance 1e-8 (W = 7): these mixtures are near
    equilibrium, where Q is a few percent of Q+ and the default 1e-6 (relative
    to sum |q|) would leave more than 1e-5 in Q."""
    torch = torch_cuda
    dim, N, S, map_, beta, gamma, n_sigma = case
    ora, plan = make_aniso(dim, N, S, map_, beta, gamma, n_sigma or 8, prec=prec,
                           **(dict(nufft_tol=1e-8) if prec else {}))
    bar = FP64_TOL if prec == 0 else 1e-5
    say("case: fast path, angle-dependent rate", case, "prec", prec)
    for c in range(2):
        if prec == 0:
            coeffs = I.random_coeffs((N,) * dim, seed=600 + c)
        else:
            # FP32: a velocity distribution (the transform tolerance is relative
            # to sum |q|, which random coefficients inflate by cancellation)
            u = (0.4 + 0.3 * c, -0.3, 0.2)[:dim]
            coeffs = ora.project(I.mixture(ora.interior_velocities(),
                                           [(0.6, u, 0.8), (0.4, tuple(-x for x in u), 1.3)]))
        cin = coeffs.astype(np.float32).astype(np.float64) if prec else coeffs
        q, qp = plan.coeffs_to_q(torch.tensor(cin, dtype=plan.dtype, device="cuda"), want_qplus=True)
        torch.cuda.synchronize()
        q_ref, qp_ref, _ = ora.collision(cin)
        r, rp = rel_l2(q.double().cpu().numpy(), q_ref), rel_l2(qp.double().cpu().numpy(), qp_ref)
        say("  input %d rel-L2 Q = %.3e, Q+ = %.3e" % (c, r, rp))
        assert r <= bar and rp <= bar, (case, prec, c, r, rp)
    plan.close()


def test_fast_path_angle_dependent_rate_3d_n24_sampled(torch_cuda):
    """A larger 3D case of the fast path with an angle-dependent rate: 24
    modes, S = 4, gamma = 1 with beta = 2, a two-Maxwellian input, one
    antipodal direction pair off the axes (the sign patterns of the orbit all
    carry different angles), sampled coefficients against the oracle."""
    torch = torch_cuda
    import oracle as O
    N, S = 24, 4.0
    sg64, sw64 = O.sphere_product_rule(8, 8)
    s0 = 13
    s1 = int(np.argmin(np.linalg.norm(sg64 + sg64[s0], axis=1)))
    ora, plan = make_aniso(3, N, S, 0, 2.0, 1.0, sigma=sg64[[s0, s1]], sigma_w=sw64[[s0, s1]])
    comps = [(0.6, (0.5, -0.3, 0.1), 0.7), (0.4, (-0.8, 0.6, 0.2), 1.2)]
    c = ora.project(I.mixture(ora.interior_velocities(), comps))
    say("case: fast path, angle-dependent rate, 3D N=24 direction pair")
    q, qp = plan.coeffs_to_q(torch.tensor(c, device="cuda"), want_qplus=True)
    torch.cuda.synchronize()
    q, qp = q.cpu().numpy(), qp.cpu().numpy()
    pick = [0, 1, 2, 5, 12, 22, 23]
    kidx = np.stack(np.meshgrid(pick, pick, pick, indexing="ij"), -1).reshape(-1, 3)[::9].astype(np.int32)
    ap, am = ora.collision_at(c, kidx)
    got_q, got_qp = q[tuple(kidx.T)], qp[tuple(kidx.T)]
    r, rp = rel_l2(got_q, ap - am), rel_l2(got_qp, ap)
    say("  %d sampled coefficients: rel-L2 Q = %.3e, Q+ = %.3e" % (len(kidx), r, rp))
    assert r <= FP64_TOL and rp <= FP64_TOL
    plan.close()


def test_fast_path_angle_dependent_rate_3d_n32_stored(torch_cuda):
    """The fast path with an angle-dependent rate at 32 modes (S = 5, B = b0 |u|
    (1 + 2 cos^2 theta), direction 13 of the 8 x 8 product rule and its
    antipode, a two-Maxwellian input) against oracle values stored once by
    tests/golden/make_golden.py a3 at 22 coefficients: the oracle needs
    minutes for them at this size."""
    torch = torch_cuda
    import oracle as O
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "a3_aniso3d_n32_pair.txt")
    rows = {}
    for line in open(path).read().splitlines():
        if line.startswith("# input sha256[:16] "):
            rows["sha"] = line.split()[-1]
        elif not line.startswith("#"):
            key, *vals = line.split()
            rows[key] = vals
    kidx = np.array([[int(x) for x in t.split(",")] for t in rows["kidx"]], dtype=np.int64)
    ref_p = np.array([float(x) for x in rows["qplus"]])
    ref_m = np.array([float(x) for x in rows["qminus"]])
    N, S = 32, 5.0
    sg64, sw64 = O.sphere_product_rule(8, 8)
    s0 = 13
    s1 = int(np.argmin(np.linalg.norm(sg64 + sg64[s0], axis=1)))
    ora, plan = make_aniso(3, N, S, 0, 2.0, 1.0, sigma=sg64[[s0, s1]], sigma_w=sw64[[s0, s1]])
    comps = [(0.6, (0.5, -0.3, 0.1), 0.7), (0.4, (-0.8, 0.6, 0.2), 1.2)]
    c = ora.project(I.mixture(ora.interior_velocities(), comps))
    # the input the stored values were computed from
    assert hashlib.sha256(np.ascontiguousarray(c, dtype=np.float64).tobytes()).hexdigest()[:16] == rows["sha"]
    say("case: fast path, angle-dependent rate, 3D N=32 direction pair vs stored oracle values")
    q, qp = plan.coeffs_to_q(torch.tensor(c, device="cuda"), want_qplus=True)
    torch.cuda.synchronize()
    q, qp = q.cpu().numpy(), qp.cpu().numpy()
    got_q, got_qp = q[tuple(kidx.T)], qp[tuple(kidx.T)]
    r, rp = rel_l2(got_q, ref_p - ref_m), rel_l2(got_qp, ref_p)
    say("  %d stored coefficients: rel-L2 Q = %.3e, Q+ = %.3e" % (len(kidx), r, rp))
    assert r <= FP64_TOL and rp <= FP64_TOL
    plan.close()


def test_angle_dependent_rate_refusals(torch_cuda):
    """The slab scheme (direction-free orbit sums) and the matrix-core gain
    have no per-direction orbit weights, and batches keep angle-free rates:
    they refuse an angle-dependent rate.  A surrogate over such a plan is
    accepted (it falls back to the plan)."""
    from paper_2105_08806_amd import pgc
    say("case: angle-dependent rate refusals")
    for mode in (pgc.GAIN_SLAB, pgc.GAIN_MFMA):
        with pytest.raises(pgc.PgcError):
            pgc.Plan(dim=3, n_modes=6, scale=3.0, sphere=pgc.SPHERE_PRODUCT_3D, n_theta=2, n_phi=4,
                     kernel=pgc.KERNEL_ANISO, kernel_aniso=0.5, gain_mode=mode)
    with pytest.raises(pgc.PgcError):
        pgc.Batch([8, 8], scale=3.0, n_sigma=8, kernel=pgc.KERNEL_ANISO, kernel_aniso=0.5)
    p32 = pgc.Plan(dim=2, n_modes=6, scale=3.0, n_sigma=8, precision=pgc.FP32, kernel=pgc.KERNEL_ANISO,
                   kernel_aniso=0.5)
    sur = pgc.Surrogate(p32, width=16, n_layers=2, batch_max=4)
    sur.close()
    p32.close()


@pytest.mark.parametrize("angle", [False, True])
def test_direct_rk4_vs_oracle(torch_cuda, angle):
    """Classical RK4 of every cell through the direct product against the
    oracle's RK4, for an angle-free and an angle-dependent rate (the latter has
    no fast path to step with)."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    N, dt, steps = 6, 0.05, 3
    if angle:
        ora, plan = make_aniso(2, N, 3.0, 1, 0.8, 0.5)
    else:
        ora, plan = make_pair(2, N, 3.0, 1, "maxwell", n_sigma=8)
    V = plan.interior_velocities()
    cells = [ora.project(I.mixture(V, [(0.7, (0.4 * c, -0.2), 0.8), (0.3, (-0.5, 0.3 * c), 1.3)]))
             for c in range(3)]
    say("case: direct RK4, angle-dependent rate = %s" % angle)
    d = pgc.Direct(plan, max_cells=2)   # chunks of 2 and 1
    c = torch.tensor(np.stack(cells), device="cuda")
    d.rk4(c, dt, steps)
    torch.cuda.synchronize()
    got = c.cpu().numpy()
    for i in range(3):
        ref = ora.rk4(cells[i], dt, steps)
        r = rel_l2(got[i], ref)
        say("  cell %d rel-L2 after %d steps = %.3e" % (i, steps, r))
        assert r <= FP64_TOL
    d.close()
    plan.close()


def test_direct_products_of_any_size_agree(torch_cuda):
    """The chunking of a call into products changes nothing but rounding, and
    an empty batch is a no-op."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    _, plan = make_pair(2, 6, 3.0, 0, "maxwell", n_sigma=8)
    cells = [I.random_coeffs((6, 6), seed=400 + c) for c in range(7)]
    say("case: direct chunking, 7 cells")
    q1, _ = direct_q(torch, plan, cells, max_cells=1)
    q3, _ = direct_q(torch, plan, cells, max_cells=3)
    q7, _ = direct_q(torch, plan, cells, max_cells=7)
    for other in (q3, q7):
        assert np.max(np.abs(other - q1)) <= 1e-14 * np.max(np.abs(q1))
    d = pgc.Direct(plan, max_cells=4)
    empty = torch.empty((0, 36), dtype=torch.float64, device="cuda")
    out = d.coeffs_to_q(empty)
    torch.cuda.synchronize()
    assert out.shape == (0, 36)
    d.close()
    plan.close()


def test_direct_rejects_unsupported_plans(torch_cuda):
    from paper_2105_08806_amd import pgc
    say("case: direct rejections")
    p32 = pgc.Plan(dim=2, n_modes=6, scale=3.0, n_sigma=8, precision=pgc.FP32)
    with pytest.raises(pgc.PgcError):
        pgc.Direct(p32)                      # FP64 plans only
    p32.close()
    p64 = pgc.Plan(dim=2, n_modes=6, scale=3.0, n_sigma=8)
    for bad in (0, 65536):
        with pytest.raises(pgc.PgcError):
            pgc.Direct(p64, max_cells=bad)
    p64.close()
    # the first sizes past the tensor limit (96 GiB): 2D N = 56 (115 GB) and
    # 3D N = 16 (N^3 = 4096 entries per pair, 187 GB)
    for dim, N, extra in ((2, 56, dict(n_sigma=8)),
                          (3, 16, dict(sphere=pgc.SPHERE_PRODUCT_3D, n_theta=2, n_phi=2))):
        big = pgc.Plan(dim=dim, n_modes=N, scale=6.0, **extra)
        with pytest.raises(pgc.PgcError):
            pgc.Direct(big)
        big.close()


def test_direct_n32_batched_cells(torch_cuda):
    """The batched workload's N = 32 cells (S = 6, Maxwell, 32 directions,
    perturbed Maxwellians): 24 cells against the plan's fast FP64 path, one
    against the oracle."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    cells = [c for c in I.cell_maxwellians_2d(96, seed=8806) if c["N"] == 32][:24]
    ora, plan = make_pair(2, 32, 6.0, 0, "maxwell", n_sigma=32)
    V = plan.interior_velocities()
    coeffs = [plan.project(I.perturbed_maxwellian_2d(V, c)).cpu().numpy() for c in cells]
    say("case: direct N=32, %d cells" % len(coeffs))
    q, info = direct_q(torch, plan, coeffs, max_cells=16)
    say("  tensor %.2f GB built in %.1f ms" % (info.tensor_bytes / 1e9, info.setup_ms))
    worst = 0.0
    for c in range(len(coeffs)):
        qf, qp = plan.coeffs_to_q(torch.tensor(coeffs[c], device="cuda"), want_qplus=True)
        torch.cuda.synchronize()
        qf, qp = qf.cpu().numpy(), qp.cpu().numpy()
        d = np.linalg.norm(q[c].reshape(qf.shape) - qf) / np.linalg.norm(qp)
        worst = max(worst, d)
        assert d <= FP64_TOL, (c, d)
    say("  fast path vs direct, normalised by |Q+|: worst %.3e" % worst)
    kidx = np.array([[0, 0], [2, 0], [0, 2], [1, 1], [3, 1], [5, 4], [10, 3], [7, 12], [15, 15], [31, 0],
                     [0, 31], [20, 17]])
    ap, am = ora.collision_at(coeffs[0], kidx)
    got = q[0].reshape(32, 32)[kidx[:, 0], kidx[:, 1]]
    r = rel_l2(got, ap - am)
    say("  cell 0 against the oracle, 12 sampled modes: rel-L2 Q = %.3e" % r)
    assert r <= FP64_TOL
    plan.close()


def test_reproducibility_of_the_two_algorithms(torch_cuda):
    """The direct algorithm repeats itself bit for bit (no atomics: a fixed
    tensor and one library product); the fast path flushes its bins into the
    fine grid with FP64 atomics, whose order varies, so repeats agree to
    rounding only."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    cells = [c for c in I.cell_maxwellians_2d(96, seed=8806) if c["N"] == 32][:8]
    _, plan = make_pair(2, 32, 6.0, 0, "maxwell", n_sigma=32)
    V = plan.interior_velocities()
    c = torch.stack([plan.project(I.perturbed_maxwellian_2d(V, cell)).reshape(-1) for cell in cells])
    say("case: reproducibility, 8 cells at N=32")
    d = pgc.Direct(plan, max_cells=8)
    a = d.coeffs_to_q(c).clone()
    b = d.coeffs_to_q(c).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    d.close()
    x = c[0].reshape(32, 32).contiguous()
    q1 = plan.coeffs_to_q(x).clone()
    q2 = plan.coeffs_to_q(x).clone()
    torch.cuda.synchronize()
    diff = float(torch.linalg.norm(q1 - q2) / torch.linalg.norm(q1))
    say("  fast path, two runs: rel-L2 difference %.2e" % diff)
    assert diff <= 1e-13
    plan.close()


def test_direct_graph_replays(torch_cuda):
    """A captured evaluation (three chunked products) replayed several times,
    the input buffer refilled and eager evaluations run between the replays:
    every replay equals the eager result for its input."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    _, plan = make_pair(2, 6, 3.0, 0, "maxwell", n_sigma=8)
    d = pgc.Direct(plan, max_cells=2)
    c = torch.tensor(np.stack([I.random_coeffs((6, 6), seed=700 + i) for i in range(5)]), device="cuda")
    q = torch.empty_like(c)
    say("case: direct graph capture, 5 cells in products of 2")
    with pytest.raises(pgc.PgcError):
        d.graph_launch()                     # nothing captured yet
    d.capture(c, q)
    for r in range(3):
        fresh = torch.tensor(np.stack([I.random_coeffs((6, 6), seed=800 + 10 * r + i) for i in range(5)]),
                             device="cuda")
        c.copy_(fresh)
        ref = d.coeffs_to_q(fresh.clone())
        torch.cuda.synchronize()
        d.graph_launch()
        torch.cuda.synchronize()
        diff = float(torch.max(torch.abs(q - ref)) / torch.max(torch.abs(ref)))
        say("  replay %d: max difference to eager %.2e" % (r, diff))
        assert diff <= 1e-14
    d.close()
    plan.close()


@pytest.mark.parametrize("N,n_cells,max_cells", [(20, 37, 37), (8, 300, 300), (8, 300, 128)])
def test_direct_product_ragged_tiles(torch_cuda, N, n_cells, max_cells):
    """The library's FP64 matrix-core product at shapes that leave partial
    tiles everywhere: N^2 = 400 columns (three full 128-column tiles and 16),
    37 or 300 rows (one or three row tiles, the last partial), n_pairs = 65341
    or 1225 (K not a multiple of the 16-long chunks), and the split-K partial
    sums the small products use.  Sampled cells against the oracle."""
    torch = torch_cuda
    ora, plan = make_pair(2, N, 3.0, 0, "vhs", 1.0, n_sigma=8)
    cells = [I.random_coeffs((N, N), seed=900 + c) for c in range(n_cells)]
    say("case: direct product N=%d, %d cells in products of %d" % (N, n_cells, max_cells))
    q, info = direct_q(torch, plan, cells, max_cells=max_cells)
    worst = 0.0
    for c in sorted({0, 1, n_cells // 2, 127 % n_cells, 128 % n_cells, n_cells - 1}):
        q_ref, _, _ = ora.collision(cells[c])
        r = rel_l2(q[c].reshape(N, N), q_ref)
        worst = max(worst, r)
        assert r <= FP64_TOL, (c, r)
    say("  worst sampled cell rel-L2 vs oracle %.3e" % worst)
    plan.close()


def test_direct_graph_survives_eager_calls_of_other_sizes(torch_cuda):
    """A graph captured for 200 cells (two products: one full 128-row tile
    pair and a ragged one) is replayed after eager calls of 3 and 150 cells on
    the same object: the replay still equals its own eager result bit for bit
    (the product's workspace is sized at creation and never regrown)."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    _, plan = make_pair(2, 8, 3.0, 0, "maxwell", n_sigma=8)
    d = pgc.Direct(plan, max_cells=160)
    c = torch.tensor(np.stack([I.random_coeffs((8, 8), seed=1100 + i) for i in range(200)]), device="cuda")
    q = torch.empty_like(c)
    say("case: direct graph, then eager calls of other sizes")
    d.capture(c, q)
    ref = d.coeffs_to_q(c.clone()).clone()
    for n in (3, 150):
        other = torch.tensor(np.stack([I.random_coeffs((8, 8), seed=1400 + i) for i in range(n)]), device="cuda")
        d.coeffs_to_q(other)
    q.zero_()
    torch.cuda.synchronize()
    d.graph_launch()
    torch.cuda.synchronize()
    assert torch.equal(q, ref)
    d.close()
    plan.close()
