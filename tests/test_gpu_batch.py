"""GPU checks of the batched path: many 2D cells with mixed N in one
evaluation (FP32 gain, FP64 dense stages), through the C ABI.

Bar: rel-L2 <= 1e-5 per cell against the FP64 oracle (small N, the whole
operator) or against the FP64 single-cell path (workload sizes; that path is
itself held to 1e-11 against the oracle).  The cells are perturbed Maxwellians,
close to equilibrium, where Q is 1-5% of Q+ and every error of the gain is
amplified 20-70 times in Q; the batches therefore ask for a transform
tolerance of 1e-8 (kernel width 7 at upsampling 3).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2105_08806_amd import inputs as I

pytestmark = pytest.mark.gpu
FP32_TOL = 1e-5
TOL = 1e-8  # transform tolerance of the near-equilibrium batches


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


def cell_coeffs(cells, S, n_sigma):
    """Coefficients of the perturbed Maxwellian of every cell, by the oracle's projection."""
    sg, sw = O.circle_rule(n_sigma)
    probs, out = {}, []
    for c in cells:
        N = c["N"]
        if N not in probs:
            probs[N] = O.Problem(2, N, S, 0, sphere=sg, sphere_w=sw)
        p = probs[N]
        out.append(p.project(I.perturbed_maxwellian_2d(p.interior_velocities(), c)))
    return out, probs


def test_batch_small_mixed_vs_oracle(torch_cuda):
    """Seven cells with N in {6, 9, 12}: every cell's Q against the oracle, for
    every supported number of cells per work unit."""
    from paper_2105_08806_amd import pgc
    S, M = 3.0, 8
    cells = I.cell_maxwellians_2d(7, seed=8806, modes=(6, 9, 12))
    coeffs, probs = cell_coeffs(cells, S, M)
    coeffs = [c.astype(np.float32).astype(np.float64) for c in coeffs]
    refs = [probs[c["N"]].collision(x)[0] for c, x in zip(cells, coeffs)]
    b = pgc.Batch([c["N"] for c in cells], scale=S, n_sigma=M, nufft_tol=TOL, autotune=False)
    say("batch: groups", list(b.info.group_n_modes)[:b.info.n_groups], "W", b.info.kernel_width,
        "units", b.info.n_units)
    packed = b.pack(coeffs)
    W = b.info.kernel_width
    for C in (1, 2, 4, 8, 16, 32, 64):
        if C <= 8 and C * W * W > 200:  # beyond the register tile the kernel is built for
            with pytest.raises(pgc.PgcError):
                b.set_tile(C)
            continue
        b.set_tile(C)
        q = b.coeffs_to_q(packed)
        torch_cuda.cuda.synchronize()
        errs = [rel(g, r) for g, r in zip(b.unpack(q), refs)]
        say("  C=%d units=%d max rel-L2 %.3e" % (C, b.info.n_units, max(errs)))
        assert max(errs) <= FP32_TOL, (C, errs)
    b.close()


def test_batch_custom_offsets_and_zero_cells(torch_cuda):
    """Cells stored at caller-chosen offsets (reverse order with gaps), one cell
    all zero: Q lands at the same offsets and the zero cell gives Q = 0."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    S, M = 3.0, 8
    cells = I.cell_maxwellians_2d(5, seed=11, modes=(7, 10))
    coeffs, probs = cell_coeffs(cells, S, M)
    coeffs[2] = np.zeros_like(coeffs[2])
    b = pgc.Batch([c["N"] for c in cells], scale=S, n_sigma=M, nufft_tol=TOL, autotune=False)
    q_dense = b.coeffs_to_q(b.pack(coeffs))
    sizes = [c["N"] ** 2 for c in cells]
    offs, pos = [0] * len(cells), 3
    for c in reversed(range(len(cells))):
        offs[c] = pos
        pos += sizes[c] + 5
    buf = np.zeros(pos, dtype=np.float32)
    for c in range(len(cells)):
        buf[offs[c]:offs[c] + sizes[c]] = coeffs[c].ravel()
    packed = torch.tensor(buf, device="cuda")
    qbuf = torch.full((pos,), 7.0, dtype=torch.float32, device="cuda")
    off_dev = torch.tensor(offs, dtype=torch.int64, device="cuda")
    b.coeffs_to_q(packed, qbuf, offsets=off_dev)
    torch.cuda.synchronize()
    qd = b.unpack(q_dense)
    qb = qbuf.cpu().numpy()
    for c in range(len(cells)):
        got = qb[offs[c]:offs[c] + sizes[c]].reshape(cells[c]["N"], -1)
        if c == 2:
            assert np.all(got == 0)
        else:
            assert rel(got, qd[c]) <= 1e-6
    # the gaps are untouched
    mask = np.ones(pos, dtype=bool)
    for c in range(len(cells)):
        mask[offs[c]:offs[c] + sizes[c]] = False
    assert np.all(qb[mask] == 7.0)
    b.close()


def test_batch_unit_orders_agree(torch_cuda):
    """The four orders of the gain's work units (bin runs longest first or in
    raster order, bin-run or cell-group major) give the same Q up to FP64
    summation order, for a register-tile and a lane-per-cell C; flags other
    than 0 and 1 are rejected."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    S, M = 3.0, 8
    cells = I.cell_maxwellians_2d(40, seed=13, modes=(7, 10))
    coeffs, _ = cell_coeffs(cells, S, M)
    b = pgc.Batch([c["N"] for c in cells], scale=S, n_sigma=M, nufft_tol=TOL, autotune=False)
    packed = b.pack(coeffs)
    for C in (2, 16):
        b.set_tile(C)
        ref = None
        for raster in (0, 1):
            for major in (0, 1):
                b.set_order(raster, major)
                assert (b.info.spatial_order, b.info.group_major) == (raster, major)
                got = b.unpack(b.coeffs_to_q(packed))
                if ref is None:
                    ref = got
                    continue
                for c in range(len(cells)):
                    assert rel(got[c], ref[c]) <= 1e-6, (C, raster, major, c)
    with pytest.raises(pgc.PgcError):
        b.set_order(2, 0)
    b.close()


def test_batch_graph_replays(torch_cuda):
    """The captured graph, replayed three times with new input and eager work
    in between, matches the eager batched call every time."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    S, M = 3.0, 8
    cells = I.cell_maxwellians_2d(6, seed=5, modes=(8, 11))
    b = pgc.Batch([c["N"] for c in cells], scale=S, n_sigma=M, nufft_tol=TOL)
    say("autotuned C =", b.info.cells_per_wave, "ms per C:", list(b.info.tuned_ms))
    packed = torch.zeros(b.total, dtype=torch.float32, device="cuda")
    q = torch.zeros_like(packed)
    b.capture(packed, q)
    assert b.info.has_graph
    for r in range(3):
        src = [I.random_coeffs((n, n), seed=100 + 10 * r + c) for c, n in enumerate(b.n_modes)]
        packed.copy_(b.pack(src))
        b.graph_launch()
        torch.cuda.synchronize()
        eager = b.coeffs_to_q(packed.clone())
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        d = rel(q.double().cpu().numpy(), eager.double().cpu().numpy())
        say("  replay %d: rel-L2 vs eager %.2e (%.1f)" % (r, d, float(junk)))
        assert d <= 1e-6
    b.close()


def test_batch_order_change_drops_the_graph(torch_cuda):
    """Changing the unit order drops a captured graph (a replay is refused
    until the next capture); the graph captured in the new order replays to
    the eager result, and the eager results of both orders agree."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    S, M = 3.0, 8
    cells = I.cell_maxwellians_2d(70, seed=9, modes=(8, 11))
    b = pgc.Batch([c["N"] for c in cells], scale=S, n_sigma=M, nufft_tol=TOL, autotune=False)
    b.set_tile(64)
    src = [I.random_coeffs((n, n), seed=300 + c) for c, n in enumerate(b.n_modes)]
    packed = b.pack(src)
    q = torch.zeros_like(packed)
    b.set_order(1, 0)
    eager0 = b.coeffs_to_q(packed.clone()).double().cpu().numpy()
    b.capture(packed, q)
    assert b.info.has_graph
    b.set_order(1, 1)
    assert not b.info.has_graph
    with pytest.raises(pgc.PgcError):
        b.graph_launch()
    eager1 = b.coeffs_to_q(packed.clone()).double().cpu().numpy()
    assert rel(eager1, eager0) <= 1e-6
    b.capture(packed, q)
    for _ in range(2):
        q.zero_()
        b.graph_launch()
        torch.cuda.synchronize()
        assert rel(q.double().cpu().numpy(), eager1) <= 1e-6
    b.close()


def test_batch_workload_sizes_vs_fp64_plans(torch_cuda):
    """The batched workload's discretisation (S = 6, 32 directions, Maxwell,
    N in {32, 48, 64}) on 12 cells: each cell against the FP64 single-cell path."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    S, M = 6.0, 32
    cells = I.cell_maxwellians_2d(12, seed=8806)
    plans = {N: pgc.Plan(dim=2, n_modes=N, scale=S, n_sigma=M, precision=pgc.FP64)
             for N in sorted({c["N"] for c in cells})}
    coeffs = [plans[c["N"]].project(I.perturbed_maxwellian_2d(plans[c["N"]].interior_velocities(), c))
              for c in cells]
    c32 = [x.float().double() for x in coeffs]
    refs = [plans[c["N"]].coeffs_to_q(x).cpu().numpy() for c, x in zip(cells, c32)]
    b = pgc.Batch([c["N"] for c in cells], scale=S, n_sigma=M, nufft_tol=TOL)
    say("workload batch: C=%d waves=%d units=%d points=%d" % (b.info.cells_per_wave, b.info.waves,
                                                              b.info.n_units, b.info.n_points))
    q = b.coeffs_to_q(b.pack([x.cpu().numpy() for x in c32]))
    torch.cuda.synchronize()
    errs = [rel(g, r) for g, r in zip(b.unpack(q), refs)]
    say("  per-cell rel-L2 vs FP64 path: max %.3e" % max(errs))
    assert max(errs) <= FP32_TOL
    b.close()
    for p in plans.values():
        p.close()


def test_batch_workload_n32_cells_vs_oracle(torch_cuda):
    """Cells of the batched workload itself (4096 cells drawn with its seed, S =
    6, 32 directions, Maxwell) at N = 32, taken from a 256-cell batch of mixed
    N: three of them against the oracle's full evaluation."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    S, M = 6.0, 32
    cells = I.cell_maxwellians_2d(256, seed=8806)
    coeffs, probs = cell_coeffs(cells, S, M)
    c32 = [x.astype(np.float32).astype(np.float64) for x in coeffs]
    b = pgc.Batch([c["N"] for c in cells], scale=S, n_sigma=M, nufft_tol=TOL)
    say("workload batch of 256 cells against the oracle at N = 32")
    q = b.unpack(b.coeffs_to_q(b.pack(c32)))
    torch.cuda.synchronize()
    picks = [i for i, c in enumerate(cells) if c["N"] == 32][:3]
    for i in picks:
        ref, _, _ = probs[32].collision(c32[i])
        r = rel(q[i], ref)
        say("  cell %d (N=32) rel-L2 vs oracle %.3e" % (i, r))
        assert r <= FP32_TOL
    b.close()
