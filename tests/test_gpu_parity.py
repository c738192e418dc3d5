"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars (written here): rel-L2 over all coefficients <= 1e-11 for FP64 plans and
<= 1e-5 for FP32 plans, element by element on identical seeded inputs.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2105_08806_amd import inputs as I

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
FP32_TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    return torch


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def make_pair(dim, N, S, map_=0, kernel="maxwell", gamma=0.0, b0=None, n_sigma=8, prec=0, m_v=None,
              n_theta=2, n_phi=4, **tune):
    from paper_2105_08806_amd import pgc
    if dim == 2:
        sg, sw = O.circle_rule(n_sigma)
        sph = dict(sphere=pgc.SPHERE_UNIFORM_2D, n_sigma=n_sigma)
    else:
        sg, sw = O.sphere_product_rule(n_theta, n_phi)
        sph = dict(sphere=pgc.SPHERE_PRODUCT_3D, n_theta=n_theta, n_phi=n_phi)
    ora = O.Problem(dim, N, S, map_, m_v=m_v, kernel=kernel, b0=b0, gamma=gamma, sphere=sg, sphere_w=sw)
    plan = pgc.Plan(dim=dim, n_modes=N, scale=S, map=map_, m_v=m_v or 0,
                    kernel=pgc.KERNEL_MAXWELL if kernel == "maxwell" else pgc.KERNEL_VHS,
                    kernel_b0=b0 or 0.0, kernel_gamma=gamma, precision=prec, **sph, **tune)
    return ora, plan


def gpu_q(torch, plan, coeffs):
    c = torch.tensor(coeffs, dtype=plan.dtype, device="cuda")
    q, qp = plan.coeffs_to_q(c, want_qplus=True)
    torch.cuda.synchronize()
    return q.double().cpu().numpy(), qp.double().cpu().numpy()


def check_q(torch, ora, plan, coeffs, tol, label):
    say("case:", label, plan.info.n_triples, "triples,", plan.info.n_points, "points, W =",
        plan.info.kernel_width, "mode =", plan.info.gain_mode, "slabs =", plan.info.n_slabs,
        "bin items =", plan.info.n_bin_items)
    # the binned gain's per-cell offset polynomials reproduce the exact kernel
    # offset to the rounding of their coefficients
    assert 0.0 < plan.info.offset_fit_err <= 1e-15, plan.info.offset_fit_err
    q, qp = gpu_q(torch, plan, coeffs)
    q_ref, qp_ref, _ = ora.collision(coeffs)
    r, rp = rel_l2(q, q_ref), rel_l2(qp, qp_ref)
    say("  rel-L2 Q = %.3e  Q+ = %.3e" % (r, rp))
    assert r <= tol, (label, r)
    assert rp <= tol, (label, rp)
    return q, q_ref


# ----------------------------------------------------------------- tables


def test_nodes_match_oracle(torch_cuda):
    for map_ in (0, 1):
        ora, plan = make_pair(2, 9, 2.5, map_=map_)
        xi, v, w = plan.nodes()
        oxi, ov, ow, _ = O.cgl(ora.m_v, map_, 2.5)
        assert np.allclose(xi, oxi, rtol=0, atol=1e-15)
        assert np.allclose(w, ow, rtol=1e-15, atol=0)
        assert np.allclose(v[1:-1], ov[1:-1], rtol=1e-13, atol=1e-14)
        assert np.isinf(v[0]) and np.isinf(v[-1])
        plan.close()


# ----------------------------------------------------------------- FP64 parity


@pytest.mark.parametrize("map_", [0, 1])
@pytest.mark.parametrize("kernel", ["maxwell", "vhs"])
def test_q_parity_2d_fp64(torch_cuda, map_, kernel):
    ora, plan = make_pair(2, 13, 2.5, map_=map_, kernel=kernel, gamma=1.0 if kernel == "vhs" else 0.0,
                          b0=1.0 / (2 * np.pi), n_sigma=8)
    c = I.random_coeffs((13, 13), seed=11 + map_)
    check_q(torch_cuda, ora, plan, c, FP64_TOL, "2D N=13 map=%d %s random" % (map_, kernel))
    plan.close()


def test_q_parity_2d_bkw_config1(torch_cuda):
    """2D BKW at t0 = 0, N = 16, S = 4, Maxwell 1/(2 pi), 16 circle directions."""
    ora, plan = make_pair(2, 16, 4.0, n_sigma=16)
    c = ora.project(I.bkw_f(0.0, ora.interior_velocities()))
    check_q(torch_cuda, ora, plan, c, FP64_TOL, "2D BKW N=16")
    plan.close()


@pytest.mark.parametrize("map_", [0, 1])
def test_q_parity_3d_fp64(torch_cuda, map_):
    ora, plan = make_pair(3, 8, 2.0, map_=map_, n_theta=2, n_phi=4)
    comps = [(0.6, (0.4, -0.3, 0.2), 0.8), (0.4, (-0.7, 0.5, -0.1), 1.3)]
    c = ora.project(I.mixture(ora.interior_velocities(), comps))
    check_q(torch_cuda, ora, plan, c, FP64_TOL, "3D N=8 map=%d mixture" % map_)
    plan.close()


def test_q_parity_3d_vhs_many_slabs(torch_cuda):
    """Ragged slabs and chunks: 3 planes per slab, 7 chunks."""
    ora, plan = make_pair(3, 9, 2.2, kernel="vhs", gamma=1.0, b0=0.3, n_theta=2, n_phi=4,
                          slab_planes=3, n_chunks=7)
    assert plan.info.n_slabs > 5
    c = I.random_coeffs((9, 9, 9), seed=4)
    check_q(torch_cuda, ora, plan, c, FP64_TOL, "3D N=9 VHS slabs=3")
    plan.close()


def test_q_parity_2d_slabs_and_odd_mv(torch_cuda):
    ora, plan = make_pair(2, 11, 3.0, m_v=15, n_sigma=6, slab_planes=5, n_chunks=3)
    c = I.random_coeffs((11, 11), seed=9)
    check_q(torch_cuda, ora, plan, c, FP64_TOL, "2D N=11 m_v=15 slabs=5")
    plan.close()


def test_minimum_size_and_zero_input(torch_cuda):
    ora, plan = make_pair(2, 3, 1.5, n_sigma=4)
    c = I.random_coeffs((3, 3), seed=1)
    check_q(torch_cuda, ora, plan, c, FP64_TOL, "2D N=3")
    q, qp = gpu_q(torch_cuda, plan, np.zeros((3, 3)))
    assert np.all(q == 0) and np.all(qp == 0)
    plan.close()


# ----------------------------------------------------------------- FP32 parity


@pytest.mark.parametrize("dim", [2, 3])
def test_q_parity_fp32(torch_cuda, dim):
    if dim == 2:
        ora, plan = make_pair(2, 16, 3.0, n_sigma=16, prec=1)
        c = ora.project(I.mixture(ora.interior_velocities(), I.two_maxwellians_2d()))
    else:
        ora, plan = make_pair(3, 8, 2.0, n_theta=2, n_phi=4, prec=1)
        c = I.random_coeffs((8, 8, 8), seed=2)
    check_q(torch_cuda, ora, plan, c.astype(np.float32).astype(np.float64), FP32_TOL,
            "%dD FP32" % dim)
    plan.close()


# ----------------------------------------------------------------- other entry points


def test_project_moments_eval(torch_cuda):
    import torch
    for map_ in (0, 1):
        ora, plan = make_pair(2, 14, 2.5, map_=map_)
        V = ora.interior_velocities()
        f = I.mixture(V, [(0.7, (0.3, -0.2), 0.9), (0.3, (-0.5, 0.4), 1.4)])
        c_ref = ora.project(f)
        c = plan.project(f)
        torch.cuda.synchronize()
        assert np.max(np.abs(c.cpu().numpy() - c_ref)) < 1e-13
        m = plan.moments(torch.tensor(c_ref, device="cuda"))
        m_ref = ora.moments(c_ref)
        assert np.allclose(m.cpu().numpy(), m_ref, rtol=1e-12, atol=1e-13)
        pts = np.random.default_rng(0).uniform(-5, 5, size=(300, 2))
        e = plan.eval(torch.tensor(c_ref, device="cuda"), pts)
        e_ref = ora.eval(c_ref, pts)
        assert np.allclose(e.cpu().numpy(), e_ref, rtol=1e-12, atol=1e-15)
        plan.close()


@pytest.mark.parametrize("dim,N,m_v", [(2, 6, 258), (2, 6, 260), (3, 12, None), (3, 20, None)])
def test_projection_transform_forms(torch_cuda, dim, N, m_v):
    """The projection is one separable transform with the matrix C^T (N x n_i)
    along every axis.  The library takes one of three forms by size: all
    passes in one workgroup (3D N=12), pass by pass with the operands staged
    in LDS (n_i = 256, its largest case, and 3D N=20, above the fused form's
    work limit), or the plain pass for n_i > 256 (n_i = 258).  Each is
    checked against the oracle's projection."""
    import torch
    ora, plan = make_pair(dim, N, 3.0, m_v=m_v, n_sigma=2, n_theta=2, n_phi=2)
    assert plan.info.m_v == ora.m_v
    V = ora.interior_velocities()
    f = I.mixture(V, [(0.6, (0.4,) * dim, 0.8), (0.4, (-0.3,) * dim, 1.3)])
    c_ref = ora.project(f)
    c = plan.project(f)
    torch.cuda.synchronize()
    r = rel_l2(c.cpu().numpy(), c_ref)
    say("case: projection %dD N=%d n_i=%d: rel-L2 %.2e" % (dim, N, ora.n_int, r))
    assert r <= 1e-13
    plan.close()


def test_rk4_parity(torch_cuda):
    import torch
    ora, plan = make_pair(2, 12, 3.0, n_sigma=8)
    c0 = ora.project(I.bkw_f(0.0, ora.interior_velocities()))
    ref = ora.rk4(c0, 0.1, 3)
    state = torch.tensor(c0, dtype=torch.float64, device="cuda")
    plan.rk4(state, 0.1, 3)
    torch.cuda.synchronize()
    assert rel_l2(state.cpu().numpy(), ref) < 1e-12
    plan.close()


def test_invalid_arguments(torch_cuda):
    from paper_2105_08806_amd import pgc
    with pytest.raises(pgc.PgcError):
        pgc.Plan(dim=2, n_modes=8, n_sigma=7)          # odd circle rule
    with pytest.raises(pgc.PgcError):
        pgc.Plan(dim=4, n_modes=8)
    with pytest.raises(pgc.PgcError):
        pgc.Plan(dim=2, n_modes=2)
    s = np.array([[1.0, 0.0], [0.0, 1.0]])
    with pytest.raises(pgc.PgcError):
        pgc.Plan(dim=2, n_modes=8, sigma=s, sigma_w=np.ones(2))   # not antipodal


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_q_parity_both_gain_modes(torch_cuda, dim, prec):
    """The LDS-slab scheme and the binned scheme give the same Q within the bar."""
    from paper_2105_08806_amd import pgc
    N = 12 if dim == 2 else 8
    shape = (N,) * dim
    c = I.random_coeffs(shape, seed=21 + dim)
    tol = FP64_TOL if prec == 0 else FP32_TOL
    for mode in (pgc.GAIN_SLAB, pgc.GAIN_BINNED):
        if dim == 2:
            ora, plan = make_pair(2, N, 2.5, n_sigma=8, prec=prec, gain_mode=mode)
        else:
            ora, plan = make_pair(3, N, 2.0, n_theta=2, n_phi=4, prec=prec, gain_mode=mode)
        assert plan.info.gain_mode == mode
        check_q(torch_cuda, ora, plan, c.astype(np.float32).astype(np.float64) if prec else c, tol,
                "%dD mode=%d prec=%d" % (dim, mode, prec))
        plan.close()


@pytest.mark.parametrize("upsample", [2.0, 4.0])
@pytest.mark.parametrize("map_", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_q_parity_fp64_other_upsampling(torch_cuda, dim, map_, upsample):
    """The binned FP64 gain at upsampling 2 and 4 (other grid spacings for the
    per-cell offset fits, other kernel widths from the same tolerance) against
    the oracle."""
    N = 12 if dim == 2 else 7
    rule = dict(n_sigma=8) if dim == 2 else dict(n_theta=2, n_phi=4)
    ora, plan = make_pair(dim, N, 2.5, map_=map_, upsample=upsample, **rule)
    assert plan.info.upsample == upsample
    c = I.random_coeffs((N,) * dim, seed=41 + dim + 2 * map_)
    check_q(torch_cuda, ora, plan, c, FP64_TOL, "%dD N=%d map=%d upsample %.0f" % (dim, N, map_, upsample))
    plan.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_binned_matches_slabs_every_width(torch_cuda, dim, prec):
    """For every kernel width the binned gain is built for (W = 4 .. 14: lane
    layouts with one, two or more points per step, partial last passes and
    the reduction of lane groups), the binned and the LDS-slab schemes, which
    share no spreading code, give the same Q whatever the transform accuracy
    of that width: up to summation order in FP64; in FP32 within 1e-6 (the
    slab scheme evaluates the kernel polynomial in FP32, the binned one in FP64
    rounded once)."""
    from paper_2105_08806_amd import pgc
    torch = torch_cuda
    N = 10 if dim == 2 else 6
    c = I.random_coeffs((N,) * dim, seed=31 + dim)
    if prec:
        c = c.astype(np.float32).astype(np.float64)
    rule = dict(n_sigma=8) if dim == 2 else dict(n_theta=2, n_phi=4)
    tol_qp, tol_q = (1e-13, 1e-12) if prec == 0 else (1e-6, 1e-6)
    for W in range(4, 15):
        out = []
        for mode in (pgc.GAIN_SLAB, pgc.GAIN_BINNED):
            _, plan = make_pair(dim, N, 2.5, kernel_width=W, gain_mode=mode, prec=prec, **rule)
            assert plan.info.kernel_width == W and plan.info.gain_mode == mode
            out.append(gpu_q(torch, plan, c))
            plan.close()
        (q_s, qp_s), (q_b, qp_b) = out
        r, rp = rel_l2(q_b, q_s), rel_l2(qp_b, qp_s)
        say("%dD prec=%d W=%d binned vs slabs: rel-L2 Q %.2e Q+ %.2e" % (dim, prec, W, r, rp))
        assert rp <= tol_qp and r <= tol_q, (W, r, rp)


@pytest.mark.parametrize("map_", [0, 1])
def test_velocity_fits_cover_the_grid(torch_cuda, map_):
    """The binned gain takes a point's kernel offset and map factor from a
    per-cell polynomial in v/S wherever the plan found one within 5e-16 (the
    cell's velocity interval narrow against the distance of the map's
    singularities from the real axis): all bin coordinates but the few at the
    ends of the grid, 93 of the 97 of the N = 32 grid for the logarithmic map
    and 87 for the algebraic one (computed for this grid in long double).  The
    other cells go through the map to w.  Both kinds of cell carry points of
    one plan, whose Q agrees with the slab scheme, which maps every point
    through the exact arctangent, to rounding."""
    from paper_2105_08806_amd import pgc
    torch = torch_cuda
    N = 32
    c = I.random_coeffs((N, N), seed=41 + map_)
    out = []
    for mode in (pgc.GAIN_SLAB, pgc.GAIN_BINNED):
        plan = pgc.Plan(dim=2, n_modes=N, scale=5.0, map=map_, kernel=pgc.KERNEL_MAXWELL, n_sigma=8,
                        precision=pgc.FP64, gain_mode=mode)
        info = plan.info
        say("case: map=%d mode=%d grid_folded=%d velocity_fit_cells=%d" % (
            map_, mode, info.grid_folded, info.velocity_fit_cells))
        assert info.grid_folded == 97
        assert info.velocity_fit_cells == (93 if map_ == 0 else 87)
        out.append(gpu_q(torch, plan, c))
        plan.close()
    (q_s, qp_s), (q_b, qp_b) = out
    r, rp = rel_l2(q_b, q_s), rel_l2(qp_b, qp_s)
    say("  binned vs slabs: rel-L2 Q %.2e Q+ %.2e" % (r, rp))
    assert rp <= 1e-13 and r <= 1e-12
    # FP32 plans fit to degree 7 within 2e-10, which covers 93 (r = 0) and 85
    # (r = 1) of the cells; their Q meets the FP32 bar against the FP64 plan's
    plan = pgc.Plan(dim=2, n_modes=N, scale=5.0, map=map_, kernel=pgc.KERNEL_MAXWELL, n_sigma=8,
                    precision=pgc.FP32, nufft_tol=1e-8)
    say("case: FP32 map=%d velocity_fit_cells=%d" % (map_, plan.info.velocity_fit_cells))
    assert plan.info.velocity_fit_cells == (93 if map_ == 0 else 85)
    q32, qp32 = gpu_q(torch, plan, c)
    plan.close()
    r32 = rel_l2(qp32, qp_b)
    say("  FP32 binned vs FP64 binned: rel-L2 Q+ %.2e" % r32)
    assert r32 <= FP32_TOL


def test_binned_limits_at_the_largest_node_count(torch_cuda):
    """The binned scheme's point ids hold a first-dimension node in 8 bits: at
    the largest node count (2D, m_v = 258, 256 interior nodes) binned and slab
    schemes agree within 5e-12 (2.2e9 points summed in different orders, with
    kernel offsets from the direct map in one and the cell fits in the other:
    measured 9e-13); one node more falls back to the slabs automatically and
    is refused when the bins are asked for."""
    from paper_2105_08806_amd import pgc
    torch = torch_cuda
    N = 6
    c = I.random_coeffs((N, N), seed=51)
    out = []
    for mode in (pgc.GAIN_SLAB, pgc.GAIN_BINNED):
        plan = pgc.Plan(dim=2, n_modes=N, m_v=258, scale=4.0, sphere=pgc.SPHERE_UNIFORM_2D, n_sigma=2,
                        gain_mode=mode)
        assert plan.info.gain_mode == mode and plan.info.m_v - 2 == 256
        out.append(gpu_q(torch, plan, c))
        plan.close()
    (q_s, qp_s), (q_b, qp_b) = out
    r, rp = rel_l2(q_b, q_s), rel_l2(qp_b, qp_s)
    say("2D 256 interior nodes binned vs slabs: rel-L2 Q %.2e Q+ %.2e" % (r, rp))
    assert rp <= 5e-12 and r <= 5e-12
    plan = pgc.Plan(dim=2, n_modes=N, m_v=259, scale=4.0, sphere=pgc.SPHERE_UNIFORM_2D, n_sigma=2)
    assert plan.info.gain_mode == pgc.GAIN_SLAB
    plan.close()
    with pytest.raises(pgc.PgcError):
        pgc.Plan(dim=2, n_modes=N, m_v=259, scale=4.0, sphere=pgc.SPHERE_UNIFORM_2D, n_sigma=2,
                 gain_mode=pgc.GAIN_BINNED)


@pytest.mark.parametrize("map_", [0, 1])
@pytest.mark.parametrize("kernel", ["maxwell", "vhs"])
def test_q_parity_3d_fp64_matrix_cores(torch_cuda, map_, kernel):
    """The FP64 binned gain on the matrix cores (gain_mode 3) against the oracle."""
    from paper_2105_08806_amd import pgc
    ora, plan = make_pair(3, 8, 2.0, map_=map_, kernel=kernel, gamma=1.0 if kernel == "vhs" else 0.0,
                          b0=0.3 if kernel == "vhs" else None, n_theta=2, n_phi=4, gain_mode=pgc.GAIN_MFMA)
    assert plan.info.gain_mode == pgc.GAIN_MFMA
    c = I.random_coeffs((8, 8, 8), seed=31 + map_)
    check_q(torch_cuda, ora, plan, c, FP64_TOL, "3D N=8 map=%d %s matrix cores" % (map_, kernel))
    plan.close()


def test_matrix_core_gain_rejects_unsupported_plans(torch_cuda):
    from paper_2105_08806_amd import pgc
    with pytest.raises(pgc.PgcError):
        pgc.Plan(dim=3, n_modes=8, sphere=pgc.SPHERE_PRODUCT_3D, n_theta=2, n_phi=4, precision=pgc.FP32,
                 gain_mode=pgc.GAIN_MFMA)
    with pytest.raises(pgc.PgcError):
        pgc.Plan(dim=2, n_modes=8, n_sigma=8, gain_mode=pgc.GAIN_MFMA)
