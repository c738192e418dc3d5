"""GPU parity of the spatial transport and the split step (pgc_transport_*,
pgc_split_step) against the transport oracle (oracle/transport.py: the
matrix exponential of the semi-discrete system per Fourier mode) and the
oracle's RK4 of the collisions.  Bars: rel-L2 1e-12 for the transport (no
transform tolerance is involved), 1e-11 for the split step (FP64)."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import transport as OT
from paper_2105_08806_amd import inputs as I

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def modulated(p, L, n_x, seed):
    """Per cell: a Maxwellian with a seeded density and bulk-velocity wave in x."""
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 3)
    V = p.interior_velocities()
    out = []
    for c in range(n_x):
        x = 2 * np.pi * c / n_x
        u = [0.4 * np.sin(x + ph[0]), 0.3 * np.cos(2 * x + ph[1]), 0.2][:p.dim]
        rho = 1.0 + 0.3 * np.cos(x + ph[2])
        out.append(p.project(I.maxwellian(V, rho, tuple(u), 0.9 + 0.1 * np.sin(x))))
    return np.stack(out)


@pytest.mark.parametrize("dim,N,n_x,dt", [(2, 12, 9, 0.4), (2, 9, 1, 0.3), (3, 6, 5, -0.25), (2, 16, 31, 1.7)])
def test_transport_step_vs_oracle(torch_cuda, dim, N, n_x, dt):
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    S, L = 3.0, 7.0
    if dim == 2:
        sg, sw = O.circle_rule(4)
        plan = pgc.Plan(dim=2, n_modes=N, scale=S, n_sigma=4)
    else:
        sg, sw = O.sphere_product_rule(2, 2)
        plan = pgc.Plan(dim=3, n_modes=N, scale=S, sphere=pgc.SPHERE_PRODUCT_3D, n_theta=2, n_phi=2)
    ora = O.Problem(dim, N, S, 0, sphere=sg, sphere_w=sw)
    c0 = modulated(ora, L, n_x, seed=N)
    ref = OT.transport_step(c0, N, S, L, dt)
    say("case: transport dim=%d N=%d n_x=%d dt=%g" % (dim, N, n_x, dt))
    t = pgc.Transport(plan, n_x, L, dt)
    speeds = t.speeds()
    assert np.allclose(np.sort(speeds), np.sort(np.linalg.eigvalsh(OT.velocity_matrix(N, S))), atol=1e-12)
    st = torch.tensor(c0.reshape(n_x, -1), device="cuda")
    t.step(st)
    torch.cuda.synchronize()
    got = st.cpu().numpy().reshape(c0.shape)
    r = rel(got, ref) if n_x > 1 else float(np.max(np.abs(got - c0)))
    say("  rel-L2 vs oracle %.3e (max speed %.3f)" % (r, t.info.max_speed))
    assert r <= 1e-12
    t.close()
    plan.close()


@pytest.mark.parametrize("use_direct", [False, True])
def test_split_step_vs_oracle(torch_cuda, use_direct):
    """Two Strang steps (transport dt/2, RK4 collisions over dt in every cell,
    transport dt/2) of the full equation, against the same composition of the
    oracle's transport and RK4."""
    torch = torch_cuda
    from paper_2105_08806_amd import pgc
    N, S, L, n_x, dt, M = 10, 3.0, 6.0, 5, 0.2, 8
    sg, sw = O.circle_rule(M)
    ora = O.Problem(2, N, S, 0, sphere=sg, sphere_w=sw)
    plan = pgc.Plan(dim=2, n_modes=N, scale=S, n_sigma=M)
    c = modulated(ora, L, n_x, seed=3)
    ref = c.copy()
    for _ in range(2):
        ref = OT.transport_step(ref, N, S, L, dt / 2)
        ref = np.stack([ora.rk4(ref[i], dt, 1) for i in range(n_x)])
        ref = OT.transport_step(ref, N, S, L, dt / 2)
    say("case: split step, collisions through %s" % ("the direct algorithm" if use_direct else "the plan"))
    half = pgc.Transport(plan, n_x, L, dt / 2)
    d = pgc.Direct(plan, max_cells=n_x) if use_direct else None
    st = torch.tensor(c.reshape(n_x, -1), device="cuda")
    half.split_step(st, n_steps=2, direct=d)
    torch.cuda.synchronize()
    got = st.cpu().numpy().reshape(c.shape)
    r = rel(got, ref)
    say("  rel-L2 vs oracle %.3e (change over the steps %.3e)" % (r, rel(ref, c)))
    assert r <= 1e-11
    if d is not None:
        d.close()
    half.close()
    plan.close()


def test_transport_refusals(torch_cuda):
    from paper_2105_08806_amd import pgc
    say("case: transport refusals")
    p1 = pgc.Plan(dim=2, n_modes=6, scale=3.0, n_sigma=4, map=pgc.MAP_ALGEBRAIC)
    with pytest.raises(pgc.PgcError):
        pgc.Transport(p1, 5, 1.0, 0.1)        # V is infinite for r = 1
    p1.close()
    p0 = pgc.Plan(dim=2, n_modes=6, scale=3.0, n_sigma=4)
    for bad in (dict(n_x=4, length=1.0, dt=0.1), dict(n_x=5, length=0.0, dt=0.1),
                dict(n_x=5, length=1.0, dt=float("nan"))):
        with pytest.raises(pgc.PgcError):
            pgc.Transport(p0, **bad)
    p0.close()
