"""Pins of the transport oracle (oracle/transport.py) against what the
mathematics fixes: the velocity matrix against an independent quadrature of
(v T~_l, T^_k), and the exact semi-discrete transport against the exact
free-streaming solution f(x - v_1 t, v) of f_t + v_1 f_x = 0 (Sec. 1: the
transport part of the full equation)."""
import numpy as np
import pytest
from scipy import integrate

import oracle as O
from oracle import transport as T
from closed_forms import t_hat, t_tilde
from paper_2105_08806_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


def test_velocity_matrix_by_quadrature():
    N, S = 7, 2.5
    V = T.velocity_matrix(N, S)
    for k in range(N):
        for l in range(N):
            val, _ = integrate.quad(lambda v: v * t_tilde(l, v, S, 0) * t_hat(k, v, S, 0), -60 * S, 60 * S,
                                    limit=800, points=[0.0])
            assert abs(V[k, l] - val) < 1e-10 * max(1.0, abs(val)), (k, l, V[k, l], val)
    assert np.allclose(V, V.T)


def cells_of(p, L, n_x, t, eps=0.5, wave=1):
    """Coefficients, cell by cell, of M(v) (1 + eps cos(2 pi wave (x - v_1 t) / L))."""
    V = p.interior_velocities()
    M = I.maxwellian(V, 1.0, (0.3, -0.2), 0.9)
    out = []
    for c in range(n_x):
        x = c * L / n_x
        out.append(p.project(M * (1.0 + eps * np.cos(2 * np.pi * wave * (x - V[:, 0] * t) / L))))
    return np.stack(out)


def test_transport_converges_to_free_streaming():
    """The Galerkin transport of a modulated Maxwellian approaches the
    projection of the exact free-streaming solution spectrally in N."""
    L, n_x, t, S = 8 * np.pi, 9, 0.8, 3.0
    errs = []
    for N in (8, 12, 16):
        sg, sw = O.circle_rule(4)
        p = O.Problem(2, N, S, 0, sphere=sg, sphere_w=sw)
        c0 = cells_of(p, L, n_x, 0.0)
        exact = cells_of(p, L, n_x, t)
        got = T.transport_step(c0, N, S, L, t)
        errs.append(np.linalg.norm(got - exact) / np.linalg.norm(exact - c0))
    assert errs[0] > 5 * errs[1] > 25 * errs[2], errs
    assert errs[2] < 2e-3, errs


def test_transport_invariants():
    """Mass (the wave-number 0 mode) is unchanged, steps compose, and a step
    of -dt undoes a step of dt."""
    N, S, L, n_x = 8, 2.5, 5.0, 7
    rng = np.random.default_rng(4)
    c = rng.standard_normal((n_x, N, N))
    a = T.transport_step(c, N, S, L, 0.3)
    assert np.allclose(a.sum(axis=0), c.sum(axis=0), atol=1e-12)
    b = T.transport_step(T.transport_step(c, N, S, L, 0.15), N, S, L, 0.15)
    assert np.allclose(a, b, atol=1e-12)
    assert np.allclose(T.transport_step(a, N, S, L, -0.3), c, atol=1e-12)
    with pytest.raises(ValueError):
        T.transport_step(np.zeros((6, N, N)), N, S, L, 0.1)
