"""Closed forms printed in arXiv 2105.08806, used as pins for the oracle.

* 2D BKW: f and Q_BKW of Sec. 5.1.1 (eqs. 2d_bkw_initial, 2d_bkw_rhs).
* 3D BKW: f and Q_BKW of Sec. 5.2.
* Mapped Chebyshev test functions T^_k of eq. (1DCheby), written directly from
  the definition with numpy's arccos-based Chebyshev polynomials.
"""
import os

import numpy as np

from paper_2105_08806_amd.inputs import bkw_f, bkw_k

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def q_bkw(t, v):
    v = np.asarray(v, dtype=np.float64)
    dim = v.shape[-1]
    K = bkw_k(t, dim)
    r2 = np.sum(v * v, axis=-1)
    f = bkw_f(t, v)
    if dim == 2:
        Kp = np.exp(-t / 8.0) / 16.0
        return ((-2.0 / K + r2 / (2 * K * K)) * f
                + np.exp(-r2 / (2 * K)) / (2 * np.pi * K * K) * (2.0 - r2 / (2 * K * K))) * Kp
    Kp = np.exp(-t / 6.0) / 6.0
    return ((-1.5 / K + r2 / (2 * K * K)) * f
            + np.exp(-r2 / (2 * K)) / (2 * (2 * np.pi * K) ** 1.5) * (3.0 / K ** 2 + (K - 2.0) / K ** 3 * r2)) * Kp


def xi_of_v(v, S, map_):
    return np.tanh(v / S) if map_ == 0 else v / np.sqrt(S * S + v * v)


def mu2_of_xi(xi, S, map_):
    return (1.0 - xi * xi) ** ((1 + map_) / 2.0) / S


def cheb(k, x):
    return np.cos(k * np.arccos(np.clip(x, -1.0, 1.0)))


def c_k(k):
    return np.pi if k == 0 else np.pi / 2


def one_minus_xi2(v, S, map_):
    """1 - xi(v)^2 written in v (sech^2(v/S), resp. S^2/(S^2 + v^2))."""
    v = np.asarray(v, dtype=np.float64)
    if map_ == 0:
        e = np.exp(-2.0 * np.abs(v / S))   # sech^2 x = 4 e^{-2|x|} / (1 + e^{-2|x|})^2, no overflow
        return 4.0 * e / (1.0 + e) ** 2
    return S * S / (S * S + v * v)


def t_hat(k, v, S, map_):
    """T^_k(v) = mu(xi(v))^-2 T_k(xi(v)) / sqrt(c_k), mu^2 = (1 - xi^2)^{(1+r)/2} / S."""
    xi = xi_of_v(v, S, map_)
    mu2 = one_minus_xi2(v, S, map_) ** ((1 + map_) / 2.0) / S
    return cheb(k, xi) / (mu2 * np.sqrt(c_k(k)))


def t_tilde(k, v, S, map_):
    """T~_k(v) = mu(xi(v))^4 T_k(xi(v)) / sqrt(c_k)."""
    xi = xi_of_v(v, S, map_)
    mu2 = one_minus_xi2(v, S, map_) ** ((1 + map_) / 2.0) / S
    return cheb(k, xi) * mu2 * mu2 / np.sqrt(c_k(k))


def load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


def uniform_grid(dim, n, half=6.3):
    x = np.linspace(-half, half, n)
    g = np.meshgrid(*([x] * dim), indexing="ij")
    return np.stack([a.ravel() for a in g], axis=1), x[1] - x[0]
