"""Seeded synthetic inputs shared by the tests, the benchmark and the examples.

This module holds initial data only -- velocity distributions written as plain
functions of v, and seeded draws of their parameters.  It contains none of the
collision method's arithmetic (no nodes, maps, transforms or quadrature), so
the GPU library and the CPU oracle can both be fed from it without sharing
code.  Every draw uses numpy's PCG64 with an explicit seed.

Recipes (one per workload of the paper, Sec. 5):
  * BKW 2D / 3D: the closed-form BKW solutions of Sec. 5.1.1 / 5.2 at a time t.
  * two_maxwellians_2d: the initial data of the 2D moments test (Sec. 5.1.2),
    and the VHS workload: two isotropic Maxwellians of mass 1/2 each at
    +-(1.5, 0) with temperatures drawn from U[0.5, 1.5].
  * cell_maxwellians_2d: per spatial cell, density U[0.5, 2], bulk velocity
    U[-1, 1]^2, temperature U[0.5, 2], times 1 + 0.05 sum_{|a|=3} c_a He_a(c)
    with c = (v - u)/sqrt(T) and c_a ~ U[-1, 1] normalised to sum |c_a| = 1
    (third-order Hermite terms leave density, momentum and energy unchanged).
  * gaussian_mixtures_3d: 2-4 anisotropic (diagonal) Gaussians, means
    U[-2, 2]^3, variances U[0.3, 2], weights U[0.2, 1] normalised to unit mass.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ---------------------------------------------------------------- BKW data


def bkw_k(t: float, dim: int) -> float:
    """K(t) of the BKW solutions: 1 - exp(-t/8)/2 in 2D, 1 - exp(-t/6) in 3D."""
    return 1.0 - 0.5 * np.exp(-t / 8.0) if dim == 2 else 1.0 - np.exp(-t / 6.0)


def bkw_f(t: float, v: np.ndarray) -> np.ndarray:
    """The BKW distribution f(t, v) for Maxwell molecules with int B dsigma = 1.

    ``v`` has shape (..., dim) with dim 2 or 3.
    """
    v = np.asarray(v, dtype=np.float64)
    dim = v.shape[-1]
    K = bkw_k(t, dim)
    r2 = np.sum(v * v, axis=-1)
    if dim == 2:
        return (1.0 / (2 * np.pi * K * K)) * np.exp(-r2 / (2 * K)) * (2 * K - 1 + (1 - K) / (2 * K) * r2)
    return (1.0 / (2 * (2 * np.pi * K) ** 1.5)) * np.exp(-r2 / (2 * K)) * ((5 * K - 3) / K + (1 - K) / (K * K) * r2)


def bkw_q(t: float, v: np.ndarray) -> np.ndarray:
    """The exact collision operator of the BKW solution, df/dt (Sec. 5.1.1,
    eq. 2d_bkw_rhs, and its 3D counterpart of Sec. 5.2): the reference of the
    accuracy studies."""
    v = np.asarray(v, dtype=np.float64)
    dim = v.shape[-1]
    K = bkw_k(t, dim)
    r2 = np.sum(v * v, axis=-1)
    f = bkw_f(t, v)
    g = np.exp(-r2 / (2 * K))
    if dim == 2:
        dK = np.exp(-t / 8.0) / 16.0
        return ((-2.0 / K + r2 / (2 * K * K)) * f + g / (2 * np.pi * K * K) * (2.0 - r2 / (2 * K * K))) * dK
    dK = np.exp(-t / 6.0) / 6.0
    return ((-1.5 / K + r2 / (2 * K * K)) * f
            + g / (2 * (2 * np.pi * K) ** 1.5) * (3.0 / K ** 2 + (K - 2.0) / K ** 3 * r2)) * dK


# ---------------------------------------------------------- Maxwellian mixtures


def maxwellian(v, rho, u, T):
    """rho (2 pi T)^{-d/2} exp(-|v - u|^2 / (2T))."""
    v = np.asarray(v, dtype=np.float64)
    dim = v.shape[-1]
    d = v - np.asarray(u, dtype=np.float64)
    return rho / (2 * np.pi * T) ** (dim / 2) * np.exp(-np.sum(d * d, axis=-1) / (2 * T))


def mixture(v, comps):
    """Sum of Maxwellians; ``comps`` is a list of (rho, u, T)."""
    out = 0.0
    for rho, u, T in comps:
        out = out + maxwellian(v, rho, u, T)
    return out


def two_maxwellians_2d(seed: int = 2105):
    """Two isotropic Maxwellians of mass 1/2 at +-(1.5, 0), T ~ U[0.5, 1.5]."""
    T = rng(seed).uniform(0.5, 1.5, size=2)
    return [(0.5, (1.5, 0.0), float(T[0])), (0.5, (-1.5, 0.0), float(T[1]))]


def moments_test_2d():
    """Initial data of the paper's 2D moments test: rho = 1/2, T = 1, V1 = (-1, 2), V2 = (3, -3)."""
    return [(0.5, (-1.0, 2.0), 1.0), (0.5, (3.0, -3.0), 1.0)]


def _hermite(n, x):
    """Probabilists' Hermite polynomials He_0..He_3."""
    return [np.ones_like(x), x, x * x - 1.0, x * x * x - 3.0 * x][n]


def cell_maxwellians_2d(n_cells: int, seed: int = 8806, modes=(32, 48, 64)):
    """Per-cell parameters of the batched workload: a list of dicts."""
    g = rng(seed)
    Ns = g.choice(np.asarray(modes), size=n_cells)
    rho = g.uniform(0.5, 2.0, size=n_cells)
    u = g.uniform(-1.0, 1.0, size=(n_cells, 2))
    T = g.uniform(0.5, 2.0, size=n_cells)
    a = g.uniform(-1.0, 1.0, size=(n_cells, 4))
    a /= np.sum(np.abs(a), axis=1, keepdims=True)
    return [dict(N=int(Ns[c]), rho=float(rho[c]), u=u[c].copy(), T=float(T[c]), a=a[c].copy())
            for c in range(n_cells)]


def perturbed_maxwellian_2d(v, cell):
    """M (1 + 0.05 sum_{a1+a2=3} c_a He_a1(c1) He_a2(c2)), c = (v - u)/sqrt(T)."""
    v = np.asarray(v, dtype=np.float64)
    c = (v - cell["u"]) / np.sqrt(cell["T"])
    pert = 0.0
    for m, (a1, a2) in enumerate(((3, 0), (2, 1), (1, 2), (0, 3))):
        pert = pert + cell["a"][m] * _hermite(a1, c[..., 0]) * _hermite(a2, c[..., 1])
    return maxwellian(v, cell["rho"], cell["u"], cell["T"]) * (1.0 + 0.05 * pert)


def gaussian_mixtures_3d(n: int, seed: int = 2024):
    """``n`` mixtures of 2-4 diagonal Gaussians (list of lists of (w, mean, var))."""
    g = rng(seed)
    out = []
    for _ in range(n):
        m = int(g.integers(2, 5))
        w = g.uniform(0.2, 1.0, size=m)
        w /= w.sum()
        means = g.uniform(-2.0, 2.0, size=(m, 3))
        var = g.uniform(0.3, 2.0, size=(m, 3))
        out.append([(float(w[c]), means[c].copy(), var[c].copy()) for c in range(m)])
    return out


def gaussian_mixture(v, comps):
    """sum_c w_c prod_l N(v_l; mean_cl, var_cl)."""
    v = np.asarray(v, dtype=np.float64)
    out = 0.0
    for w, mean, var in comps:
        d = v - mean
        out = out + w * np.prod(np.exp(-d * d / (2 * var)) / np.sqrt(2 * np.pi * var), axis=-1)
    return out


def random_coeffs(shape, seed: int, decay: float = 0.35) -> np.ndarray:
    """Random coefficient tensor with geometric decay exp(-decay * sum k).

    Generic smooth-spectrum input for parity tests: any coefficient tensor is a
    valid argument of the collision map.
    """
    g = rng(seed)
    c = g.uniform(-1.0, 1.0, size=shape)
    ks = np.indices(shape).sum(axis=0)
    return c * np.exp(-decay * ks)
