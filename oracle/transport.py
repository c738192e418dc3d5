"""Transport step of the spatially inhomogeneous Boltzmann equation in the
coefficient space of the Petrov-Galerkin method (plain numpy / scipy, FP64).

TEST INFRASTRUCTURE ONLY: this module checks the GPU library and shares no
code with it.  Only tests/, __graft_entry__.smoke() and the cpu_baseline leg
of bench.py may import it.

The full equation adds the free-streaming term v . grad_x f to the
homogeneous equation the paper solves, and the two parts are usually treated
separately by operator splitting (Sec. 1, before eq. Boltz_eqn).  Here x is
one periodic space dimension along the first velocity component.  Testing
f_t + v_1 f_x = 0 for f_N = sum_l f_l T~_l against T^_k (the Petrov-Galerkin
step of Sec. 3, eq. petrov, with biorthogonality, eq. ortho) gives

    d/dt f_k + sum_l V_kl d/dx f_l = 0,     V_kl = (v_1 T~_l, T^_k),

acting on the first index of every coefficient tensor.  Only the logarithmic
map (r = 0) has a finite V: for r = 1, v T~_l T^_k decays like 1/|v|.
"""
from __future__ import annotations

import numpy as np
from scipy import linalg


def velocity_matrix(n_modes: int, S: float) -> np.ndarray:
    """V_kl = (v T~_l, T^_k) for the logarithmic map v = S atanh(xi) (Sec. 2.1).

    With T~_l = mu^4 T_l / sqrt(c_l), T^_k = mu^-2 T_k / sqrt(c_k) and
    dv = omega / mu^2 dxi (eq. 1D_mapping),
        V_kl = S / sqrt(c_k c_l) int_{-1}^{1} atanh(xi) T_k T_l omega dxi
             = S / sqrt(c_k c_l) int_0^pi ln cot(t/2) cos(kt) cos(lt) dt
    (xi = cos t).  The cosine series ln cot(t/2) = 2 sum_{n odd} cos(nt)/n
    gives int_0^pi ln cot(t/2) cos(mt) dt = pi/|m| for odd m and 0 otherwise,
    and cos(kt) cos(lt) = (cos((k-l)t) + cos((k+l)t))/2.
    """
    def I(m):
        m = abs(m)
        return np.pi / m if m % 2 == 1 else 0.0

    c = np.array([np.pi if k == 0 else np.pi / 2 for k in range(n_modes)])
    V = np.zeros((n_modes, n_modes))
    for k in range(n_modes):
        for l in range(n_modes):
            V[k, l] = S / np.sqrt(c[k] * c[l]) * 0.5 * (I(k - l) + I(k + l))
    return V


def transport_step(coeffs: np.ndarray, n_modes: int, S: float, length: float, dt: float) -> np.ndarray:
    """One exact step of the semi-discrete transport system over dt.

    coeffs has shape (n_x, N, ...) (cell index first, then the coefficient
    tensor with k_1 first) on the periodic grid x_c = c length / n_x, n_x odd.
    In x the state is a trigonometric polynomial; its Fourier mode of wave
    number kappa = 2 pi m / length evolves by exp(-i kappa dt V) along k_1.
    """
    n_x = coeffs.shape[0]
    if n_x % 2 != 1:
        raise ValueError("n_x must be odd (every Fourier mode has its conjugate partner)")
    V = velocity_matrix(n_modes, S)
    F = np.fft.fft(coeffs, axis=0)
    m = np.fft.fftfreq(n_x, d=1.0 / n_x)
    out = np.empty_like(F)
    for r in range(n_x):
        kappa = 2.0 * np.pi * m[r] / length
        E = linalg.expm(-1j * kappa * dt * V)
        out[r] = np.tensordot(E, F[r], axes=([1], [0]))
    return np.real(np.fft.ifft(out, axis=0))
