"""FP64 CPU oracle for the Petrov-Galerkin mapped-Chebyshev collision operator.

TEST INFRASTRUCTURE ONLY.  This package checks the GPU library and shares no
code with it.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never does.

The arithmetic lives in ``pgc_oracle.c`` (plain C99 + OpenMP, FP64).  This
module only marshals numpy arrays into it and holds the plain set-up of the
paper's test problems (sphere rules, kernel constants).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile pgc_oracle.c into liboracle.so next to it (gcc, OpenMP)."""
    src = os.path.join(_HERE, "pgc_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
               src, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n_modes", ctypes.c_int),
        ("m_v", ctypes.c_int),
        ("map", ctypes.c_int),
        ("S", ctypes.c_double),
        ("kernel", ctypes.c_int),
        ("b0", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("n_sigma", ctypes.c_int),
        ("sigma", ctypes.POINTER(ctypes.c_double)),
        ("sigma_w", ctypes.POINTER(ctypes.c_double)),
        ("aniso", ctypes.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed with %d" % (what, rc))


def num_threads() -> int:
    return int(lib().ora_num_threads())


def cgl(m_v: int, map_: int, S: float):
    """CGL nodes xi, mapped v, weights w and mu^2 (endpoints included)."""
    xi, v, w, mu2 = (np.zeros(m_v) for _ in range(4))
    _check(lib().ora_cgl(m_v, map_, ctypes.c_double(S), _dp(xi), _dp(v), _dp(w), _dp(mu2)), "cgl")
    return xi, v, w, mu2


def gauss_legendre(n: int):
    x, w = np.zeros(n), np.zeros(n)
    _check(lib().ora_gauss_legendre(n, _dp(x), _dp(w)), "gauss_legendre")
    return x, w


def circle_rule(m: int):
    s, w = np.zeros((m, 2)), np.zeros(m)
    _check(lib().ora_circle_rule(m, _dp(s), _dp(w)), "circle_rule")
    return s, w


def sphere_product_rule(n_t: int, n_p: int):
    s, w = np.zeros((n_t * n_p, 3)), np.zeros(n_t * n_p)
    _check(lib().ora_sphere_product_rule(n_t, n_p, _dp(s), _dp(w)), "sphere_product_rule")
    return s, w


class Problem:
    """One discretised collision operator: dimension, modes, map, kernel, sphere rule.

    ``kernel`` is "maxwell" (B = b0), "vhs" (B = b0 |u|^gamma) or "aniso"
    (B = b0 |u|^gamma (1 + aniso cos^2 theta), cos theta = u.sigma/|u|).
    ``sphere`` is an (n_sigma x dim) array of unit vectors with ``sphere_w``
    its weights.
    """

    def __init__(self, dim, n_modes, S, map_=0, m_v=None, kernel="maxwell", b0=None,
                 gamma=0.0, sphere=None, sphere_w=None, aniso=0.0):
        self.dim = int(dim)
        self.n_modes = int(n_modes)
        self.m_v = int(m_v) if m_v else self.n_modes + 1
        self.map = int(map_)
        self.S = float(S)
        self.kernel = {"maxwell": 0, "vhs": 1, "aniso": 2}[kernel]
        self.aniso = float(aniso)
        if b0 is None:
            # Maxwell molecules normalised to int B dsigma = 1 (the BKW kernels)
            b0 = 1.0 / (2 * np.pi) if self.dim == 2 else 1.0 / (4 * np.pi)
        self.b0 = float(b0)
        self.gamma = float(gamma)
        self.sphere = np.ascontiguousarray(sphere, dtype=np.float64)
        self.sphere_w = np.ascontiguousarray(sphere_w, dtype=np.float64)
        assert self.sphere.shape == (self.sphere_w.size, self.dim)
        self._c = _Problem(self.dim, self.n_modes, self.m_v, self.map, self.S, self.kernel,
                           self.b0, self.gamma, int(self.sphere_w.size),
                           _dp(self.sphere), _dp(self.sphere_w), self.aniso)

    @property
    def n_int(self):
        return self.m_v - 2

    def shape(self):
        return (self.n_modes,) * self.dim

    def node_shape(self):
        return (self.n_int,) * self.dim

    def interior_velocities(self):
        """Interior node velocities as an (n_i^dim x dim) array, row-major."""
        _, v, _, _ = cgl(self.m_v, self.map, self.S)
        vi = v[1:-1]
        grids = np.meshgrid(*([vi] * self.dim), indexing="ij")
        return np.stack([g.ravel() for g in grids], axis=1)

    def project(self, f_int):
        f_int = np.ascontiguousarray(f_int, dtype=np.float64).reshape(-1)
        out = np.zeros(self.shape())
        _check(lib().ora_project(ctypes.byref(self._c), _dp(f_int), _dp(out)), "project")
        return out

    def nodal(self, coeffs):
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        out = np.zeros(self.node_shape())
        _check(lib().ora_nodal(ctypes.byref(self._c), _dp(c), _dp(out)), "nodal")
        return out

    def collision(self, coeffs):
        """(Q, Q+, Q-) as N^dim arrays."""
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        q, qp, qm = (np.zeros(self.shape()) for _ in range(3))
        _check(lib().ora_collision(ctypes.byref(self._c), _dp(c), _dp(q), _dp(qp), _dp(qm)),
               "collision")
        return q, qp, qm

    def collision_at(self, coeffs, kidx, gain=True):
        """(Q+, Q-) at the multi-indices kidx (n_k x dim); Q+ is None when
        gain is False (only the loss is formed)."""
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        k = np.ascontiguousarray(kidx, dtype=np.int32).reshape(-1, self.dim)
        qp, qm = np.zeros(len(k)), np.zeros(len(k))
        _check(lib().ora_collision_at(ctypes.byref(self._c), _dp(c), len(k), _ip(k),
                                      _dp(qp) if gain else None, _dp(qm)), "collision_at")
        return (qp if gain else None), qm

    def gain_units(self, coeffs, u_lo, u_hi):
        """Q+ restricted to the collision units [u_lo, u_hi), u = s * n_i^dim + i."""
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        out = np.zeros(self.shape())
        _check(lib().ora_gain_units(ctypes.byref(self._c), _dp(c), ctypes.c_int64(u_lo),
                                    ctypes.c_int64(u_hi), _dp(out)), "gain_units")
        return out

    def eval(self, coeffs, v):
        return eval_expansion(self.dim, self.n_modes, self.map, self.S, coeffs, v)

    def moments(self, coeffs):
        return moments(self.dim, self.n_modes, self.map, self.S, coeffs)

    def rk4(self, coeffs, dt, n_steps):
        c = np.array(coeffs, dtype=np.float64, copy=True, order="C")
        _check(lib().ora_rk4(ctypes.byref(self._c), _dp(c), ctypes.c_double(dt), int(n_steps)),
               "rk4")
        return c


def eval_expansion(dim, n_modes, map_, S, coeffs, v):
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, dim)
    out = np.zeros(len(v))
    _check(lib().ora_eval(dim, n_modes, map_, ctypes.c_double(S), _dp(c), ctypes.c_int64(len(v)),
                          _dp(v), _dp(out)), "eval")
    return out


def moment_functionals(n_modes, map_, S, pmax=2):
    out = np.zeros((pmax + 1, n_modes))
    _check(lib().ora_moment_functionals(n_modes, map_, ctypes.c_double(S), pmax, _dp(out)),
           "moment_functionals")
    return out


def moments(dim, n_modes, map_, S, coeffs):
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    out = np.zeros(dim + 2)
    _check(lib().ora_moments(dim, n_modes, map_, ctypes.c_double(S), _dp(c), _dp(out)), "moments")
    return out


def cosine_sum(z, q, n_modes):
    z = np.ascontiguousarray(z, dtype=np.float64)
    dim = z.shape[1]
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros((n_modes,) * dim)
    _check(lib().ora_cosine_sum(dim, ctypes.c_int64(len(q)), _dp(z), _dp(q), n_modes, _dp(out)),
           "cosine_sum")
    return out


__all__ = [
    "build", "lib", "cgl", "gauss_legendre", "circle_rule", "sphere_product_rule", "Problem",
    "eval_expansion", "moment_functionals", "moments", "cosine_sum", "num_threads",
]
