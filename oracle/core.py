"""ctypes binding of the plain C oracle loops (oracle/sv_core.c).

Test infrastructure only.  ``build()`` compiles sv_core.c with gcc/OpenMP
into oracle/_sv_core.so; the functions below take numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_core.c")
_LIB = os.path.join(_HERE, "_sv_core.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build() -> str:
    """Compile the oracle core (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_prepare.argtypes = [_dp, ctypes.c_int, ctypes.c_uint64]
        L.orc_apply_exp.argtypes = [_dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double]
        L.orc_apply_product.argtypes = [_dp, ctypes.c_int, _u64p, _u64p, _dp, ctypes.c_int64, ctypes.c_int]
        L.orc_energy.argtypes = [_dp, ctypes.c_int, _u64p, _u64p, _dp, _i64p, ctypes.c_int64]
        L.orc_energy.restype = ctypes.c_double
        L.orc_sigma.argtypes = [_dp, _dp, ctypes.c_int, _u64p, _u64p, _dp, ctypes.c_int64]
        L.orc_vdot.argtypes = [_dp, _dp, ctypes.c_int, _dp, _dp]
        L.orc_energy_grad.argtypes = [ctypes.c_int, ctypes.c_uint64, _u64p, _u64p, _dp, ctypes.c_int64,
                                      _u64p, _u64p, _dp, ctypes.c_int64, _dp, _dp, _dp]
        L.orc_pool_grad.argtypes = [_dp, _dp, ctypes.c_int, _u64p, _u64p, _dp, _i64p, ctypes.c_int64, _dp]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the following calls."""
    lib().orc_set_threads(int(n))


def prepare(n: int, occ: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_prepare(_p(psi.view(np.float64), _dp), n, occ)
    return psi


def apply_product(psi: np.ndarray, n: int, xs, zs, th, inverse=False) -> np.ndarray:
    """In place on psi (complex128, contiguous); returns psi."""
    xs, zs, th = _u64(xs), _u64(zs), _f64(th)
    lib().orc_apply_product(_p(psi.view(np.float64), _dp), n, _p(xs, _u64p), _p(zs, _u64p),
                            _p(th, _dp), len(xs), int(inverse))
    return psi


def energy(psi: np.ndarray, n: int, xs, zs, cs, goff) -> float:
    xs, zs, cs = _u64(xs), _u64(zs), _f64(cs)
    goff = np.ascontiguousarray(goff, dtype=np.int64)
    return float(lib().orc_energy(_p(psi.view(np.float64), _dp), n, _p(xs, _u64p), _p(zs, _u64p),
                                  _p(cs, _dp), _p(goff, _i64p), len(goff) - 1))


def sigma(psi: np.ndarray, n: int, xs, zs, cs) -> np.ndarray:
    xs, zs, cs = _u64(xs), _u64(zs), _f64(cs)
    out = np.empty_like(psi)
    lib().orc_sigma(_p(psi.view(np.float64), _dp), _p(out.view(np.float64), _dp), n,
                    _p(xs, _u64p), _p(zs, _u64p), _p(cs, _dp), len(xs))
    return out


def vdot(a: np.ndarray, b: np.ndarray, n: int) -> complex:
    re = ctypes.c_double()
    im = ctypes.c_double()
    lib().orc_vdot(_p(a.view(np.float64), _dp), _p(b.view(np.float64), _dp), n,
                   ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def energy_grad(n: int, occ: int, ax, az, th, hx, hz, hc):
    """(E, dE/dtheta) by the adjoint sweep; allocates two states."""
    ax, az, th = _u64(ax), _u64(az), _f64(th)
    hx, hz, hc = _u64(hx), _u64(hz), _f64(hc)
    work = np.empty(4 << n, dtype=np.float64)
    E = ctypes.c_double()
    grad = np.zeros(len(ax))
    lib().orc_energy_grad(n, occ, _p(ax, _u64p), _p(az, _u64p), _p(th, _dp), len(ax),
                          _p(hx, _u64p), _p(hz, _u64p), _p(hc, _dp), len(hx),
                          _p(work, _dp), ctypes.byref(E), _p(grad, _dp))
    return float(E.value), grad


def pool_grad(psi: np.ndarray, lam: np.ndarray, n: int, xs, zs, cs, off) -> np.ndarray:
    """g_nu = -2 sum_{k in nu} c_k Im <lam|P_k|psi> (ADAPT pool gradients, lam = H psi)."""
    xs, zs, cs = _u64(xs), _u64(zs), _f64(cs)
    off = np.ascontiguousarray(off, dtype=np.int64)
    g = np.zeros(len(off) - 1)
    lib().orc_pool_grad(_p(psi.view(np.float64), _dp), _p(lam.view(np.float64), _dp), n, _p(xs, _u64p),
                        _p(zs, _u64p), _p(cs, _dp), _p(off, _i64p), len(off) - 1, _p(g, _dp))
    return g
