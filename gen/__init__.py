"""Seeded synthetic inputs for the oracle, the tests and the benchmark.

Holds no arithmetic of the Dirac operator: it only draws random numbers
(Philox4x32-10) and shapes them into gauge links, U(1) angles, spinors and
gauge transformations in the lexicographic site order of eq. (lexi) of the
paper (Sec. 4.1.1: time first, x3 fastest).  Both sides of every parity check
take their inputs from here; nothing here reads anything that either side
computes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "gen.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, u64, u32, dbl, ptr = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p
        lib.gen_philox4x32_10.argtypes = [ptr, ptr, ptr]
        lib.gen_su3_field.argtypes = [i64, dbl, u64, ptr]
        lib.gen_u1_field.argtypes = [i64, dbl, u64, ptr]
        lib.gen_spinor_field.argtypes = [i64, u64, u32, ptr]
        lib.gen_gauge_transform.argtypes = [i64, dbl, u64, ptr, ptr]
        lib.gen_uniforms.argtypes = [i64, u64, u32, ptr]
        _lib = lib
    return _lib


def volume(dims) -> int:
    return int(np.prod([int(d) for d in dims]))


def philox4x32_10(counter, key) -> np.ndarray:
    """One Philox4x32-10 block: counter (4 x uint32), key (2 x uint32) -> 4 x uint32."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().gen_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def su3_field(dims, eps: float, seed: int) -> np.ndarray:
    """U[site, mu, a, b] = exp(i eps H), H random traceless Hermitian (Gell-Mann, N(0,1) coefficients)."""
    V = volume(dims)
    out = np.empty((V, 4, 3, 3), dtype=np.complex128)
    _load().gen_su3_field(V, float(eps), int(seed), out.ctypes.data)
    return out


def u1_field(dims, theta_max: float, seed: int) -> np.ndarray:
    """theta[site, mu] uniform in (-theta_max, theta_max); the U(1) link is exp(i theta)."""
    V = volume(dims)
    out = np.empty((V, 4), dtype=np.float64)
    _load().gen_u1_field(V, float(theta_max), int(seed), out.ctypes.data)
    return out


def gaussian_spinor(dims, seed: int, index: int = 0) -> np.ndarray:
    """psi[site, spin, colour], complex128 with re, im ~ N(0,1)."""
    V = volume(dims)
    out = np.empty((V, 4, 3), dtype=np.complex128)
    _load().gen_spinor_field(V, int(seed), int(index), out.ctypes.data)
    return out


def point_source(dims, spin: int, colour: int, site: int = 0) -> np.ndarray:
    """eta(x)_{alpha a} = delta_{x, site} delta_{alpha, spin} delta_{a, colour}."""
    out = np.zeros((volume(dims), 4, 3), dtype=np.complex128)
    out[site, spin, colour] = 1.0
    return out


def gauge_transform(dims, seed: int, eps: float = 2.0):
    """Random local transformation: Omega[site] in SU(3) (3x3) and lambda[site] in (-pi, pi)."""
    V = volume(dims)
    om = np.empty((V, 3, 3), dtype=np.complex128)
    lam = np.empty(V, dtype=np.float64)
    _load().gen_gauge_transform(V, float(eps), int(seed), om.ctypes.data, lam.ctypes.data)
    return om, lam


def uniforms(n: int, seed: int, stream: int = 99) -> np.ndarray:
    out = np.empty(int(n), dtype=np.float64)
    _load().gen_uniforms(int(n), int(seed), int(stream), out.ctypes.data)
    return out


def unit_links(dims) -> np.ndarray:
    U = np.zeros((volume(dims), 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U
