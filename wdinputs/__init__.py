"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Nothing here computes any step of the Wilson-Dirac method: this module only
draws counter-based random numbers (Philox4x64-10) and turns them into SU(3)
links, Gaussian or uniform spinor components, point sources and random gauge
transformations.  The C source (``gen.c``) is compiled with gcc into
``libwdinputs.so`` next to it.

Layouts (float64 numpy arrays, complex numbers as trailing (re, im)):
  gauge          ``U[Lt, Lz, Ly, Lx, 4, 3, 3, 2]`` (x fastest, mu = x, y, z, t)
  full spinor    ``psi[Lt, Lz, Ly, Lx, 4, 3, 2]`` (spin, colour)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libwdinputs.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libwdinputs.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u64, i64, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.wdg_philox4x64_10.argtypes = [u64p, u64p, u64p]
        lib.wdg_gauge_random.argtypes = [dp, i64, dbl, u64]
        lib.wdg_su3_random.argtypes = [dp, i64, dbl, u64, u64]
        lib.wdg_spinor_gaussian.argtypes = [dp, i64, u64, u64]
        lib.wdg_uniform.argtypes = [dp, i64, u64, u64]
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox4x64_10(counter, key) -> np.ndarray:
    """One Philox4x64-10 block: four uint64 words for (counter[4], key[2])."""
    lib = _load()
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    p = ctypes.POINTER(ctypes.c_uint64)
    lib.wdg_philox4x64_10(c.ctypes.data_as(p), k.ctypes.data_as(p), out.ctypes.data_as(p))
    return out


def volume(dims) -> int:
    lx, ly, lz, lt = dims
    return int(lx) * int(ly) * int(lz) * int(lt)


def gauge_random(dims, eps: float, seed: int) -> np.ndarray:
    """Links U = exp(i eps H), H traceless Hermitian with Gaussian entries."""
    lx, ly, lz, lt = dims
    U = np.empty((lt, lz, ly, lx, 4, 3, 3, 2), dtype=np.float64)
    _load().wdg_gauge_random(_dptr(U), volume(dims), float(eps), int(seed))
    return U


def gauge_unit(dims) -> np.ndarray:
    """Free field: every link is the identity."""
    lx, ly, lz, lt = dims
    U = np.zeros((lt, lz, ly, lx, 4, 3, 3, 2), dtype=np.float64)
    for a in range(3):
        U[..., a, a, 0] = 1.0
    return U


def su3_random(n: int, eps: float, seed: int, stream: int = 0) -> np.ndarray:
    """n SU(3) matrices, shape (n, 3, 3, 2)."""
    W = np.empty((n, 3, 3, 2), dtype=np.float64)
    _load().wdg_su3_random(_dptr(W), int(n), float(eps), int(seed), int(stream))
    return W


def spinor_gaussian(dims, seed: int, stream: int = 1, nrhs: int | None = None) -> np.ndarray:
    """Gaussian source(s): re and im of every spin-colour component ~ N(0,1).

    With ``nrhs`` given, right-hand side k uses stream ``stream + k``.
    """
    lx, ly, lz, lt = dims
    if nrhs is None:
        psi = np.empty((lt, lz, ly, lx, 4, 3, 2), dtype=np.float64)
        _load().wdg_spinor_gaussian(_dptr(psi), volume(dims), int(seed), int(stream))
        return psi
    out = np.empty((nrhs, lt, lz, ly, lx, 4, 3, 2), dtype=np.float64)
    for k in range(nrhs):
        _load().wdg_spinor_gaussian(_dptr(out[k]), volume(dims), int(seed), int(stream + k))
    return out


def spinor_uniform(dims, seed: int, stream: int = 2) -> np.ndarray:
    """Spinor with every real component uniform in (0, 1)."""
    lx, ly, lz, lt = dims
    psi = np.empty((lt, lz, ly, lx, 4, 3, 2), dtype=np.float64)
    _load().wdg_uniform(_dptr(psi), psi.size, int(seed), int(stream))
    return psi


def point_sources(dims, site=(0, 0, 0, 0)) -> np.ndarray:
    """The 12 spin-colour unit vectors at one site, shape (12, Lt, Lz, Ly, Lx, 4, 3, 2)."""
    lx, ly, lz, lt = dims
    x, y, z, t = site
    out = np.zeros((12, lt, lz, ly, lx, 4, 3, 2), dtype=np.float64)
    for s in range(4):
        for c in range(3):
            out[3 * s + c, t, z, y, x, s, c, 0] = 1.0
    return out
