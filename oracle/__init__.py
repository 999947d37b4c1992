"""FP64 CPU oracle for the even-odd Wilson-Dirac path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library neither links nor calls
it, and it imports nothing from the GPU package.

The arithmetic lives in ``wd_oracle.c`` (plain C99 complex double, OpenMP over
sites), compiled with gcc into ``libwdoracle.so``; this module only marshals
numpy arrays.  What each function follows in the paper:

  dslash_full, dslash_parity, dslash_parity_sites
      hopping term D of the Wilson-Dirac matrix (Section 3, Eq. 1), gamma
      matrices of the DeGrand-Rossi basis (Appendix B)
  mhat        even-odd Schur complement 1 - kappa^2 D_eo D_oe (Eq. 2)
  mfull       1 - kappa D, with kappa = 1/(2(4+m)) (Eq. 1 and Section 3)
  prepare, reconstruct
      the even-odd source and solution maps ("trivially reconstructed",
      Section 3), from the block form of 1 - kappa D
  bicgstab, cgnr
      BiCGstab on M_hat and CG on the normal equations (Section 5.1)
  encode_spinor16, decode_spinor16, encode_link16, decode_link16
      16-bit storage with a per-site norm (Section 4.6)
  encode_link8, decode_link8
      the 8-real SU(3) parametrization (Appendix A.2)
  gauge_fix_temporal, gauge_rotate_spinor
      the temporal gauge of Section 4.3 (all temporal links the unit matrix
      but on the last time slice) and the matching spinor rotation

Pins (tests marked "not gpu"): a dense brute-force matrix built from the
printed projector tables, the Clifford algebra, gamma5-hermiticity, the
free-field plane-wave spectrum, gauge covariance, locality, dense solves,
numpy's binary16 rounding, SU(3) unitarity and determinant of rebuilt
links, gauge covariance of D under the temporal-gauge rotation.

Layouts: gauge ``[V,4,3,3,2]``, full spinor ``[V,4,3,2]``, parity spinor
``[Vh,4,3,2]`` (any shape with those sizes, float64, C order).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wd_oracle.c")
_LIB = os.path.join(_HERE, "libwdoracle.so")
_LIB_SAN = os.path.join(_HERE, "libwdoracle_san.so")
_lib = None


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math: IEEE semantics are relied on).
    sanitize: libwdoracle_san.so, built with clang (the runtime of the
    sanitized HIP library) under AddressSanitizer and UndefinedBehaviorSanitizer,
    without OpenMP (its loops are correct serially); loaded when WD_ORACLE_LIB
    names it."""
    if sanitize:
        clang = "/opt/rocm/llvm/bin/clang"
        tmp = _LIB_SAN + ".tmp"
        subprocess.check_call([clang, "-O1", "-g", "-shared", "-fPIC", "-std=c11", "-fno-fast-math",
                               "-ffp-contract=off", "-fsanitize=address,undefined",
                               "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                               "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_SAN)
        return _LIB_SAN
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("WD_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u16p = ctypes.POINTER(ctypes.c_uint16)
        fp = ctypes.POINTER(ctypes.c_float)
        I, D, L = ctypes.c_int, ctypes.c_double, ctypes.c_int64
        lib.wdo_gamma.argtypes = [I, dp]
        lib.wdo_dslash_full.argtypes = [ip, I, dp, dp, dp, I]
        lib.wdo_dslash_parity.argtypes = [ip, I, dp, dp, dp, I, I]
        lib.wdo_dslash_parity_sites.argtypes = [ip, I, dp, dp, I, I, i64p, L, dp]
        lib.wdo_mhat.argtypes = [ip, I, dp, D, dp, dp, I]
        lib.wdo_mfull.argtypes = [ip, I, dp, D, dp, dp]
        lib.wdo_split.argtypes = [ip, dp, dp, dp]
        lib.wdo_join.argtypes = [ip, dp, dp, dp]
        lib.wdo_prepare.argtypes = [ip, I, dp, D, dp, dp]
        lib.wdo_reconstruct.argtypes = [ip, I, dp, D, dp, dp, dp]
        lib.wdo_true_relres.argtypes = [ip, I, dp, D, dp, dp]
        lib.wdo_true_relres.restype = D
        lib.wdo_bicgstab.argtypes = [ip, I, dp, D, dp, dp, D, I, dp]
        lib.wdo_cgnr.argtypes = [ip, I, dp, D, dp, dp, D, I, dp]
        lib.wdo_f32_to_f16.argtypes = [fp, u16p, L]
        lib.wdo_f16_to_f32.argtypes = [u16p, fp, L]
        lib.wdo_encode_spinor16.argtypes = [I, L, dp, u16p, fp]
        lib.wdo_decode_spinor16.argtypes = [I, L, u16p, fp, dp]
        lib.wdo_encode_link16.argtypes = [I, L, dp, u16p]
        lib.wdo_decode_link16.argtypes = [I, L, u16p, dp]
        lib.wdo_encode_link8.argtypes = [L, dp, dp]
        lib.wdo_decode_link8.argtypes = [L, dp, dp]
        lib.wdo_gauge_fix_temporal.argtypes = [ip, dp, dp, dp]
        lib.wdo_gauge_rotate_spinor.argtypes = [ip, dp, dp, dp, I, I]
        _lib = lib
    return _lib


def _dims(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    assert d.shape == (4,)
    return d, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _in(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _out(shape):
    a = np.zeros(shape, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vol(dims):
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def gamma(mu: int) -> np.ndarray:
    """The oracle's gamma_mu (mu = 0..3 for x, y, z, t) as a complex 4x4."""
    out, p = _out((4, 4, 2))
    _load().wdo_gamma(mu, p)
    return out[..., 0] + 1j * out[..., 1]


def dslash_full(dims, U, psi, dagger=False, antiperiodic_t=True):
    """D psi on the full lattice (Eq. 1 without the factor -1/2 and the mass)."""
    d, dp = _dims(dims)
    U, Up = _in(U)
    psi, pp = _in(psi)
    out, op = _out(psi.shape)
    _load().wdo_dslash_full(dp, int(antiperiodic_t), Up, pp, op, int(dagger))
    return out


def dslash_parity(dims, U, psi_in, out_parity, dagger=False, antiperiodic_t=True):
    """D_{p,1-p}: parity-(1-p) spinor in, parity-p spinor out (cb order)."""
    d, dp = _dims(dims)
    U, Up = _in(U)
    psi, pp = _in(psi_in)
    out, op = _out(psi.shape)
    _load().wdo_dslash_parity(dp, int(antiperiodic_t), Up, pp, op, int(out_parity), int(dagger))
    return out


def dslash_parity_sites(dims, U, psi_in, out_parity, cbs, dagger=False, antiperiodic_t=True):
    """D_{p,1-p} psi evaluated only at the output sites with cb indices ``cbs``."""
    d, dp = _dims(dims)
    U, Up = _in(U)
    psi, pp = _in(psi_in)
    cb = np.ascontiguousarray(cbs, dtype=np.int64)
    out, op = _out((cb.size, 4, 3, 2))
    _load().wdo_dslash_parity_sites(dp, int(antiperiodic_t), Up, pp, int(out_parity),
                                    int(dagger), cb.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    cb.size, op)
    return out


def mhat(dims, U, kappa, psi_e, dagger=False, antiperiodic_t=True):
    """M_hat psi_e = psi_e - kappa^2 D_eo D_oe psi_e (Eq. 2); dagger: its adjoint."""
    d, dp = _dims(dims)
    U, Up = _in(U)
    psi, pp = _in(psi_e)
    out, op = _out(psi.shape)
    _load().wdo_mhat(dp, int(antiperiodic_t), Up, float(kappa), pp, op, int(dagger))
    return out


def mfull(dims, U, kappa, psi, antiperiodic_t=True):
    """(1 - kappa D) psi on the full lattice."""
    d, dp = _dims(dims)
    U, Up = _in(U)
    psi, pp = _in(psi)
    out, op = _out(psi.shape)
    _load().wdo_mfull(dp, int(antiperiodic_t), Up, float(kappa), pp, op)
    return out


def split(dims, full):
    """Full-lattice spinor -> (even, odd) parity spinors in cb order."""
    d, dp = _dims(dims)
    full, fp = _in(full)
    vh = _vol(dims) // 2
    e, ep = _out((vh, 4, 3, 2))
    o, opp = _out((vh, 4, 3, 2))
    _load().wdo_split(dp, fp, ep, opp)
    return e, o


def join(dims, even, odd):
    d, dp = _dims(dims)
    e, ep = _in(even)
    o, opp = _in(odd)
    full, fp = _out((_vol(dims), 4, 3, 2))
    _load().wdo_join(dp, ep, opp, fp)
    return full


def prepare(dims, U, kappa, b_full, antiperiodic_t=True):
    """b_hat_e = b_e + kappa D_eo b_o."""
    d, dp = _dims(dims)
    U, Up = _in(U)
    b, bp = _in(b_full)
    out, op = _out((_vol(dims) // 2, 4, 3, 2))
    _load().wdo_prepare(dp, int(antiperiodic_t), Up, float(kappa), bp, op)
    return out


def reconstruct(dims, U, kappa, b_full, x_e, antiperiodic_t=True):
    """x_full from x_e: x_o = b_o + kappa D_oe x_e."""
    d, dp = _dims(dims)
    U, Up = _in(U)
    b, bp = _in(b_full)
    xe, xp = _in(x_e)
    out, op = _out((_vol(dims), 4, 3, 2))
    _load().wdo_reconstruct(dp, int(antiperiodic_t), Up, float(kappa), bp, xp, op)
    return out


def true_relres(dims, U, kappa, b_full, x_full, antiperiodic_t=True) -> float:
    """||b - (1 - kappa D) x|| / ||b|| in FP64 on the full lattice."""
    d, dp = _dims(dims)
    U, Up = _in(U)
    b, bp = _in(b_full)
    x, xp = _in(x_full)
    return float(_load().wdo_true_relres(dp, int(antiperiodic_t), Up, float(kappa), bp, xp))


def _solve(fn, dims, U, kappa, b_full, tol, maxiter, antiperiodic_t):
    d, dp = _dims(dims)
    U, Up = _in(U)
    b, bp = _in(b_full)
    x, xp = _out((_vol(dims), 4, 3, 2))
    info, ip = _out(4)
    fn(dp, int(antiperiodic_t), Up, float(kappa), bp, xp, float(tol), int(maxiter), ip)
    return x, {"iters": int(info[0]), "updates": int(info[1]), "converged": bool(info[2]),
               "true_relres": float(info[3])}


def bicgstab(dims, U, kappa, b_full, tol=1e-12, maxiter=10000, antiperiodic_t=True):
    """Solve (1 - kappa D) x = b via BiCGstab on M_hat; returns (x_full, info)."""
    return _solve(_load().wdo_bicgstab, dims, U, kappa, b_full, tol, maxiter, antiperiodic_t)


def cgnr(dims, U, kappa, b_full, tol=1e-12, maxiter=20000, antiperiodic_t=True):
    """Solve (1 - kappa D) x = b via CG on M_hat^dag M_hat; returns (x_full, info)."""
    return _solve(_load().wdo_cgnr, dims, U, kappa, b_full, tol, maxiter, antiperiodic_t)


def f32_to_f16_bits(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.zeros(x.shape, dtype=np.uint16)
    _load().wdo_f32_to_f16(x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)), x.size)
    return out


def f16_bits_to_f32(h) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint16)
    out = np.zeros(h.shape, dtype=np.float32)
    _load().wdo_f16_to_f32(h.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), h.size)
    return out


KIND = {"i16": 0, "f16": 1}


def encode_spinor16(kind: str, psi):
    """psi [n,4,3,2] float64 -> (q [n,24] uint16 bit patterns, norm [n] float32)."""
    psi, pp = _in(psi)
    n = psi.size // 24
    q = np.zeros((n, 24), dtype=np.uint16)
    nm = np.zeros(n, dtype=np.float32)
    _load().wdo_encode_spinor16(KIND[kind], n, pp, q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                nm.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return q, nm


def decode_spinor16(kind: str, q, norm):
    q = np.ascontiguousarray(q, dtype=np.uint16)
    nm = np.ascontiguousarray(norm, dtype=np.float32)
    n = nm.size
    out, op = _out((n, 4, 3, 2))
    _load().wdo_decode_spinor16(KIND[kind], n, q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                nm.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), op)
    return out


def encode_link16(kind: str, u):
    u, up = _in(u)
    q = np.zeros(u.shape, dtype=np.uint16)
    _load().wdo_encode_link16(KIND[kind], u.size, up, q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)))
    return q


def decode_link16(kind: str, q):
    q = np.ascontiguousarray(q, dtype=np.uint16)
    out, op = _out(q.shape)
    _load().wdo_decode_link16(KIND[kind], q.size, q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)), op)
    return out


def encode_link8(U):
    """links [..., 3, 3, 2] -> [..., 8]: Re/Im a2, a3, b1, arg a1, arg c1 (Appendix A.2)."""
    U, up = _in(U)
    n = U.size // 18
    out = np.zeros(U.shape[:-3] + (8,))
    _load().wdo_encode_link8(n, up, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def decode_link8(p):
    """[..., 8] -> links [..., 3, 3, 2] rebuilt as in Appendix A.2."""
    p, pp = _in(p)
    n = p.size // 8
    out, op = _out(p.shape[:-1] + (3, 3, 2))
    _load().wdo_decode_link8(n, pp, op)
    return out


def gauge_fix_temporal(dims, U):
    """(U in temporal gauge, g [V,3,3,2]) with U'_mu(x) = g(x) U_mu(x) g(x+mu)^dagger."""
    U, up = _in(U)
    V = _vol(dims)
    Uo, uop = _out((V, 4, 3, 3, 2))
    g, gp = _out((V, 3, 3, 2))
    d, dp = _dims(dims)
    _load().wdo_gauge_fix_temporal(dp, up, uop, gp)
    return Uo, g


def gauge_rotate_spinor(dims, g, psi, adjoint=False):
    """psi'(x) = g(x) psi(x) (or g(x)^dagger psi(x)); psi [nrhs?, V, 4, 3, 2]."""
    g, gp = _in(g)
    psi, pp = _in(psi)
    V = _vol(dims)
    nrhs = psi.size // (V * 24)
    out, op = _out(psi.shape)
    d, dp = _dims(dims)
    _load().wdo_gauge_rotate_spinor(dp, gp, pp, op, nrhs, 1 if adjoint else 0)
    return out
