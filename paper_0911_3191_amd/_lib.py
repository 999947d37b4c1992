"""ctypes binding of libwdslash.so (argument marshalling only).

Every function here forwards to the C entry point of the same name declared
in include/wd.h.  Device buffers are PyTorch tensors (their data_ptr() is
passed through), streams are torch streams.  Nothing is computed in Python:
if the shared library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# WD_LIB_PATH selects another build of the same library (e.g. a sanitizer build)
LIB_PATH = os.environ.get("WD_LIB_PATH") or os.path.join(HERE, "libwdslash.so")

WD_OK, WD_NOT_CONVERGED = 0, 1
WD_EINVAL, WD_ENOMEM, WD_EDEVICE, WD_EBREAKDOWN, WD_EUNSUPPORTED = -1, -2, -3, -4, -5
WD_FP64, WD_FP32, WD_HALF_I16, WD_HALF_F16 = 0, 1, 2, 3
PREC = {"fp64": WD_FP64, "fp32": WD_FP32, "i16": WD_HALF_I16, "f16": WD_HALF_F16}
STATUS_NAMES = {0: "WD_OK", 1: "WD_NOT_CONVERGED", -1: "WD_EINVAL", -2: "WD_ENOMEM",
                -3: "WD_EDEVICE", -4: "WD_EBREAKDOWN", -5: "WD_EUNSUPPORTED"}


class WDError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("t_antiperiodic", ctypes.c_int32)]

    @classmethod
    def make(cls, dims, t_antiperiodic: bool = True) -> "Lattice":
        lat = cls()
        for i, d in enumerate(dims):
            lat.dims[i] = int(d)
        lat.t_antiperiodic = 1 if t_antiperiodic else 0
        return lat


_lib = None


def lib():
    """Load libwdslash.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_0911_3191_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double, ctypes.c_size_t
        lp = ctypes.POINTER(Lattice)
        L.wd_last_error.restype = ctypes.c_char_p
        L.wd_version.restype = ctypes.c_char_p
        L.wd_gauge_bytes.argtypes = [lp, u32]
        L.wd_gauge_bytes.restype = sz
        L.wd_gauge_create.argtypes = [lp, vp, u32, vp, sz, vp, ctypes.POINTER(vp)]
        L.wd_gauge_create.restype = i32
        L.wd_gauge_bytes_ex.argtypes = [lp, u32, i32, u32]
        L.wd_gauge_bytes_ex.restype = sz
        L.wd_gauge_create_ex.argtypes = [lp, vp, u32, i32, u32, vp, sz, vp, ctypes.POINTER(vp)]
        L.wd_gauge_create_ex.restype = i32
        L.wd_gauge_fix_temporal.argtypes = [lp, vp, vp, vp, vp]
        L.wd_gauge_fix_temporal.restype = i32
        L.wd_gauge_rotate_spinor.argtypes = [lp, vp, vp, vp, i32, i32, vp]
        L.wd_gauge_rotate_spinor.restype = i32
        L.wd_gauge_destroy.argtypes = [vp]
        L.wd_gauge_destroy.restype = None
        L.wd_spinor_bytes.argtypes = [lp, i32, i32]
        L.wd_spinor_bytes.restype = sz
        for name in ("wd_spinor_encode", "wd_spinor_decode"):
            getattr(L, name).argtypes = [lp, i32, i32, vp, vp, vp]
            getattr(L, name).restype = i32
        for name in ("wd_spinor_encode_full", "wd_spinor_decode_full"):
            getattr(L, name).argtypes = [lp, i32, i32, i32, vp, vp, vp]
            getattr(L, name).restype = i32
        for name in ("wd_spinor_encode_basis", "wd_spinor_decode_basis"):
            getattr(L, name).argtypes = [lp, i32, i32, i32, vp, vp, vp]
            getattr(L, name).restype = i32
        L.wd_operator_workspace_bytes.argtypes = [lp, i32, i32]
        L.wd_operator_workspace_bytes.restype = sz
        L.wilson_dslash.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, sz, vp]
        L.wilson_dslash.restype = i32
        L.wilson_mat_pc.argtypes = [vp, dbl, vp, vp, i32, i32, i32, vp, sz, vp]
        L.wilson_mat_pc.restype = i32
        L.mdagm.argtypes = [vp, dbl, vp, vp, i32, i32, vp, sz, vp]
        L.mdagm.restype = i32
        L.mdagm_noalloc.argtypes = [vp, dbl, vp, vp, i32, i32, vp]
        L.mdagm_noalloc.restype = i32
        L.wd_dslash_field.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp]
        L.wd_dslash_field.restype = i32
        L.wd_dslash_field_basis.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, vp]
        L.wd_dslash_field_basis.restype = i32
        L.wd_mat_pc_field.argtypes = [vp, dbl, vp, vp, vp, i32, i32, i32, vp]
        L.wd_mat_pc_field.restype = i32
        L.wd_mdagm_field.argtypes = [vp, dbl, vp, vp, vp, vp, i32, i32, vp]
        L.wd_mdagm_field.restype = i32
        _declare_solver(L)
        _lib = L
    return _lib


def _declare_solver(L):
    """Solver and serving entry points."""
    from ._solver_types import declare, declare_server
    declare(L)
    declare_server(L)


def check(status: int, where: str) -> int:
    if status < 0:
        raise WDError(status, where, lib().wd_last_error().decode())
    return status


def ptr(t) -> ctypes.c_void_p:
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(t.data_ptr())


def stream_ptr(stream=None) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)
