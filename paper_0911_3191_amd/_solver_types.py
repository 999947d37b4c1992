"""ctypes declarations of the solver part of the C ABI (include/wd.h)."""
from __future__ import annotations

import ctypes


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("delta", ctypes.c_double), ("nrhs", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("x0_given", ctypes.c_int32), ("restart", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("status", ctypes.c_int32),
                ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("gflops", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def declare(L) -> None:
    from ._lib import Lattice
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    pp = ctypes.POINTER(SolveParams)
    ip = ctypes.POINTER(SolveInfo)
    L.wd_solve_workspace_bytes.argtypes = [ctypes.POINTER(Lattice), pp, i32]
    L.wd_solve_workspace_bytes.restype = sz
    for name in ("bicgstab_solve", "cg_solve"):
        fn = getattr(L, name)
        fn.argtypes = [vp, dbl, vp, vp, pp, ip, vp, sz, vp]
        fn.restype = i32
    L.wd_solver_begin.argtypes = [i32, vp, dbl, vp, vp, pp, vp, sz, vp, ctypes.POINTER(vp)]
    L.wd_solver_begin.restype = i32
    L.wd_solver_step.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.wd_solver_step.restype = i32
    L.wd_solver_end.argtypes = [vp, ip]
    L.wd_solver_end.restype = i32
    L.wd_solver_residuals.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.wd_solver_residuals.restype = i32


class ServeParams(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("iters_per_pump", ctypes.c_int32)]


def declare_server(L) -> None:
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    L.wd_server_create.argtypes = [vp, sz, ctypes.POINTER(ServeParams), ctypes.POINTER(vp)]
    L.wd_server_create.restype = i32
    L.wd_server_submit.argtypes = [vp, i32, vp, dbl, vp, vp, ctypes.POINTER(SolveParams), ctypes.POINTER(i64)]
    L.wd_server_submit.restype = i32
    L.wd_server_pump.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.wd_server_pump.restype = i32
    L.wd_server_poll.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(SolveInfo)]
    L.wd_server_poll.restype = i32
    L.wd_server_destroy.argtypes = [vp]
    L.wd_server_destroy.restype = i32
