"""MI355X (gfx950) Wilson-Dirac dslash and mixed-precision solvers.

Thin Python layer over the C ABI of libwdslash.so (include/wd.h).  Functions
keep the C names; device memory comes from PyTorch tensors and streams from
torch.cuda.  Every operation runs in the library's HIP kernels -- there is no
Python or CPU fallback.
"""
from __future__ import annotations

import ctypes

from ._lib import (PREC, WD_EBREAKDOWN, WD_EDEVICE, WD_EINVAL, WD_ENOMEM, WD_EUNSUPPORTED, WD_FP32, WD_FP64,
                   WD_HALF_F16, WD_HALF_I16, WD_NOT_CONVERGED, WD_OK, Lattice, WDError, check, lib, ptr,
                   stream_ptr)

__all__ = [
    "Lattice", "WDError", "Gauge", "PREC", "WD_FP64", "WD_FP32", "WD_HALF_I16", "WD_HALF_F16",
    "lattice", "prec_of", "wd_gauge_bytes", "wd_spinor_bytes", "new_field", "wd_spinor_encode",
    "wd_spinor_decode", "wd_spinor_encode_full", "wd_spinor_decode_full", "wilson_dslash",
    "wd_spinor_encode_basis", "wd_spinor_decode_basis", "wd_dslash_field", "wd_dslash_field_basis",
    "wd_mat_pc_field", "wd_mdagm_field", "wd_operator_workspace_bytes", "new_operator_workspace",
    "WD_BASIS_DEGRAND_ROSSI", "WD_BASIS_UKQCD",
    "wilson_mat_pc", "mdagm", "mdagm_noalloc", "gauge_fix_temporal", "wd_gauge_rotate_spinor", "WD_GAUGE_TEMPORAL",
]


def prec_of(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


def lattice(dims, t_antiperiodic: bool = True) -> Lattice:
    return Lattice.make(dims, t_antiperiodic)


def wd_gauge_bytes(lat: Lattice, prec_mask: int) -> int:
    return int(lib().wd_gauge_bytes(ctypes.byref(lat), prec_mask))


def wd_spinor_bytes(lat: Lattice, prec, nrhs: int = 1) -> int:
    return int(lib().wd_spinor_bytes(ctypes.byref(lat), prec_of(prec), nrhs))


def new_field(lat: Lattice, prec, nrhs: int = 1, device="cuda"):
    """Uninitialised device buffer for one encoded parity field."""
    import torch
    n = wd_spinor_bytes(lat, prec, nrhs)
    if n == 0:
        raise WDError(-1, "new_field", "invalid lattice, precision or nrhs")
    return torch.empty(n, dtype=torch.uint8, device=device)


WD_GAUGE_TEMPORAL = 1
WD_BASIS_DEGRAND_ROSSI, WD_BASIS_UKQCD = 0, 1


class Gauge:
    """A resident gauge field: device buffer (torch) + library handle.

    recon: 12 or 8 reals per stored link; temporal: the field is in temporal
    gauge (see gauge_fix_temporal) and the unit time links are not read."""

    def __init__(self, lat: Lattice, U_dev, precs=("fp64", "fp32", "i16", "f16"), stream=None, recon=12,
                 temporal=False):
        import torch
        self.lat = lat
        self.mask = 0
        for p in precs:
            self.mask |= 1 << prec_of(p)
        self.recon = recon
        self.flags = WD_GAUGE_TEMPORAL if temporal else 0
        nbytes = lib().wd_gauge_bytes_ex(ctypes.byref(lat), self.mask, recon, self.flags)
        if nbytes == 0:
            raise WDError(-1, "Gauge", "invalid lattice, precision mask, recon or flags")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=U_dev.device)
        h = ctypes.c_void_p()
        check(lib().wd_gauge_create_ex(ctypes.byref(lat), ptr(U_dev), self.mask, recon, self.flags, ptr(self.buf),
                                       nbytes, stream_ptr(stream), ctypes.byref(h)), "wd_gauge_create_ex")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().wd_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gauge_fix_temporal(lat: Lattice, U_dev, stream=None):
    """(U in temporal gauge, g) as new device tensors: U'_mu(x) = g(x) U_mu(x) g(x+mu)^dagger."""
    import torch
    V = int(U_dev.numel() // 72)
    Uo = torch.empty_like(U_dev)
    g = torch.empty((V, 3, 3, 2), dtype=torch.float64, device=U_dev.device)
    check(lib().wd_gauge_fix_temporal(ctypes.byref(lat), ptr(U_dev), ptr(Uo), ptr(g), stream_ptr(stream)),
          "wd_gauge_fix_temporal")
    return Uo, g


def wd_gauge_rotate_spinor(lat: Lattice, g, out, inp, nrhs: int = 1, adjoint: bool = False, stream=None):
    return check(lib().wd_gauge_rotate_spinor(ctypes.byref(lat), ptr(g), ptr(out), ptr(inp), nrhs,
                                              1 if adjoint else 0, stream_ptr(stream)), "wd_gauge_rotate_spinor")


def wd_spinor_encode(lat, prec, nrhs, field, canon, stream=None):
    return check(lib().wd_spinor_encode(ctypes.byref(lat), prec_of(prec), nrhs, ptr(field), ptr(canon),
                                        stream_ptr(stream)), "wd_spinor_encode")


def wd_spinor_decode(lat, prec, nrhs, canon, field, stream=None):
    return check(lib().wd_spinor_decode(ctypes.byref(lat), prec_of(prec), nrhs, ptr(canon), ptr(field),
                                        stream_ptr(stream)), "wd_spinor_decode")


def wd_spinor_encode_basis(lat, prec, nrhs, basis, field, canon, stream=None):
    return check(lib().wd_spinor_encode_basis(ctypes.byref(lat), prec_of(prec), nrhs, basis, ptr(field),
                                              ptr(canon), stream_ptr(stream)), "wd_spinor_encode_basis")


def wd_spinor_decode_basis(lat, prec, nrhs, basis, canon, field, stream=None):
    return check(lib().wd_spinor_decode_basis(ctypes.byref(lat), prec_of(prec), nrhs, basis, ptr(canon),
                                              ptr(field), stream_ptr(stream)), "wd_spinor_decode_basis")


def wd_spinor_encode_full(lat, prec, nrhs, parity, field, canon_full, stream=None):
    return check(lib().wd_spinor_encode_full(ctypes.byref(lat), prec_of(prec), nrhs, parity, ptr(field),
                                             ptr(canon_full), stream_ptr(stream)), "wd_spinor_encode_full")


def wd_spinor_decode_full(lat, prec, nrhs, parity, canon_full, field, stream=None):
    return check(lib().wd_spinor_decode_full(ctypes.byref(lat), prec_of(prec), nrhs, parity,
                                             ptr(canon_full), ptr(field), stream_ptr(stream)),
                 "wd_spinor_decode_full")


def wd_operator_workspace_bytes(lat: Lattice, prec, nrhs: int = 1) -> int:
    return int(lib().wd_operator_workspace_bytes(ctypes.byref(lat), prec_of(prec), nrhs))


def new_operator_workspace(lat: Lattice, prec, nrhs: int = 1, device="cuda"):
    """Device workspace of wilson_dslash / wilson_mat_pc / mdagm."""
    import torch
    n = wd_operator_workspace_bytes(lat, prec, nrhs)
    if n == 0:
        raise WDError(-1, "new_operator_workspace", "invalid lattice, precision or nrhs")
    return torch.empty(n, dtype=torch.uint8, device=device)


def wilson_dslash(gauge: Gauge, out, inp, out_parity: int, dagger: int, prec, nrhs: int, workspace,
                  stream=None):
    """out, inp: canonical FP64 parity spinors (device tensors)."""
    return check(lib().wilson_dslash(gauge.handle, ptr(out), ptr(inp), out_parity, dagger, prec_of(prec), nrhs,
                                     ptr(workspace), workspace.numel(), stream_ptr(stream)), "wilson_dslash")


def wilson_mat_pc(gauge: Gauge, kappa: float, out, inp, dagger: int, prec, nrhs: int, workspace, stream=None):
    return check(lib().wilson_mat_pc(gauge.handle, kappa, ptr(out), ptr(inp), dagger, prec_of(prec), nrhs,
                                     ptr(workspace), workspace.numel(), stream_ptr(stream)), "wilson_mat_pc")


def mdagm(gauge: Gauge, kappa: float, out, inp, prec, nrhs: int, workspace, stream=None):
    return check(lib().mdagm(gauge.handle, kappa, ptr(out), ptr(inp), prec_of(prec), nrhs, ptr(workspace),
                             workspace.numel(), stream_ptr(stream)), "mdagm")


def mdagm_noalloc(gauge: Gauge, kappa: float, out, inp, prec, nrhs: int, stream=None):
    """mdagm with its scratch in the library's static device array (no workspace)."""
    return check(lib().mdagm_noalloc(gauge.handle, kappa, ptr(out), ptr(inp), prec_of(prec), nrhs,
                                     stream_ptr(stream)), "mdagm_noalloc")


def wd_dslash_field(gauge: Gauge, out, inp, out_parity: int, dagger: int, prec, nrhs: int = 1, stream=None):
    """Fast path on encoded fields (see wd_spinor_encode*)."""
    return check(lib().wd_dslash_field(gauge.handle, ptr(out), ptr(inp), out_parity, dagger, prec_of(prec),
                                       nrhs, stream_ptr(stream)), "wd_dslash_field")


def wd_dslash_field_basis(gauge: Gauge, out, inp, out_parity: int, dagger: int, prec, nrhs: int = 1,
                          basis: int = 1, stream=None):
    return check(lib().wd_dslash_field_basis(gauge.handle, ptr(out), ptr(inp), out_parity, dagger,
                                             prec_of(prec), nrhs, basis, stream_ptr(stream)),
                 "wd_dslash_field_basis")


def wd_mat_pc_field(gauge: Gauge, kappa: float, out, inp, tmp_odd, dagger: int, prec, nrhs: int = 1,
                    stream=None):
    return check(lib().wd_mat_pc_field(gauge.handle, kappa, ptr(out), ptr(inp), ptr(tmp_odd), dagger,
                                       prec_of(prec), nrhs, stream_ptr(stream)), "wd_mat_pc_field")


def wd_mdagm_field(gauge: Gauge, kappa: float, out, inp, tmp_odd, tmp_even, prec, nrhs: int = 1, stream=None):
    return check(lib().wd_mdagm_field(gauge.handle, kappa, ptr(out), ptr(inp), ptr(tmp_odd), ptr(tmp_even),
                                      prec_of(prec), nrhs, stream_ptr(stream)), "wd_mdagm_field")


# ---- solvers ------------------------------------------------------------------------
from ._solver_types import SolveInfo, SolveParams  # noqa: E402

WD_SOLVER_BICGSTAB, WD_SOLVER_CG = 0, 1
SOLVER = {"bicgstab": WD_SOLVER_BICGSTAB, "cg": WD_SOLVER_CG}


def solve_params(tol=1e-12, maxiter=10000, inner="fp64", delta=0.1, nrhs=1, use_graph=False,
                 restart=False, check_every=0) -> SolveParams:
    """restart=False: reliable updates (Algorithm 2); True: defect correction
    (Algorithm 1) with inner tolerance delta.  check_every: iterations per
    read of the flags by the host (0 or 1: every iteration)."""
    return SolveParams(tol=tol, maxiter=maxiter, inner=prec_of(inner), delta=delta, nrhs=nrhs,
                       use_graph=1 if use_graph else 0, check_every=int(check_every), x0_given=0,
                       restart=1 if restart else 0)


def wd_solve_workspace_bytes(lat: Lattice, params: SolveParams, solver) -> int:
    kind = SOLVER[solver] if isinstance(solver, str) else int(solver)
    return int(lib().wd_solve_workspace_bytes(ctypes.byref(lat), ctypes.byref(params), kind))


def new_workspace(lat: Lattice, params: SolveParams, solver, device="cuda"):
    import torch
    n = wd_solve_workspace_bytes(lat, params, solver)
    if n == 0:
        raise WDError(-1, "new_workspace", "invalid lattice or solve parameters")
    return torch.empty(n, dtype=torch.uint8, device=device)


def _solve(name, gauge, kappa, x, b, params, workspace, stream=None):
    infos = (SolveInfo * params.nrhs)()
    st = getattr(lib(), name)(gauge.handle, kappa, ptr(x), ptr(b), ctypes.byref(params), infos, ptr(workspace),
                              workspace.numel(), stream_ptr(stream))
    if st != WD_EBREAKDOWN:  # a breakdown still reports per-RHS info (see last_error())
        check(st, name)
    return st, [i.as_dict() for i in infos]


def last_error() -> str:
    return lib().wd_last_error().decode()


def bicgstab_solve(gauge: Gauge, kappa: float, x, b, params: SolveParams, workspace, stream=None):
    """Returns (status, [info per RHS]); x, b: full-lattice FP64 device tensors."""
    return _solve("bicgstab_solve", gauge, kappa, x, b, params, workspace, stream)


def cg_solve(gauge: Gauge, kappa: float, x, b, params: SolveParams, workspace, stream=None):
    return _solve("cg_solve", gauge, kappa, x, b, params, workspace, stream)


def solve_full(solver: str, gauge: Gauge, lat: Lattice, kappa: float, b, tol=1e-12, inner="fp64",
               delta=0.1, nrhs=1, use_graph=False, maxiter=10000, stream=None, restart=False):
    """Allocate x and the workspace (torch) and run bicgstab_solve / cg_solve."""
    import torch
    params = solve_params(tol, maxiter, inner, delta, nrhs, use_graph, restart)
    ws = new_workspace(lat, params, solver, b.device)
    x = torch.zeros_like(b)
    fn = bicgstab_solve if solver == "bicgstab" else cg_solve
    st, infos = fn(gauge, kappa, x, b, params, ws, stream)
    return x, (infos[0] if nrhs == 1 else infos)


class Solver:
    """Step API: begin / step / end of one (possibly multi-RHS) solve."""

    def __init__(self, solver: str, gauge: Gauge, kappa: float, x, b, params: SolveParams, workspace,
                 stream=None):
        self.params = params
        self.stream = stream
        self._keep = (gauge, x, b, workspace)
        h = ctypes.c_void_p()
        check(lib().wd_solver_begin(SOLVER[solver], gauge.handle, kappa, ptr(x), ptr(b), ctypes.byref(params),
                                    ptr(workspace), workspace.numel(), stream_ptr(stream), ctypes.byref(h)),
              "wd_solver_begin")
        self.handle = h

    def step(self, n_iters: int = 1) -> bool:
        done = ctypes.c_int32(0)
        check(lib().wd_solver_step(self.handle, n_iters, ctypes.byref(done)), "wd_solver_step")
        return bool(done.value)

    def residuals(self):
        """[(|r^|^2, |r_true|^2 at the last update, |b|^2) per RHS]."""
        buf = (ctypes.c_double * (3 * self.params.nrhs))()
        check(lib().wd_solver_residuals(self.handle, buf), "wd_solver_residuals")
        return [tuple(buf[3 * k:3 * k + 3]) for k in range(self.params.nrhs)]

    def end(self):
        infos = (SolveInfo * self.params.nrhs)()
        st = lib().wd_solver_end(self.handle, infos)
        self.handle = None
        check(st, "wd_solver_end")
        return st, [i.as_dict() for i in infos]
