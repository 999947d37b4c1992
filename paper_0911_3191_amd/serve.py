"""Serving: continuous batching of independent Wilson-Dirac solves.

`Server` wraps the C scheduler (wd_server_* in include/wd.h): requests are
admitted by the HBM footprint of their solver workspace into a device arena,
each in-flight solve iterates on its own HIP stream, and finished solves free
their slot and memory for queued ones.  `serve_stream` drives it with Poisson
arrivals of single-RHS mixed-precision reliable-update BiCGstab solves over
several resident gauge fields of different lattice sizes and reports latency
percentiles (arrival to result) and solves per second.  Sources come from the
seeded input generator (wdinputs), a pool per lattice size built before the
stream starts.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from ._lib import WDError, check, lib, ptr
from ._solver_types import ServeParams, SolveInfo, SolveParams

WD_SOLVER = {"bicgstab": 0, "cg": 1}


class Server:
    """One scheduler over a device arena of `arena_bytes` (a torch allocation)."""

    def __init__(self, arena_bytes: int, max_slots: int = 8, iters_per_pump: int = 1, device="cuda"):
        import torch
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        prm = ServeParams(max_slots=max_slots, iters_per_pump=iters_per_pump)
        h = ctypes.c_void_p()
        check(lib().wd_server_create(ptr(self.arena), self.arena.numel(), ctypes.byref(prm), ctypes.byref(h)),
              "wd_server_create")
        self.handle = h
        self._live = {}  # request id -> objects that must outlive the request

    def submit(self, solver: str, gauge, kappa: float, x, b, params: SolveParams) -> int:
        rid = ctypes.c_int64()
        check(lib().wd_server_submit(self.handle, WD_SOLVER[solver], gauge.handle, kappa, ptr(x), ptr(b),
                                     ctypes.byref(params), ctypes.byref(rid)), "wd_server_submit")
        self._live[rid.value] = (gauge, x, b, params)
        return rid.value

    def pump(self):
        """One scheduling round; returns (in flight, queued)."""
        na, nq = ctypes.c_int32(), ctypes.c_int32()
        check(lib().wd_server_pump(self.handle, ctypes.byref(na), ctypes.byref(nq)), "wd_server_pump")
        return na.value, nq.value

    def poll(self, rid: int):
        """None while pending, else (status, [info per RHS])."""
        nrhs = self._live[rid][3].nrhs if rid in self._live else 1
        done, st = ctypes.c_int32(), ctypes.c_int32()
        infos = (SolveInfo * nrhs)()
        check(lib().wd_server_poll(self.handle, rid, ctypes.byref(done), ctypes.byref(st), infos), "wd_server_poll")
        if not done.value:
            return None
        self._live.pop(rid, None)
        return st.value, [i.as_dict() for i in infos]

    def close(self):
        if self.handle is not None:
            lib().wd_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Resident fields of the serving workload: (dims, seed), links exp(i 0.3 H).
SERVE_FIELDS = [((16, 16, 16, 32), 40), ((16, 16, 16, 32), 41), ((16, 16, 16, 32), 42),
                ((24, 24, 24, 32), 43), ((24, 24, 24, 32), 44), ((24, 24, 24, 32), 45),
                ((32, 32, 32, 64), 46), ((32, 32, 32, 64), 47)]


def make_fields(spec=SERVE_FIELDS, eps=0.3, inner="f16", keep_host=False):
    """Gauge handles (FP64 + inner precision) for every (dims, seed):
    [(dims, lattice, Gauge[, host links])]."""
    import torch
    import wdinputs
    from . import Gauge, lattice
    out = []
    for dims, seed in spec:
        lat = lattice(dims)
        Uh = wdinputs.gauge_random(dims, eps, seed)
        U = torch.from_numpy(Uh).cuda()
        out.append((dims, lat, Gauge(lat, U, precs=("fp64", inner))) + ((Uh,) if keep_host else ()))
        torch.cuda.synchronize()
        del U
    return out


def source_seed(size_index: int, j: int) -> int:
    """Seed of source j of the pool of lattice size number size_index."""
    return 10000 + 100 * size_index + j


def source_pool(sizes, per_size: int = 8, device="cuda"):
    """Seeded complex Gaussian full-lattice sources [1][V][4][3][2] (re, im of
    every component ~ N(0, 1), wdinputs' counter-based generator), per_size
    of them per lattice size, uploaded once: {dims: [(seed, tensor)]}."""
    import torch
    import wdinputs
    pool = {}
    for si, d in enumerate(sizes):
        pool[d] = []
        for j in range(per_size):
            seed = source_seed(si, j)
            pool[d].append((seed, torch.from_numpy(wdinputs.spinor_gaussian(d, seed)[None]).to(device)))
    torch.cuda.synchronize()
    return pool


def serve_stream(fields, n_requests=600, rate=20.0, seed=7, arena_bytes=None, max_slots=16,
                 iters_per_pump=1, inner="f16", delta=0.1, tol=1e-12, kappa_range=(0.120, 0.1245),
                 log=None, check_every=0, pool=None, keep_every=0) -> dict:
    """Poisson arrivals (exponential gaps of mean 1/rate, seeded) of single-RHS
    RU-BiCGstab solves: lattice size uniform over the sizes in `fields`, then
    a field of that size uniform, kappa uniform in kappa_range, and the next
    source of that size's seeded pool (see source_pool; built here if not
    given).  Returns latency percentiles and solves/s.  With keep_every = n,
    the solutions of every n-th request are copied to the host after the run
    and returned under "kept" as (request, field index, kappa, source seed,
    x) for an independent check."""
    import torch
    from . import solve_params, wd_solve_workspace_bytes
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    arrivals = np.cumsum(gaps)
    sizes = sorted({f[0] for f in fields})
    by_size = {d: [k for k, f in enumerate(fields) if f[0] == d] for d in sizes}
    if pool is None:
        pool = source_pool(sizes)
    used = {d: 0 for d in sizes}
    choice = []
    for _ in range(n_requests):
        d = sizes[rng.integers(len(sizes))]
        fk = by_size[d][rng.integers(len(by_size[d]))]
        kappa = float(rng.uniform(*kappa_range))
        src = pool[d][used[d] % len(pool[d])]
        used[d] += 1
        choice.append((fk, kappa, src))
    prm = solve_params(tol=tol, maxiter=20000, inner=inner, delta=delta, nrhs=1, use_graph=True,
                       check_every=check_every)
    need = {d: wd_solve_workspace_bytes(fields[by_size[d][0]][1], prm, "bicgstab") for d in sizes}
    if arena_bytes is None:
        free, _ = torch.cuda.mem_get_info()
        arena_bytes = int(min(free * 0.5, max_slots * max(need.values()) * 1.05))
    srv = Server(arena_bytes, max_slots=max_slots, iters_per_pump=iters_per_pump)

    # warm-up: one solve per lattice size (the dslash launch shapes are tuned here)
    for d in sizes:
        f = fields[by_size[d][0]]
        b = pool[d][0][1]
        x = torch.zeros_like(b)
        torch.cuda.current_stream().synchronize()
        rid = srv.submit("bicgstab", f[2], 0.12, x, b, prm)
        while srv.poll(rid) is None:
            srv.pump()
    torch.cuda.synchronize()

    pending = {}  # rid -> (index, arrival time, x)
    kept = {}
    lat = np.full(n_requests, np.nan)
    status = [None] * n_requests
    iters = np.zeros(n_requests, dtype=np.int64)
    resid = np.zeros(n_requests)
    max_active = 0
    max_queued = 0
    i = 0
    t0 = time.perf_counter()
    first = None
    last_done = t0
    ndone = 0
    while ndone < n_requests:
        now = time.perf_counter() - t0
        while i < n_requests and arrivals[i] <= now:
            fk, kappa, (_, b) = choice[i]
            x = torch.zeros_like(b)
            torch.cuda.current_stream().synchronize()  # the slot streams do not wait on it
            rid = srv.submit("bicgstab", fields[fk][2], kappa, x, b, prm)
            pending[rid] = (i, arrivals[i], x)
            if first is None:
                first = t0 + arrivals[i]
            i += 1
        if pending:
            na, nq = srv.pump()
            max_active, max_queued = max(max_active, na), max(max_queued, nq)
            tdone = time.perf_counter()
            for rid in list(pending):
                res = srv.poll(rid)
                if res is None:
                    continue
                k, arr, x = pending.pop(rid)
                lat[k] = tdone - t0 - arr
                status[k] = res[0]
                iters[k] = res[1][0]["iters"]
                resid[k] = res[1][0]["true_rel_resid"]
                if keep_every and k % keep_every == 0:
                    kept[k] = x
                ndone += 1
                last_done = tdone
        elif i < n_requests:
            time.sleep(max(0.0, min(arrivals[i] - (time.perf_counter() - t0), 0.01)))
    srv.close()
    if any(s != 0 for s in status):
        bad = [k for k, s in enumerate(status) if s != 0]
        raise WDError(-1, "serve_stream", f"{len(bad)} requests did not converge (first: {bad[:5]})")
    span = last_done - first
    per_size = {}
    for d in sizes:
        idx = [k for k in range(n_requests) if fields[choice[k][0]][0] == d]
        if idx:
            per_size["x".join(map(str, d))] = {"requests": len(idx),
                                               "p50_ms": round(float(np.percentile(lat[idx], 50)) * 1e3, 2),
                                               "p99_ms": round(float(np.percentile(lat[idx], 99)) * 1e3, 2)}
    out = {
        "requests": n_requests, "rate_per_s": rate, "arena_bytes": arena_bytes, "max_slots": max_slots,
        "footprint_bytes": {"x".join(map(str, d)): need[d] for d in sizes},
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
        "mean_ms": round(float(np.mean(lat)) * 1e3, 2),
        "per_lattice": per_size,
        "solves_per_s": round(n_requests / span, 2),
        "max_in_flight": max_active, "max_queued": max_queued,
        "iters_mean": round(float(iters.mean()), 1), "true_rel_resid_max": float(resid.max()),
        "sources": f"{len(pool[sizes[0]])} seeded Gaussian sources per lattice size, used in turn",
    }
    if log:
        log(f"serve: {out}")
    if keep_every:
        torch.cuda.synchronize()
        out["kept"] = [(k, choice[k][0], choice[k][1], choice[k][2][0], kept[k].cpu().numpy())
                       for k in sorted(kept)]
    return out
