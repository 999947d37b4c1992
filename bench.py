#!/usr/bin/env python3
"""Benchmark of the even-odd Wilson-Dirac hot path on one MI355X.

Workload (one "step"): the 48^3x96 lattice (links exp(i 0.3 H), seed 5,
antiperiodic in t), kappa = 0.124, the 12 spin-colour point sources at the
origin solved together by reliable-update BiCGstab with binary16 storage +
per-site norm (FP32 arithmetic, FP64 reductions, FP64 reliable updates and
solution), 12-real links, delta = 0.1, to a true FP64 residual of 1e-12.
One step runs the whole path: even-odd source preparation, the multi-RHS
M_hat applications, the fused BLAS-1 kernels and reductions, the reliable
updates and the reconstruction of the full-lattice solution.

Reported:
  value            algorithmic GB/s of the whole step (sum of every kernel's
                   algorithmic bytes under the method's storage formats, divided
                   by the step's wall time)
  roofline         the dominant kernel (12-RHS binary16 dslash): algorithmic
                   bytes per launch / average launch time (HIP events on its
                   stream), against 8 TB/s; traffic = HBM-side bytes per launch
                   (FETCH_SIZE + WRITE_SIZE from the committed counter summary,
                   when it was taken on the current kernel source)
  time_to_solution mixed 12-RHS batch vs the plain FP64 single-RHS BiCGstab
  dslash_single_rhs the single-RHS dslash in every storage precision
  stream_GBps      what plain torch streaming kernels reach on the same device
                   (read only, write only, copy, two reads + one write): the
                   practical ceiling beside the nominal 8 TB/s
  dslash_rhs_scan  (--rhs-scan) dslash time against the RHS count per launch
  other_configs    time to solution on the smaller lattices, mixed vs FP64
  next1            8-real links and temporal gauge (Section 4.3, Appendix A.2):
                   the dslash in every format with 1 and 12 RHS on recon-8,
                   temporal-gauge recon-12 and temporal-gauge recon-8 handles,
                   and the 12-RHS solve on the temporal-gauge recon-8 handle
  serve            the Poisson serving run (latency percentiles, solves/s)
  cpu_baseline     the FP64 oracle's own BiCGstab on source 0, stopped after one
                   and after two iterations: the difference is one iteration;
                   the same CPU leg has the oracle compute the FP64 true
                   residual of every GPU solution of the step, of the FP64
                   reference, of sampled temporal-gauge solutions and of every
                   10th served request (oracle_check)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector FMA rate without packed-FP32 instructions (the library is compiled
# without them): 256 CUs x 64 lanes x 2 flops x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
DIMS = (48, 48, 48, 96)
KAPPA = 0.124
EPS, SEED = 0.3, 5
NRHS = 12

# Algorithmic bytes per site (one parity) under the storage formats:
# spinor 24 reals (+ a 4-byte norm for 16-bit), link 12 reals.
SPINOR_B = {"fp64": 192, "fp32": 96, "i16": 52, "f16": 52}
LINK_B = {"fp64": 96, "fp32": 48, "i16": 24, "f16": 24}
# The paper's own per-site count for one RHS (Section 4.3, no reuse of
# neighbours): 8 x (24 spinor + 12 link) reals loaded and 24 stored, plus, in
# 16-bit storage, 9 norms.
PAPER_MODEL_B = {"fp64": 8 * 36 * 8 + 24 * 8, "fp32": 8 * 36 * 4 + 24 * 4,
                 "i16": 8 * 36 * 2 + 24 * 2 + 9 * 4, "f16": 8 * 36 * 2 + 24 * 2 + 9 * 4}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def dslash_bytes(prec: str, nrhs: int, xpay: int = 0) -> int:
    """Per output site: 8 links once per launch, nrhs input and output spinors
    (+ xpay extra spinor reads per RHS)."""
    return 8 * LINK_B[prec] + nrhs * SPINOR_B[prec] * (2 + xpay)


def dslash_bytes_links(prec: str, nrhs: int, recon: int, temporal: bool, lt: int) -> float:
    """As dslash_bytes, for recon-12 or recon-8 links (Appendix A), optionally
    in temporal gauge (Section 4.3: the two time links of a site are read only
    where they cross the last time slice, 2 of every lt sites)."""
    per_link = LINK_B[prec] * recon // 12
    links = 6 + (2.0 / lt if temporal else 2)
    return links * per_link + nrhs * SPINOR_B[prec] * 2


def bicgstab_iter_bytes(prec: str, nrhs: int) -> int:
    """One BiCGstab iteration for nrhs RHS, per site: 2 M_hat (4 dslash, the
    second of each with the xpay read and, for v, the <r~,v> read of r~) and
    the BLAS-1 passes (p: 3R+1W, s: 2R+1W, x/r: 5R+2W)."""
    s = SPINOR_B[prec]
    return (dslash_bytes(prec, nrhs) * 2 + dslash_bytes(prec, nrhs, 1) * 2 + nrhs * s  # <r~,v>
            + nrhs * s * (4 + 3 + 7))


def ru_bytes(prec: str, nrhs: int) -> int:
    """One reliable update (FP64): x += x^ (R x, R x^, W x), M_hat x (2 dslash),
    r = b - r (2R+1W), re-encode (R r, R r~, W r^, W x^, R r^)."""
    s64, s = SPINOR_B["fp64"], SPINOR_B[prec]
    return (nrhs * (2 * s64 + s) + dslash_bytes("fp64", nrhs) + dslash_bytes("fp64", nrhs, 1)
            + nrhs * 3 * s64 + nrhs * (s64 + 4 * s))


def prepare_bytes(nrhs: int) -> int:
    """Even-odd prepare and reconstruct in FP64 (per site of one parity):
    encode b_e, b_o (2 x 192 read + write), |b|^2, b_hat dslash, x = 0,
    first residual (M_hat + r = b - r), reconstruct (encode b_o, dslash, decode 2)."""
    s64 = SPINOR_B["fp64"]
    return (nrhs * 4 * s64 + nrhs * 2 * s64 + dslash_bytes("fp64", nrhs, 1) + nrhs * s64
            + dslash_bytes("fp64", nrhs) + dslash_bytes("fp64", nrhs, 1) + nrhs * 3 * s64
            + nrhs * 2 * s64 + dslash_bytes("fp64", nrhs, 1) + nrhs * 4 * s64)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in ("wd_dslash_impl.h", "wd_dslash.hip", "wd_device.h", "wd_reduce.h"):
        with open(os.path.join(ROOT, "paper_0911_3191_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str, dims) -> dict | None:
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source (same hash); otherwise None."""
    path = os.path.join(ROOT, "profiles", "dslash_traffic_48x48x48x96.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("| ") and kernel in line:
                cells = [c.strip() for c in line.strip().strip("|").split("|")]
                rec = {"fetch_bytes": float(cells[1]), "write_bytes": float(cells[2]),
                       "source_hash": cells[3]}
    if not rec or rec["source_hash"] != kernel_source_hash():
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def other_configs(wd, torch, wdinputs, stream) -> dict:
    """8^4 plain FP64 BiCGstab to 1e-10; 24^3x32 Gaussian source by RU-BiCGstab
    with FP32, int16 and binary16 inner solvers against FP64 (eps 0.3, seed 2,
    kappa 0.124); 24^3x32 CG on 12 point sources in FP32 and binary16 storage
    under hipGraph (eps 0.5, seed 3, kappa 0.1245).  These small solves read
    the flags every 4 iterations (one graph of 4 iterations per host check).
    Each solve runs once untimed (launch shapes are tuned) and once timed."""
    dev = torch.device("cuda:0")

    def timed(gauge, lat, kappa, b, solver, **kw):
        p = wd.solve_params(maxiter=20000, use_graph=True, check_every=4, **kw)
        ws = wd.new_workspace(lat, p, solver)
        fn = wd.bicgstab_solve if solver == "bicgstab" else wd.cg_solve
        x = torch.zeros_like(b)
        with torch.cuda.stream(stream):
            fn(gauge, kappa, x, b, p, ws, stream)
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        with torch.cuda.stream(stream):
            st, infos = fn(gauge, kappa, x, b, p, ws, stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        return {"seconds": round(dt, 4), "status": st, "iters_max": max(i["iters"] for i in infos),
                "reliable_updates_max": max(i["reliable_updates"] for i in infos),
                "true_rel_resid_max": max(i["true_rel_resid"] for i in infos)}

    out = {}
    dims = (8, 8, 8, 8)
    lat = wd.lattice(dims)
    U = torch.from_numpy(wdinputs.gauge_random(dims, 0.3, 1)).to(dev)
    g = wd.Gauge(lat, U, ("fp64",))
    b = torch.from_numpy(wdinputs.spinor_gaussian(dims, 1001)).to(dev).reshape(1, -1)
    out["8x8x8x8_fp64_bicgstab_1e-10"] = timed(g, lat, 0.12, b, "bicgstab", tol=1e-10, inner="fp64", delta=0.0)
    dims = (24, 24, 24, 32)
    lat = wd.lattice(dims)
    U = torch.from_numpy(wdinputs.gauge_random(dims, 0.3, 2)).to(dev)
    g = wd.Gauge(lat, U)
    b = torch.from_numpy(wdinputs.spinor_gaussian(dims, 1002)).to(dev).reshape(1, -1)
    c2 = {"fp64": timed(g, lat, 0.124, b, "bicgstab", tol=1e-12, inner="fp64", delta=0.0)}
    for inner in ("fp32", "i16", "f16"):
        c2[inner] = timed(g, lat, 0.124, b, "bicgstab", tol=1e-12, inner=inner, delta=0.1)
        c2[inner]["speedup_vs_fp64"] = round(c2["fp64"]["seconds"] / c2[inner]["seconds"], 2)
    out["24x24x24x32_ru_bicgstab_1e-12"] = c2
    U = torch.from_numpy(wdinputs.gauge_random(dims, 0.5, 3)).to(dev)
    g = wd.Gauge(lat, U, ("fp64", "fp32", "f16"))
    V = int(np.prod(dims))
    bp = torch.zeros((NRHS, V, 4, 3, 2), dtype=torch.float64, device=dev)
    for sp in range(4):
        for c in range(3):
            bp[3 * sp + c, 0, sp, c, 0] = 1.0
    out["24x24x24x32_cg_12_point_sources_1e-12"] = {
        inner: timed(g, lat, 0.1245, bp, "cg", tol=1e-12, inner=inner, delta=0.1, nrhs=NRHS)
        for inner in ("fp32", "f16")}
    return out


def time_dslash(wd, torch, gauge, lat, prec: str, n: int, gsrc, stream, reps: int) -> float:
    """Seconds per launch of the n-RHS dslash (UKQCD-basis fields, as in the
    solvers) on `gauge`, HIP events on the launch stream."""
    UK = wd.WD_BASIS_UKQCD
    fi = wd.new_field(lat, prec, n)
    fo = wd.new_field(lat, prec, n)
    with torch.cuda.stream(stream):
        wd.wd_spinor_encode_basis(lat, prec, n, UK, fi, gsrc[0:n], stream)
        for _ in range(3):
            wd.wd_dslash_field_basis(gauge, fo, fi, 0, 0, prec, n, UK, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            wd.wd_dslash_field_basis(gauge, fo, fi, 0, 0, prec, n, UK, stream)
        e1.record(stream)
    e1.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    del fi, fo
    return t


def measure_next1(wd, torch, args, lat, dims, U, gauge, gsrc, b, stream):
    """8-real links and temporal gauge fixing (Section 4.3, Appendix A.2): the
    dslash on recon-12, recon-8, temporal-gauge recon-12 and temporal-gauge
    recon-8 handles of the same field, in every format with 1 and 12 RHS
    (algorithmic bytes from dslash_bytes_links), and the step's 12-RHS solve
    on the temporal-gauge recon-8 handle: sources rotated by the gauge
    transformation g, solutions rotated back by g^dagger, so they solve the
    original system (checked by the oracle in the CPU leg).  Returns the
    report and host copies of RHS 0, 5 and 11 of that solve."""
    dev = torch.device("cuda:0")
    Vh = int(np.prod(dims)) // 2
    lt = dims[3]
    precs = ("fp64", "fp32", "i16", "f16")
    U_dev = torch.from_numpy(U).to(dev)
    handles = {"recon12": (gauge, 12, False), "recon8": (wd.Gauge(lat, U_dev, precs, recon=8), 8, False)}
    Ug, gmat = wd.gauge_fix_temporal(lat, U_dev)
    del U_dev
    handles["recon12_temporal"] = (wd.Gauge(lat, Ug, precs, recon=12, temporal=True), 12, True)
    handles["recon8_temporal"] = (wd.Gauge(lat, Ug, precs, recon=8, temporal=True), 8, True)
    del Ug
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    dsl = {}
    for name, (g, recon, tg) in handles.items():
        rows = {}
        for prec in precs:
            row = {}
            for n in (1, NRHS):
                t = time_dslash(wd, torch, g, lat, prec, n, gsrc, stream, args.dslash_reps)
                per_site = dslash_bytes_links(prec, n, recon, tg, lt)
                gbs = per_site * Vh / t / 1e9
                row[str(n)] = {"us": round(t * 1e6, 1), "alg_B_per_site": round(per_site, 2),
                               "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                               "gflops": round(1320 * Vh * n / t / 1e9, 1)}
            rows[prec] = row
        dsl[name] = rows
        log(f"next1 dslash {name}: {rows}")
    # the step's solve on the temporal-gauge recon-8 handle
    g8t = handles["recon8_temporal"][0]
    p = wd.solve_params(tol=1e-12, maxiter=20000, inner=args.inner, delta=0.1, nrhs=NRHS, use_graph=True)
    ws = wd.new_workspace(lat, p, "bicgstab")
    bt = torch.empty_like(b)
    xt = torch.zeros_like(b)
    wd.wd_gauge_rotate_spinor(lat, gmat, bt, b, NRHS, False)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):  # untimed: tunes the recon-8 temporal-gauge launch shapes
        wd.bicgstab_solve(g8t, KAPPA, xt, bt, p, ws, stream)
    xt.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        st, infos = wd.bicgstab_solve(g8t, KAPPA, xt, bt, p, ws, stream)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    wd.wd_gauge_rotate_spinor(lat, gmat, xt, xt, NRHS, True)
    torch.cuda.synchronize()
    kept = [(k, xt[k].cpu().numpy()) for k in (0, 5, NRHS - 1)] if not args.no_oracle_check else None
    solve = {"batch_s": round(t_solve, 3), "status": st, "iters_max": max(i["iters"] for i in infos),
             "reliable_updates_max": max(i["reliable_updates"] for i in infos),
             "true_rel_resid_max": max(i["true_rel_resid"] for i in infos)}
    log(f"next1 solve (temporal gauge, recon 8): {solve}")
    del ws, bt, xt, gmat, handles, g8t
    torch.cuda.empty_cache()
    return {"dslash": dsl, "solve_recon8_temporal": solve,
            "bytes_model": "per site: links (8, or 6 + 2/Lt in temporal gauge) x (12 or 8 reals) + "
                           "nrhs x (input + output spinor)"}, kept


def oracle_checks(oracle, dims, U, x_host, x64_host, xtg_host, serve_kept, serve_fields) -> dict:
    """The FP64 oracle's true residual ||b - (1 - kappa D) x|| / ||b|| of the
    GPU solutions kept from this run (Section 5.3: the stopping contract of
    Algorithm 2 is a true residual of 1e-12)."""
    import wdinputs
    V = int(np.prod(dims))
    t0 = time.perf_counter()
    bsrc = np.zeros((V, 4, 3, 2))
    out = {}

    def point(k):
        bsrc[:] = 0.0
        bsrc[0, k // 3, k % 3, 0] = 1.0
        return bsrc

    if x_host is not None:
        res = [oracle.true_relres(dims, U, KAPPA, point(k), x_host[k]) for k in range(len(x_host))]
        out["step_per_rhs"] = [float(f"{r:.3e}") for r in res]
        out["step_max"] = max(res)
    if x64_host is not None:
        out["fp64_reference"] = oracle.true_relres(dims, U, KAPPA, point(0), x64_host)
    if xtg_host is not None:
        res = {k: oracle.true_relres(dims, U, KAPPA, point(k), xk) for k, xk in xtg_host}
        out["recon8_temporal_sampled"] = {str(k): float(f"{r:.3e}") for k, r in res.items()}
        out["recon8_temporal_max"] = max(res.values())
    if serve_kept and serve_fields is not None:
        res = []
        for k, fk, kappa, seed, x in serve_kept:
            d, Uf = serve_fields[fk]
            res.append(oracle.true_relres(d, Uf, kappa, wdinputs.spinor_gaussian(d, seed), x[0]))
        out["serve_checked"] = len(res)
        out["serve_max"] = max(res)
    out["seconds"] = round(time.perf_counter() - t0, 1)
    return out


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--inner", default="f16", choices=["f16", "i16", "fp32"])
    ap.add_argument("--dims", default="x".join(map(str, DIMS)))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--no-defect-correction", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true")
    ap.add_argument("--dslash-reps", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=600,
                    help="requests of the Poisson serving run (0: skip it)")
    ap.add_argument("--no-next1", action="store_true",
                    help="skip the 8-real / temporal-gauge measurements")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the oracle's true residuals of the GPU solutions")
    ap.add_argument("--copy-probe-gb", type=float, default=0.0,
                    help="also run a plain device copy of this many GB (counter scaling)")
    ap.add_argument("--rhs-scan", action="store_true",
                    help="also time the FP64 and inner-precision dslash against the number of RHS "
                         "per launch (1, 2, 3, 4, 6, 12)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the library has no "
                                   "multi-GPU path (--gpus must be 1)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_0911_3191_amd as wd
    import wdinputs

    dims = tuple(int(v) for v in args.dims.split("x"))
    V = int(np.prod(dims))
    Vh = V // 2
    dev = torch.device("cuda:0")
    inner = args.inner

    log(f"generating links {dims} eps={EPS} seed={SEED}")
    t0 = time.time()
    U = wdinputs.gauge_random(dims, EPS, SEED)
    log(f"links generated in {time.time() - t0:.1f}s")
    lat = wd.lattice(dims, True)
    U_dev = torch.from_numpy(U).to(dev)
    gauge = wd.Gauge(lat, U_dev, ("fp64", "fp32", "i16", "f16"))
    torch.cuda.synchronize()
    del U_dev
    torch.cuda.empty_cache()

    # 12 spin-colour point sources at the origin, built in place on the device
    b = torch.zeros((NRHS, V, 4, 3, 2), dtype=torch.float64, device=dev)
    for s in range(4):
        for c in range(3):
            b[3 * s + c, 0, s, c, 0] = 1.0
    x = torch.zeros_like(b)
    stream = torch.cuda.Stream()
    params = wd.solve_params(tol=1e-12, maxiter=20000, inner=inner, delta=0.1, nrhs=NRHS, use_graph=True)
    ws = wd.new_workspace(lat, params, "bicgstab")
    log(f"workspace {ws.numel() / 1e9:.1f} GB; warmup {args.warmup}, steps {args.steps}")

    def step():
        with torch.cuda.stream(stream):
            st, infos = wd.bicgstab_solve(gauge, KAPPA, x, b, params, ws, stream)
        return st, infos

    for i in range(args.warmup):
        st, infos = step()
        log(f"warmup {i}: status {st} iters {[inf['iters'] for inf in infos]}")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    all_infos = []
    for i in range(args.steps):
        st, infos = step()
        all_infos.append(infos)
        log(f"step {i}: status {st} iters max {max(inf['iters'] for inf in infos)}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed / args.steps * 1e3
    infos = all_infos[-1]
    # the step's solutions, kept on the host for the oracle's check (CPU leg)
    x_host = None if args.no_oracle_check else [x[k].cpu().numpy() for k in range(NRHS)]
    iters = [inf["iters"] for inf in infos]
    rus = [inf["reliable_updates"] for inf in infos]
    worst_res = max(inf["true_rel_resid"] for inf in infos)
    loops = max(iters)  # batch iterations (k + l), the batch runs until the slowest RHS is done
    n_it = max(i - r for i, r in zip(iters, rus))
    n_ru = max(rus)
    step_bytes = Vh * (n_it * bicgstab_iter_bytes(inner, NRHS) + n_ru * ru_bytes(inner, NRHS)
                       + prepare_bytes(NRHS))
    value = step_bytes / (ms_per_step * 1e-3) / 1e9

    # ---- the same batch by defect correction (Algorithm 1), inner tolerance = delta ----
    dc = None
    if not args.no_defect_correction:
        pdc = wd.solve_params(tol=1e-12, maxiter=20000, inner=inner, delta=0.1, nrhs=NRHS, use_graph=True,
                              restart=True)
        xdc = torch.zeros_like(b)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        with torch.cuda.stream(stream):
            stdc, infdc = wd.bicgstab_solve(gauge, KAPPA, xdc, b, pdc, ws, stream)
        torch.cuda.synchronize()
        tdc = time.perf_counter() - t2
        dc = {"batch_s": round(tdc, 3), "status": stdc, "iters_max": max(i["iters"] for i in infdc),
              "restarts_max": max(i["reliable_updates"] for i in infdc),
              "true_rel_resid_max": max(i["true_rel_resid"] for i in infdc),
              "time_vs_reliable_updates": round(tdc / (ms_per_step * 1e-3), 3)}
        log(f"defect correction: {dc}")
        del xdc

    # ---- FP64 single-RHS reference solve (same source 0) ----
    fp64 = None
    x64_host = None
    if not args.no_fp64_reference:
        p64 = wd.solve_params(tol=1e-12, maxiter=20000, inner="fp64", delta=0.0, nrhs=1, use_graph=True)
        ws = None
        torch.cuda.empty_cache()
        ws64 = wd.new_workspace(lat, p64, "bicgstab")
        b0 = b[0:1].contiguous()
        x0 = torch.zeros_like(b0)
        with torch.cuda.stream(stream):  # untimed: tunes the single-RHS FP64 launch shape
            wd.bicgstab_solve(gauge, KAPPA, x0, b0, p64, ws64, stream)
        x0.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        with torch.cuda.stream(stream):
            st64, inf64 = wd.bicgstab_solve(gauge, KAPPA, x0, b0, p64, ws64, stream)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        fp64 = {"seconds": t64, "iters": inf64[0]["iters"], "true_rel_resid": inf64[0]["true_rel_resid"],
                "status": st64}
        x64_host = None if args.no_oracle_check else x0[0].cpu().numpy()
        log(f"fp64 reference: {t64:.3f}s iters {inf64[0]['iters']}")
        del ws64
        # the same single source by the mixed solver (warmed once, then timed)
        p1 = wd.solve_params(tol=1e-12, maxiter=20000, inner=inner, delta=0.1, nrhs=1, use_graph=True)
        ws1 = wd.new_workspace(lat, p1, "bicgstab")
        with torch.cuda.stream(stream):
            wd.bicgstab_solve(gauge, KAPPA, x0, b0, p1, ws1, stream)
        x0.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        with torch.cuda.stream(stream):
            st1, inf1 = wd.bicgstab_solve(gauge, KAPPA, x0, b0, p1, ws1, stream)
        torch.cuda.synchronize()
        fp64["mixed_single_rhs"] = {"seconds": time.perf_counter() - t1, "iters": inf1[0]["iters"],
                                    "reliable_updates": inf1[0]["reliable_updates"],
                                    "true_rel_resid": inf1[0]["true_rel_resid"], "status": st1}
        log(f"mixed single RHS: {fp64['mixed_single_rhs']}")
        del ws1, b0, x0
        torch.cuda.empty_cache()

    # ---- dominant kernel: 12-RHS dslash in the inner precision, HIP events on its stream ----
    # The solvers run the dslash on UKQCD-basis fields, so that is the kernel timed.
    # input: 12 complex Gaussian odd-parity fields (torch's device generator, seed 11)
    UK = wd.WD_BASIS_UKQCD
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    gsrc = torch.randn((NRHS, Vh, 4, 3, 2), dtype=torch.float64, device=dev, generator=gen)
    torch.cuda.synchronize()
    fin = wd.new_field(lat, inner, NRHS)
    fout = wd.new_field(lat, inner, NRHS)
    with torch.cuda.stream(stream):
        wd.wd_spinor_encode_basis(lat, inner, NRHS, UK, fin, gsrc, stream)
        for _ in range(3):
            wd.wd_dslash_field_basis(gauge, fout, fin, 0, 0, inner, NRHS, UK, stream)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.dslash_reps):
            wd.wd_dslash_field_basis(gauge, fout, fin, 0, 0, inner, NRHS, UK, stream)
        ev1.record(stream)
    ev1.synchronize()
    t_dslash = ev0.elapsed_time(ev1) / args.dslash_reps * 1e-3
    dbytes = dslash_bytes(inner, NRHS) * Vh
    achieved = dbytes / t_dslash / 1e9
    dflops = 1320 * Vh * NRHS
    tflops = dflops / t_dslash / 1e12
    traffic = profiled_traffic(f"dslash_{inner}_{NRHS}rhs", dims)
    del fin, fout

    # single-RHS dslash in every precision (context for the roofline)
    table = {}
    for prec in ("fp64", "fp32", "i16", "f16"):
        fi = wd.new_field(lat, prec, 1)
        fo = wd.new_field(lat, prec, 1)
        with torch.cuda.stream(stream):
            wd.wd_spinor_encode_basis(lat, prec, 1, UK, fi, gsrc[0:1], stream)
            for _ in range(3):
                wd.wd_dslash_field_basis(gauge, fo, fi, 0, 0, prec, 1, UK, stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.dslash_reps):
                wd.wd_dslash_field_basis(gauge, fo, fi, 0, 0, prec, 1, UK, stream)
            e1.record(stream)
        e1.synchronize()
        t = e0.elapsed_time(e1) / args.dslash_reps * 1e-3
        gbs = dslash_bytes(prec, 1) * Vh / t / 1e9
        table[prec] = {"us": round(t * 1e6, 1), "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                       "gflops": round(1320 * Vh / t / 1e9, 1),
                       "paper_model_GB/s": round(PAPER_MODEL_B[prec] * Vh / t / 1e9, 1)}
        del fi, fo
    log(f"dslash table {table}")
    next1 = None
    xtg_host = None
    if not args.no_next1:
        next1, xtg_host = measure_next1(wd, torch, args, lat, dims, U, gauge, gsrc, b, stream)
    rhs_scan = None
    if args.rhs_scan:
        # cost of each added right-hand side in one launch (tuned shapes)
        rhs_scan = {}
        for prec in ("fp64", inner):
            rows = {}
            for n in (1, 2, 3, 4, 6, NRHS):
                fi = wd.new_field(lat, prec, n)
                fo = wd.new_field(lat, prec, n)
                with torch.cuda.stream(stream):
                    wd.wd_spinor_encode_basis(lat, prec, n, UK, fi, gsrc[0:n], stream)
                    for _ in range(3):
                        wd.wd_dslash_field_basis(gauge, fo, fi, 0, 0, prec, n, UK, stream)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(args.dslash_reps):
                        wd.wd_dslash_field_basis(gauge, fo, fi, 0, 0, prec, n, UK, stream)
                    e1.record(stream)
                e1.synchronize()
                t = e0.elapsed_time(e1) / args.dslash_reps * 1e-3
                rows[n] = {"us": round(t * 1e6, 1),
                           "alg_GB/s": round(dslash_bytes(prec, n) * Vh / t / 1e9, 1)}
                del fi, fo
            rhs_scan[prec] = rows
        log(f"rhs scan {rhs_scan}")
    del gsrc
    torch.cuda.empty_cache()

    # practical bandwidth of a plain device copy (read + write), HIP events
    ncopy = int(max(args.copy_probe_gb, 4.0) * 1e9) // 8
    src = torch.ones(ncopy, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        dst.copy_(src)
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(5):
            dst.copy_(src)
        c1.record(stream)
    c1.synchronize()
    copy_gbs = 2 * ncopy * 8 / (c0.elapsed_time(c1) / 5 * 1e-3) / 1e9
    log(f"copy: {ncopy * 8 / 1e9:.2f} GB read + written at {copy_gbs:.0f} GB/s")

    # practical streaming rates of plain torch kernels on the same buffers (context for
    # the 8 TB/s peak): read only, write only, and two reads + one write
    def stream_rate(fn, nbytes):
        with torch.cuda.stream(stream):
            fn()
            s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record(stream)
            for _ in range(5):
                fn()
            s1.record(stream)
        s1.synchronize()
        return round(nbytes / (s0.elapsed_time(s1) / 5 * 1e-3) / 1e9, 1)
    nb = ncopy * 8
    stream_gbs = {"read": stream_rate(lambda: src.sum(), nb),
                  "write": stream_rate(lambda: dst.fill_(1.0), nb),
                  "copy": round(copy_gbs, 1),
                  "read2_write1": stream_rate(lambda: dst.add_(src), 3 * nb)}
    log(f"streaming rates {stream_gbs}")
    del src, dst

    # ---- the smaller configurations: time to solution, mixed against FP64 ----
    others = None
    if not args.no_other_configs:
        others = other_configs(wd, torch, wdinputs, stream)
        log(f"other configurations: {others}")

    # ---- serving: Poisson arrivals over 8 resident fields of three lattice sizes ----
    serve = None
    serve_kept, serve_fields_host = [], None
    if args.serve_requests > 0:
        from paper_0911_3191_amd.serve import make_fields, serve_stream, source_pool
        b = x = ws = None
        torch.cuda.empty_cache()
        t3 = time.time()
        fields = make_fields(inner=inner, keep_host=not args.no_oracle_check)
        pool = source_pool(sorted({f[0] for f in fields}))
        log(f"serving fields and sources built in {time.time() - t3:.1f}s")
        serve = serve_stream(fields, n_requests=args.serve_requests, rate=20.0, seed=7, max_slots=16,
                             inner=inner, log=log, check_every=2, pool=pool,
                             keep_every=0 if args.no_oracle_check else 10)
        serve_kept = serve.pop("kept", [])
        # the same stream with the arena cut to about twice the largest footprint,
        # so that admission by HBM footprint binds
        tight = 2 * max(serve["footprint_bytes"].values()) + 4096
        serve_tight = serve_stream(fields, n_requests=max(args.serve_requests // 3, 20), rate=20.0, seed=8,
                                   arena_bytes=tight, max_slots=16, inner=inner, log=log, check_every=2,
                                   pool=pool)
        serve["budget_2x_largest"] = {k: serve_tight[k] for k in
                                      ("requests", "arena_bytes", "p50_ms", "p99_ms", "solves_per_s",
                                       "max_in_flight", "max_queued")}
        serve_fields_host = [(f[0], f[3]) for f in fields] if not args.no_oracle_check else None
        del fields, pool
        torch.cuda.empty_cache()

    # ---- CPU baseline: the FP64 oracle on a bounded sample ----
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        b0h = np.zeros((V, 4, 3, 2))
        b0h[0, 0, 0, 0] = 1.0  # the batch's first point source
        oracle.dslash_parity_sites(dims, U, np.zeros((Vh, 4, 3, 2)), 0, np.arange(64))  # load the library
        times = {}
        for k in (1, 2):
            t2 = time.perf_counter()
            oracle.bicgstab(dims, U, KAPPA, b0h, tol=1e-12, maxiter=k)
            times[k] = time.perf_counter() - t2
        t_iter = max(times[2] - times[1], 1e-9)
        # the same step on the oracle: every iteration of every RHS (reliable updates not counted)
        cpu_value = bicgstab_iter_bytes(inner, NRHS) * Vh / (t_iter * NRHS) / 1e9
        cpu = {"value": round(cpu_value, 3), "unit": "GB/s", "cores": nthreads, "kind": "oracle",
               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "sample": (f"FP64 oracle BiCGstab on source 0 of {args.dims}, stopped after 1 and after 2 "
                          f"iterations ({times[1]:.1f} s, {times[2]:.1f} s); one iteration = {t_iter:.2f} s; "
                          f"value = the step's algorithmic bytes per batch iteration / ({NRHS} x that time)")}
        log(f"cpu baseline {cpu}")
        if not args.no_oracle_check:
            cpu["oracle_check"] = oracle_checks(oracle, dims, U, x_host, x64_host, xtg_host, serve_kept,
                                                serve_fields_host)
            log(f"oracle check {cpu['oracle_check']}")

    per_rhs_mixed = ms_per_step * 1e-3 / NRHS
    out = {
        "metric": "dslash GB/s & % HBM roofline; time-to-1e-12 mixed vs FP64; serve p50/p99",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.dims} 12-RHS {inner}-storage RU-BiCGstab to 1e-12",
                   "lattice": args.dims, "kappa": KAPPA, "eps": EPS, "seed": SEED, "nrhs": NRHS,
                   "sources": "12 spin-colour point sources at the origin", "inner": inner,
                   "delta": 0.1, "recon": 12, "graph": True, "spin_basis": "UKQCD (solver-internal)",
                   "arith": "f32 inner, f64 reductions/updates"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": f"dslash_kernel<{inner}> {NRHS}-RHS, UKQCD basis",
                     "bytes_per_launch": dbytes, "us_per_launch": round(t_dslash * 1e6, 1),
                     "flops_per_launch": dflops, "alu_achieved_TFLOPs": round(tflops, 2),
                     "alu_frac": round(tflops / ALU_PEAK_TFLOPS, 4),
                     "paper_model_GBps": round(NRHS * PAPER_MODEL_B[inner] * Vh / t_dslash / 1e9, 1)},
        "time_to_solution": {"mixed_batch_s": round(ms_per_step * 1e-3, 3),
                             "mixed_per_rhs_s": round(per_rhs_mixed, 4),
                             "fp64_single_rhs_s": round(fp64["seconds"], 3) if fp64 else None,
                             "speedup_per_rhs": round(fp64["seconds"] / per_rhs_mixed, 2) if fp64 else None,
                             "iters_mixed_max": max(iters), "reliable_updates_max": n_ru,
                             "iters_fp64": fp64["iters"] if fp64 else None,
                             "true_rel_resid_max": worst_res,
                             "oracle_true_rel_resid_max": (cpu or {}).get("oracle_check", {}).get(
                                 "step_max"),
                             "fp64_true_rel_resid": fp64["true_rel_resid"] if fp64 else None,
                             "mixed_single_rhs_s": (round(fp64["mixed_single_rhs"]["seconds"], 3)
                                                    if fp64 else None),
                             "speedup_single_rhs": (round(fp64["seconds"] / fp64["mixed_single_rhs"]["seconds"], 2)
                                                    if fp64 else None),
                             "defect_correction": dc},
        "dslash_single_rhs": table,
        "next1": next1,
        "dslash_rhs_scan": rhs_scan,
        "copy_GBps": round(copy_gbs, 1),
        "stream_GBps": stream_gbs,
        "other_configs": others,
        "serve": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
