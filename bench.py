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


# ---- counter and trace summaries (no GPU: reads rocprofv3's CSV output) -------------
DOT_NAMES = {0: "", 1: " <y,out>", 2: " <out,x>,|out|^2", 3: " |out|^2", 4: " res |r|^2", 5: " res->enc"}
PREC_OF = {"SF64": "fp64", "SF32": "fp32", "SI16": "i16", "SF16": "f16"}


def _csv_rows(root: str, suffix: str) -> list[dict]:
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows += list(csv.DictReader(f))
    return rows


def _col(row: dict, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(names)


def dslash_launch(name: str, grid: int, block: int, Vh: int, slab: bool) -> dict | None:
    """What a dslash dispatch computed, from its kernel template arguments and
    launch size: precision, form, basis, kernel, RHS groups."""
    if "dslash_kernel<" not in name and "dslash16_rloop_kernel<" not in name:
        return None
    a = name.index("<")
    depth, b = 0, a
    for b in range(a, len(name)):
        depth += {"<": 1, ">": -1}.get(name[b], 0)
        if depth == 0:
            break
    args = [t.strip().replace("wd::", "") for t in name[a + 1:b].split(",")]
    if "rloop" in name:  # <DAGGER, XPAY, DOT, BASIS, LDS, S2>
        prec, dag, xpay, dot, basis, lds, kind, nr = "f16", args[0], args[1], int(args[2]), int(args[3]), args[4], \
            "rhs loop", 0
    else:  # <S, DAGGER, XPAY, DOT, NR, RECON, LDS, BASIS, S2>
        prec, dag, xpay, dot, nr = PREC_OF.get(args[0], args[0]), args[1], args[2], int(args[3]), int(args[4])
        lds, basis, kind = args[6], int(args[7]), f"{nr} slot" + ("s" if nr > 1 else "")
        if args[5] == "8":
            kind += ", 8-real links"
    per_group = (8 * -(-(Vh // 8) // block) if slab else -(-Vh // block)) * block
    groups = grid // per_group if per_group else 0
    form = ("D^dag" if dag == "true" else "D") if xpay == "false" else \
        ("x + a D^dag" if dag == "true" else "x + a D") + DOT_NAMES.get(dot, f" dot {dot}")
    return {"prec": prec, "form": form, "basis": "UKQCD" if basis == 1 else "DR", "kind": kind,
            "lds": lds == "true", "block": block, "groups": groups,
            "nrhs": (nr * groups) if nr else None, "xpay": xpay == "true", "dot": dot}


def profile_summary(args) -> None:
    """Print the counter/trace summary tables of the dslash launches found in a
    directory of rocprofv3 CSV output (kernel trace + stats, FETCH_SIZE run,
    WRITE_SIZE run), FETCH/WRITE scaled by the plain device copy of the same runs."""
    import statistics
    root = args.profile_summary
    dims = tuple(int(v) for v in args.dims.split("x"))
    Vh = int(np.prod(dims)) // 2
    slab = dims[2] % 8 == 0
    copy_bytes = int(max(args.copy_probe_gb, 4.0) * 1e9) // 8 * 8

    def group_key(r):
        name = _col(r, "Kernel_Name")
        grid = int(_col(r, "Grid_Size", "Grid_Size_X"))
        block = int(_col(r, "Workgroup_Size", "Workgroup_Size_X"))
        return name, grid, block

    # kernel trace: durations per (name, grid, block)
    dur = {}
    trace = sorted(_csv_rows(root, "kernel_trace.csv"), key=lambda r: int(r["Dispatch_Id"]))
    for r in trace:
        k = group_key(r)
        dur.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    # counters: per dispatch value, per counter
    cnt = {}
    for r in _csv_rows(root, "counter_collection.csv"):
        cnt.setdefault(_col(r, "Counter_Name"), {}).setdefault(group_key(r), []).append(float(r["Counter_Value"]))
    scale = {}
    for c, rows in cnt.items():  # the copy: the largest FETCH/WRITE among kernels named *copy*
        cands = [max(v) for (n, _, _), v in rows.items() if "copy" in n.lower()]
        if cands:
            scale[c] = copy_bytes / (max(cands) * 1024.0)
    keys = set(dur) | {k for rows in cnt.values() for k in rows}
    table = []
    for k in keys:
        d = dslash_launch(k[0], k[1], k[2], Vh, slab)
        if not d:
            continue
        f = cnt.get("FETCH_SIZE", {}).get(k)
        w = cnt.get("WRITE_SIZE", {}).get(k)
        t = dur.get(k)
        if f or w:  # launch shapes of the run itself (tuning candidates carry no counters)
            table.append((d, k, f, w, t))
    # algorithmic reads of a launch: links once + per RHS the input spinor, the
    # xpay source and y where the form reads them
    def alg_reads(d):
        n = d["nrhs"] or NRHS
        per = SPINOR_B[d["prec"]] * (1 + d["xpay"] + (d["dot"] in (1, 4, 5)))
        return Vh * (8 * LINK_B[d["prec"]] + n * per)

    def label(d):
        if d["form"] == "D" and d["basis"] == "UKQCD" and (d["nrhs"] in (1, NRHS) or d["kind"] == "rhs loop"):
            return f"dslash_{d['prec']}_{d['nrhs'] or NRHS}rhs"
        return ""

    h = kernel_source_hash()
    if args.profile_part == "trace":
        print(f"Kernel source hash (wd_dslash_impl.h + wd_dslash.hip + wd_device.h + wd_reduce.h): `{h}`\n")
        print(f"## Timed dslash launches (the last {args.dslash_reps} of each group: the back-to-back launches "
              "bench.py times with HIP events)\n")
        print("| label | kernel | form | grid | launches | mean us | median us | min us | max us | algorithmic GB/s |")
        print("|---|---|---|---|---|---|---|---|---|---|")
        for k, t in dur.items():
            d = dslash_launch(k[0], k[1], k[2], Vh, slab)
            if not d or not label(d) or k not in cnt.get("FETCH_SIZE", {}):
                continue
            last = t[-args.dslash_reps:]
            m = statistics.mean(last)
            gbs = dslash_bytes(d["prec"], d["nrhs"] or NRHS) * Vh / (m * 1e-6) / 1e9
            kind = d["kind"] + (", LDS" if d["lds"] else "") + f", {d['block']} threads"
            print(f"| {label(d)} | {d['prec']} {kind} | {d['form']} ({d['basis']}) | {k[1]} | {len(last)} | "
                  f"{m:.1f} | {statistics.median(last):.1f} | {min(last):.1f} | {max(last):.1f} | {gbs:.0f} |")
        stats = _csv_rows(root, "kernel_stats.csv")
        tot = sum(float(r["TotalDurationNs"]) for r in stats)
        print("\n## Kernels by total time in the run (all calls, every grid)\n")
        print("| kernel | calls | total ms | share | mean us |")
        print("|---|---|---|---|---|")
        for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:20]:
            name = r["Name"].split("(")[0].replace("void ", "").replace("wd::", "")
            print(f"| `{name[:110]}` | {r['Calls']} | {float(r['TotalDurationNs']) * 1e-6:.1f} | "
                  f"{float(r['TotalDurationNs']) / tot:.3f} | {float(r['AverageNs']) * 1e-3:.1f} |")
        return
    if args.profile_part == "counters":
        # every counter of the run, median per labelled dslash group, with derived rates
        print(f"Kernel source hash (wd_dslash_impl.h + wd_dslash.hip + wd_device.h + wd_reduce.h): `{h}`\n")
        names = sorted(cnt)
        groups = []
        for k in {k for rows in cnt.values() for k in rows}:
            d = dslash_launch(k[0], k[1], k[2], Vh, slab)
            if d and label(d):
                groups.append((label(d), d, k))
        print("| label | kernel | " + " | ".join(names) + " |")
        print("|---|---|" + "---|" * len(names))
        med = {}
        for lab, d, k in sorted(groups):
            med[lab] = {c: statistics.median(cnt[c][k]) for c in names if k in cnt[c]}
            kind = d["kind"] + (", LDS" if d["lds"] else "") + f", {d['block']} threads"
            print(f"| {lab} | {d['prec']} {kind} | " +
                  " | ".join(f"{med[lab].get(c, float('nan')):.4g}" for c in names) + " |")
        print("\nDerived (per launch; GRBM_GUI_ACTIVE counts the 8 XCDs):\n")
        print("| label | VALU busy | TA busy avg / max | TCP pending-stall share | L1->L2 latency (clk) | "
              "L2 hit rate | waves issuing nothing (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES) |")
        print("|---|---|---|---|---|---|---|")
        for lab, m in med.items():
            cyc = m.get("GRBM_GUI_ACTIVE", float("nan")) / 8  # clocks of one XCD
            f = lambda v: f"{v:.2f}" if v == v else "-"
            valu = m.get("SQ_INSTS_VALU", float("nan")) * 4 / 1024 / cyc
            ta = (m.get("TA_BUSY_avr", float("nan")) / cyc, m.get("TA_BUSY_max", float("nan")) / cyc)
            tcp = m.get("TCP_PENDING_STALL_CYCLES_sum", float("nan")) / 256 / cyc
            lat = m.get("TCP_TCC_READ_REQ_LATENCY_sum", float("nan")) / m.get("TCP_TCC_READ_REQ_sum", float("nan"))
            hit = m.get("TCC_HIT_sum", float("nan")) / (m.get("TCC_HIT_sum", float("nan"))
                                                         + m.get("TCC_MISS_sum", float("nan")))
            wait = m.get("SQ_WAIT_INST_ANY", float("nan")) / m.get("SQ_WAVE_CYCLES", float("nan"))
            print(f"| {lab} | {f(valu)} | {f(ta[0])} / {f(ta[1])} | {f(tcp)} | {lat:.0f} | {f(hit)} | {f(wait)} |")
        return
    print(f"Counter scaling from the plain device copy of {copy_bytes / 1e9:.1f} GB in the same runs: "
          + ", ".join(f"{c} x {v:.3f}" for c, v in sorted(scale.items())) + ".\n")
    print("Per launch, median over the launches of each group.  `fetch`/`write` are bytes; "
          "`ratio` = fetch / algorithmic reads; `us` = mean kernel-trace duration of the group "
          f"(solver launches late in a solve skip converged RHS), `last {args.dslash_reps}` = mean of "
          f"its last {args.dslash_reps} launches (for the labelled dslash rows: the bench's timed, "
          "back-to-back launches).  A RHS-loop launch covers every RHS of its launch (12 here).\n")
    print(f"| label | fetch | write | source hash | launches | us | last {args.dslash_reps} us | kernel | "
          "form | RHS | algorithmic reads | ratio |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|")
    order = sorted(table, key=lambda e: -(sum(e[4]) if e[4] else 0))
    for d, k, f, w, t in order:
        fb = statistics.median(f) * 1024 * scale.get("FETCH_SIZE", 1.0) if f else None
        wb = statistics.median(w) * 1024 * scale.get("WRITE_SIZE", 1.0) if w else None
        n = len(t) if t else (len(f) if f else 0)
        alg = alg_reads(d)
        kind = d["kind"] + (", LDS" if d["lds"] else "") + f", {d['block']} threads"
        def e(v):
            return f"{v:.4e}" if v is not None else "-"
        us = f"{statistics.mean(t):.1f}" if t else "-"
        last = f"{statistics.mean(t[-args.dslash_reps:]):.1f}" if t else "-"
        ratio = f"{fb / alg:.2f}" if fb is not None else "-"
        print(f"| {label(d)} | {e(fb)} | {e(wb)} | {h} | {n} | {us} | {last} | {d['prec']} {kind} | "
              f"{d['form']} ({d['basis']}) | {d['nrhs'] or NRHS} | {alg:.4e} | {ratio} |")


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
    ap.add_argument("--profile-summary", metavar="DIR", default=None,
                    help="print the dslash counter/trace tables of the rocprofv3 CSV output under DIR "
                         "(kernel trace, FETCH_SIZE and WRITE_SIZE runs) and exit; no GPU")
    ap.add_argument("--profile-part", choices=["traffic", "trace", "counters"], default="traffic",
                    help="with --profile-summary: the FETCH/WRITE table, the kernel-trace tables, or the "
                         "medians of every counter of the run")
    ap.add_argument("--rhs-scan", action="store_true",
                    help="also time the FP64 and inner-precision dslash against the number of RHS "
                         "per launch (1, 2, 3, 4, 6, 12)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.profile_summary:
        profile_summary(args)
        return
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
        # untimed first: tunes the subset launches of the update sizes this solve meets
        with torch.cuda.stream(stream):
            wd.bicgstab_solve(gauge, KAPPA, xdc, b, pdc, ws, stream)
        xdc.zero_()
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
                   "arith": (("inner dslash: binary16 projections and binary16 x binary16 products "
                              "summed in f32 (v_dot2_f32_f16), f32 accumulation" if inner == "f16" else
                              "inner: f32 arithmetic") + "; f64 reductions, reliable updates and solution")},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": f"{inner} dslash, {NRHS} RHS per launch at the tuned launch shape, UKQCD basis",
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
