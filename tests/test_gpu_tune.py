"""Autotuner of the dslash launch shape.  The first eager launch of a key
(lattice, precision, RHS count, link format, basis, form) times the
candidates -- RHS slots per thread, y-sub-slabs, LDS staging and the binary16
RHS loop, then the workgroup size of the winner, then an occupancy cap on it
-- and appends its choice to the file named by WD_TUNE_CACHE.  The form
separates the adjoint, xpay and the fused dot products, and subset launches
over part of a batch; the solvers tune the forms of their iteration before
capturing it.  Later launches reuse the choice without timing, and the chosen
shape gives the same bits as a forced one."""
import re

import numpy as np
import pytest

import oracle
import paper_0911_3191_amd as wd
import wdinputs
from gpu_helpers import DEV, Setup, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

UK = wd.WD_BASIS_UKQCD
LINE = re.compile(r"\[wd tune\] (\S+) prec (\d+) nrhs (\d+) form (\d+): nr (\d+) nsub (\d+) lds (\d+) rloop (\d+) "
                  r"block (\d+) wgs (\d+) -> ")


RETIMED = re.compile(r"\[wd tune\] (\S+) prec (\d+) nrhs (\d+) form (\d+): nr (\d+) nsub (\d+) lds (\d+) "
                     r"rloop (\d+) block (\d+) wgs (\d+) re-timed -> ")


def _cache_entries(path):
    """Cache file lines as (key, shape) dicts."""
    out = []
    if path.exists():
        for line in path.read_text().splitlines():
            v = [int(t) for t in line.split()]
            if len(v) == 16:
                out.append(dict(dims=tuple(v[:4]), prec=v[4], nrhs=v[5], flags=v[6], form=v[7], nr=v[8],
                                block=v[9], gslow=v[10], nsub=v[11], link_nt=v[12], lds=v[13], rloop=v[14],
                                wgs=v[15]))
    return out


def _timed(err, dims, pattern=LINE):
    tag = "x".join(map(str, dims))
    return [dict(zip(("form", "nr", "nsub", "lds", "rloop", "block", "wgs"), map(int, m.groups()[3:])))
            for m in map(pattern.match, err.splitlines()) if m and m.group(1) == tag]


def test_first_launch_tunes_once_and_records_its_choice(tmp_path, monkeypatch, capfd):
    dims, nrhs = (6, 10, 16, 4), 3  # a lattice and RHS count that no other test launches
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("WD_TUNE_CACHE", str(cache))
    monkeypatch.setenv("WD_TUNE_VERBOSE", "1")
    monkeypatch.delenv("WD_TUNE", raising=False)
    monkeypatch.delenv("WD_DSLASH_SHAPE", raising=False)
    U = wdinputs.gauge_random(dims, 0.4, 71)
    s = Setup(dims, U, precs=("f16",))
    srcs = wdinputs.spinor_gaussian(dims, 72, nrhs=nrhs)
    po = np.stack([oracle.split(dims, srcs[k])[1] for k in range(nrhs)])
    fin = s.encode_parity("f16", po, nrhs, basis=UK)
    capfd.readouterr()

    def run(dagger=0):
        fout = s.field("f16", nrhs)
        wd.wd_dslash_field_basis(s.gauge, fout, fin, 0, dagger, "f16", nrhs, UK)
        return s.decode("f16", fout, nrhs, basis=UK)

    first = run()
    err = capfd.readouterr().err
    timed = _timed(err, dims)
    retimed = _timed(err, dims, RETIMED)
    assert timed and all(t["form"] == 0 for t in timed)
    # stage 1: 1-3 RHS slots x 1 or 2 y-sub-slabs (Ly = 10) x LDS staging off / on, and
    # the RHS loop with 1 or 2 y-sub-slabs x LDS off / on, all at 256 threads, no cap
    stage1 = [t for t in timed if t["block"] == 256 and t["wgs"] == 0]
    assert len(stage1) == 16 and sum(t["rloop"] for t in stage1) == 4, timed
    # stage 2: the winner at 128 threads (and 512 if it is the RHS loop)
    stage2 = [t for t in timed if t["block"] != 256 and t["wgs"] == 0]
    assert {t["block"] for t in stage2} <= {128, 512} and 1 <= len(stage2) <= 2, timed
    assert all(t["rloop"] for t in stage2 if t["block"] == 512)
    # stage 3: the winner under caps of 2, 3, 4 and 6 workgroups per CU (at most 8 waves per SIMD)
    stage3 = [t for t in timed if t["wgs"] != 0]
    assert {t["wgs"] for t in stage3} <= {2, 3, 4, 6} and 3 <= len(stage3) <= 4, timed
    assert len(timed) == len(stage1) + len(stage2) + len(stage3)
    # stage 4: none, or two to four of the timed shapes timed again; the choice is one of them
    assert len(retimed) == 0 or 2 <= len(retimed) <= 4, retimed
    assert all(t in timed for t in retimed)
    entries = _cache_entries(cache)
    assert len(entries) == 1, entries
    e = entries[0]
    if retimed:
        keys = ("nr", "nsub", "lds", "rloop", "block", "wgs")
        assert {k: e[k] for k in keys} in [{k: t[k] for k in keys} for t in retimed]
    assert (e["dims"], e["prec"], e["nrhs"], e["flags"], e["form"]) == (dims, 3, 3, 4, 0)  # UKQCD, D
    assert e["block"] in (128, 256, 512) and e["gslow"] == 0 and e["link_nt"] == 0 and e["wgs"] in (0, 2, 3, 4, 6)
    assert 1 <= e["nr"] <= 3 and e["nsub"] in (1, 2) and e["lds"] in (0, 1) and e["rloop"] in (0, 1)
    assert not (e["rloop"] and e["nr"] != 1) and not (e["block"] == 512 and not e["rloop"])

    # the choice is reused: nothing timed, nothing appended, the same bits
    second = run()
    assert not _timed(capfd.readouterr().err, dims)
    assert len(_cache_entries(cache)) == 1
    assert np.array_equal(first, second)

    # the adjoint is a key of its own
    run(dagger=1)
    timed = _timed(capfd.readouterr().err, dims)
    assert timed and all(t["form"] == 1 for t in timed)
    assert [x["form"] for x in _cache_entries(cache)] == [0, 1]

    # a forced one-slot shape redistributes the same arithmetic: the same bits
    monkeypatch.setenv("WD_DSLASH_SHAPE", "1,0,1")
    forced = run()
    assert np.array_equal(first, forced)
    for k in range(nrhs):
        assert rel_l2(first[k], oracle.dslash_parity(dims, U, po[k], 0)) <= 2e-3


@pytest.mark.parametrize("prec", ["fp64", "f16"])
def test_block_size_and_occupancy_cap_keep_the_bits(prec, monkeypatch):
    """The workgroup size and the occupancy cap that the tuner searches only
    redistribute work: every combination gives the bits of the default
    shape (binary16 also through the RHS loop, up to 512 threads)."""
    dims, nrhs = (6, 10, 16, 4), 2
    U = wdinputs.gauge_random(dims, 0.4, 73)
    s = Setup(dims, U, precs=(prec,))
    srcs = wdinputs.spinor_gaussian(dims, 74, nrhs=nrhs)
    po = np.stack([oracle.split(dims, srcs[k])[1] for k in range(nrhs)])
    fin = s.encode_parity(prec, po, nrhs, basis=UK)

    def run(shape):
        monkeypatch.setenv("WD_DSLASH_SHAPE", shape)
        fout = s.field(prec, nrhs)
        wd.wd_dslash_field_basis(s.gauge, fout, fin, 0, 0, prec, nrhs, UK)
        return s.decode(prec, fout, nrhs, basis=UK)

    ref = run("2,0,1")
    shapes = [f"{nr},0,2,0,0,{wgs},0,0,{block}" for nr in (1, 2) for wgs in (0, 3) for block in (128, 256)]
    if prec == "f16":
        shapes += [f"1,0,2,0,0,{wgs},{lds},1,{block}" for wgs in (0, 2) for lds in (0, 1) for block in (128, 256, 512)]
    for shape in shapes:
        assert np.array_equal(run(shape), ref), shape
    for k in range(nrhs):
        assert rel_l2(ref[k], oracle.dslash_parity(dims, U, po[k], 0)) <= (1e-13 if prec == "fp64" else 2e-3)


@pytest.mark.parametrize("solver", ["bicgstab", "cg"])
def test_solver_tunes_every_form_before_capture(solver, tmp_path, monkeypatch, capfd):
    """A solve records a key for every inner-precision form of its iteration
    (tuned before the graph capture), for the FP64 forms of prepare and of
    the reliable updates, and for subset launches over the updating RHS; the
    solution still meets the oracle's residual."""
    # lattices no other test launches (keys are tuned once per process)
    dims, kappa = ((6, 10, 8, 6) if solver == "bicgstab" else (6, 10, 8, 4)), 0.124
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("WD_TUNE_CACHE", str(cache))
    monkeypatch.delenv("WD_TUNE", raising=False)
    monkeypatch.delenv("WD_DSLASH_SHAPE", raising=False)
    U = wdinputs.gauge_random(dims, 0.4, 75)
    s = Setup(dims, U, precs=("fp64", "f16"))
    bs = wdinputs.spinor_gaussian(dims, 76, nrhs=4)
    bs[1] = 0.0
    bs[1][0, 0, 0, 0, 2, 1, 0] = 1.0  # a point source converges on its own schedule
    bs[3] = bs[3] * np.linspace(0.01, 3.0, bs[3].shape[0])[:, None, None, None, None, None, None]
    bt = torch.from_numpy(np.ascontiguousarray(bs)).to(DEV)
    params = wd.solve_params(tol=1e-12, inner="f16", delta=0.1, nrhs=4, use_graph=True)
    ws = wd.new_workspace(s.lat, params, solver)
    x = torch.zeros_like(bt)
    fn = wd.bicgstab_solve if solver == "bicgstab" else wd.cg_solve
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        st, infos = fn(s.gauge, kappa, x, bt, params, ws, stream)
    torch.cuda.synchronize()
    assert st == wd.WD_OK
    xs = x.cpu().numpy()
    for k in range(4):
        assert oracle.true_relres(dims, U, kappa, bs[k], xs[k]) <= 1e-12
    entries = [e for e in _cache_entries(cache) if e["dims"] == dims]
    inner = {e["form"] for e in entries if e["prec"] == 3 and e["nrhs"] == 4}
    dot = {"YO": 1, "OX": 2, "OO": 3}
    if solver == "bicgstab":  # D, xpay + <r~, v>, xpay + <t, s> and |t|^2
        assert inner == {0, 2 + 4 * dot["YO"], 2 + 4 * dot["OX"]}, inner
    else:  # D, xpay + |M p|^2, D^dag, xpay with D^dag
        assert inner == {0, 2 + 4 * dot["OO"], 1, 3}, inner
    fp64 = {(e["form"], e["nrhs"]) for e in entries if e["prec"] == 0}
    assert any(f & 32 for f, _ in fp64), fp64  # some reliable update covered a subset
    assert all(n < 4 for f, n in fp64 if f & 32)
    if solver == "cg":  # the re-seed's adjoint xpay launch encodes M^dag r into r^ (dot mode 6)
        assert any(f & 31 == 1 + 2 + 4 * 6 for f, _ in fp64), fp64
    for e in entries:  # fused dots keep one sub-slab and 256-thread workgroups
        if e["form"] & 2 and e["form"] >> 2 & 7:
            assert e["nsub"] == 1 and e["block"] == 256
    capfd.readouterr()


def test_pretuning_does_not_depend_on_what_is_cached(monkeypatch):
    """A CG solve tunes the plain binary16 form; a BiCGstab solve after it on
    the same lattice finds that key cached and tunes only its xpay forms.  Its
    pre-tuning must still leave the iteration's fields as prepare left them:
    the solve converges to the oracle's residual with the iterations and bits
    of the same solve with every key already cached."""
    dims, kappa = (4, 10, 8, 6), 0.1205  # a lattice no other test launches
    monkeypatch.delenv("WD_TUNE", raising=False)
    monkeypatch.delenv("WD_TUNE_CACHE", raising=False)
    monkeypatch.delenv("WD_DSLASH_SHAPE", raising=False)
    U = wdinputs.gauge_random(dims, 0.3, 77)
    s = Setup(dims, U, precs=("fp64", "f16"))
    b = wdinputs.spinor_gaussian(dims, 78)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(DEV)

    def solve(solver):
        params = wd.solve_params(tol=1e-12, inner="f16", delta=0.1, use_graph=True)
        ws = wd.new_workspace(s.lat, params, solver)
        x = torch.zeros_like(bt)
        fn = wd.bicgstab_solve if solver == "bicgstab" else wd.cg_solve
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            st, infos = fn(s.gauge, kappa, x, bt, params, ws, stream)
        torch.cuda.synchronize()
        return st, x.cpu().numpy(), infos[0]

    st_cg, _, _ = solve("cg")
    st1, x1, i1 = solve("bicgstab")   # pre-tunes with the plain form cached
    st2, x2, i2 = solve("bicgstab")   # every key cached
    assert st_cg == st1 == st2 == wd.WD_OK, (st_cg, st1, st2, wd.last_error())
    assert i1["iters"] == i2["iters"] and np.array_equal(x1, x2)
    assert oracle.true_relres(dims, U, kappa, b, x1) <= 1e-12
