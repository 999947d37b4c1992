"""Autotuner of the dslash launch shape (RHS slots per thread, y-sub-slabs, LDS
staging, the binary16 RHS loop).  The first eager launch for a key (lattice, precision, RHS count, link
format, basis) times every candidate once and appends its choice to the file
named by WD_TUNE_CACHE.  Later launches reuse the choice without timing, and
the chosen shape gives the same bits as a forced one."""
import numpy as np
import pytest

import oracle
import paper_0911_3191_amd as wd
import wdinputs
from gpu_helpers import Setup, rel_l2

pytestmark = pytest.mark.gpu

UK = wd.WD_BASIS_UKQCD


def _cache_lines(path):
    return [l for l in path.read_text().splitlines() if l.strip()] if path.exists() else []


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

    def run():
        fout = s.field("f16", nrhs)
        wd.wd_dslash_field_basis(s.gauge, fout, fin, 0, 0, "f16", nrhs, UK)
        return s.decode("f16", fout, nrhs, basis=UK)

    first = run()
    timed = [l for l in capfd.readouterr().err.splitlines() if l.startswith("[wd tune] 6x10x16x4 prec 3 nrhs 3:")]
    # candidates: 1-3 RHS slots x 1 or 2 y-sub-slabs (Ly = 10) x LDS staging off / on,
    # and the one-thread-per-site RHS loop with 1 or 2 y-sub-slabs x LDS staging off / on
    assert len(timed) == 16, timed
    assert sum("rhs loop" in t for t in timed) == 4, timed
    lines = _cache_lines(cache)
    assert len(lines) == 1, lines
    v = [int(t) for t in lines[0].split()]
    assert v[:7] == [6, 10, 16, 4, 3, 3, 4]  # dims, binary16, 3 RHS, UKQCD basis with 12-real links
    nr, block, gslow, nsub, link_nt, lds, rloop = v[7:]
    assert 1 <= nr <= 3 and block == 256 and gslow == 0 and nsub in (1, 2) and link_nt == 0 and lds in (0, 1)
    assert rloop in (0, 1) and not (rloop and nr != 1)

    # the choice is reused: nothing timed, nothing appended, the same bits
    second = run()
    assert "[wd tune]" not in capfd.readouterr().err
    assert len(_cache_lines(cache)) == 1
    assert np.array_equal(first, second)

    # a forced one-slot shape redistributes the same arithmetic: the same bits
    monkeypatch.setenv("WD_DSLASH_SHAPE", "1,0,1")
    forced = run()
    assert np.array_equal(first, forced)
    for k in range(nrhs):
        assert rel_l2(first[k], oracle.dslash_parity(dims, U, po[k], 0)) <= 2e-3
