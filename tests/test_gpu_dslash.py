"""Parity of the HIP dslash, M_hat and M_hat^dag M_hat with the FP64 oracle.

Bars (relative L2 over the output field): 1e-13 in FP64, 1e-6 in FP32, 2e-3 in
the two 16-bit storage formats.  Lattices span several 256-site workgroups and
ragged tails; multi-RHS results must equal the single-RHS ones bit for bit.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import wdinputs  # noqa: E402

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0911_3191_amd as wd  # noqa: E402
from gpu_helpers import Setup, rel_l2  # noqa: E402

TOL = {"fp64": 1e-13, "fp32": 1e-6, "i16": 2e-3, "f16": 2e-3}
PRECS = ["fp64", "fp32", "i16", "f16"]
SHAPES = [(2, 2, 2, 2), (4, 4, 4, 4), (6, 4, 6, 10), (10, 6, 4, 8), (8, 8, 8, 8)]


@pytest.fixture(scope="module", params=SHAPES, ids=lambda d: "x".join(map(str, d)))
def setup(request):
    dims = request.param
    U = wdinputs.gauge_random(dims, 0.5, 17)
    return Setup(dims, U)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dagger", [0, 1])
def test_dslash_matches_oracle(setup, prec, dagger):
    s = setup
    psi = wdinputs.spinor_gaussian(s.dims, 5)
    pe, po = oracle.split(s.dims, psi)
    for p in (0, 1):
        fin = s.encode_full(prec, psi, 1 - p)
        fout = s.field(prec)
        wd.wd_dslash_field(s.gauge, fout, fin, p, dagger, prec)
        got = s.decode(prec, fout)
        ref = oracle.dslash_parity(s.dims, s.U, po if p == 0 else pe, p, dagger=bool(dagger))
        err = rel_l2(got, ref)
        assert err <= TOL[prec], f"{prec} parity {p} dagger {dagger}: rel err {err:.3e}"


@pytest.mark.parametrize("prec", PRECS)
def test_periodic_t(prec):
    dims = (4, 4, 6, 6)
    U = wdinputs.gauge_random(dims, 0.3, 23)
    s = Setup(dims, U, tap=False)
    psi = wdinputs.spinor_gaussian(dims, 24)
    _, po = oracle.split(dims, psi)
    fin = s.encode_full(prec, psi, 1)
    fout = s.field(prec)
    wd.wd_dslash_field(s.gauge, fout, fin, 0, 0, prec)
    ref = oracle.dslash_parity(dims, U, po, 0, antiperiodic_t=False)
    assert rel_l2(s.decode(prec, fout), ref) <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dagger", [0, 1])
def test_mat_pc_and_mdagm(setup, prec, dagger):
    s = setup
    kappa = 0.124
    psi = wdinputs.spinor_gaussian(s.dims, 6)
    pe, _ = oracle.split(s.dims, psi)
    fin = s.encode_parity(prec, pe)
    fout, tmp = s.field(prec), s.field(prec)
    wd.wd_mat_pc_field(s.gauge, kappa, fout, fin, tmp, dagger, prec)
    ref = oracle.mhat(s.dims, s.U, kappa, pe, dagger=bool(dagger))
    assert rel_l2(s.decode(prec, fout), ref) <= TOL[prec]
    if dagger == 0:
        tmpe = s.field(prec)
        wd.wd_mdagm_field(s.gauge, kappa, fout, fin, tmp, tmpe, prec)
        ref2 = oracle.mhat(s.dims, s.U, kappa, oracle.mhat(s.dims, s.U, kappa, pe), dagger=True)
        assert rel_l2(s.decode(prec, fout), ref2) <= 2 * TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_multi_rhs_equals_single_rhs_bitwise(prec):
    dims = (6, 4, 6, 10)
    U = wdinputs.gauge_random(dims, 0.5, 31)
    s = Setup(dims, U)
    srcs = wdinputs.spinor_gaussian(dims, 32, nrhs=3)
    fin = s.encode_full(prec, srcs, 1, nrhs=3)
    fout = s.field(prec, 3)
    wd.wd_dslash_field(s.gauge, fout, fin, 0, 0, prec, 3)
    batch = s.decode(prec, fout, 3)
    for k in range(3):
        f1 = s.encode_full(prec, srcs[k], 1)
        o1 = s.field(prec)
        wd.wd_dslash_field(s.gauge, o1, f1, 0, 0, prec)
        assert np.array_equal(s.decode(prec, o1), batch[k])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", [(4, 6, 8, 4), (6, 4, 16, 2), (6, 4, 6, 10)], ids=lambda d: "x".join(map(str, d)))
def test_every_launch_shape_gives_identical_results(prec, dims, monkeypatch):
    """RHS per thread, RHS-group order, y-sub-slabs and LDS staging only
    redistribute work: every shape must give the same bits, and match the
    oracle."""
    U = wdinputs.gauge_random(dims, 0.5, 61)
    s = Setup(dims, U)
    srcs = wdinputs.spinor_gaussian(dims, 62, nrhs=3)
    fin = s.encode_full(prec, srcs, 1, nrhs=3)
    results = {}
    for nr in (1, 2, 3, 4):
        for gslow in (0, 1):
            for nsub in (1, 2, 3):
                for lds in ((0, 1) if prec in ("i16", "f16") else (0,)):
                    monkeypatch.setenv("WD_DSLASH_SHAPE", f"{nr},{gslow},{nsub},0,0,0,{lds}")
                    fout = s.field(prec, 3)
                    wd.wd_dslash_field(s.gauge, fout, fin, 0, 1, prec, 3)
                    results[(nr, gslow, nsub, lds, 0)] = s.decode(prec, fout, 3)
    if prec == "f16":  # one thread per site over every RHS
        for nsub in (1, 2, 3):
            for lds in (0, 1):
                monkeypatch.setenv("WD_DSLASH_SHAPE", f"1,0,{nsub},0,0,0,{lds},1")
                fout = s.field(prec, 3)
                wd.wd_dslash_field(s.gauge, fout, fin, 0, 1, prec, 3)
                results[(1, 0, nsub, lds, 1)] = s.decode(prec, fout, 3)
    ref = results[(1, 0, 1, 0, 0)]
    for key, val in results.items():
        assert np.array_equal(val, ref), key
    for k in range(3):
        _, po = oracle.split(dims, srcs[k])
        expect = oracle.dslash_parity(dims, U, po, 0, dagger=True)
        assert rel_l2(ref[k], expect) <= TOL[prec]


@pytest.mark.parametrize("kind", ["i16", "f16"])
def test_spinor16_encode_is_bit_exact_with_oracle(kind):
    dims = (4, 4, 4, 6)
    s = Setup(dims, wdinputs.gauge_unit(dims))
    rng = np.random.default_rng(3)
    psi = rng.normal(size=(s.Vh, 4, 3, 2)) * np.exp(rng.normal(size=(s.Vh, 1, 1, 1)) * 2)
    psi[5] = 0.0
    f = s.encode_parity(kind, psi)
    got = s.decode(kind, f)
    q, nm = oracle.encode_spinor16(kind, psi)
    ref = oracle.decode_spinor16(kind, q, nm)
    assert np.array_equal(got, ref)


def check_on_quantised_inputs(kind, dims, U, seed, sparse=False):
    """Feed the oracle the 16-bit-rounded links and spinor.  int16: what
    remains is FP32 arithmetic plus one output rounding, bounded per site by
    the output norm.  binary16 also rounds the projected half spinor and the
    rebuilt third link row to binary16 (one rounding each); with `sparse`
    the input has only the upper two spins and the first two colours, which
    makes both exact for the first two output colours (the half spinor is the
    upper spins themselves, and only stored link rows meet nonzero colours),
    so those are held to the int16 bound; otherwise every component is
    bounded by eight hops of half-spinor rounding, 2^-10 of the neighbour
    norm each, through a unitary link, expanded to the upper and lower
    spins."""
    s = Setup(dims, U)
    Uq = oracle.decode_link16(kind, oracle.encode_link16(kind, U))
    uq = Uq[..., 0] + 1j * Uq[..., 1]
    c = np.conj(np.cross(uq[..., 0, :], uq[..., 1, :]))  # the third row the kernel rebuilds
    Uq[..., 2, :, 0], Uq[..., 2, :, 1] = c.real, c.imag
    psi = wdinputs.spinor_gaussian(dims, seed)
    if sparse:
        psi[..., 2:, :, :] = 0.0
        psi[..., :, 2, :] = 0.0
    _, po = oracle.split(dims, psi)
    q, nm = oracle.encode_spinor16(kind, po)
    po_q = oracle.decode_spinor16(kind, q, nm)
    fin = s.encode_parity(kind, po)
    fout = s.field(kind)
    wd.wd_dslash_field(s.gauge, fout, fin, 0, 0, kind)
    got = s.decode(kind, fout).reshape(s.Vh, 24)
    ref = oracle.dslash_parity(dims, Uq, po_q, 0).reshape(s.Vh, 24)
    site_norm = np.abs(ref).max(axis=1, keepdims=True)
    lsb = site_norm / 32767 if kind == "i16" else site_norm * 2.0 ** -11
    bound = 0.5 * lsb * 1.01 + 64 * 6e-8 * site_norm
    if kind == "f16" and sparse:
        keep = np.zeros((4, 3, 2), dtype=bool)
        keep[:, :2, :] = True
        got, ref = got[:, keep.reshape(-1)], ref[:, keep.reshape(-1)]
        bound = np.broadcast_to(bound, got.shape)
    elif kind == "f16":
        bound = bound + 8 * 2 * 2.0 ** -10 * float(np.max(nm))
    ratio = np.abs(got - ref) / bound
    i, j = np.unravel_index(np.argmax(ratio), ratio.shape)
    assert ratio.max() <= 1.0, (f"site {i} comp {j}: got {got[i, j]!r} ref {ref[i, j]!r} "
                                f"norm {site_norm[i, 0]!r} ratio {ratio.max():.3f}")


@pytest.mark.parametrize("kind", ["i16", "f16"])
def test_16bit_dslash_against_oracle_on_quantised_inputs(kind):
    dims = (6, 4, 6, 10)
    check_on_quantised_inputs(kind, dims, wdinputs.gauge_random(dims, 0.5, 41), 42)
    check_on_quantised_inputs(kind, dims, wdinputs.gauge_random(dims, 0.5, 41), 42, sparse=True)


def test_binary16_links_round_through_binary32():
    """A link real just above a binary16 rounding tie that binary32 rounding
    lands on exactly: binary32 first (the format's definition) rounds the tie
    to even, a direct FP64 -> binary16 rounding goes up.  Every link carries
    one such real, so the two roundings disagree on every link."""
    dims = (6, 4, 6, 10)
    U = wdinputs.gauge_random(dims, 0.5, 43)
    tie = 2457 / 8192          # halfway between the binary16 values 1228/4096 and 1229/4096
    v = tie + 2.0 ** -27       # below half a binary32 ulp above the tie
    assert np.float16(np.float32(v)) != np.float16(v)
    U[..., 0, 0, 0] = v
    check_on_quantised_inputs("f16", dims, U, 44, sparse=True)


@pytest.mark.parametrize("prec", ["fp32", "f16"])
def test_sixty_four_rhs_in_one_launch_equal_single_rhs(prec):
    """The largest batch the ABI accepts (64 RHS, 32 groups of two slots)."""
    dims = (4, 4, 8, 4)
    U = wdinputs.gauge_random(dims, 0.5, 71)
    s = Setup(dims, U, precs=("fp64", prec))
    srcs = wdinputs.spinor_gaussian(dims, 72, nrhs=64)
    fin = s.encode_full(prec, srcs, 1, nrhs=64)
    fout = s.field(prec, 64)
    wd.wd_dslash_field(s.gauge, fout, fin, 0, 0, prec, 64)
    multi = s.decode(prec, fout, 64)
    for k in (0, 1, 31, 62, 63):
        f1 = s.encode_full(prec, srcs[k], 1)
        o1 = s.field(prec)
        wd.wd_dslash_field(s.gauge, o1, f1, 0, 0, prec)
        assert np.array_equal(s.decode(prec, o1), multi[k]), k
