"""The UKQCD spin basis on the GPU (Appendix B).

Fields rotated into the UKQCD basis (psi_UK = S psi_DR, S pinned against both
printed projector tables) must give, after rotating back, the oracle's
DeGrand-Rossi dslash: FP64 1e-13, FP32 1e-6, 16-bit 2e-3 relative L2, for
both parities, the adjoint, 12- and 8-real links, the temporal gauge, slab
and non-slab lattices, every launch shape, and several right-hand sides.
The 16-bit kernels are also checked site by site against the oracle fed the
same quantised inputs, and the encode / decode rotation against S itself.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import wdinputs  # noqa: E402
from dense_ref import UKQCD_S  # noqa: E402

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0911_3191_amd as wd  # noqa: E402
from gpu_helpers import Setup, rel_l2  # noqa: E402

UK = wd.WD_BASIS_UKQCD
TOL = {"fp64": 1e-13, "fp32": 1e-6, "i16": 2e-3, "f16": 2e-3}
PRECS = ["fp64", "fp32", "i16", "f16"]
SHAPES = [(4, 6, 8, 4), (6, 4, 6, 10), (2, 2, 2, 2), (8, 8, 16, 8)]


def to_uk(psi):
    """S psi on the spin index of [..., 4, 3, 2] spinors (FP64, each entry one
    sum and one product by the double nearest 1/sqrt(2), as a rounding-order
    reference for the encode)."""
    r = np.sqrt(0.5)  # correctly rounded; 1 / np.sqrt(2) is one ulp below it
    a = [psi[..., s, :, :] for s in range(4)]
    return np.stack([r * (a[1] + a[3]), -r * (a[0] + a[2]), r * (a[1] - a[3]), r * (a[2] - a[0])], axis=-3)


def from_uk(psi):
    return np.einsum("ts,...tcr->...scr", UKQCD_S, psi)


def test_rotation_helper_is_s():
    psi = wdinputs.spinor_gaussian((2, 2, 2, 2), 1)
    assert np.allclose(to_uk(psi), np.einsum("st,...tcr->...scr", UKQCD_S, psi), rtol=0, atol=1e-15)
    assert np.allclose(from_uk(to_uk(psi)), psi, rtol=0, atol=1e-15)


@pytest.mark.parametrize("prec", PRECS)
def test_encode_rotates_by_s(prec):
    dims = (4, 6, 8, 4)
    s = Setup(dims, wdinputs.gauge_unit(dims))
    psi = wdinputs.spinor_gaussian(dims, 2)
    pe, _ = oracle.split(dims, psi)
    f = s.encode_parity(prec, pe, basis=UK)
    raw = s.decode(prec, f)                # the stored UKQCD components
    back = s.decode(prec, f, basis=UK)     # rotated back to DeGrand-Rossi
    if prec == "fp64":
        assert np.array_equal(raw, to_uk(pe))
        assert rel_l2(back, pe) <= 1e-15
    else:
        assert rel_l2(raw, to_uk(pe)) <= TOL[prec] / 10
        assert rel_l2(back, pe) <= TOL[prec] / 10
    if prec in ("i16", "f16"):
        q, nm = oracle.encode_spinor16(prec, to_uk(pe))
        assert np.array_equal(raw, oracle.decode_spinor16(prec, q, nm))


@pytest.fixture(scope="module", params=SHAPES, ids=lambda d: "x".join(map(str, d)))
def setup(request):
    dims = request.param
    return Setup(dims, wdinputs.gauge_random(dims, 0.5, 71))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dagger", [0, 1])
def test_ukqcd_dslash_matches_oracle(setup, prec, dagger):
    s = setup
    psi = wdinputs.spinor_gaussian(s.dims, 72)
    pe, po = oracle.split(s.dims, psi)
    for p in (0, 1):
        src = po if p == 0 else pe
        fin = s.encode_parity(prec, src, basis=UK)
        fout = s.field(prec)
        wd.wd_dslash_field_basis(s.gauge, fout, fin, p, dagger, prec, 1, UK)
        got = s.decode(prec, fout, basis=UK)
        ref = oracle.dslash_parity(s.dims, s.U, src, p, dagger=bool(dagger))
        err = rel_l2(got, ref)
        assert err <= TOL[prec], f"{prec} parity {p} dagger {dagger}: rel err {err:.3e}"


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("recon,temporal", [(8, False), (12, True), (8, True)])
def test_ukqcd_dslash_compressed_links(prec, recon, temporal):
    dims = (4, 6, 8, 6)
    U = wdinputs.gauge_random(dims, 0.5, 73)
    if temporal:
        U, _ = oracle.gauge_fix_temporal(dims, U)
    s = Setup(dims, U, recon=recon, temporal=temporal)
    psi = wdinputs.spinor_gaussian(dims, 74)
    _, po = oracle.split(dims, psi)
    for dagger in (0, 1):
        fin = s.encode_parity(prec, po, basis=UK)
        fout = s.field(prec)
        wd.wd_dslash_field_basis(s.gauge, fout, fin, 0, dagger, prec, 1, UK)
        ref = oracle.dslash_parity(dims, U, po, 0, dagger=bool(dagger))
        assert rel_l2(s.decode(prec, fout, basis=UK), ref) <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_ukqcd_periodic_t(prec):
    dims = (4, 4, 8, 6)
    U = wdinputs.gauge_random(dims, 0.3, 75)
    s = Setup(dims, U, tap=False)
    psi = wdinputs.spinor_gaussian(dims, 76)
    pe, _ = oracle.split(dims, psi)
    fin = s.encode_parity(prec, pe, basis=UK)
    fout = s.field(prec)
    wd.wd_dslash_field_basis(s.gauge, fout, fin, 1, 0, prec, 1, UK)
    ref = oracle.dslash_parity(dims, U, pe, 1, antiperiodic_t=False)
    assert rel_l2(s.decode(prec, fout, basis=UK), ref) <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", [(4, 6, 8, 4), (6, 4, 6, 10)], ids=lambda d: "x".join(map(str, d)))
def test_ukqcd_every_launch_shape_and_rhs_count(prec, dims, monkeypatch):
    """Every launch shape gives the same bits on 5 right-hand sides (ragged RHS
    groups), each equal to its single-RHS launch, and the oracle's result."""
    U = wdinputs.gauge_random(dims, 0.5, 77)
    s = Setup(dims, U)
    srcs = wdinputs.spinor_gaussian(dims, 78, nrhs=5)
    po = np.stack([oracle.split(dims, srcs[k])[1] for k in range(5)])
    fin = s.encode_parity(prec, po, nrhs=5, basis=UK)
    results = {}
    for nr in (1, 2, 3, 4):
        for nsub in (1, 2):
            for lds in ((0, 1) if prec in ("i16", "f16") else (0,)):
                monkeypatch.setenv("WD_DSLASH_SHAPE", f"{nr},0,{nsub},0,0,0,{lds}")
                fout = s.field(prec, 5)
                wd.wd_dslash_field_basis(s.gauge, fout, fin, 0, 1, prec, 5, UK)
                results[(nr, nsub, lds, 0)] = s.decode(prec, fout, 5)
    if prec == "f16":  # one thread per site over every RHS
        for nsub in (1, 2):
            for lds in (0, 1):
                monkeypatch.setenv("WD_DSLASH_SHAPE", f"1,0,{nsub},0,0,0,{lds},1")
                fout = s.field(prec, 5)
                wd.wd_dslash_field_basis(s.gauge, fout, fin, 0, 1, prec, 5, UK)
                results[(1, nsub, lds, 1)] = s.decode(prec, fout, 5)
    ref = results[(2, 1, 0, 0)]
    for key, val in results.items():
        assert np.array_equal(val, ref), key
    monkeypatch.delenv("WD_DSLASH_SHAPE")
    for k in range(5):
        f1 = s.encode_parity(prec, po[k], basis=UK)
        o1 = s.field(prec)
        wd.wd_dslash_field_basis(s.gauge, o1, f1, 0, 1, prec, 1, UK)
        assert np.array_equal(s.decode(prec, o1), s.decode(prec, fout, 5)[k])
        expect = oracle.dslash_parity(dims, U, po[k], 0, dagger=True)
        assert rel_l2(from_uk(ref[k]), expect) <= TOL[prec]


@pytest.mark.parametrize("kind", ["i16", "f16"])
@pytest.mark.parametrize("dagger", [0, 1])
@pytest.mark.parametrize("sparse", [False, True])
def test_ukqcd_16bit_dslash_on_quantised_inputs(kind, dagger, sparse):
    """The oracle fed the 16-bit links and the UKQCD-basis spinor quantised as
    the kernel stores it.  int16: what remains is FP32 arithmetic and one
    output rounding, bounded per site by the output norm.  binary16 also
    rounds the projected half spinor and the rebuilt third link row once
    each; with `sparse` (stored lower spins and colour 2 zero) both are exact
    for output colours 0 and 1, which keep the int16 bound, otherwise eight
    hops of half-spinor rounding (2^-10 of the neighbour norm each) are
    allowed."""
    dims = (6, 4, 8, 10)
    U = wdinputs.gauge_random(dims, 0.5, 79)
    s = Setup(dims, U)
    Uq = oracle.decode_link16(kind, oracle.encode_link16(kind, U))
    uq = Uq[..., 0] + 1j * Uq[..., 1]
    c = np.conj(np.cross(uq[..., 0, :], uq[..., 1, :]))  # the third row the kernel rebuilds
    Uq[..., 2, :, 0], Uq[..., 2, :, 1] = c.real, c.imag
    psi = wdinputs.spinor_gaussian(dims, 80)
    _, po = oracle.split(dims, psi)
    if sparse:
        pu = to_uk(po)
        pu[:, 2:, :, :] = 0.0
        pu[:, :, 2, :] = 0.0
        po = from_uk(pu)
    q, nm = oracle.encode_spinor16(kind, to_uk(po))
    po_q = from_uk(oracle.decode_spinor16(kind, q, nm))
    fin = s.encode_parity(kind, po, basis=UK)
    fout = s.field(kind)
    wd.wd_dslash_field_basis(s.gauge, fout, fin, 0, dagger, kind, 1, UK)
    got = s.decode(kind, fout).reshape(s.Vh, 24)  # UKQCD components as stored
    ref = to_uk(oracle.dslash_parity(dims, Uq, po_q, 0, dagger=bool(dagger))).reshape(s.Vh, 24)
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


def test_unknown_basis_is_rejected():
    dims = (4, 4, 4, 4)
    s = Setup(dims, wdinputs.gauge_unit(dims), precs=("fp32",))
    f, g = s.field("fp32"), s.field("fp32")
    with pytest.raises(wd.WDError) as e:
        wd.wd_dslash_field_basis(s.gauge, f, g, 0, 0, "fp32", 1, 2)
    assert e.value.status == wd.WD_EINVAL


@pytest.mark.parametrize("basis", [0, UK], ids=["dr", "uk"])
@pytest.mark.parametrize("tap", [True, False], ids=["antiperiodic", "periodic"])
def test_rhs_loop_kernel_matches_slot_kernels_in_every_form(basis, tap, monkeypatch):
    """The binary16 kernel in which one thread runs over every RHS must give
    the slot kernels' bits for D and its adjoint, on both output parities, and
    (DeGrand-Rossi fast path) for M_hat and its adjoint, which fuse the
    x + a D y update into the second dslash."""
    dims = (6, 4, 8, 6)
    U = wdinputs.gauge_random(dims, 0.5, 81)
    s = Setup(dims, U, tap=tap, precs=("f16",))
    srcs = wdinputs.spinor_gaussian(dims, 82, nrhs=5)
    pe = np.stack([oracle.split(dims, srcs[k])[0] for k in range(5)])
    fin = s.encode_parity("f16", pe, nrhs=5, basis=basis)

    def run(shape):
        monkeypatch.setenv("WD_DSLASH_SHAPE", shape)
        out = {}
        for par in (0, 1):
            for dag in (0, 1):
                fo = s.field("f16", 5)
                wd.wd_dslash_field_basis(s.gauge, fo, fin, par, dag, "f16", 5, basis)
                out[("D", par, dag)] = s.decode("f16", fo, 5, basis=basis)
        if basis == 0:
            for dag in (0, 1):
                fo, ft = s.field("f16", 5), s.field("f16", 5)
                wd.wd_mat_pc_field(s.gauge, 0.124, fo, fin, ft, dag, "f16", 5)
                out[("M", 0, dag)] = s.decode("f16", fo, 5)
        return out

    ref = run("2,0,1,0,0,0,0,0")
    for nsub in (1, 2):
        for lds in (0, 1):
            got = run(f"1,0,{nsub},0,0,0,{lds},1")
            for key in ref:
                assert np.array_equal(got[key], ref[key]), (nsub, lds, key)
