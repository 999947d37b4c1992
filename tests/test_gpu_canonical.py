"""The operator entry points on canonical FP64 parity spinors (wilson_dslash,
wilson_mat_pc, mdagm): the statement of Section 3 (D of Eq. 1, M_hat of
Eq. 2) and the normal operator of the CG solver (Section 5.1), with the
conversion into the storage format inside the call.  Compared with the FP64
oracle at the stated bars (relative L2): 1e-13 in FP64, 1e-6 in FP32, 2e-3 in
the 16-bit formats; the canonical calls equal the encoded-field fast path bit
for bit.
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
from gpu_helpers import DEV, Setup, rel_l2  # noqa: E402

TOL = {"fp64": 1e-13, "fp32": 1e-6, "i16": 2e-3, "f16": 2e-3}
PRECS = ["fp64", "fp32", "i16", "f16"]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


@pytest.fixture(scope="module", params=[(4, 4, 4, 4), (6, 4, 6, 10), (8, 8, 8, 8)],
                ids=lambda d: "x".join(map(str, d)))
def setup(request):
    dims = request.param
    return Setup(dims, wdinputs.gauge_random(dims, 0.5, 71))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dagger", [0, 1])
def test_canonical_dslash_matches_oracle(setup, prec, dagger):
    s = setup
    nrhs = 3
    psi = wdinputs.spinor_gaussian(s.dims, 72, nrhs=nrhs)
    ws = wd.new_operator_workspace(s.lat, prec, nrhs)
    for p in (0, 1):
        src = np.stack([oracle.split(s.dims, psi[k])[1 - p] for k in range(nrhs)])
        out = torch.zeros(nrhs * s.Vh * 24, dtype=torch.float64, device=DEV)
        wd.wilson_dslash(s.gauge, out, dev(src), p, dagger, prec, nrhs, ws)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(nrhs, s.Vh, 4, 3, 2)
        for k in range(nrhs):
            ref = oracle.dslash_parity(s.dims, s.U, src[k], p, dagger=bool(dagger))
            err = rel_l2(got[k], ref)
            assert err <= TOL[prec], f"{prec} parity {p} dagger {dagger} rhs {k}: {err:.3e}"


@pytest.mark.parametrize("prec", PRECS)
def test_canonical_mat_pc_and_mdagm_match_oracle(setup, prec):
    s = setup
    kappa = 0.124
    nrhs = 2
    psi = wdinputs.spinor_gaussian(s.dims, 73, nrhs=nrhs)
    pe = np.stack([oracle.split(s.dims, psi[k])[0] for k in range(nrhs)])
    ws = wd.new_operator_workspace(s.lat, prec, nrhs)
    for dagger in (0, 1):
        out = torch.zeros(nrhs * s.Vh * 24, dtype=torch.float64, device=DEV)
        wd.wilson_mat_pc(s.gauge, kappa, out, dev(pe), dagger, prec, nrhs, ws)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(nrhs, s.Vh, 4, 3, 2)
        for k in range(nrhs):
            ref = oracle.mhat(s.dims, s.U, kappa, pe[k], dagger=bool(dagger))
            assert rel_l2(got[k], ref) <= TOL[prec], (prec, dagger, k)
    out = torch.zeros(nrhs * s.Vh * 24, dtype=torch.float64, device=DEV)
    wd.mdagm(s.gauge, kappa, out, dev(pe), prec, nrhs, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(nrhs, s.Vh, 4, 3, 2)
    for k in range(nrhs):
        ref = oracle.mhat(s.dims, s.U, kappa, oracle.mhat(s.dims, s.U, kappa, pe[k]), dagger=True)
        # two encodes of an intermediate in the 16-bit formats: twice the bar
        assert rel_l2(got[k], ref) <= 2 * TOL[prec], (prec, k)


@pytest.mark.parametrize("prec", PRECS)
def test_canonical_calls_equal_the_field_fast_path_bitwise(prec):
    dims = (6, 4, 6, 10)
    s = Setup(dims, wdinputs.gauge_random(dims, 0.5, 74))
    psi = wdinputs.spinor_gaussian(dims, 75)
    pe, po = oracle.split(dims, psi)
    ws = wd.new_operator_workspace(s.lat, prec, 1)
    # dslash
    out = torch.zeros(s.Vh * 24, dtype=torch.float64, device=DEV)
    wd.wilson_dslash(s.gauge, out, dev(po), 0, 1, prec, 1, ws)
    fin = s.encode_parity(prec, po)
    fout = s.field(prec)
    wd.wd_dslash_field(s.gauge, fout, fin, 0, 1, prec)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(s.Vh, 4, 3, 2), s.decode(prec, fout))
    # M_hat^dagger M_hat, in place (out aliases in)
    x = dev(pe)
    wd.mdagm(s.gauge, 0.12, x, x, prec, 1, ws)
    fin = s.encode_parity(prec, pe)
    fo, t1, t2 = s.field(prec), s.field(prec), s.field(prec)
    wd.wd_mdagm_field(s.gauge, 0.12, fo, fin, t1, t2, prec)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy().reshape(s.Vh, 4, 3, 2), s.decode(prec, fo))


def test_canonical_calls_refuse_a_short_workspace():
    dims = (4, 4, 4, 4)
    s = Setup(dims, wdinputs.gauge_random(dims, 0.3, 76), precs=("fp32",))
    need = wd.wd_operator_workspace_bytes(s.lat, "fp32", 2)
    ws = torch.empty(need - 256, dtype=torch.uint8, device=DEV)
    x = torch.zeros(2 * s.Vh * 24, dtype=torch.float64, device=DEV)
    with pytest.raises(wd.WDError, match="workspace too small"):
        wd.mdagm(s.gauge, 0.12, x, x, "fp32", 2, ws)
    with pytest.raises(wd.WDError, match="does not hold"):
        wd.wilson_dslash(s.gauge, x, x, 0, 0, "fp64", 1, torch.empty(need, dtype=torch.uint8, device=DEV))
