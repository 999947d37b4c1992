"""mdagm_noalloc (scratch in the library's static device array, no
workspace) against mdagm with a caller workspace: the same kernels on the
same inputs, so the results must agree bit for bit, on two calls in a row,
the second with a smaller input than the first; and against the FP64
oracle's M_hat^dagger M_hat at the precision bars."""
import ctypes

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


def even_sources(dims, seed, nrhs):
    psi = wdinputs.spinor_gaussian(dims, seed, nrhs=nrhs)
    return np.stack([oracle.split(dims, psi[k])[0] for k in range(nrhs)])


def noalloc(s, kappa, out, inp, prec, nrhs):
    """Through the C ABI directly."""
    st = wd.lib().mdagm_noalloc(s.gauge.handle, kappa, ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(inp.data_ptr()), wd.prec_of(prec), nrhs,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, wd.last_error()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "i16", "f16"])
def test_noalloc_equals_workspace_mdagm_on_two_calls(prec):
    big = Setup((8, 8, 8, 8), wdinputs.gauge_random((8, 8, 8, 8), 0.5, 81))
    small = Setup((4, 4, 6, 4), wdinputs.gauge_random((4, 4, 6, 4), 0.5, 82))
    for s, nrhs, seed in ((big, 3, 83), (small, 1, 84)):  # the second call is smaller
        pe = even_sources(s.dims, seed, nrhs)
        inp = torch.from_numpy(np.ascontiguousarray(pe)).to(DEV)
        out_na = torch.full_like(inp, np.nan)
        noalloc(s, 0.124, out_na, inp, prec, nrhs)
        out_ws = torch.full_like(inp, np.nan)
        wd.mdagm(s.gauge, 0.124, out_ws, inp, prec, nrhs, wd.new_operator_workspace(s.lat, prec, nrhs))
        torch.cuda.synchronize()
        a, b = out_na.cpu().numpy(), out_ws.cpu().numpy()
        assert np.array_equal(a, b), (prec, s.dims)
        for k in range(nrhs):
            ref = oracle.mhat(s.dims, s.U, 0.124, oracle.mhat(s.dims, s.U, 0.124, pe[k]), dagger=True)
            assert rel_l2(a[k], ref) <= 2 * TOL[prec], (prec, s.dims, k)


def test_noalloc_in_place_and_size_limit():
    s = Setup((4, 4, 4, 4), wdinputs.gauge_random((4, 4, 4, 4), 0.3, 85), precs=("fp32",))
    pe = even_sources(s.dims, 86, 2)
    x = torch.from_numpy(np.ascontiguousarray(pe)).to(DEV)
    ref = torch.empty_like(x)
    wd.mdagm(s.gauge, 0.12, ref, x, "fp32", 2, wd.new_operator_workspace(s.lat, "fp32", 2))
    wd.mdagm_noalloc(s.gauge, 0.12, x, x, "fp32", 2)  # out aliases in
    torch.cuda.synchronize()
    assert torch.equal(x, ref)
    # one FP64 field of 24^3x32 is 42.5 MB: four exceed the 64 MiB array
    dims = (24, 24, 24, 32)
    big = Setup(dims, wdinputs.gauge_random(dims, 0.3, 87), precs=("fp64",))
    y = torch.zeros(big.Vh * 24, dtype=torch.float64, device=DEV)
    with pytest.raises(wd.WDError, match="static maximum"):
        wd.mdagm_noalloc(big.gauge, 0.12, y, y, "fp64", 1)
