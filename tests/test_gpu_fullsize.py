"""Parity at the full benchmark lattice, in the launch configurations the
benchmark times.

48^3 x 96, links exp(i 0.3 H) with seed 5, antiperiodic in t.  The 12
right-hand sides of the batched launch are four host-generated Gaussian
sources, RHS k = 2^(k // 4) * source(k mod 4): every RHS of a launch holds
different values, and scaling by a power of two is exact, so the oracle's
expected output for RHS k is 2^(k // 4) times that of its source.  The
oracle computes sampled output sites one by one: random sites plus every
lattice corner, the t boundary (antiperiodic sign) and the z-slab edges of
the XCD work split.
"""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]

import oracle  # noqa: E402
import wdinputs  # noqa: E402

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0911_3191_amd as wd  # noqa: E402
from gpu_helpers import DEV, Setup, rel_l2  # noqa: E402

DIMS = (48, 48, 48, 96)
NRHS, NSRC = 12, 4
TOL = {"fp64": 1e-13, "fp32": 1e-6, "i16": 2e-3, "f16": 2e-3}


def sample_sites(dims, n, seed):
    """Checkerboard indices of even output sites: n random ones plus corners,
    t-boundary and z-slab-edge sites."""
    Lx, Ly, Lz, Lt = dims
    rng = np.random.default_rng(seed)
    picks = set(int(c) for c in rng.choice(Lx * Ly * Lz * Lt // 2, size=n, replace=False))
    zs = sorted({z for k in range(8) for z in (k * Lz // 8, (k + 1) * Lz // 8 - 1)})
    for t in (0, 1, Lt - 2, Lt - 1):
        for z in zs:
            for y in (0, Ly - 1):
                for x in (0, 1, Lx - 2, Lx - 1):
                    if (x + y + z + t) & 1 == 0:
                        picks.add((x + Lx * (y + Ly * (z + Lz * t))) // 2)
    return np.array(sorted(picks), dtype=np.int64)


@pytest.fixture(scope="module")
def big():
    """(setup, full-lattice sources, sampled sites, oracle outputs per source,
    canonical odd-parity sources)."""
    U = wdinputs.gauge_random(DIMS, 0.3, 5)
    s = Setup(DIMS, U)
    V = s.V
    cbs = sample_sites(DIMS, 4000, 9)
    src = torch.empty((NRHS, V, 4, 3, 2), dtype=torch.float64, device=DEV)
    src_odd = torch.empty((NRHS, s.Vh, 4, 3, 2), dtype=torch.float64, device=DEV)  # canonical odd parity
    expect = np.empty((NSRC, len(cbs), 4, 3, 2))
    for j in range(NSRC):
        psi = wdinputs.spinor_gaussian(DIMS, 900 + j)
        _, odd = oracle.split(DIMS, psi)
        expect[j] = oracle.dslash_parity_sites(DIMS, U, odd, 0, cbs)
        dev = torch.from_numpy(psi.reshape(V, 4, 3, 2)).to(DEV)
        dev_odd = torch.from_numpy(np.ascontiguousarray(odd)).to(DEV)
        for k in range(j, NRHS, NSRC):
            src[k] = dev * float(2 ** (k // NSRC))
            src_odd[k] = dev_odd * float(2 ** (k // NSRC))
        del psi, odd, dev, dev_odd
    torch.cuda.synchronize()
    yield s, src, cbs, expect, src_odd
    del src, src_odd
    torch.cuda.empty_cache()


def run(s, src, cbs, prec, nrhs):
    fin = wd.new_field(s.lat, prec, nrhs)
    fout = wd.new_field(s.lat, prec, nrhs)
    wd.wd_spinor_encode_full(s.lat, prec, nrhs, 1, fin, src[:nrhs].contiguous())
    wd.wd_dslash_field(s.gauge, fout, fin, 0, 0, prec, nrhs)
    out = torch.empty((nrhs, s.Vh, 4, 3, 2), dtype=torch.float64, device=DEV)
    wd.wd_spinor_decode(s.lat, prec, nrhs, out, fout)
    idx = torch.from_numpy(cbs).to(DEV)
    got = out[:, idx].cpu().numpy()
    del fin, fout, out
    return got


@pytest.mark.parametrize("prec", ["f16", "i16", "fp32"])
def test_12rhs_launch_at_full_size(big, prec):
    s, src, cbs, expect, _ = big
    got = run(s, src, cbs, prec, NRHS)
    for k in range(NRHS):
        ref = expect[k % NSRC] * float(2 ** (k // NSRC))
        err = rel_l2(got[k], ref)
        assert err <= TOL[prec], f"{prec} rhs {k}: rel L2 {err:.3e} on {len(cbs)} sampled sites"


@pytest.mark.parametrize("prec", ["fp64", "fp32", "i16", "f16"])
def test_single_rhs_launch_at_full_size(big, prec):
    s, src, cbs, expect, _ = big
    got = run(s, src, cbs, prec, 1)
    err = rel_l2(got[0], expect[0])
    assert err <= TOL[prec], f"{prec}: rel L2 {err:.3e} on {len(cbs)} sampled sites"


@pytest.mark.parametrize("prec", ["f16", "i16", "fp32"])
def test_12rhs_ukqcd_launch_at_full_size(big, prec):
    """The launch the benchmark times: 12 RHS on UKQCD-basis fields at the tuned
    shape (binary16: the RHS-loop kernel), canonical odd-parity sources
    encoded into the basis, the output decoded back to DeGrand-Rossi."""
    s, _, cbs, expect, src_odd = big
    fin = wd.new_field(s.lat, prec, NRHS)
    fout = wd.new_field(s.lat, prec, NRHS)
    wd.wd_spinor_encode_basis(s.lat, prec, NRHS, wd.WD_BASIS_UKQCD, fin, src_odd)
    wd.wd_dslash_field_basis(s.gauge, fout, fin, 0, 0, prec, NRHS, wd.WD_BASIS_UKQCD)
    out = torch.empty((NRHS, s.Vh, 4, 3, 2), dtype=torch.float64, device=DEV)
    wd.wd_spinor_decode_basis(s.lat, prec, NRHS, wd.WD_BASIS_UKQCD, out, fout)
    got = out[:, torch.from_numpy(cbs).to(DEV)].cpu().numpy()
    del fin, fout, out
    for k in range(NRHS):
        ref = expect[k % NSRC] * float(2 ** (k // NSRC))
        err = rel_l2(got[k], ref)
        assert err <= TOL[prec], f"{prec} rhs {k}: rel L2 {err:.3e} on {len(cbs)} sampled sites"
