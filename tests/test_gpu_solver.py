"""Solvers on the GPU against the FP64 oracle.

Every GPU solution is checked with the oracle's own FP64 true residual
||b - (1 - kappa D) x|| / ||b|| of the full system, and, where the oracle can
solve the same system, against the oracle's solution.
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
from gpu_helpers import DEV, Setup  # noqa: E402


def run(setup, solver, b, kappa, **kw):
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(DEV)
    nrhs = kw.get("nrhs", 1)
    params = wd.solve_params(**kw)
    ws = wd.new_workspace(setup.lat, params, solver)
    x = torch.zeros_like(bt)
    stream = torch.cuda.Stream() if kw.get("use_graph") else None
    fn = wd.bicgstab_solve if solver == "bicgstab" else wd.cg_solve
    if stream is not None:
        with torch.cuda.stream(stream):
            st, infos = fn(setup.gauge, kappa, x, bt, params, ws, stream)
    else:
        st, infos = fn(setup.gauge, kappa, x, bt, params, ws)
    torch.cuda.synchronize()
    return st, x.cpu().numpy(), (infos[0] if nrhs == 1 else infos)


def test_config1_fp64_bicgstab_8x4():
    """8^4, eps 0.3 seed 1, kappa 0.12, Gaussian source, plain FP64 BiCGstab to 1e-10."""
    dims, kappa = (8, 8, 8, 8), 0.12
    U = wdinputs.gauge_random(dims, 0.3, 1)
    s = Setup(dims, U, precs=("fp64",))
    b = wdinputs.spinor_gaussian(dims, 1001)
    st, x, info = run(s, "bicgstab", b, kappa, tol=1e-10, inner="fp64", delta=0.0)
    assert st == wd.WD_OK and info["converged"]
    rr = oracle.true_relres(dims, U, kappa, b, x)
    assert rr <= 1e-10 and abs(rr - info["true_rel_resid"]) <= 1e-3 * rr + 1e-15
    xo, oinfo = oracle.bicgstab(dims, U, kappa, b, tol=1e-12)
    xo = xo.reshape(x.shape)
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("solver", ["bicgstab", "cg"])
@pytest.mark.parametrize("inner", ["fp64", "fp32", "i16", "f16"])
def test_reliable_update_solves_reach_1e12(solver, inner):
    dims, kappa = (6, 4, 6, 10), 0.124
    U = wdinputs.gauge_random(dims, 0.3, 7)
    s = Setup(dims, U)
    b = wdinputs.spinor_gaussian(dims, 8)
    st, x, info = run(s, solver, b, kappa, tol=1e-12, inner=inner, delta=0.1, maxiter=5000)
    assert st == wd.WD_OK, info
    rr = oracle.true_relres(dims, U, kappa, b, x)
    assert rr <= 1e-12, f"{solver}/{inner}: oracle true residual {rr:.3e}, info {info}"
    if inner != "fp64":
        assert info["reliable_updates"] >= 2


def test_multi_rhs_batch_equals_each_rhs_alone():
    """Continuous-batching invariant: a RHS's result is the same alone and in a batch."""
    dims, kappa = (6, 4, 6, 10), 0.124
    U = wdinputs.gauge_random(dims, 0.3, 9)
    s = Setup(dims, U)
    bs = wdinputs.spinor_gaussian(dims, 10, nrhs=3)
    bs[2] *= 1e-3  # different scales converge at different iterations
    for solver, inner in (("bicgstab", "i16"), ("cg", "fp32")):
        st, xb, infos = run(s, solver, bs, kappa, tol=1e-12, inner=inner, delta=0.1, nrhs=3)
        assert st == wd.WD_OK
        for k in range(3):
            st1, x1, info1 = run(s, solver, bs[k], kappa, tol=1e-12, inner=inner, delta=0.1)
            assert np.array_equal(x1, xb[k]), f"{solver}/{inner} rhs {k}"
            assert info1["iters"] == infos[k]["iters"]


@pytest.mark.parametrize("solver,restart", [("bicgstab", False), ("cg", False), ("bicgstab", True)])
def test_batch_of_five_with_staggered_updates_equals_each_rhs_alone(solver, restart):
    """Five RHS of different structure reach their reliable updates at different
    iterations, so the updates run on packed subsets of the batch (BiCGstab
    re-encodes the residual inside the FP64 dslash; CG forms M_hat^dag r on the
    same subset and encodes it into r^ inside the second of those launches;
    defect correction also restarts there): every RHS must still
    come out bit for bit as when solved alone, and solve the system."""
    dims, kappa = (8, 4, 8, 6), 0.124
    U = wdinputs.gauge_random(dims, 0.4, 13)
    s = Setup(dims, U)
    bs = wdinputs.spinor_gaussian(dims, 14, nrhs=5)
    bs[1] = 0.0
    bs[1][0, 0, 0, 0, 2, 1, 0] = 1.0                 # a point source
    bs[3] = bs[3] * np.linspace(0.01, 3.0, bs[3].shape[0])[:, None, None, None, None, None, None]
    for inner in ("f16", "fp32"):
        st, xb, infos = run(s, solver, bs, kappa, tol=1e-12, inner=inner, delta=0.1, nrhs=5, restart=restart)
        assert st == wd.WD_OK
        for k in range(5):
            assert oracle.true_relres(dims, U, kappa, bs[k], xb[k]) <= 1e-12
            st1, x1, info1 = run(s, solver, bs[k], kappa, tol=1e-12, inner=inner, delta=0.1, restart=restart)
            assert np.array_equal(x1, xb[k]), f"{inner} rhs {k}"
            assert info1["iters"] == infos[k]["iters"]
            assert info1["reliable_updates"] == infos[k]["reliable_updates"]


@pytest.mark.parametrize("solver,restart,use_graph", [("bicgstab", False, False), ("bicgstab", False, True),
                                                       ("cg", False, False), ("cg", False, True),
                                                       ("bicgstab", True, True)])
def test_iterations_between_flag_reads_do_not_change_the_result(solver, restart, use_graph):
    """check_every = 3 runs three iterations (one graph) between two reads of
    the flags by the host.  An RHS that triggers a reliable update (or, with
    restart, ends an inner solve) waits on the device for the rest of the
    batch, so x and the iteration and update counts equal those of a read
    after every iteration."""
    dims, kappa = (8, 4, 8, 6), 0.124
    U = wdinputs.gauge_random(dims, 0.4, 13)
    s = Setup(dims, U)
    bs = wdinputs.spinor_gaussian(dims, 14, nrhs=5)
    bs[1] = 0.0
    bs[1][0, 0, 0, 0, 2, 1, 0] = 1.0
    bs[3] = bs[3] * np.linspace(0.01, 3.0, bs[3].shape[0])[:, None, None, None, None, None, None]
    kw = dict(tol=1e-12, inner="f16", delta=0.1, nrhs=5, use_graph=use_graph, restart=restart)
    st1, x1, i1 = run(s, solver, bs, kappa, **kw)
    st3, x3, i3 = run(s, solver, bs, kappa, check_every=3, **kw)
    assert st1 == st3 == wd.WD_OK
    assert np.array_equal(x1, x3)
    for k in range(5):
        assert i1[k]["iters"] == i3[k]["iters"], k
        assert i1[k]["reliable_updates"] == i3[k]["reliable_updates"], k
        assert oracle.true_relres(dims, U, kappa, bs[k], x3[k]) <= 1e-12


def test_check_every_out_of_range_is_refused():
    dims = (4, 4, 4, 4)
    s = Setup(dims, wdinputs.gauge_random(dims, 0.3, 3))
    bt = torch.from_numpy(wdinputs.spinor_gaussian(dims, 4)).to(DEV)
    x = torch.zeros_like(bt)
    ws = wd.new_workspace(s.lat, wd.solve_params(tol=1e-10), "bicgstab")
    with pytest.raises(wd.WDError, match="check_every"):
        wd.bicgstab_solve(s.gauge, 0.12, x, bt, wd.solve_params(tol=1e-10, check_every=65), ws)


@pytest.mark.parametrize("shape", ["3,0,2,1,0,0,0", "4,1,2,0,0,0,0", "1,1,2,0,0,0,1", "1,0,2,0,0,0,0,1",
                                   "1,0,2,0,0,0,1,1"])
def test_batch_under_any_launch_shape_equals_each_rhs_alone(shape, monkeypatch):
    """Launches with a fused dot product keep one sub-slab, so their partial
    records cover the same sites whatever else the shape says (RHS per thread,
    group order, link cache policy, LDS staging): a batch solved under a forced
    shape matches each RHS solved alone, bit for bit (the last shape is the
    binary16 kernel in which one thread loops over every RHS of the batch,
    without and with LDS staging)."""
    dims, kappa = (8, 4, 8, 6), 0.124
    U = wdinputs.gauge_random(dims, 0.4, 15)
    s = Setup(dims, U)
    bs = wdinputs.spinor_gaussian(dims, 16, nrhs=5)
    monkeypatch.setenv("WD_DSLASH_SHAPE", shape)
    st, xb, infos = run(s, "bicgstab", bs, kappa, tol=1e-12, inner="f16", delta=0.1, nrhs=5)
    assert st == wd.WD_OK
    monkeypatch.delenv("WD_DSLASH_SHAPE")
    for k in range(5):
        st1, x1, info1 = run(s, "bicgstab", bs[k], kappa, tol=1e-12, inner="f16", delta=0.1)
        assert np.array_equal(x1, xb[k]), f"{shape} rhs {k}"
        assert info1["iters"] == infos[k]["iters"]


@pytest.mark.parametrize("solver", ["bicgstab", "cg"])
def test_graph_replay_matches_direct_launches(solver):
    dims, kappa = (8, 8, 8, 8), 0.12
    U = wdinputs.gauge_random(dims, 0.3, 11)
    s = Setup(dims, U)
    b = wdinputs.spinor_gaussian(dims, 12, nrhs=2)
    st0, x0, i0 = run(s, solver, b, kappa, tol=1e-12, inner="f16", delta=0.1, nrhs=2)
    st1, x1, i1 = run(s, solver, b, kappa, tol=1e-12, inner="f16", delta=0.1, nrhs=2, use_graph=True)
    assert st0 == st1 == wd.WD_OK
    assert np.array_equal(x0, x1)
    for k in range(2):
        assert oracle.true_relres(dims, U, kappa, b[k], x1[k]) <= 1e-12


def test_maxiter_returns_not_converged_with_best_iterate():
    dims, kappa = (8, 8, 8, 8), 0.12
    U = wdinputs.gauge_random(dims, 0.3, 13)
    s = Setup(dims, U)
    b = wdinputs.spinor_gaussian(dims, 14)
    st, x, info = run(s, "bicgstab", b, kappa, tol=1e-12, inner="fp32", delta=0.1, maxiter=3)
    assert st == wd.WD_NOT_CONVERGED and not info["converged"]
    assert info["status"] == wd.WD_NOT_CONVERGED
    assert np.all(np.isfinite(x))


@pytest.mark.parametrize("solver,inner", [("bicgstab", "f16"), ("cg", "i16")])
@pytest.mark.parametrize("e", [133, -133])
def test_solution_scales_with_the_source_bit_for_bit(solver, inner, e):
    """The solve runs on b / |b| and scales x back, so a source times 2^e (here
    beyond the binary32 range the 16-bit formats keep their norms in) gives
    exactly 2^e times the solution of the unscaled source: powers of two scale
    every rounding step of the path exactly."""
    dims, kappa = (8, 4, 8, 6), 0.124
    U = wdinputs.gauge_random(dims, 0.4, 13)
    s = Setup(dims, U)
    b = wdinputs.spinor_gaussian(dims, 31)
    c = 2.0 ** e
    st0, x0, info0 = run(s, solver, b, kappa, tol=1e-12, inner=inner, delta=0.1)
    st1, x1, info1 = run(s, solver, b * c, kappa, tol=1e-12, inner=inner, delta=0.1)
    assert st0 == wd.WD_OK and st1 == wd.WD_OK
    assert np.array_equal(x1, x0 * c)
    assert info1["iters"] == info0["iters"] and info1["true_rel_resid"] == info0["true_rel_resid"]
    assert oracle.true_relres(dims, U, kappa, b * c, x1) <= 1e-12


def test_zero_source_gives_zero_solution():
    dims, kappa = (4, 4, 4, 4), 0.12
    U = wdinputs.gauge_random(dims, 0.3, 15)
    s = Setup(dims, U)
    b = np.zeros((4, 4, 4, 4, 4, 3, 2))
    st, x, info = run(s, "bicgstab", b, kappa, tol=1e-12, inner="fp32")
    assert st == wd.WD_OK and info["converged"] and info["iters"] == 0
    assert not np.any(x)


def test_nan_source_is_rejected():
    dims, kappa = (4, 4, 4, 4), 0.12
    U = wdinputs.gauge_random(dims, 0.3, 15)
    s = Setup(dims, U)
    b = wdinputs.spinor_gaussian(dims, 16)
    b[1, 2, 3, 0, 1, 1, 0] = np.nan
    with pytest.raises(wd.WDError) as e:
        run(s, "bicgstab", b, kappa, tol=1e-12, inner="fp32")
    assert e.value.status == -1


def test_config2_mixed_vs_fp64_24x32():
    """24^3x32, eps 0.3 seed 2, kappa 0.124: FP64 BiCGstab and reliable-update
    BiCGstab with FP32, int16 and binary16 inner solvers, all to 1e-12."""
    dims, kappa = (24, 24, 24, 32), 0.124
    U = wdinputs.gauge_random(dims, 0.3, 2)
    s = Setup(dims, U)
    b = wdinputs.spinor_gaussian(dims, 1002)
    iters = {}
    for inner in ("fp64", "fp32", "i16", "f16"):
        st, x, info = run(s, "bicgstab", b, kappa, tol=1e-12, inner=inner,
                          delta=0.0 if inner == "fp64" else 0.1)
        assert st == wd.WD_OK, (inner, info)
        rr = oracle.true_relres(dims, U, kappa, b, x)
        assert rr <= 1e-12, f"{inner}: {rr:.3e}"
        iters[inner] = info["iters"]
    # reliable updates cost few extra iterations (Table 5: within ~15% single, ~34% half)
    assert iters["fp32"] <= 1.5 * iters["fp64"] + 10
    assert iters["i16"] <= 2.0 * iters["fp64"] + 10


def test_config3_cg_twelve_point_sources_graph():
    """24^3x32, eps 0.5, kappa 0.1245: CG on M^dag M for the 12 spin-colour point
    sources at the origin in one batch under hipGraph, FP32 and 16-bit storage."""
    dims, kappa = (24, 24, 24, 32), 0.1245
    U = wdinputs.gauge_random(dims, 0.5, 3)
    s = Setup(dims, U)
    b = wdinputs.point_sources(dims)
    for inner in ("fp32", "f16"):
        st, x, infos = run(s, "cg", b, kappa, tol=1e-12, inner=inner, delta=0.1, nrhs=12,
                           use_graph=True, maxiter=20000)
        assert st == wd.WD_OK, (inner, wd.last_error(), [(i["iters"], i["status"]) for i in infos])
        for k in range(12):
            rr = oracle.true_relres(dims, U, kappa, b[k], x[k])
            assert rr <= 1e-12, f"{inner} rhs {k}: {rr:.3e}"
            assert abs(rr - infos[k]["true_rel_resid"]) <= 1e-2 * rr + 1e-15, (inner, k)


@pytest.mark.parametrize("solver", ["bicgstab", "cg"])
@pytest.mark.parametrize("inner,eps_in", [("fp32", 1e-4), ("f16", 1e-2), ("f16", 0.1)])
def test_defect_correction_solves_reach_1e12(solver, inner, eps_in):
    """Algorithm 1: inner solves to eps_in relative to the residual they start
    from, each restarted from the FP64 residual, until the true residual is
    below 1e-12."""
    dims, kappa = (6, 4, 6, 10), 0.124
    U = wdinputs.gauge_random(dims, 0.3, 7)
    s = Setup(dims, U, precs=("fp64", inner))
    b = wdinputs.spinor_gaussian(dims, 8)
    st, x, info = run(s, solver, b, kappa, tol=1e-12, inner=inner, delta=eps_in, maxiter=5000, restart=True)
    assert st == wd.WD_OK, info
    rr = oracle.true_relres(dims, U, kappa, b, x)
    assert rr <= 1e-12, f"{solver}/{inner}: oracle true residual {rr:.3e}, info {info}"
    assert info["reliable_updates"] >= 2  # outer corrections


def test_config2_defect_correction_against_reliable_updates():
    """24^3x32, eps 0.3 seed 2, kappa 0.124: both mixed schemes reach 1e-12
    (the iteration counts are printed; the benchmark reports the comparison)."""
    dims, kappa = (24, 24, 24, 32), 0.124
    U = wdinputs.gauge_random(dims, 0.3, 2)
    s = Setup(dims, U, precs=("fp64", "fp32", "f16"))
    b = wdinputs.spinor_gaussian(dims, 1002)
    res = {}
    for inner in ("fp32", "f16"):
        st, x, ru = run(s, "bicgstab", b, kappa, tol=1e-12, inner=inner, delta=0.1, maxiter=20000,
                        use_graph=True)
        assert st == wd.WD_OK and oracle.true_relres(dims, U, kappa, b, x) <= 1e-12
        st, x, dc = run(s, "bicgstab", b, kappa, tol=1e-12, inner=inner, delta=0.1, maxiter=20000,
                        use_graph=True, restart=True)
        assert st == wd.WD_OK and oracle.true_relres(dims, U, kappa, b, x) <= 1e-12
        res[inner] = (ru["iters"], dc["iters"])
    print("config2 iterations (reliable updates, defect correction):", res)


def test_smallest_lattice_mixed_solve():
    """2^4: every neighbour wraps; both parities have 8 sites."""
    dims, kappa = (2, 2, 2, 2), 0.124
    U = wdinputs.gauge_random(dims, 0.5, 74)
    s = Setup(dims, U)
    b = wdinputs.spinor_gaussian(dims, 75)
    for solver in ("bicgstab", "cg"):
        st, x, info = run(s, solver, b, kappa, tol=1e-12, inner="f16", delta=0.1, maxiter=2000)
        assert st == wd.WD_OK, (solver, info)
        assert oracle.true_relres(dims, U, kappa, b, x) <= 1e-12


def test_vanishing_kappa_returns_the_source():
    """kappa -> 0: 1 - kappa D -> 1, so x = b within a few iterations."""
    dims = (4, 4, 4, 4)
    U = wdinputs.gauge_random(dims, 0.3, 76)
    s = Setup(dims, U)
    b = wdinputs.spinor_gaussian(dims, 77)
    st, x, info = run(s, "bicgstab", b, 1e-14, tol=1e-12, inner="fp32", delta=0.1)
    assert st == wd.WD_OK
    assert np.linalg.norm(x.reshape(b.shape) - b) <= 1e-11 * np.linalg.norm(b)
    assert info["iters"] <= 6
