"""Serving scheduler on the GPU: continuous batching of independent solves.

Each request's result must be the same whether it runs alone or in the mix
with others on concurrent streams, admission must respect the arena budget
(the HBM footprint of each solver workspace), and bad requests must fail
alone without disturbing the rest.
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
from paper_0911_3191_amd.serve import Server, serve_stream  # noqa: E402
from gpu_helpers import DEV, Setup  # noqa: E402

# (dims, gauge seed, eps): two lattice sizes, three fields
FIELDS = [((8, 8, 8, 8), 71, 0.3), ((8, 8, 8, 8), 72, 0.4), ((8, 8, 16, 8), 73, 0.3)]


@pytest.fixture(scope="module")
def setups():
    out = [Setup(d, wdinputs.gauge_random(d, e, s), precs=("fp64", "fp32", "f16")) for d, s, e in FIELDS]
    torch.cuda.synchronize()
    return out


def requests(setups, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        s = setups[int(rng.integers(len(setups)))]
        kappa = float(rng.uniform(0.120, 0.1245))
        solver = "bicgstab" if k % 3 else "cg"
        inner = ("f16", "fp32")[k % 2]
        b = wdinputs.spinor_gaussian(s.dims, 500 + k)[None]
        reqs.append((s, solver, kappa, inner, b))
    return reqs


def params_of(inner, use_graph=True, check_every=0):
    return wd.solve_params(tol=1e-12, maxiter=5000, inner=inner, delta=0.1, nrhs=1, use_graph=use_graph,
                           check_every=check_every)


def solve_alone(s, solver, kappa, inner, b):
    p = params_of(inner)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(DEV)
    x = torch.zeros_like(bt)
    ws = wd.new_workspace(s.lat, p, solver)
    stream = torch.cuda.Stream()
    fn = wd.bicgstab_solve if solver == "bicgstab" else wd.cg_solve
    with torch.cuda.stream(stream):
        st, info = fn(s.gauge, kappa, x, bt, p, ws, stream)
    torch.cuda.synchronize()
    return st, x.cpu().numpy(), info[0]


def run_mix(reqs, arena_bytes, max_slots, iters_per_pump=1, check_every=0):
    srv = Server(arena_bytes, max_slots=max_slots, iters_per_pump=iters_per_pump)
    ids, keep = [], []
    for s, solver, kappa, inner, b in reqs:
        bt = torch.from_numpy(np.ascontiguousarray(b)).to(DEV)
        x = torch.zeros_like(bt)
        torch.cuda.synchronize()
        ids.append(srv.submit(solver, s.gauge, kappa, x, bt, params_of(inner, check_every=check_every)))
        keep.append(x)
    results = {}
    trace = []
    for _ in range(100000):
        na, nq = srv.pump()
        trace.append((na, nq))
        for rid in ids:
            if rid not in results:
                r = srv.poll(rid)
                if r is not None:
                    results[rid] = r
        if len(results) == len(ids):
            break
    srv.close()
    assert len(results) == len(ids), "server did not drain"
    xs = [keep[k].cpu().numpy() for k in range(len(ids))]
    return [results[rid] for rid in ids], xs, trace


def test_each_result_is_the_same_alone_and_in_the_mix(setups):
    reqs = requests(setups, 9, 3)
    alone = [solve_alone(*r) for r in reqs]
    need = max(wd.wd_solve_workspace_bytes(r[0].lat, params_of(r[3]), r[1]) for r in reqs)
    res, xs, trace = run_mix(reqs, arena_bytes=16 * need, max_slots=4)
    assert max(na for na, _ in trace) >= 2, "the solves never overlapped"
    for k, ((st, info), x) in enumerate(zip(res, xs)):
        st_a, x_a, info_a = alone[k]
        assert st == st_a == wd.WD_OK, k
        assert info[0]["iters"] == info_a["iters"], k
        assert np.array_equal(x, x_a), f"request {k}: result differs from the same solve alone"
        s, _, kappa, _, b = reqs[k]
        assert oracle.true_relres(s.dims, s.U, kappa, b[0], x[0]) <= 1e-12


def test_mix_with_several_iterations_per_flag_read_equals_each_solve_alone(setups):
    """Solves that read their flags every 3 iterations, interleaved by the
    scheduler, give the bits and iteration counts of the same solves alone
    reading them every iteration."""
    reqs = requests(setups, 6, 5)
    alone = [solve_alone(*r) for r in reqs]
    need = max(wd.wd_solve_workspace_bytes(r[0].lat, params_of(r[3]), r[1]) for r in reqs)
    res, xs, _ = run_mix(reqs, arena_bytes=16 * need, max_slots=4, check_every=3)
    for k, ((st, info), x) in enumerate(zip(res, xs)):
        st_a, x_a, info_a = alone[k]
        assert st == st_a == wd.WD_OK, k
        assert info[0]["iters"] == info_a["iters"], k
        assert info[0]["reliable_updates"] == info_a["reliable_updates"], k
        assert np.array_equal(x, x_a), f"request {k}"


def test_admission_binds_on_the_arena_budget(setups):
    """Six requests with one footprint and an arena for two: never more than
    two in flight, the rest wait, and every one still converges."""
    same = [s for s in setups if s.dims == (8, 8, 8, 8)]
    reqs = [(same[k % 2], "bicgstab", 0.1205 + 0.0005 * k, "f16",
             wdinputs.spinor_gaussian(same[0].dims, 600 + k)[None]) for k in range(6)]
    need = wd.wd_solve_workspace_bytes(same[0].lat, params_of("f16"), "bicgstab")
    res, xs, trace = run_mix(reqs, arena_bytes=2 * need + 4096, max_slots=6)
    assert max(na for na, _ in trace) == 2
    assert max(nq for _, nq in trace) >= 1, "admission never held a request back"
    for (st, info), x, r in zip(res, xs, reqs):
        assert st == wd.WD_OK
        assert oracle.true_relres(r[0].dims, r[0].U, r[2], r[4][0], x[0]) <= 1e-12


def test_request_larger_than_the_arena_is_refused(setups):
    s = setups[0]
    p = params_of("f16")
    need = wd.wd_solve_workspace_bytes(s.lat, p, "bicgstab")
    srv = Server(need // 2, max_slots=2)
    b = torch.zeros((1, int(np.prod(s.dims)), 4, 3, 2), dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    with pytest.raises(wd.WDError) as e:
        srv.submit("bicgstab", s.gauge, 0.12, x, b, p)
    assert e.value.status == wd.WD_ENOMEM
    srv.close()


def test_bad_request_fails_alone(setups):
    reqs = requests(setups, 3, 21)
    s, solver, kappa, inner, b = reqs[1]
    bad = b.copy()
    bad[0, 5, 1, 1, 0] = np.nan
    reqs_bad = [reqs[0], (s, solver, kappa, inner, bad), reqs[2]]
    res, xs, _ = run_mix(reqs_bad, arena_bytes=1 << 30, max_slots=3)
    assert res[1][0] == wd.WD_EINVAL
    for k in (0, 2):
        st_a, x_a, _ = solve_alone(*reqs[k])
        assert res[k][0] == wd.WD_OK
        assert np.array_equal(xs[k], x_a)


def test_poisson_stream_small():
    """The Poisson driver end to end on two small lattice sizes."""
    spec = [((8, 8, 8, 8), 81), ((8, 8, 8, 16), 82), ((8, 8, 8, 16), 83)]
    from paper_0911_3191_amd.serve import make_fields
    fields = make_fields(spec)
    out = serve_stream(fields, n_requests=24, rate=200.0, seed=7, max_slots=4)
    assert out["true_rel_resid_max"] <= 1e-12
    assert out["p99_ms"] >= out["p50_ms"] > 0
    assert out["solves_per_s"] > 0
