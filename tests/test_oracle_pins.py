"""Pins of the FP64 oracle to facts other than itself (CPU only).

Each test ties one part of the oracle to something it does not compute itself:
the projector tables printed in Appendix B, the Clifford algebra, a dense
brute-force matrix built entry by entry from Eq. 1, the dense Schur complement
(Eq. 2), gamma5-hermiticity, the free-field plane-wave spectrum, gauge
covariance, locality, translation invariance, dense linear solves, and numpy's
IEEE binary16 rounding.
"""
import numpy as np
import pytest

import oracle
import wdinputs
from dense_ref import PROJ, UKQCD_S, dense_hopping, enumerate_sites, from_vec, gammas, parity_masks, to_vec
from golden_io import read_projectors

TINY = [(2, 2, 2, 2), (2, 4, 2, 6), (4, 2, 2, 4)]


# ---- random numbers and links --------------------------------------------------
def test_philox_known_answer_and_numpy():
    # Known-answer vector of Philox4x64-10 for zero counter and key (Random123 KAT).
    out = wdinputs.philox4x64_10([0, 0, 0, 0], [0, 0])
    assert [int(v) for v in out] == [0x16554d9eca36314c, 0xdb20fe9d672d0fdc,
                                      0xd7e772cee186176b, 0x7e68b68aec7ba23b]
    # numpy's Philox bit generator increments its counter before each block.
    for key in ([0, 0], [12345, 987654321]):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array([41, 0, 0, 0], dtype=np.uint64))
        ref = bg.random_raw(8)
        ours = np.concatenate([wdinputs.philox4x64_10([42, 0, 0, 0], key),
                               wdinputs.philox4x64_10([43, 0, 0, 0], key)])
        assert np.array_equal(ref, ours)


def test_links_are_su3_and_recon12_exact():
    U = wdinputs.gauge_random((4, 4, 4, 4), 0.3, 1)
    u = U[..., 0] + 1j * U[..., 1]
    eye = np.eye(3)
    assert np.abs(np.einsum("...ab,...cb->...ac", u, u.conj()) - eye).max() < 4e-15
    assert np.abs(np.linalg.det(u) - 1).max() < 4e-15
    c = np.conj(np.cross(u[..., 0, :], u[..., 1, :]))
    assert np.abs(c - u[..., 2, :]).max() < 4e-15
    # Gaussian traceless Hermitian generator: <Re tr U>/3 ~ 0.885 at eps = 0.3
    # (exp(i eps H) with E tr H^2 = 8 gives 1 - eps^2 * 8 / 6 + O(eps^4)).
    Ub = wdinputs.gauge_random((8, 8, 8, 8), 0.3, 7)
    plaq = (Ub[..., 0, 0, 0] + Ub[..., 1, 1, 0] + Ub[..., 2, 2, 0]).mean() / 3
    assert abs(plaq - 0.885) < 0.01


def test_inputs_are_deterministic_and_seed_dependent():
    a = wdinputs.gauge_random((2, 2, 2, 4), 0.3, 5)
    b = wdinputs.gauge_random((2, 2, 2, 4), 0.3, 5)
    c = wdinputs.gauge_random((2, 2, 2, 4), 0.3, 6)
    assert np.array_equal(a, b) and not np.allclose(a, c)
    s = wdinputs.spinor_gaussian((2, 2, 2, 4), 3)
    assert abs(s.std() - 1) < 0.2


# ---- gamma matrices -----------------------------------------------------------
def test_oracle_gammas_match_printed_projectors():
    for mu in range(4):
        g = oracle.gamma(mu)
        assert np.array_equal(np.eye(4) + g, PROJ[("+", mu + 1)])
        assert np.array_equal(np.eye(4) - g, PROJ[("-", mu + 1)])


def test_clifford_algebra_and_projector_rank():
    g = [oracle.gamma(mu) for mu in range(4)]
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * (a == b) * np.eye(4))
        for s in (+1, -1):
            P = np.eye(4) + s * g[a]
            assert np.allclose(P @ P, 2 * P)
            assert np.linalg.matrix_rank(P) == 2
        assert np.allclose((np.eye(4) + g[a]) @ (np.eye(4) - g[a]), 0)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


def test_ukqcd_table_is_a_valid_basis_change_of_the_degrand_rossi_table():
    uk = read_projectors("projectors_ukqcd.txt")
    gd = gammas(PROJ)
    gu = gammas(uk)
    for a in range(4):
        for b in range(4):
            assert np.allclose(gu[a] @ gu[b] + gu[b] @ gu[a], 2 * (a == b) * np.eye(4))
    assert np.allclose(gu[3], np.diag([1, 1, -1, -1]))
    S = UKQCD_S
    assert np.allclose(S @ S.conj().T, np.eye(4))
    for a in range(4):
        assert np.allclose(S @ gd[a] @ S.conj().T, gu[a])


# ---- dslash against the dense brute force ------------------------------------------
@pytest.mark.parametrize("dims", TINY)
@pytest.mark.parametrize("tap", [True, False])
def test_dslash_full_matches_dense(dims, tap):
    U = wdinputs.gauge_random(dims, 0.5, 11)
    psi = wdinputs.spinor_gaussian(dims, 12)
    D = dense_hopping(dims, U, antiperiodic_t=tap)
    ref = D @ to_vec(psi)
    got = to_vec(oracle.dslash_full(dims, U, psi, antiperiodic_t=tap))
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
    got_dag = to_vec(oracle.dslash_full(dims, U, psi, dagger=True, antiperiodic_t=tap))
    ref_dag = D.conj().T @ to_vec(psi)
    assert np.linalg.norm(got_dag - ref_dag) <= 1e-14 * np.linalg.norm(ref_dag)


@pytest.mark.parametrize("dims", TINY)
def test_dslash_parity_blocks_match_dense(dims):
    U = wdinputs.gauge_random(dims, 0.5, 21)
    psi = wdinputs.spinor_gaussian(dims, 22)
    D = dense_hopping(dims, U)
    even, odd = parity_masks(dims)
    pe, po = oracle.split(dims, psi)
    for p, (m_out, m_in, src) in enumerate([(even, odd, po), (odd, even, pe)]):
        ref = D[np.ix_(m_out, m_in)] @ to_vec(src)
        got = to_vec(oracle.dslash_parity(dims, U, src, p))
        assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
        cbs = np.array([0, 3, len(src) - 1])
        got_s = oracle.dslash_parity_sites(dims, U, src, p, cbs)
        assert np.allclose(got_s, from_vec(got)[cbs], rtol=0, atol=1e-14)


@pytest.mark.parametrize("dims", TINY)
def test_mhat_is_the_dense_schur_complement(dims):
    kappa = 0.13
    U = wdinputs.gauge_random(dims, 0.5, 31)
    D = dense_hopping(dims, U)
    M = np.eye(D.shape[0]) - kappa * D
    even, odd = parity_masks(dims)
    Mee, Meo, Moe, Moo = (M[np.ix_(a, b)] for a, b in [(even, even), (even, odd), (odd, even), (odd, odd)])
    S = Mee - Meo @ np.linalg.solve(Moo, Moe)
    x = wdinputs.spinor_gaussian(dims, 32)
    xe, _ = oracle.split(dims, x)
    got = to_vec(oracle.mhat(dims, U, kappa, xe))
    ref = S @ to_vec(xe)
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
    got_d = to_vec(oracle.mhat(dims, U, kappa, xe, dagger=True))
    ref_d = S.conj().T @ to_vec(xe)
    assert np.linalg.norm(got_d - ref_d) <= 1e-14 * np.linalg.norm(ref_d)


def test_mfull_matches_dense():
    dims, kappa = (2, 4, 2, 6), 0.11
    U = wdinputs.gauge_random(dims, 0.3, 41)
    x = wdinputs.spinor_gaussian(dims, 42)
    M = np.eye(12 * 96) - kappa * dense_hopping(dims, U)
    ref = M @ to_vec(x)
    assert np.linalg.norm(to_vec(oracle.mfull(dims, U, kappa, x)) - ref) <= 1e-14 * np.linalg.norm(ref)


# ---- invariants on larger lattices -------------------------------------------------
def test_gamma5_hermiticity_and_adjoint():
    dims = (4, 4, 4, 6)
    U = wdinputs.gauge_random(dims, 0.5, 51)
    x = wdinputs.spinor_gaussian(dims, 52)
    y = wdinputs.spinor_gaussian(dims, 53)
    g5 = np.array([1, 1, -1, -1], dtype=float)[:, None, None]
    lhs = oracle.dslash_full(dims, U, x, dagger=True)
    rhs = g5 * oracle.dslash_full(dims, U, g5 * x)
    assert np.abs(lhs - rhs).max() < 1e-13
    ip1 = np.vdot(to_vec(y), to_vec(oracle.dslash_full(dims, U, x)))
    ip2 = np.vdot(to_vec(oracle.dslash_full(dims, U, y, dagger=True)), to_vec(x))
    assert abs(ip1 - ip2) <= 1e-13 * abs(ip1)
    xe, _ = oracle.split(dims, x)
    ye, _ = oracle.split(dims, y)
    a = np.vdot(to_vec(ye), to_vec(oracle.mhat(dims, U, 0.12, xe)))
    b = np.vdot(to_vec(oracle.mhat(dims, U, 0.12, ye, dagger=True)), to_vec(xe))
    assert abs(a - b) <= 1e-13 * abs(a)


def _plane_wave(dims, p, chi):
    coords, _ = enumerate_sites(dims)
    X = np.array(coords, dtype=float)
    phase = np.exp(1j * X @ np.asarray(p))
    return phase[:, None] * chi[None, :], X


@pytest.mark.parametrize("tap", [True, False])
def test_free_field_plane_wave_spectrum(tap):
    dims, kappa = (4, 6, 4, 8), 0.12
    U = wdinputs.gauge_unit(dims)
    g = gammas()
    rng = np.random.default_rng(0)
    for n in ([0, 0, 0, 0], [1, 2, 3, 1], [3, 5, 1, 6]):
        p = [2 * np.pi * n[m] / dims[m] for m in range(3)]
        p.append(((2 * n[3] + 1) if tap else 2 * n[3]) * np.pi / dims[3])
        chi = rng.normal(size=12) + 1j * rng.normal(size=12)
        wave, _ = _plane_wave(dims, p, chi)
        Dp = sum(2 * np.cos(p[m]) * np.eye(4) - 2j * np.sin(p[m]) * g[m] for m in range(4))
        Dp12 = np.kron(Dp, np.eye(3))
        psi = from_vec(wave.reshape(-1))
        got = to_vec(oracle.mfull(dims, U, kappa, psi, antiperiodic_t=tap))
        ref = (wave @ (np.eye(12) - kappa * Dp12).T).reshape(-1)
        assert np.abs(got - ref).max() < 1e-13
        # even-site restriction: M_hat phi_e = (1 - kappa^2 D(p)^2) phi_e
        pe, _ = oracle.split(dims, psi)
        got_e = to_vec(oracle.mhat(dims, U, kappa, pe, antiperiodic_t=tap))
        ref_e = (to_vec(pe).reshape(-1, 12) @ (np.eye(12) - kappa ** 2 * Dp12 @ Dp12).T).reshape(-1)
        assert np.abs(got_e - ref_e).max() < 1e-13
        # eigenvalues of 1 - kappa^2 D(p)^2 against the closed form
        s2 = sum(np.sin(p[m]) ** 2 for m in range(4))
        c = sum(np.cos(p[m]) for m in range(4))
        lam = [1 - kappa ** 2 * (2 * c + sg * 2j * np.sqrt(s2)) ** 2 for sg in (1, -1)]
        ev = np.linalg.eigvals(np.eye(4) - kappa ** 2 * Dp @ Dp)
        for e in ev:
            assert min(abs(e - l) for l in lam) < 1e-12


def test_gauge_covariance():
    dims = (4, 4, 2, 6)
    V = 4 * 4 * 2 * 6
    U = wdinputs.gauge_random(dims, 0.5, 61)
    psi = wdinputs.spinor_gaussian(dims, 62)
    W = wdinputs.su3_random(V, 2.0, 63)
    Om = (W[..., 0] + 1j * W[..., 1]).reshape(dims[3], dims[2], dims[1], dims[0], 3, 3)
    Uc = U[..., 0] + 1j * U[..., 1]
    Up = np.empty_like(Uc)
    for mu in range(4):
        axis = 3 - mu  # array axes are (t, z, y, x)
        Om_next = np.roll(Om, -1, axis=axis)
        Up[..., mu, :, :] = Om @ Uc[..., mu, :, :] @ np.conj(np.swapaxes(Om_next, -1, -2))
    Up_r = np.stack([Up.real, Up.imag], axis=-1)
    pc = psi[..., 0] + 1j * psi[..., 1]
    pt = np.einsum("tzyxab,tzyxsb->tzyxsa", Om, pc)
    pt_r = np.stack([pt.real, pt.imag], axis=-1)
    lhs = oracle.dslash_full(dims, Up_r, pt_r)
    d = oracle.dslash_full(dims, U, psi)
    dc = d[..., 0] + 1j * d[..., 1]
    rhs = np.einsum("tzyxab,tzyxsb->tzyxsa", Om, dc.reshape(pc.shape))
    assert np.abs((lhs[..., 0] + 1j * lhs[..., 1]).reshape(rhs.shape) - rhs).max() < 1e-13


def test_locality_point_source_hits_its_eight_neighbours():
    dims = (4, 4, 4, 4)
    U = wdinputs.gauge_random(dims, 0.3, 71)
    psi = np.zeros((4, 4, 4, 4, 4, 3, 2))
    psi[1, 2, 3, 0, 2, 1, 0] = 1.0  # t=1, z=2, y=3, x=0
    out = oracle.dslash_full(dims, U, psi)
    nz = np.argwhere(np.abs(out).reshape(4, 4, 4, 4, -1).max(axis=-1) > 0)
    expect = set()
    for mu, axis in enumerate([3, 2, 1, 0]):
        for d in (1, -1):
            c = [1, 2, 3, 0]
            c[axis] = (c[axis] + d) % 4
            expect.add(tuple(c))
    assert set(map(tuple, nz)) == expect


def test_translation_invariance_spatial():
    dims = (4, 4, 4, 4)
    U = wdinputs.gauge_random(dims, 0.5, 81)
    psi = wdinputs.spinor_gaussian(dims, 82)
    out = oracle.dslash_full(dims, U, psi).reshape(4, 4, 4, 4, 4, 3, 2)
    for axis in (1, 2, 3):  # z, y, x (periodic)
        Us = np.roll(U, 1, axis=axis)
        ps = np.roll(psi, 1, axis=axis)
        o2 = oracle.dslash_full(dims, Us, ps).reshape(out.shape)
        assert np.abs(o2 - np.roll(out, 1, axis=axis)).max() < 1e-14


# ---- even-odd solve ----------------------------------------------------------
def test_prepare_and_reconstruct_give_the_dense_solution():
    dims, kappa = (2, 4, 2, 6), 0.12
    U = wdinputs.gauge_random(dims, 0.3, 91)
    b = wdinputs.spinor_gaussian(dims, 92)
    M = np.eye(12 * 96) - kappa * dense_hopping(dims, U)
    x_ref = np.linalg.solve(M, to_vec(b))
    bhat = oracle.prepare(dims, U, kappa, b)
    # solve the Schur system densely from the oracle's b_hat
    even, odd = parity_masks(dims)
    Dd = dense_hopping(dims, U)
    S = np.eye(even.sum()) - kappa ** 2 * Dd[np.ix_(even, odd)] @ Dd[np.ix_(odd, even)]
    xe = np.linalg.solve(S, to_vec(bhat))
    x_full = oracle.reconstruct(dims, U, kappa, b, from_vec(xe))
    assert np.linalg.norm(to_vec(x_full) - x_ref) <= 1e-13 * np.linalg.norm(x_ref)
    assert oracle.true_relres(dims, U, kappa, b, x_full) < 1e-14


@pytest.mark.parametrize("tap", [True, False])
def test_true_relres_is_the_dense_residual_at_non_solutions(tap):
    """The checker behind every solver parity claim, ||b - (1 - kappa D) x|| /
    ||b|| of the full system (Section 3), against the dense matrix of Eq. 1
    at points that are not solutions: x = 0 gives exactly 1; x = the dense
    solution plus a perturbation gives the dense residual norm (a dropped
    square root, a missing normalisation by ||b||, a sign of kappa or a
    residual of the Schur system alone would all fail here)."""
    dims, kappa = (2, 4, 2, 6), 0.12
    U = wdinputs.gauge_random(dims, 0.3, 111)
    b = wdinputs.spinor_gaussian(dims, 112)
    M = np.eye(12 * 96) - kappa * dense_hopping(dims, U, antiperiodic_t=tap)
    bv = to_vec(b)
    assert oracle.true_relres(dims, U, kappa, b, np.zeros_like(b), antiperiodic_t=tap) == 1.0
    # x = b: residual kappa D b, whose norm is independent of the solve
    expect = np.linalg.norm(bv - M @ bv) / np.linalg.norm(bv)
    got = oracle.true_relres(dims, U, kappa, b, b, antiperiodic_t=tap)
    assert abs(got - expect) <= 1e-14 * expect
    # scaled b: the relative residual does not depend on the scale of b and x
    got2 = oracle.true_relres(dims, U, kappa, 3.0 * b, 3.0 * b, antiperiodic_t=tap)
    assert abs(got2 - expect) <= 1e-14 * expect
    x_ref = np.linalg.solve(M, bv)
    rng = np.random.default_rng(113)
    for scale in (1e-3, 1e-7, 1e-11):
        dx = scale * (rng.standard_normal(x_ref.shape) + 1j * rng.standard_normal(x_ref.shape))
        xv = x_ref + dx
        expect = np.linalg.norm(bv - M @ xv) / np.linalg.norm(bv)
        got = oracle.true_relres(dims, U, kappa, b, from_vec(xv), antiperiodic_t=tap)
        # the dense residual itself carries ~1e-16 * ||b|| of rounding
        assert abs(got - expect) <= 1e-12 * expect + 1e-15, (scale, got, expect)
        # and it is linear in the perturbation: ||M dx|| / ||b||
        lin = np.linalg.norm(M @ dx) / np.linalg.norm(bv)
        assert abs(got - lin) <= 1e-3 * lin + 1e-15
    # the odd-site residual counts too: perturbing only the odd sites of the
    # dense solution moves the result
    even, odd = parity_masks(dims)
    xv = x_ref.copy()
    xv[odd] += 1e-6
    expect = np.linalg.norm(bv - M @ xv) / np.linalg.norm(bv)
    got = oracle.true_relres(dims, U, kappa, b, from_vec(xv), antiperiodic_t=tap)
    assert abs(got - expect) <= 1e-9 * expect and expect > 1e-7


@pytest.mark.parametrize("solver", ["bicgstab", "cgnr"])
def test_solvers_match_dense_solve(solver):
    dims, kappa = (2, 4, 2, 6), 0.12
    U = wdinputs.gauge_random(dims, 0.3, 101)
    b = wdinputs.spinor_gaussian(dims, 102)
    M = np.eye(12 * 96) - kappa * dense_hopping(dims, U)
    x_ref = np.linalg.solve(M, to_vec(b))
    x, info = getattr(oracle, solver)(dims, U, kappa, b, tol=1e-12)
    assert info["converged"] and info["true_relres"] <= 1e-12
    r = to_vec(b) - M @ to_vec(x)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(to_vec(b))
    cond = np.linalg.cond(M)
    assert np.linalg.norm(to_vec(x) - x_ref) <= 10 * cond * 1e-12 * np.linalg.norm(x_ref)


def test_bicgstab_on_8x4_config_converges():
    dims, kappa = (8, 8, 8, 8), 0.12
    U = wdinputs.gauge_random(dims, 0.3, 1)
    b = wdinputs.spinor_gaussian(dims, 1001)
    x, info = oracle.bicgstab(dims, U, kappa, b, tol=1e-10)
    assert info["converged"] and info["true_relres"] <= 1e-10
    assert 5 < info["iters"] < 200


# ---- 16-bit formats ------------------------------------------------------------
def test_f16_rounding_matches_numpy():
    rng = np.random.default_rng(1)
    vals = np.concatenate([
        rng.normal(size=20000).astype(np.float32),
        (rng.normal(size=20000) * 1e-5).astype(np.float32),
        (rng.normal(size=5000) * 1e-8).astype(np.float32),
        (rng.normal(size=5000) * 3e4).astype(np.float32),
        np.array([0.0, -0.0, 65504.0, 65519.99, 65519.0, 1e-7, 5.960464477539063e-08,
                  2.980232238769531e-08, 2.9802326e-08, 1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11,
                  np.inf, -np.inf], dtype=np.float32),
    ])
    ours = oracle.f32_to_f16_bits(vals)
    ref = vals.astype(np.float16).view(np.uint16)
    assert np.array_equal(ours, ref)
    back = oracle.f16_bits_to_f32(ref)
    assert np.array_equal(back, ref.view(np.float16).astype(np.float32))


@pytest.mark.parametrize("kind", ["i16", "f16"])
def test_spinor16_encoding_properties(kind):
    rng = np.random.default_rng(2)
    psi = rng.normal(size=(500, 4, 3, 2)) * np.exp(rng.normal(size=(500, 1, 1, 1)) * 3)
    psi[7] = 0.0
    q, nm = oracle.encode_spinor16(kind, psi)
    f = psi.reshape(500, 24).astype(np.float32)
    assert np.array_equal(nm, np.abs(f).max(axis=1))
    assert np.all(q[7] == 0) and nm[7] == 0
    dec = oracle.decode_spinor16(kind, q, nm).reshape(500, 24)
    if kind == "i16":
        qs = q.view(np.int16)
        assert np.abs(qs).max() <= 32767
        assert np.all(np.abs(qs).max(axis=1)[nm > 0] == 32767)  # the largest element maps to full scale
        bound = nm[:, None] / 32767 * (0.5 + 5e-3)  # binary32 scale and product roundings
    else:
        bound = nm[:, None] * 2.0 ** -11 * (1 + 1e-3) + nm[:, None] * 2.0 ** -25
    assert np.all(np.abs(dec - f) <= bound)


@pytest.mark.parametrize("kind", ["i16", "f16"])
def test_spinor16_tiny_sites_are_stored_as_zero(kind):
    """Sites whose norm is below 2^-100 (where 32767/norm would overflow binary32)
    are stored as zero; just above the threshold the scale stays finite."""
    psi = np.zeros((3, 4, 3, 2))
    psi[0, 1, 2, 0] = 3e-39    # binary32 denormal
    psi[1, 0, 0, 1] = 2.0 ** -101
    psi[2, 3, 1, 0] = 2.0 ** -99
    q, nm = oracle.encode_spinor16(kind, psi)
    assert nm[0] == 0 and nm[1] == 0 and not q[:2].any()
    dec = oracle.decode_spinor16(kind, q, nm)
    assert np.all(np.isfinite(dec)) and dec[2, 3, 1, 0] == 2.0 ** -99


@pytest.mark.parametrize("kind", ["i16", "f16"])
def test_link16_encoding_properties(kind):
    U = wdinputs.gauge_random((2, 2, 2, 2), 0.5, 3)
    q = oracle.encode_link16(kind, U)
    dec = oracle.decode_link16(kind, q)
    if kind == "i16":
        assert np.all(np.abs(dec - U) <= 0.5 / 32767 + 1e-7)
    else:
        assert np.all(np.abs(dec - U) <= 2.0 ** -11 * np.abs(U) + 2.0 ** -25)


# ---- 8-real links (Appendix A.2) and the temporal gauge (Section 4.3) ----------------

def _cx(U):
    return U[..., 0] + 1j * U[..., 1]


@pytest.mark.parametrize("eps", [0.3, 1.0, 3.0])
def test_link8_round_trip_restores_the_matrix(eps):
    U = wdinputs.su3_random(2000, eps, 41)
    p = oracle.encode_link8(U)
    assert p.shape == (2000, 8)
    R = oracle.decode_link8(p)
    assert np.abs(R - U).max() < 1e-12


def test_link8_rebuilds_special_unitary_matrices_from_any_parameters():
    """For any a2, a3 (|a2|^2 + |a3|^2 < 1), b1 (|b1|^2 <= |a2|^2 + |a3|^2) and
    phases, the rebuilt matrix is in SU(3) and carries the given entries; a
    sign slip in b', c' or the plane rotation breaks unitarity or the
    determinant."""
    rng = np.random.default_rng(5)
    n = 500
    a23 = rng.normal(size=(n, 4))
    a23 *= (rng.uniform(0.05, 0.95, n) / np.linalg.norm(a23, axis=1))[:, None]
    N = np.linalg.norm(a23, axis=1)
    ang = rng.uniform(0, 2 * np.pi, n)
    b1 = (N * rng.uniform(0, 1, n))[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    p = np.concatenate([a23, b1, rng.uniform(-np.pi, np.pi, (n, 2))], axis=1)
    M = _cx(oracle.decode_link8(p))
    eye = np.eye(3)
    assert np.abs(M @ np.conj(np.swapaxes(M, 1, 2)) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(M) - 1).max() < 1e-13
    assert np.allclose(M[:, 0, 1], p[:, 0] + 1j * p[:, 1]) and np.allclose(M[:, 0, 2], p[:, 2] + 1j * p[:, 3])
    assert np.allclose(M[:, 1, 0], p[:, 4] + 1j * p[:, 5])
    assert np.allclose(np.angle(M[:, 0, 0]), np.angle(np.exp(1j * p[:, 6])))
    assert np.allclose(np.angle(M[:, 2, 0]), np.angle(np.exp(1j * p[:, 7])))


def test_link8_negative_square_root_argument_is_taken_as_zero():
    p = np.array([[0.8, 0.0, 0.0, 0.6000001, 0.0, 0.0, 0.3, 0.2]])
    M = _cx(oracle.decode_link8(p))
    assert np.all(np.isfinite(M))
    assert M[0, 0, 0] == 0.0 and M[0, 2, 0] != 0.0


def test_temporal_gauge_makes_time_links_unit_but_on_the_last_slice():
    dims = (4, 2, 4, 6)
    U = wdinputs.gauge_random(dims, 0.5, 17)
    Uf, g = oracle.gauge_fix_temporal(dims, U)
    Ut = _cx(Uf.reshape(dims[::-1] + (4, 3, 3, 2))[..., 3, :, :, :])
    assert np.abs(Ut[:-1] - np.eye(3)).max() < 1e-13
    # the last slice carries the time line's product: same trace as the ordered product
    Uo = _cx(U.reshape(dims[::-1] + (4, 3, 3, 2))[..., 3, :, :, :])
    P = np.broadcast_to(np.eye(3, dtype=complex), Uo.shape[1:]).copy()
    for t in range(dims[3]):
        P = P @ Uo[t]
    assert np.abs(np.trace(Ut[-1], axis1=-2, axis2=-1) - np.trace(P, axis1=-2, axis2=-1)).max() < 1e-12
    G = _cx(g)
    assert np.abs(G @ np.conj(np.swapaxes(G, -1, -2)) - np.eye(3)).max() < 1e-13
    # the links stay in SU(3)
    M = _cx(Uf).reshape(-1, 3, 3)
    assert np.abs(np.linalg.det(M) - 1).max() < 1e-12


@pytest.mark.parametrize("tap", [True, False])
def test_temporal_gauge_rotation_is_a_similarity_transform_of_d(tap):
    """D[U'] (G psi) = G (D[U] psi), with the antiperiodic sign untouched."""
    dims = (4, 2, 4, 6)
    U = wdinputs.gauge_random(dims, 0.5, 18)
    Uf, g = oracle.gauge_fix_temporal(dims, U)
    psi = wdinputs.spinor_gaussian(dims, 19)
    lhs = oracle.dslash_full(dims, Uf, oracle.gauge_rotate_spinor(dims, g, psi), antiperiodic_t=tap)
    rhs = oracle.gauge_rotate_spinor(dims, g, oracle.dslash_full(dims, U, psi, antiperiodic_t=tap))
    assert np.abs(lhs - rhs).max() < 1e-12
    back = oracle.gauge_rotate_spinor(dims, g, oracle.gauge_rotate_spinor(dims, g, psi), adjoint=True)
    assert np.abs(back - psi).max() < 1e-13
