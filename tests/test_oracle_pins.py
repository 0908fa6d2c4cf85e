"""Pins of the FP64 oracle to the paper's equations (CPU only).

Each test compares the oracle with a route that does not go through the
oracle's code: closed forms, brute-force diagonalisation, the spin-orbital
form of the equations, the Dyson equation, frequency integration, the MP2
self-energy, four-index integrals, invariances.  The mutation tests at the end
plant mistakes in a copy of an oracle step and check that a pin catches them.
"""
import numpy as np
import pytest

import oracle as O
import pins
from qsgw_inputs import cfg1_omega_grid, make_config, make_mo_tensor, make_problem


def tiny(nbf=6, naux=14, nocc=2, seed=3, coupling=1.0):
    return make_problem(nbf, naux, nocc, naux, 0.9, seed, coupling=coupling)


def chain(p, eps=None, C=None):
    eps = p.eps0 if eps is None else eps
    C = p.C0 if C is None else C
    B_mo = O.mo_transform(p.B_ao, C)
    M, sq = O.rpa_hermitian(B_mo, eps, p.nocc)
    Om, XpY = O.rpa_solve(M, sq)
    w = O.residues(B_mo, XpY, p.nocc)
    return B_mo, M, sq, Om, XpY, w


# --------------------------------------------------------------- P1 ------
@pytest.mark.parametrize("b,B00,B11", [(0.3, 0.7, -0.2), (1.1, 0.0, 0.4), (0.05, -0.3, 0.9)])
def test_p1_one_transition_closed_form(b, B00, B11):
    eps = np.array([-0.8, 0.45])
    eta = 1e-3
    B_ao = np.array([[[B00, b], [b, B11]]])
    C = np.eye(2)
    B_mo = O.mo_transform(B_ao, C)
    M, sq = O.rpa_hermitian(B_mo, eps, 1)
    Om, XpY = O.rpa_solve(M, sq)
    w = O.residues(B_mo, XpY, 1)
    grid = np.linspace(-2, 2, 41)
    Om_ref, w_ref, sig_ref = pins.one_transition_closed_form(eps[0], eps[1], b, B00, B11, eta, grid)
    assert abs(Om[0] - Om_ref) <= 1e-15 * Om_ref
    # w is fixed up to the sign of the Casida eigenvector
    s = np.sign(w[0, 1, 0] / w_ref[0, 1])
    np.testing.assert_allclose(s * w[:, :, 0], w_ref, rtol=1e-14, atol=1e-16)
    for m in range(2):
        sig = O.sigma_element(w, eps, Om, 1, eta, m, m, grid)
        np.testing.assert_allclose(sig, sig_ref[m], rtol=1e-13, atol=1e-16)
    # qsGW potential, Eq. (19), from the closed-form residues
    V = O.sigma_qs(w, eps, Om, 1, eta)
    G = np.zeros((2, 2))
    for m in range(2):
        for n in range(2):
            x0 = eps[m] - eps[0] + Om_ref
            x1 = eps[m] - eps[1] - Om_ref
            G[m, n] = (w_ref[m, 0] * w_ref[n, 0] * x0 / (x0 ** 2 + eta ** 2)
                       + w_ref[m, 1] * w_ref[n, 1] * x1 / (x1 ** 2 + eta ** 2))
    np.testing.assert_allclose(V, 0.5 * (G + G.T), rtol=1e-13, atol=1e-16)


# --------------------------------------------------------------- P2 ------
@pytest.mark.parametrize("seed", [1, 2])
def test_p2_nonhermitian_casida(seed):
    p = tiny(seed=seed)
    B_mo, M, sq, Om, XpY, w = chain(p)
    Om_b, XpY_b = pins.casida_nonhermitian(B_mo, p.eps0, p.nocc)
    np.testing.assert_allclose(Om, Om_b, rtol=1e-12)
    for s in range(Om.size):
        sgn = np.sign(XpY[:, s] @ XpY_b[:, s])
        np.testing.assert_allclose(XpY[:, s], sgn * XpY_b[:, s], rtol=1e-9, atol=1e-11)


# --------------------------------------------------------------- P3 ------
def test_p3_spin_orbital_equations():
    p = tiny(nbf=5, naux=9, nocc=2, seed=7)
    eta = 1e-2
    B_mo, M, sq, Om, XpY, w = chain(p)
    grid = np.array([-1.3, 0.2, 0.9, 2.5])
    Om_so, sig_so = pins.spin_orbital_gw(B_mo, p.eps0, p.nocc, eta, grid, 1, 3)
    # singlets are the spin-adapted Omega, triplets are Delta (A = Delta, B = 0)
    delta = O.transition_energies(p.eps0, p.nocc)
    expect = np.sort(np.concatenate([Om, delta]))
    np.testing.assert_allclose(Om_so, expect, rtol=1e-12)
    sig = O.sigma_element(w, p.eps0, Om, p.nocc, eta, 1, 3, grid)
    np.testing.assert_allclose(sig, sig_so, rtol=1e-11, atol=1e-14)


# --------------------------------------------------------------- P4 ------
@pytest.mark.parametrize("nu", [0.0, 0.37, 2.0, 11.0])
def test_p4_dyson_screened_interaction(nu):
    p = tiny(nbf=7, naux=12, nocc=3, seed=11)
    B_mo, M, sq, Om, XpY, w = chain(p)
    Wd = pins.screened_dyson(B_mo, p.eps0, p.nocc, nu)
    Ws = pins.screened_spectral(w, Om, nu)
    np.testing.assert_allclose(Ws, Wd, rtol=1e-10, atol=1e-13 * np.abs(Wd).max())


# --------------------------------------------------------------- P5 ------
@pytest.mark.parametrize("m,n,xi", [(1, 1, 0.3), (1, 3, 0.3), (0, 4, 1.5), (5, 2, 0.05)])
def test_p5_frequency_integration_of_iGW(m, n, xi):
    p = tiny(seed=3)
    B_mo, M, sq, Om, XpY, w = chain(p)
    mu = 0.5 * (p.eps0[p.nocc - 1] + p.eps0[p.nocc])
    z = mu + 1j * xi
    ref = O.sigma_element(w, p.eps0, Om, p.nocc, 0.0, m, n, [z])[0]
    q = pins.sigma_frequency_integral(B_mo, p.eps0, p.nocc, z, m, n, npts=400)
    assert abs(q - ref) < 1e-9 * max(1.0, abs(ref))


# --------------------------------------------------------------- P6 ------
def test_p6_weak_coupling_is_mp2_direct():
    p = tiny(nbf=5, naux=10, nocc=2, seed=5)
    eta = 0.05
    om = 0.37
    diffs, sigs = [], []
    for lam in (0.01, 0.02):
        B = p.B_ao * lam
        B_mo = O.mo_transform(B, p.C0)
        M, sq = O.rpa_hermitian(B_mo, p.eps0, p.nocc)
        Om, XpY = O.rpa_solve(M, sq)
        w = O.residues(B_mo, XpY, p.nocc)
        gw = O.sigma_element(w, p.eps0, Om, p.nocc, eta, 1, 2, [om])[0]
        mp2 = pins.sigma_mp2_direct(B_mo, p.eps0, p.nocc, eta, om, 1, 2)
        diffs.append(abs(gw - mp2))
        sigs.append(abs(gw))
    # Sigma ~ lambda^4, Sigma^GW - Sigma^MP2,direct ~ lambda^6
    assert 14.0 < sigs[1] / sigs[0] < 18.0
    assert 54.0 < diffs[1] / diffs[0] < 74.0


# --------------------------------------------------------------- P7 ------
def test_p7_sum_rules():
    p = tiny(nbf=8, naux=16, nocc=3, seed=9)
    B_mo, M, sq, Om, XpY, w = chain(p)
    A, B = O.casida_AB(B_mo, p.eps0, p.nocc)
    delta = O.transition_energies(p.eps0, p.nocc)
    np.testing.assert_allclose((XpY * Om[None, :]) @ XpY.T, np.diag(delta), atol=1e-11)
    np.testing.assert_allclose((XpY / Om[None, :]) @ XpY.T, np.linalg.inv(A + B), atol=1e-11)
    assert abs(np.sum(Om ** 2) - np.trace(M)) < 1e-10 * np.trace(M)
    np.testing.assert_allclose(A - B, np.diag(delta), atol=1e-13)


# --------------------------------------------------------------- P8 ------
def test_p8_invariances():
    p = tiny(nbf=7, naux=12, nocc=3, seed=13)
    eta = 1e-2
    h = O.hf_core(p.B_ao, p.C0, p.eps0, p.nocc)
    ref = O.qsgw_step(p.B_ao, h, p.C0, p.eps0, p.nocc, eta)
    rng = np.random.default_rng(99)
    # auxiliary rotation
    Oa, _ = np.linalg.qr(rng.standard_normal((p.naux, p.naux)))
    Brot = np.einsum("pq,qmn->pmn", Oa, p.B_ao)
    r1 = O.qsgw_step(Brot, O.hf_core(Brot, p.C0, p.eps0, p.nocc), p.C0, p.eps0, p.nocc, eta)
    np.testing.assert_allclose(r1["eps"], ref["eps"], atol=1e-11)
    np.testing.assert_allclose(r1["Omega"], ref["Omega"], rtol=1e-11)
    np.testing.assert_allclose(r1["V"], ref["V"], atol=1e-11)
    # AO rotation
    R, _ = np.linalg.qr(rng.standard_normal((p.nbf, p.nbf)))
    B2 = np.einsum("am,pab,bn->pmn", R, p.B_ao, R)
    C2 = R.T @ p.C0
    h2 = R.T @ h @ R
    r2 = O.qsgw_step(B2, h2, C2, p.eps0, p.nocc, eta)
    np.testing.assert_allclose(r2["eps"], ref["eps"], atol=1e-11)
    np.testing.assert_allclose(r2["V"], ref["V"], atol=1e-11)
    np.testing.assert_allclose(R @ r2["F"] @ R.T, ref["F"], atol=1e-11)
    # MO sign flips
    sg = np.array([1, -1, -1, 1, -1, 1, -1.0])
    r3 = O.qsgw_step(p.B_ao, h, p.C0 * sg[None, :], p.eps0, p.nocc, eta)
    np.testing.assert_allclose(r3["eps"], ref["eps"], atol=1e-11)
    np.testing.assert_allclose(r3["V"], ref["V"] * np.outer(sg, sg), atol=1e-11)


# --------------------------------------------------------------- P9 ------
def test_p9_ri_hartree_exchange_four_index():
    p = tiny(nbf=6, naux=10, nocc=2, seed=17)
    D = O.density(p.C0, p.nocc)
    J4, K4 = pins.jk_four_index(p.B_ao, D)
    np.testing.assert_allclose(O.hartree(p.B_ao, D), J4, atol=1e-12)
    np.testing.assert_allclose(O.exchange(p.B_ao, D), K4, atol=1e-12)


# --------------------------------------------------------------- P10 -----
def test_p10_hf_fixed_point():
    p = make_config("cfg1")
    h = O.hf_core(p.B_ao, p.C0, p.eps0, p.nocc)
    F = O.fock(h, p.B_ao, p.C0, p.nocc, np.zeros((p.nbf, p.nbf)))
    e, C = O.diagonalize(F)
    np.testing.assert_allclose(e, p.eps0, atol=1e-12)
    np.testing.assert_allclose(np.abs(C.T @ p.C0), np.eye(p.nbf), atol=1e-9)
    np.testing.assert_allclose(F, F.T, atol=0)


# ------------------------------------------------ iteration properties ---
def test_sigma_real_symmetric_and_cfg1_grid():
    p = make_config("cfg1")
    B_mo, M, sq, Om, XpY, w = chain(p)
    assert Om.size == 95
    V = O.sigma_qs(w, p.eps0, Om, p.nocc, 1e-3)
    np.testing.assert_array_equal(V, V.T)
    grid = cfg1_omega_grid()
    assert grid.size == 201 and grid[0] == -2.0 and abs(grid[-1] - 2.0) < 1e-15
    homo = p.nocc - 1
    sig = O.sigma_element(w, p.eps0, Om, p.nocc, 1e-3, homo, homo, grid)
    # Sigma(conj z) = conj Sigma(z) with eta -> 0 (real residues)
    z = 0.1 + 0.4j
    a = O.sigma_element(w, p.eps0, Om, p.nocc, 0.0, homo, homo + 1, [z, np.conj(z)])
    assert abs(a[1] - np.conj(a[0])) < 1e-14 * abs(a[0])


def test_iterate_records_and_mixing():
    p = tiny(nbf=8, naux=16, nocc=3, seed=21, coupling=0.1)
    h = O.hf_core(p.B_ao, p.C0, p.eps0, p.nocc)
    eps, C, hist = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0, p.nocc, 1e-2, 1e-10, 40)
    assert hist[-1]["max_deps"] < 1e-10
    np.testing.assert_allclose(C.T @ C, np.eye(p.nbf), atol=1e-12)
    # at the fixed point, one more step returns the same energies
    st = O.qsgw_step(p.B_ao, h, C, eps, p.nocc, 1e-2)
    np.testing.assert_allclose(st["eps"], eps, atol=1e-9)
    # linear mixing reaches the same fixed point
    eps2, _, _ = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0, p.nocc, 1e-2, 1e-11, 200, mix=0.6)
    np.testing.assert_allclose(eps2, eps, atol=1e-9)


# ------------------------------------------- P19, P20: per-state features --
@pytest.mark.parametrize("eta", [1e-2, 1e-3])
def test_p19_sigma_derivative_is_finite_difference_of_eq17(eta):
    """d Sigma_mm / d omega against a central difference of Eq. (17) itself
    (sigma_element), at several states and frequencies between the poles."""
    p = make_config("cfg1")
    B_mo, M, sq, Om, XpY, w = chain(p)
    for m in (0, p.nocc - 2, p.nocc - 1, p.nocc, p.nocc + 3, p.nbf - 1):
        for om in (p.eps0[m], p.eps0[m] + 0.013, -0.71):
            der = O.sigma_diag_derivative(w, p.eps0, Om, p.nocc, eta, m, om)
            # Richardson-extrapolated central difference, step << eta
            h = eta * 1e-3
            d1 = (O.sigma_element(w, p.eps0, Om, p.nocc, eta, m, m, [om + h, om - h]))
            d2 = (O.sigma_element(w, p.eps0, Om, p.nocc, eta, m, m, [om + 2 * h, om - 2 * h]))
            f1 = (d1[0] - d1[1]) / (2 * h)
            f2 = (d2[0] - d2[1]) / (4 * h)
            fd = (4 * f1 - f2) / 3
            assert abs(der - fd) <= 1e-6 * abs(fd) + 1e-9, (m, om, der, fd)


@pytest.mark.parametrize("b,B00,B11", [(0.3, 0.7, -0.2), (1.1, 0.0, 0.4)])
def test_p19_sigma_derivative_two_level_closed_form(b, B00, B11):
    """The one-transition case: the derivative of the closed-form Sigma_mm(omega)."""
    eps = np.array([-0.8, 0.45])
    B_mo = np.array([[[B00, b], [b, B11]]])
    M, sq = O.rpa_hermitian(B_mo, eps, 1)
    Om, XpY = O.rpa_solve(M, sq)
    w = O.residues(B_mo, XpY, 1)
    grid = [-1.3, -0.8, 0.0, 0.45, 1.7]
    for eta in (1e-2, 1e-3):
        ref = pins.one_transition_sigma_derivative(eps[0], eps[1], b, B00, B11, eta, grid)
        for m in range(2):
            der = np.array([O.sigma_diag_derivative(w, eps, Om, 1, eta, m, x) for x in grid])
            np.testing.assert_allclose(der, ref[m], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("nbf,naux,nocc,seed", [(6, 14, 2, 3), (7, 9, 3, 5), (5, 20, 1, 8)])
def test_p20_exchange_diagonal_is_four_index_exchange(nbf, naux, nocc, seed):
    """Sigma_x,mm against -(C^T K[D] C)_mm with K[D] of Eq. (10) built from
    explicit four-index integrals (mu nu|lambda tau) = sum_P B B."""
    p = tiny(nbf=nbf, naux=naux, nocc=nocc, seed=seed)
    # a general orthogonal C, not the generator's, so occupied columns mix
    C = np.linalg.qr(np.random.default_rng(seed + 100).standard_normal((nbf, nbf)))[0]
    D = C[:, :nocc] @ C[:, :nocc].T
    _, K = pins.jk_four_index(p.B_ao, D)
    ref = -np.diag(C.T @ K @ C)
    got = O.exchange_diagonal_mo(O.mo_transform(p.B_ao, C), nocc)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)


def test_mutant_sigma_derivative_sign_caught(monkeypatch):
    """A sign slip in d Sigma / d omega fails the finite-difference pin."""
    orig = O.sigma_diag_derivative
    monkeypatch.setattr(O, "sigma_diag_derivative", lambda *a: -orig(*a))
    with pytest.raises(AssertionError):
        test_p19_sigma_derivative_is_finite_difference_of_eq17(1e-2)


def test_mutant_exchange_diagonal_over_virtuals_caught(monkeypatch):
    """Summing the exchange diagonal over virtual instead of occupied states
    fails the four-index pin."""
    def over_virtuals(B_mo, nocc):
        return -np.einsum("pmi,pmi->m", B_mo[:, :, nocc:], B_mo[:, :, nocc:])
    monkeypatch.setattr(O, "exchange_diagonal_mo", over_virtuals)
    with pytest.raises(AssertionError):
        test_p20_exchange_diagonal_is_four_index_exchange(6, 14, 2, 3)


# ------------------------------------------- P21: frozen mean field ------
def test_p21_frozen_mean_field():
    """Eq. (6) with the mean field frozen at the start's density: with F0 the
    start's Hartree-Fock matrix, the first step equals the full step (same
    density); the converged frozen iteration is self-consistent for F0 + V."""
    p = tiny(nbf=8, naux=16, nocc=3, seed=21, coupling=0.1)
    h = O.hf_core(p.B_ao, p.C0, p.eps0, p.nocc)
    D0 = p.C0[:, :p.nocc] @ p.C0[:, :p.nocc].T
    J0, K0 = pins.jk_four_index(p.B_ao, D0)
    F0 = h + J0 - K0
    # the synthetic start is an exact Hartree-Fock fixed point: F0 = C0 diag(eps0) C0^T
    np.testing.assert_allclose(F0, (p.C0 * p.eps0) @ p.C0.T, atol=1e-12)
    eta = 1e-2
    full = O.qsgw_step(p.B_ao, h, p.C0, p.eps0, p.nocc, eta)
    frz = O.qsgw_step(p.B_ao, F0, p.C0, p.eps0, p.nocc, eta, fock_mode="frozen")
    np.testing.assert_allclose(frz["eps"], full["eps"], atol=1e-12)
    eps, C, hist = O.qsgw_iterate(p.B_ao, F0, p.C0, p.eps0, p.nocc, eta, 1e-11, 200, mix=0.6,
                                  keep=("Vao",), fock_mode="frozen")
    assert hist[-1]["max_deps"] < 1e-11
    # at the fixed point (F0 + V[eps, C]) C = C diag(eps); V from the converged orbitals
    st = O.qsgw_step(p.B_ao, F0, C, eps, p.nocc, eta, fock_mode="frozen")
    Fc = F0 + C @ st["V"] @ C.T
    np.testing.assert_allclose(Fc @ C, C * eps[None, :], atol=1e-9)
    # and the frozen and full fixed points differ once the density has moved
    eps_f, _, _ = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0, p.nocc, eta, 1e-11, 200, mix=0.6)
    assert np.max(np.abs(eps_f - eps)) > 1e-6


# ------------------------------------- P22: DIIS on the Fock matrix ------
@pytest.mark.parametrize("n", [2, 3, 6])
def test_p22_diis_weights_minimise_the_error_norm(n):
    """Pulay's weights against an independent route: eliminate the constraint
    (c_n = 1 - sum of the others) and solve the unconstrained least-squares
    problem for the residual e_n + sum_i c_i (e_i - e_n) with lstsq."""
    rng = np.random.default_rng(22 + n)
    errs = [rng.standard_normal((7, 7)) for _ in range(n)]
    errs = [e - e.T for e in errs]  # commutators of symmetric matrices are antisymmetric
    c = O.diis_coefficients(errs)
    A = np.stack([(e - errs[-1]).ravel() for e in errs[:-1]], axis=1)
    x, *_ = np.linalg.lstsq(A, -errs[-1].ravel(), rcond=None)
    ref = np.append(x, 1.0 - x.sum())
    np.testing.assert_allclose(c, ref, rtol=1e-9, atol=1e-12)
    assert abs(c.sum() - 1.0) < 1e-12
    # no other affine combination has a smaller error norm
    best = np.linalg.norm(sum(ci * e for ci, e in zip(c, errs)))
    for _ in range(20):
        d = rng.standard_normal(n)
        d -= d.mean()
        assert np.linalg.norm(sum((ci + 1e-3 * di) * e for ci, di, e in zip(c, d, errs))) >= best


def test_p22_diis_reaches_the_plain_fixed_point():
    """DIIS changes the path, not the fixed point: from the same start the
    DIIS iteration, the mixed iteration and the plain iteration end at the
    same energies; at the end the Fock matrix commutes with the density
    (the DIIS error vanishes) and one plain step no longer moves anything."""
    for seed, coupling in ((21, 0.3), (22, 0.3), (23, 0.1)):
        p = tiny(nbf=8, naux=16, nocc=3, seed=seed, coupling=coupling)
        h = O.hf_core(p.B_ao, p.C0, p.eps0, p.nocc)
        eta = 0.05
        e1, C1, h1 = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0, p.nocc, eta, 1e-11, 60, diis=6,
                                    keep=("eps", "diis_err"))
        e2, _, h2 = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0, p.nocc, eta, 1e-11, 300, mix=0.5)
        e3, _, _ = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0, p.nocc, eta, 1e-11, 300)
        assert h1[-1]["max_deps"] < 1e-11 and h2[-1]["max_deps"] < 1e-11
        np.testing.assert_allclose(e1, e2, atol=1e-9)
        np.testing.assert_allclose(e1, e3, atol=1e-9)
        assert len(h1) < len(h2)
        assert h1[-1]["diis_err"] < 1e-9 < h1[0]["diis_err"]
        st = O.qsgw_step(p.B_ao, h, C1, e1, p.nocc, eta)
        assert np.max(np.abs(st["eps"] - e1)) < 1e-9
        # the first DIIS iteration is the plain step
        np.testing.assert_allclose(h1[0]["eps"], O.qsgw_step(p.B_ao, h, p.C0, p.eps0, p.nocc,
                                                             eta)["eps"], atol=1e-13)


def test_mutant_diis_constraint_sign_caught(monkeypatch):
    """Weights summing to -1 (the border row's sign flipped) fail P22."""
    good = O.diis_coefficients

    def flipped(errors):
        return -good(errors)
    monkeypatch.setattr(O, "diis_coefficients", flipped)
    with pytest.raises(AssertionError):
        test_p22_diis_weights_minimise_the_error_norm(3)


def test_mutant_diis_anticommutator_error_caught(monkeypatch):
    """An error vector F D + D F (anticommutator) does not vanish at the
    fixed point: P22's end-of-iteration check fails."""
    import oracle.qsgw_oracle as OQ
    monkeypatch.setattr(OQ, "diis_error", lambda F, D: F @ D + D @ F)
    with pytest.raises(AssertionError):
        test_p22_diis_reaches_the_plain_fixed_point()


# ------------------------------------------------------------- mutations --
_residues = O.residues


def _mutant_residues_no_sqrt2(B_mo, XpY, nocc):
    return _residues(B_mo, XpY, nocc) / np.sqrt(2.0)


def _mutant_rpa_minus_sign(B_mo, eps, nocc):
    A, B = O.casida_AB(B_mo, eps, nocc)
    delta = O.transition_energies(eps, nocc)
    K = (A - np.diag(delta)) / 2.0
    sq = np.sqrt(delta)
    # A + B with a single factor 2 (spin sum dropped)
    return sq[:, None] * (np.diag(delta) + 2.0 * K) * sq[None, :], sq


def _mutant_residues_transposed(B_mo, XpY, nocc):
    naux, n, _ = B_mo.shape
    Bai = B_mo[:, nocc:, :nocc].transpose(0, 2, 1).reshape(naux, -1)
    rho = Bai @ XpY[::-1]
    return (np.sqrt(2.0) * (B_mo.reshape(naux, n * n).T @ rho)).reshape(n, n, -1)


@pytest.mark.parametrize("target,mutant", [
    ("residues", _mutant_residues_no_sqrt2),
    ("rpa_hermitian", _mutant_rpa_minus_sign),
    ("residues", _mutant_residues_transposed),
])
def test_pins_catch_planted_mistakes(monkeypatch, target, mutant):
    """A plausible mistake planted in the oracle makes the Dyson pin fail."""
    monkeypatch.setattr(O, target, mutant)
    p = tiny(nbf=7, naux=12, nocc=3, seed=11)
    B_mo = O.mo_transform(p.B_ao, p.C0)
    M, sq = O.rpa_hermitian(B_mo, p.eps0, p.nocc)
    Om, XpY = O.rpa_solve(M, sq)
    w = O.residues(B_mo, XpY, p.nocc)
    Wd = pins.screened_dyson(B_mo, p.eps0, p.nocc, 0.37)
    Ws = pins.screened_spectral(w, Om, 0.37)
    assert not np.allclose(Ws, Wd, rtol=1e-6, atol=1e-10)


def test_mutant_sigma_sign_caught_by_closed_form(monkeypatch):
    """Swapping the occupied/virtual pole signs of Eq. (17) fails P1."""
    import oracle.qsgw_oracle as OM
    orig = OM._pole_denominators

    def swapped(omega, eps, Omega, nocc, eta):
        d = orig(omega, eps, Omega, nocc, eta)
        return d.conj()

    monkeypatch.setattr(OM, "_pole_denominators", swapped)
    eps = np.array([-0.8, 0.45])
    B_mo = np.array([[[0.7, 0.3], [0.3, -0.2]]])
    M, sq = O.rpa_hermitian(B_mo, eps, 1)
    Om, XpY = O.rpa_solve(M, sq)
    w = O.residues(B_mo, XpY, 1)
    grid = np.array([0.1])
    _, _, sig_ref = pins.one_transition_closed_form(eps[0], eps[1], 0.3, 0.7, -0.2, 1e-3, grid)
    sig = O.sigma_element(w, eps, Om, 1, 1e-3, 0, 0, grid)
    assert not np.allclose(sig, sig_ref[0], rtol=1e-8)


# ------------------------------------------------------- P12-P14: qsMP2 --
@pytest.mark.parametrize("nbf,naux,nocc,seed", [(5, 9, 2, 1), (6, 4, 3, 2), (4, 6, 1, 7)])
def test_p12_mp2_is_spin_orbital_second_order(nbf, naux, nocc, seed):
    """Eq. (20) with the exchange reading equals the second-order self-energy
    of antisymmetrised spin-orbital integrals, complex, every (m, n)."""
    # a general RI tensor: the generator's B has fully symmetric integrals,
    # which would hide the index pairing of the exchange term
    B_mo, eps = make_mo_tensor(nbf, naux, nocc, seed, coupling=1.0)
    for om, eta in ((0.37, 0.05), (-1.3, 1e-3), (eps[0], 0.02)):
        S = O.sigma_mp2(B_mo, eps, nocc, eta, om)
        T = pins.sigma2_spin_orbital(B_mo, eps, nocc, eta, om)
        np.testing.assert_allclose(S, T, rtol=0, atol=1e-12 * np.abs(T).max())
        np.testing.assert_allclose(S, S.T, rtol=0, atol=1e-12 * np.abs(T).max())


@pytest.mark.parametrize("B00,b,B11", [(0.7, 0.3, -0.2), (-0.1, 0.8, 0.5)])
def test_p13_mp2_two_level_closed_form(B00, b, B11):
    B_mo = np.array([[[B00, b], [b, B11]]])
    eps = np.array([-0.6, 0.35])
    for om in (-0.9, 0.1, 1.7):
        S = O.sigma_mp2(B_mo, eps, 1, 1e-3, om)
        ref = pins.mp2_two_level_closed_form(B_mo[0], eps[0], eps[1], 1e-3, om)
        np.testing.assert_allclose(S, ref, rtol=1e-13, atol=1e-16)


def test_p14_qsmp2_potential_and_direct_limit():
    """Eq. (21) from elements of Eq. (20); the direct sum is the weak-coupling
    limit of the GW self-energy (Sigma^GW - Sigma^MP2,direct ~ lambda^6)."""
    B_mo, eps = make_mo_tensor(7, 12, 3, 11, coupling=1.0)
    V = O.qsmp2_potential(B_mo, eps, 3, 0.01)
    np.testing.assert_array_equal(V, V.T)
    for m, n in ((0, 0), (1, 5), (6, 2)):
        a = pins.sigma2_spin_orbital(B_mo, eps, 3, 0.01, eps[n])[m, n]
        b = pins.sigma2_spin_orbital(B_mo, eps, 3, 0.01, eps[m])[n, m]
        assert abs(V[m, n] - 0.5 * (a + b).real) < 1e-12 * abs(V).max()
        assert abs(O.qsmp2_entry(B_mo, eps, 3, 0.01, m, n) - V[m, n]) < 1e-12 * abs(V).max()
    q = tiny(nbf=5, naux=10, nocc=2, seed=5)
    diffs = []
    for lam in (0.01, 0.02):
        Bl = O.mo_transform(q.B_ao * lam, q.C0)
        M, sq = O.rpa_hermitian(Bl, q.eps0, q.nocc)
        Om, XpY = O.rpa_solve(M, sq)
        w = O.residues(Bl, XpY, q.nocc)
        gw = O.sigma_element(w, q.eps0, Om, q.nocc, 0.05, 1, 2, [0.37])[0]
        d = O.sigma_mp2(Bl, q.eps0, q.nocc, 0.05, 0.37, terms="direct")[1, 2]
        x = O.sigma_mp2(Bl, q.eps0, q.nocc, 0.05, 0.37, terms="sox")[1, 2]
        full = O.sigma_mp2(Bl, q.eps0, q.nocc, 0.05, 0.37)[1, 2]
        assert abs(full - d - x) < 1e-14 * abs(full) + 1e-300
        diffs.append(abs(gw - d))
    assert 54.0 < diffs[1] / diffs[0] < 74.0


def test_mutant_mp2_printed_exchange_caught(monkeypatch):
    """The exchange integral of Eq. (20) exactly as printed for occupied p,
    (pi|an), fails the spin-orbital pin; so does dropping the spin factor 2."""
    import oracle.qsgw_oracle as OM
    orig = OM._mp2_integrals

    def printed(B_mo, nocc, m_rows=None, n_rows=None):
        L, R, X = orig(B_mo, nocc, m_rows, n_rows)
        n_rows_ = np.arange(B_mo.shape[1]) if n_rows is None else np.asarray(n_rows)
        X = X.copy()
        X[:, :nocc] = np.einsum("Ppi,Pan->npia", B_mo[:, :nocc, :nocc],
                                B_mo[:, nocc:][:, :, n_rows_])
        return L, R, X

    def no_spin(B_mo, nocc, m_rows=None, n_rows=None):
        L, R, X = orig(B_mo, nocc, m_rows, n_rows)
        return L, 0.5 * R, X

    B_mo, eps = make_mo_tensor(5, 9, 2, 1, coupling=1.0)
    T = pins.sigma2_spin_orbital(B_mo, eps, 2, 0.05, 0.37)
    for mutant in (printed, no_spin):
        monkeypatch.setattr(OM, "_mp2_integrals", mutant)
        S = O.sigma_mp2(B_mo, eps, 2, 0.05, 0.37)
        assert np.abs(S - T).max() > 1e-6 * np.abs(T).max()
    monkeypatch.setattr(OM, "_mp2_integrals", orig)


# ------------------------------------------------- P15: four-index AO->MO --
def test_p15_ao2mo_4center():
    """Eq. (16) on explicit integrals: the literal eight-fold sum (N = 4), the
    RI route (mn|kl) = sum_P B^P_mn B^P_kl with its own MO transform, slabs of
    the first index, and the identity / permutation special cases."""
    p = tiny(nbf=4, naux=5, nocc=1, seed=2)
    B = make_mo_tensor(4, 5, 1, 8)[0]          # general symmetric RI factors
    eri = pins.mo_eri(B)
    C = p.C0
    ref = pins.ao2mo_brute_force(eri, C)
    np.testing.assert_allclose(O.ao2mo_4center(eri, C), ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(O.ao2mo_4center(eri, C, [2, 3]), ref[2:], rtol=0, atol=1e-14)
    q = tiny(nbf=9, naux=7, nocc=2, seed=4)
    B9 = make_mo_tensor(9, 7, 2, 5)[0]
    np.testing.assert_allclose(O.ao2mo_4center(pins.mo_eri(B9), q.C0), pins.ri_four_index(B9, q.C0),
                               rtol=0, atol=1e-13)
    np.testing.assert_allclose(O.ao2mo_4center(eri, np.eye(4)), eri, rtol=0, atol=0)
    perm = np.eye(4)[:, [2, 0, 3, 1]]
    np.testing.assert_array_equal(O.ao2mo_4center(eri, perm), eri[np.ix_([2, 0, 3, 1], [2, 0, 3, 1],
                                                                        [2, 0, 3, 1], [2, 0, 3, 1])])


def test_mutant_ao2mo_caught():
    """A transposed C in one slot of Eq. (16), or a dropped slot, fails P15."""
    p = tiny(nbf=4, naux=5, nocc=1, seed=2)
    eri = pins.mo_eri(make_mo_tensor(4, 5, 1, 8)[0])
    ref = pins.ao2mo_brute_force(eri, p.C0)
    bad1 = np.einsum("abcd,am,bn,kc,dl->mnkl", eri, p.C0, p.C0, p.C0, p.C0)
    bad2 = np.einsum("abcd,am,bn,ck->mnkd", eri, p.C0, p.C0, p.C0)
    for bad in (bad1, bad2):
        assert np.abs(bad - ref).max() > 1e-6 * np.abs(ref).max()


# --------------------------------------------- P16-P17: open shell (UHF) --
def _two_spins(nbf, naux, nocc_a, nocc_b, seed):
    pa = make_problem(nbf, naux, nocc_a, naux, 0.9, seed, coupling=1.0)
    pb = make_problem(nbf, naux, nocc_b, naux, 0.9, seed + 100, coupling=1.0)
    B_a = O.mo_transform(pa.B_ao, pa.C0)
    B_b = O.mo_transform(pa.B_ao, pb.C0)          # same AO integrals, other orbitals
    return [B_a, B_b], [pa.eps0, pb.eps0], [nocc_a, nocc_b]


def test_p16_unrestricted_closed_shell_reduces_to_restricted():
    """Equal spins: V_alpha = V_beta = the restricted V of Eq. (19), and the
    excitations are the singlets plus triplets at Omega = Delta."""
    p = tiny(nbf=7, naux=11, nocc=3, seed=6)
    B_mo = O.mo_transform(p.B_ao, p.C0)
    V, Om = O.gw_unrestricted([B_mo, B_mo], [p.eps0, p.eps0], [3, 3], 0.02)
    M, sq = O.rpa_hermitian(B_mo, p.eps0, 3)
    Om_r, XpY = O.rpa_solve(M, sq)
    Vr = O.sigma_qs(O.residues(B_mo, XpY, 3), p.eps0, Om_r, 3, 0.02)
    scale = np.abs(Vr).max()
    np.testing.assert_allclose(V[0], Vr, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(V[1], Vr, rtol=0, atol=1e-12 * scale)
    both = np.sort(np.concatenate([Om_r, O.transition_energies(p.eps0, 3)]))
    np.testing.assert_allclose(Om, both, rtol=1e-12)


@pytest.mark.parametrize("nocc_a,nocc_b", [(3, 2), (2, 2), (1, 3)])
def test_p17_unrestricted_spin_sums(nocc_a, nocc_b):
    """Open shell with different orbitals per spin: the Hermitian form, the
    concatenated RI sums and Eq. (19) agree with the non-Hermitian spin-block
    problem and term-by-term sums over (i, a, sigma')."""
    B_s, e_s, n_s = _two_spins(6, 9, nocc_a, nocc_b, 12)
    V, Om = O.gw_unrestricted(B_s, e_s, n_s, 0.03)
    for spin in (0, 1):
        Vp, Omp = pins.gw_unrestricted_spin_sums(B_s, e_s, n_s, 0.03, spin)
        np.testing.assert_allclose(Om, Omp, rtol=1e-10)
        np.testing.assert_allclose(V[spin], Vp, rtol=0, atol=1e-10 * np.abs(Vp).max())


def test_p18_unrestricted_fock():
    """Open-shell Fock matrices: explicit four-index J[D_alpha + D_beta] and
    K[D_sigma] (P9's route), and equal spins reduce to the closed-shell Fock."""
    p = tiny(nbf=6, naux=10, nocc=3, seed=14)
    q2 = make_problem(6, 10, 2, 10, 0.9, 15, coupling=1.0)
    C_s, n_s = [p.C0, q2.C0], [3, 2]
    rng = np.random.default_rng(3)
    V_s = [(lambda a: a + a.T)(rng.standard_normal((6, 6))) for _ in range(2)]
    h = O.hf_core(p.B_ao, p.C0, p.eps0, 3)
    F = O.fock_unrestricted(h, p.B_ao, C_s, n_s, V_s)
    D = [O.density(C, no) for C, no in zip(C_s, n_s)]
    Jt = pins.jk_four_index(p.B_ao, 0.5 * (D[0] + D[1]))[0]
    for s_ in (0, 1):
        K = pins.jk_four_index(p.B_ao, D[s_])[1]
        ref = h + Jt - K + C_s[s_] @ V_s[s_] @ C_s[s_].T
        np.testing.assert_allclose(F[s_], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    Fr = O.fock(h, p.B_ao, p.C0, 3, V_s[0])
    Fe = O.fock_unrestricted(h, p.B_ao, [p.C0, p.C0], [3, 3], [V_s[0], V_s[0]])
    np.testing.assert_allclose(Fe[0], Fr, rtol=0, atol=1e-12 * np.abs(Fr).max())
    np.testing.assert_allclose(Fe[1], Fr, rtol=0, atol=1e-12 * np.abs(Fr).max())


def test_unrestricted_step_equal_spins_is_qsgw_step():
    p = tiny(nbf=7, naux=11, nocc=3, seed=6, coupling=0.1)
    h = O.hf_core(p.B_ao, p.C0, p.eps0, 3)
    r = O.qsgw_step(p.B_ao, h, p.C0, p.eps0, 3, 0.02)
    e_r, C_r = r["eps"], r["C"]
    e_u, C_u = O.unrestricted_step(p.B_ao, h, [p.C0, p.C0], [p.eps0, p.eps0], [3, 3], 0.02)
    for s_ in (0, 1):
        np.testing.assert_allclose(e_u[s_], e_r, rtol=0, atol=1e-12)
        np.testing.assert_allclose(C_u[s_], C_r, rtol=0, atol=1e-10)


def test_mutant_unrestricted_spin_factor_caught(monkeypatch):
    """The closed-shell factor 2 of the Casida coupling left in the open-shell
    build fails P17."""
    import oracle.qsgw_oracle as OM
    orig = OM.rpa_hermitian_unrestricted

    def doubled(B_mo_s, eps_s, nocc_s):
        M, sq, Bt = orig(B_mo_s, eps_s, nocc_s)
        d = sq * sq
        return 2.0 * M - np.diag(d * d), sq, Bt

    B_s, e_s, n_s = _two_spins(6, 9, 3, 2, 12)
    Vp, Omp = pins.gw_unrestricted_spin_sums(B_s, e_s, n_s, 0.03, 0)
    monkeypatch.setattr(OM, "rpa_hermitian_unrestricted", doubled)
    V, Om = O.gw_unrestricted(B_s, e_s, n_s, 0.03)
    assert np.abs(Om - Omp).max() > 1e-6 * Omp.max()


# ------------------------------------------------------------ generator ---
def test_generator_determinism_and_structure():
    a = make_problem(10, 30, 3, 15, 0.9, 42)
    b = make_problem(10, 30, 3, 15, 0.9, 42)
    np.testing.assert_array_equal(a.B_ao, b.B_ao)
    np.testing.assert_array_equal(a.eps0, b.eps0)
    np.testing.assert_array_equal(a.B_ao, a.B_ao.transpose(0, 2, 1))
    np.testing.assert_allclose(a.C0.T @ a.C0, np.eye(10), atol=1e-13)
    assert np.all(np.diff(a.eps0) > 0)
    assert a.eps0[2] < -0.3 + 1e-12 and a.eps0[3] > 0.05 - 1e-12
    c = make_problem(10, 30, 3, 15, 0.9, 43)
    assert not np.array_equal(a.B_ao, c.B_ao)


def test_generator_coupling_scale():
    # mean diagonal (mu mu|mu mu) = 0.5 * coupling Ha in expectation
    p = make_problem(60, 240, 8, 120, 0.99, 0, coupling=1.0)
    diag = np.einsum("pmm,pmm->m", p.B_ao, p.B_ao)
    assert 0.3 < diag.mean() < 0.7
