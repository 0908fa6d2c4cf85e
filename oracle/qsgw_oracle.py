"""Plain FP64 CPU oracle for one RI qsGW iteration.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or call this module.  The product
path (the HIP library and its binding) never routes through it, and this
module shares no code with that path.

Everything here is real (the paper considers real orbitals, section
"Theoretical background"), FP64, Hartree atomic units, closed shell.  The
code follows the paper's equations in the paper's order and notation:

  * LCAO and the AO->MO transform, Eqs. (3) and (16), with the RI
    factorisation (mu nu|lambda tau) ~ sum_P B^P_{mu nu} B^P_{lambda tau}
    (section "Self-consistent field", the paragraph on the RI approximation).
  * Casida equation, Eqs. (12)-(14), closed-shell singlet block, solved in its
    Hermitian form M = (A-B)^{1/2} (A+B) (A-B)^{1/2}.
  * Residues w^s_{mn}, Eq. (18).
  * GW self-energy Sigma_{mn}(omega), Eq. (17); qsGW potential, Eq. (19).
  * Hamiltonian Eq. (6) with Hartree Eq. (7), density Eq. (9), exchange
    Eq. (10); eigenproblem Eq. (4) with S = I.

Readings of passages that are silent or ambiguous (each one is listed with
its reason in the design notes of the repository):

  * Eqs. (13)-(14) are read with "+" signs (standard direct RPA):
    A = Delta + (ia|jb), B = (ia|bj) per spin pair.  With the printed "-"
    A+B is indefinite for a positive semidefinite Coulomb kernel.
  * Closed shell: the spin sums of Eqs. (12)-(18) give the singlet block
    A = Delta + 2K, B = 2K and w = sqrt(2) sum_ia (mn|ia)(X+Y)_ia; triplet
    excitations have zero residue.
  * Normalisation X^T X - Y^T Y = 1, so X+Y = (A-B)^{1/2} Z Omega^{-1/2}.
  * Eq. (19) takes the real part: V_mn = 1/2 Re[Sigma_mn(eps_m) + Sigma_mn(eps_n)]
    with eta kept finite.
  * The one-body part of Eq. (6), T + V_ext, is a synthetic matrix h built so
    that the starting (eps0, C0) is an exact Hartree-Fock fixed point.
  * No mixing by default; convergence when max_m |eps_m' - eps_m| < tol.
    Optional accelerators of the fixed point (the paper names none): linear
    mixing of the AO-basis correlation potential, or Pulay's direct inversion
    in the iterative subspace (DIIS) on the AO Fock matrix with the
    commutator error F D - D F (Pulay, Chem. Phys. Lett. 73, 393 (1980);
    J. Comput. Chem. 3, 556 (1982), with S = I).
  * Eq. (20), second-order exchange with p occupied: the printed integral
    (pi|an) is read as (pa|in).  The printed form matches the second-order
    self-energy of antisymmetrised spin-orbital integrals for virtual p only;
    for occupied p it breaks the m <-> n symmetry that self-energy has for
    real orbitals, while (pa|in) restores both.
  * Eq. (21) takes the real part, as Eq. (19): V_mn = 1/2 Re[Sigma_mn(eps_n)
    + Sigma_nm(eps_m)].

Also here, beyond the qsGW iteration: the MP2 self-energy, Eq. (20), the
qsMP2 potential, Eq. (21), the four-index AO->MO transform of Eq. (16)
without the RI factorisation, and the open-shell (spin-unrestricted) GW
potential: Eqs. (12)-(19) with the spin labels kept, each spin with its own
orbitals, energies and occupation.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


# ---------------------------------------------------------------- O1 ------
def mo_transform(B_ao: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Eq. (16) with RI: B^P_{mn} = sum_{mu nu} C_{mu m} B^P_{mu nu} C_{nu n}.

    B_ao is [P][mu][nu]; C is [mu][m] (column m = MO m, Eq. (3)).
    Returns B_mo as [P][m][n].
    """
    return np.matmul(np.matmul(C.T[None, :, :], B_ao), C[None, :, :])


def eri_mo(B_mo: np.ndarray) -> np.ndarray:
    """(mn|pq) = sum_P B^P_{mn} B^P_{pq}, the RI form of Eq. (15).  Small cases only."""
    n = B_mo.shape[1]
    flat = B_mo.reshape(B_mo.shape[0], n * n)
    return (flat.T @ flat).reshape(n, n, n, n)


# ---------------------------------------------------------------- O2 ------
def transition_energies(eps: np.ndarray, nocc: int) -> np.ndarray:
    """Delta_t = eps_a - eps_i for t = i * n_v + (a - n_occ)."""
    return (eps[None, nocc:] - eps[:nocc, None]).reshape(-1)


def casida_AB(B_mo: np.ndarray, eps: np.ndarray, nocc: int):
    """Eqs. (13)-(14), closed-shell singlet block, "+" sign reading.

    K_{ia,jb} = (ia|jb) = sum_P B^P_{ia} B^P_{jb}; (ia|bj) = (ia|jb) for
    real orbitals.  A = diag(Delta) + 2K, B = 2K (the factor 2 is the sum
    over the spin sigma' of the partner pair).
    """
    naux = B_mo.shape[0]
    Bia = B_mo[:, :nocc, nocc:].reshape(naux, -1)
    K = Bia.T @ Bia
    delta = transition_energies(eps, nocc)
    A = np.diag(delta) + 2.0 * K
    B = 2.0 * K
    return A, B


def rpa_hermitian(B_mo: np.ndarray, eps: np.ndarray, nocc: int):
    """M = (A-B)^{1/2} (A+B) (A-B)^{1/2} with A-B = diag(Delta) for real orbitals.

    Returns (M, sqrt_delta).
    """
    A, B = casida_AB(B_mo, eps, nocc)
    delta = transition_energies(eps, nocc)
    sqrt_delta = np.sqrt(delta)
    M = sqrt_delta[:, None] * (A + B) * sqrt_delta[None, :]
    return M, sqrt_delta


# ---------------------------------------------------------------- O3 ------
def rpa_solve(M: np.ndarray, sqrt_delta: np.ndarray):
    """Solve M Z = Z Omega^2; (X+Y)^s = (A-B)^{1/2} Z^s / sqrt(Omega_s).

    Returns (Omega ascending, XpY[t][s]).
    """
    lam, Z = scipy.linalg.eigh(M)
    if lam[0] <= 0.0:
        raise ValueError("RPA instability: non-positive Omega^2")
    Omega = np.sqrt(lam)
    XpY = sqrt_delta[:, None] * Z / np.sqrt(Omega)[None, :]
    return Omega, XpY


# ---------------------------------------------------------------- O4 ------
def residues(B_mo: np.ndarray, XpY: np.ndarray, nocc: int) -> np.ndarray:
    """Eq. (18): w^s_{mn} = sum_{ia sigma'} (mn|ia sigma') (X+Y)^s_{ia sigma'}.

    With RI and the singlet spin sum, w^s_{mn} = sqrt(2) sum_P B^P_{mn} rho_{P s},
    rho_{P s} = sum_{ia} B^P_{ia} (X+Y)^s_{ia}.  Returns w as [m][n][s].
    """
    naux, n, _ = B_mo.shape
    Bia = B_mo[:, :nocc, nocc:].reshape(naux, -1)
    rho = Bia @ XpY
    w = np.sqrt(2.0) * (B_mo.reshape(naux, n * n).T @ rho)
    return w.reshape(n, n, -1)


# ---------------------------------------------------------------- O5 ------
def _pole_denominators(omega: float, eps: np.ndarray, Omega: np.ndarray,
                       nocc: int, eta: float) -> np.ndarray:
    """Denominators of Eq. (17) as a [k][s] complex array at one frequency.

    occupied k = i:  omega - eps_i + Omega_s - i eta
    virtual  k = a:  omega - eps_a - Omega_s + i eta
    """
    d = np.empty((eps.size, Omega.size), dtype=np.complex128)
    d[:nocc] = (omega - eps[:nocc, None] + Omega[None, :]) - 1j * eta
    d[nocc:] = (omega - eps[nocc:, None] - Omega[None, :]) + 1j * eta
    return d


def sigma_element(w: np.ndarray, eps: np.ndarray, Omega: np.ndarray, nocc: int,
                  eta: float, m: int, n: int, omegas) -> np.ndarray:
    """Eq. (17): <m|Sigma_c^GW(omega)|n> for each omega in ``omegas`` (complex)."""
    num = w[m] * w[n]  # [k][s]
    out = np.empty(len(omegas), dtype=np.complex128)
    for j, om in enumerate(omegas):
        out[j] = np.sum(num / _pole_denominators(om, eps, Omega, nocc, eta))
    return out


# ---------------------------------------------------------------- O6 ------
def sigma_qs(w: np.ndarray, eps: np.ndarray, Omega: np.ndarray, nocc: int,
             eta: float) -> np.ndarray:
    """Eq. (19), real part: V_mn = 1/2 Re[Sigma_mn(eps_m) + Sigma_mn(eps_n)].

    Sigma is complex symmetric in (m, n) for real orbitals, so the second
    term is the transpose of the first: with G_mn = Re Sigma_mn(eps_m),
    V = (G + G^T) / 2.
    """
    n = eps.size
    G = np.empty((n, n))
    for m in range(n):
        # w is real, so Re sum_ks w_mks w_nks / d_ks = sum_ks w_mks w_nks Re(1/d_ks)
        g = (1.0 / _pole_denominators(eps[m], eps, Omega, nocc, eta)).real
        G[m] = np.tensordot(w, w[m] * g, axes=([1, 2], [0, 1]))
    return 0.5 * (G + G.T)


# ---------------------------------------------------------------- O7 ------
def density(C: np.ndarray, nocc: int) -> np.ndarray:
    """Eq. (9) per spin, closed shell: D = sum_{i occ} C_{mu i} C_{nu i}."""
    Cocc = C[:, :nocc]
    return Cocc @ Cocc.T


def hartree(B_ao: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Eq. (7) with RI: J = sum_P B^P (B^P . sum_sigma D^sigma), sum_sigma D^sigma = 2D."""
    c = np.einsum("plt,lt->p", B_ao, 2.0 * D)
    return np.einsum("p,pmn->mn", c, B_ao)


def exchange(B_ao: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Eq. (10) with RI: K_{mu nu} = sum_{lt} D_{lt} (mu lambda|tau nu) = sum_P (B^P D B^P)_{mu nu}."""
    return np.einsum("pml,lt,ptn->mn", B_ao, D, B_ao, optimize=True)


def hf_core(B_ao: np.ndarray, C0: np.ndarray, eps0: np.ndarray, nocc: int) -> np.ndarray:
    """One-body matrix h that makes (eps0, C0) a Hartree-Fock fixed point:
    h = C0 diag(eps0) C0^T - (J - K)[D0]."""
    D0 = density(C0, nocc)
    return (C0 * eps0[None, :]) @ C0.T - hartree(B_ao, D0) + exchange(B_ao, D0)


def fock(h: np.ndarray, B_ao: np.ndarray, C: np.ndarray, nocc: int,
         V: np.ndarray, fock_mode: str = "full") -> np.ndarray:
    """Eq. (6): H = h + J - K + Sigma_c, with Sigma_c in the AO basis = C V C^T.

    fock_mode "frozen" keeps the mean field of a reference density fixed: h is
    then the whole frozen mean-field matrix F0 = T + V_ext + J[D0] - K[D0] and
    H = F0 + C V C^T (J and K are not rebuilt)."""
    if fock_mode == "frozen":
        return h + C @ V @ C.T
    if fock_mode != "full":
        raise ValueError(f"unknown fock_mode {fock_mode!r}")
    D = density(C, nocc)
    return h + hartree(B_ao, D) - exchange(B_ao, D) + C @ V @ C.T


def diagonalize(F: np.ndarray):
    """Eq. (4) with S = I.  Returns (eps ascending, C) with each column's
    largest-magnitude entry made positive (a fixed sign convention)."""
    e, C = scipy.linalg.eigh(F)
    idx = np.argmax(np.abs(C), axis=0)
    sgn = np.sign(C[idx, np.arange(C.shape[1])])
    sgn[sgn == 0] = 1.0
    return e, C * sgn[None, :]


# ---------------------------------------------------------------- O1-O8 ---
def qsgw_step(B_ao, h, C, eps, nocc, eta, fock_mode="full"):
    """One qsGW iteration from (eps, C).  Returns a dict of every intermediate.
    fock_mode as in ``fock``."""
    B_mo = mo_transform(B_ao, C)
    M, sqrt_delta = rpa_hermitian(B_mo, eps, nocc)
    Omega, XpY = rpa_solve(M, sqrt_delta)
    w = residues(B_mo, XpY, nocc)
    V = sigma_qs(w, eps, Omega, nocc, eta)
    F = fock(h, B_ao, C, nocc, V, fock_mode)
    eps_new, C_new = diagonalize(F)
    return dict(B_mo=B_mo, M=M, sqrt_delta=sqrt_delta, Omega=Omega, XpY=XpY,
                w=w, V=V, F=F, eps=eps_new, C=C_new)


def diis_error(F: np.ndarray, D: np.ndarray) -> np.ndarray:
    """DIIS error of a Fock matrix built from density D: the commutator
    F D - D F (S = I), zero exactly when F and D share eigenvectors."""
    return F @ D - D @ F


def diis_coefficients(errors) -> np.ndarray:
    """Pulay's DIIS weights: the c minimising || sum_i c_i e_i ||_F subject
    to sum_i c_i = 1, from the bordered system
        [ B   -1 ] [c]   [ 0 ]
        [ -1^T 0 ] [l] = [ -1 ],   B_ij = <e_i, e_j>_F."""
    n = len(errors)
    Bm = np.zeros((n + 1, n + 1))
    for i in range(n):
        for j in range(n):
            Bm[i, j] = float(np.sum(errors[i] * errors[j]))
    Bm[:n, n] = -1.0
    Bm[n, :n] = -1.0
    rhs = np.zeros(n + 1)
    rhs[n] = -1.0
    return np.linalg.solve(Bm, rhs)[:n]


def qsgw_iterate(B_ao, h, C0, eps0, nocc, eta, tol, max_iter, mix=1.0,
                 keep=("eps", "Omega"), fock_mode="full", diis=0):
    """Repeat the qsGW step until max|eps' - eps| < tol or max_iter.

    With mix < 1 the AO-basis correlation potential is mixed linearly with the
    previous one: Sigma_ao <- mix * Sigma_ao + (1 - mix) * Sigma_ao_prev.
    With diis = m >= 2 the Fock matrix of Eq. (6) built from (eps, C) is
    stored with its error e = F D - D F (D of Eq. (9) from the same C) among
    the last m such pairs, and the matrix diagonalised is sum_i c_i F_i with
    the weights of ``diis_coefficients`` (the first iteration is the plain
    step).  fock_mode "frozen": h is the frozen mean-field matrix F0 (see
    ``fock``).  Returns (eps, C, history) where history[j] holds the ``keep``
    entries and max|d eps| of iteration j + 1.
    """
    C, eps = C0.copy(), eps0.copy()
    hist = []
    Vao_prev = None
    F_hist, E_hist = [], []
    for _ in range(max_iter):
        B_mo = mo_transform(B_ao, C)
        M, sqrt_delta = rpa_hermitian(B_mo, eps, nocc)
        Omega, XpY = rpa_solve(M, sqrt_delta)
        w = residues(B_mo, XpY, nocc)
        V = sigma_qs(w, eps, Omega, nocc, eta)
        Vao = C @ V @ C.T
        if Vao_prev is not None and mix != 1.0:
            Vao = mix * Vao + (1.0 - mix) * Vao_prev
        Vao_prev = Vao
        D = density(C, nocc)
        if fock_mode == "frozen":
            F = h + Vao
        else:
            F = h + hartree(B_ao, D) - exchange(B_ao, D) + Vao
        if diis >= 2:
            F_hist.append(F)
            E_hist.append(diis_error(F, D))
            F_hist, E_hist = F_hist[-diis:], E_hist[-diis:]
            if len(F_hist) > 1:
                c = diis_coefficients(E_hist)
                F = sum(ci * Fi for ci, Fi in zip(c, F_hist))
        eps_new, C_new = diagonalize(F)
        d = float(np.max(np.abs(eps_new - eps)))
        rec = {"max_deps": d}
        if diis >= 2:
            rec["diis_err"] = float(np.linalg.norm(E_hist[-1]))
        loc = dict(B_mo=B_mo, M=M, Omega=Omega, XpY=XpY, w=w, V=V, Vao=Vao,
                   F=F, eps=eps_new, C=C_new)
        for k in keep:
            if k not in rec:
                rec[k] = loc[k]
        hist.append(rec)
        C, eps = C_new, eps_new
        if d < tol:
            break
    return eps, C, hist


# ------------------------------------------------- per-state features -----
def exchange_diagonal_mo(B_mo: np.ndarray, nocc: int) -> np.ndarray:
    """Diagonal of the exchange operator of Eq. (10) in the MO basis, closed
    shell: Sigma_x,mm = -(C^T K[D] C)_mm = -sum_{i occ} (mi|im)
    = -sum_i sum_P (B^P_{mi})^2."""
    return -np.einsum("pmi,pmi->m", B_mo[:, :, :nocc], B_mo[:, :, :nocc])


def sigma_diag_derivative(w, eps, Omega, nocc, eta, m, omega) -> complex:
    """d Sigma_mm / d omega of Eq. (17): omega enters every denominator d_ks
    with coefficient 1, so the derivative is -sum_{k s} w_mks^2 / d_ks^2."""
    d = _pole_denominators(omega, eps, Omega, nocc, eta)
    return complex(-np.sum(w[m] ** 2 / d ** 2))


# ------------------------------------------------------------ qsMP2 -------
def _mp2_integrals(B_mo: np.ndarray, nocc: int, m_rows=None, n_rows=None):
    """RI integrals of Eq. (20) over (p, i, a), p any state, i occupied, a virtual.

    L[m, p, i, a] = (mp|ia)              for m in m_rows
    R[n, p, i, a] = (pn|ai)              (direct, for n in n_rows)
    X[n, p, i, a] = (pi|an), p virtual;  (pa|in), p occupied  (exchange)
    every (kl|rs) = sum_P B^P_{kl} B^P_{rs}.
    """
    nb = B_mo.shape[1]
    occ, vir = slice(0, nocc), slice(nocc, nb)
    m_rows = np.arange(nb) if m_rows is None else np.asarray(m_rows)
    n_rows = np.arange(nb) if n_rows is None else np.asarray(n_rows)
    Bia = B_mo[:, occ, vir]                                   # [P][i][a]
    L = np.einsum("Pmp,Pia->mpia", B_mo[:, m_rows, :], Bia, optimize=True)
    R = np.einsum("Ppn,Pai->npia", B_mo[:, :, n_rows], B_mo[:, vir, occ], optimize=True)
    X = np.empty_like(R)
    # p virtual: (pi|an) = sum_P B^P_{pi} B^P_{an}
    X[:, nocc:] = np.einsum("Ppi,Pan->npia", B_mo[:, vir, occ], B_mo[:, vir][:, :, n_rows], optimize=True)
    # p occupied: (pa|in) = sum_P B^P_{pa} B^P_{in}
    X[:, :nocc] = np.einsum("Ppa,Pin->npia", B_mo[:, occ, vir], B_mo[:, occ][:, :, n_rows], optimize=True)
    return L, R, X


def _mp2_denominators(omega, eps: np.ndarray, nocc: int, eta: float) -> np.ndarray:
    """Bracket of Eq. (20) for one frequency, as an array over (p, i, a):
    f_p / (omega + eps_a - eps_i - eps_p - i eta) for occupied p,
    (1 - f_p) / (omega + eps_i - eps_a - eps_p + i eta) for virtual p."""
    ep = eps[:, None, None]
    ei = eps[None, :nocc, None]
    ea = eps[None, None, nocc:]
    occ_p = (np.arange(eps.size) < nocc)[:, None, None]
    return np.where(occ_p, 1.0 / (omega + ea - ei - ep - 1j * eta),
                    1.0 / (omega + ei - ea - ep + 1j * eta))


def sigma_mp2(B_mo: np.ndarray, eps: np.ndarray, nocc: int, eta: float, omegas,
              terms: str = "both") -> np.ndarray:
    """MP2 correlation self-energy, Eq. (20), closed shell, real orbitals.

    Returns the complex matrix S[m, n] = Sigma_mn(omegas[n]): column n is taken
    at its own frequency (a scalar omegas gives Sigma(omega) itself).  The sum
    over sigma' of the direct term gives its factor 2; the exchange term has
    no spin sum.  terms = "direct" or "sox" keeps one of the two sums.
    """
    nb = eps.size
    om = np.broadcast_to(np.asarray(omegas, dtype=np.float64), (nb,))
    L, R, X = _mp2_integrals(B_mo, nocc)
    fd = {"both": 1.0, "direct": 1.0, "sox": 0.0}[terms]
    fx = {"both": 1.0, "direct": 0.0, "sox": 1.0}[terms]
    S = np.empty((nb, nb), dtype=np.complex128)
    for n in range(nb):
        g = _mp2_denominators(om[n], eps, nocc, eta)
        S[:, n] = np.einsum("mpia,pia->m", L, (2.0 * fd * R[n] - fx * X[n]) * g)
    return S


def sigma_mp2_entry(B_mo: np.ndarray, eps: np.ndarray, nocc: int, eta: float, omega: float,
                    m: int, n: int) -> complex:
    """One element Sigma_mn(omega) of Eq. (20), from B_mo without the four-index
    tensor (for sampled checks at sizes where the full matrix is too costly)."""
    L, R, X = _mp2_integrals(B_mo, nocc, [m], [n])
    g = _mp2_denominators(omega, eps, nocc, eta)
    return complex(np.sum(L[0] * (2.0 * R[0] - X[0]) * g))


def qsmp2_potential(B_mo: np.ndarray, eps: np.ndarray, nocc: int, eta: float) -> np.ndarray:
    """Eq. (21): V_mn = 1/2 Re[Sigma_mn(eps_n) + Sigma_nm(eps_m)]."""
    S = sigma_mp2(B_mo, eps, nocc, eta, eps)   # S[m, n] = Sigma_mn(eps_n)
    return 0.5 * np.real(S + S.T)


def qsmp2_entry(B_mo: np.ndarray, eps: np.ndarray, nocc: int, eta: float, m: int, n: int) -> float:
    """One element of Eq. (21) from two elements of Eq. (20)."""
    a = sigma_mp2_entry(B_mo, eps, nocc, eta, eps[n], m, n)
    b = sigma_mp2_entry(B_mo, eps, nocc, eta, eps[m], n, m)
    return 0.5 * (a + b).real


# ------------------------------------------------------ four-index AO->MO --
def ao2mo_4center(eri_ao: np.ndarray, C: np.ndarray, m_rows=None) -> np.ndarray:
    """Eq. (16) on explicit four-index integrals:
    (mn|kl) = sum_{mu nu lambda tau} C_{mu m} C_{nu n} C_{lambda k} C_{tau l} (mu nu|lambda tau).

    eri_ao is [mu][nu][lambda][tau]; C is [mu][m].  m_rows selects the first MO
    index (default: all).  Returns [len(m_rows)][nbf][nbf][nbf].
    """
    Cm = C if m_rows is None else C[:, np.asarray(m_rows)]
    return np.einsum("abcd,am,bn,ck,dl->mnkl", eri_ao, Cm, C, C, C, optimize=True)


# ------------------------------------------------------ open shell (UHF) --
def rpa_hermitian_unrestricted(B_mo_s, eps_s, nocc_s):
    """Eqs. (12)-(14) with explicit spins, direct RPA ("+" reading): transitions
    t = (i, a, sigma) of both spins, spin alpha first, each in the order of
    ``transition_energies``;  A = diag(Delta) + K, B = K with
    K_{t u} = (i a sigma | j b sigma') = sum_P B^{sigma P}_{ia} B^{sigma' P}_{jb}.
    Returns (M, sqrt_delta, Bt) with M = (A-B)^{1/2} (A+B) (A-B)^{1/2} and
    Bt[P][t] = B^{sigma P}_{ia} (unscaled, [naux][ntr_alpha + ntr_beta]).
    """
    naux = B_mo_s[0].shape[0]
    Bt = np.concatenate([B[:, :no, no:].reshape(naux, -1) for B, no in zip(B_mo_s, nocc_s)],
                        axis=1)
    delta = np.concatenate([transition_energies(e, no) for e, no in zip(eps_s, nocc_s)])
    K = Bt.T @ Bt
    A = np.diag(delta) + K
    B = K
    sqrt_delta = np.sqrt(delta)
    M = sqrt_delta[:, None] * (A + B) * sqrt_delta[None, :]
    return M, sqrt_delta, Bt


def residues_unrestricted(B_mo: np.ndarray, Bt: np.ndarray, XpY: np.ndarray) -> np.ndarray:
    """Eq. (18) for one spin sigma: w^s_{mn sigma} = sum_{t sigma'} (mn sigma|t) (X+Y)^s_t
    = sum_P B^{sigma P}_{mn} rho_{P s}, rho = Bt (X+Y) over both spins' transitions."""
    naux, n, _ = B_mo.shape
    rho = Bt @ XpY
    return (B_mo.reshape(naux, n * n).T @ rho).reshape(n, n, -1)


def gw_unrestricted(B_mo_s, eps_s, nocc_s, eta):
    """Open-shell qsGW potential of each spin, Eqs. (12)-(19):
    returns ([V_alpha, V_beta], Omega) with V_sigma from Eq. (19) on the residues
    and energies of that spin (occupied k < nocc_sigma)."""
    M, sq, Bt = rpa_hermitian_unrestricted(B_mo_s, eps_s, nocc_s)
    Om, XpY = rpa_solve(M, sq)
    V = [sigma_qs(residues_unrestricted(B, Bt, XpY), e, Om, no, eta)
         for B, e, no in zip(B_mo_s, eps_s, nocc_s)]
    return V, Om


def fock_unrestricted(h, B_ao, C_s, nocc_s, V_s):
    """Eq. (6) per spin with explicit spins: F^sigma = h + J[D^alpha + D^beta] - K[D^sigma]
    + C^sigma V^sigma C^sigma^T, D^sigma from Eq. (9) with that spin's occupied
    orbitals, J[D] = sum_P B^P (B^P . D) (Eq. 7), K[D] = sum_P B^P D B^P (Eq. 10)."""
    D = [density(C, no) for C, no in zip(C_s, nocc_s)]
    Dt = D[0] + D[1]
    J = np.einsum("p,pmn->mn", np.einsum("plt,lt->p", B_ao, Dt), B_ao)
    return [h + J - exchange(B_ao, Ds) + C @ V @ C.T for Ds, C, V in zip(D, C_s, V_s)]


def unrestricted_step(B_ao, h, C_s, eps_s, nocc_s, eta):
    """One open-shell qsGW step: MO transform per spin, the open-shell GW
    potential, the Fock matrix of each spin and its eigenproblem (Eq. 4, S = I).
    Returns ([eps'_alpha, eps'_beta], [C'_alpha, C'_beta])."""
    B_mo_s = [mo_transform(B_ao, C) for C in C_s]
    V_s, _ = gw_unrestricted(B_mo_s, eps_s, nocc_s, eta)
    out = [diagonalize(F) for F in fock_unrestricted(h, B_ao, C_s, nocc_s, V_s)]
    return [e for e, _ in out], [C for _, C in out]


def qsmp2_step(B_ao, h, C, eps, nocc, eta):
    """One qsMP2 iteration: MO transform (Eq. 16), the qsMP2 potential (Eqs. 20-21)
    in place of the qsGW one, Fock matrix (Eq. 6) and its eigenproblem.
    Returns (eps', C')."""
    B_mo = mo_transform(B_ao, C)
    V = qsmp2_potential(B_mo, eps, nocc, eta)
    return diagonalize(fock(h, B_ao, C, nocc, V))
