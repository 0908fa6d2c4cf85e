"""Independent routes to the quantities the oracle computes.

Each function here re-derives a result of the qsGW iteration by a different
route than the oracle takes (a closed form, the full spin-orbital Casida
problem, the non-Hermitian Casida matrix, the Dyson equation for the screened
interaction on the imaginary axis, direct frequency integration of iGW, the
MP2 self-energy, explicit four-index integrals).  None of them imports the
oracle, so agreement pins the oracle to the paper's equations rather than to
itself.
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------ P1 ---------
def one_transition_closed_form(eps0, eps1, b, B00, B11, eta, omegas):
    """N_b = 2, n_occ = 1, N_aux = 1: the only transition t = (0, 1).

    v = (01|01) = b^2, Delta = eps1 - eps0; singlet A = Delta + 2v, B = 2v,
    Omega^2 = (A - B)(A + B) = Delta (Delta + 4v); X + Y = sqrt(Delta / Omega).
    w_mk = sqrt(2) B_mk b sqrt(Delta / Omega).  Returns Omega, the 2x2 w, and
    Sigma_00(omega), Sigma_11(omega) of Eq. (17).
    """
    v = b * b
    delta = eps1 - eps0
    Omega = np.sqrt(delta * (delta + 4.0 * v))
    xpy = np.sqrt(delta / Omega)
    Bm = np.array([[B00, b], [b, B11]])
    w = np.sqrt(2.0) * Bm * b * xpy
    omegas = np.asarray(omegas, dtype=np.complex128)
    sig = np.zeros((2, omegas.size), dtype=np.complex128)
    for m in range(2):
        sig[m] = (w[m, 0] ** 2 / (omegas - eps0 + Omega - 1j * eta)
                  + w[m, 1] ** 2 / (omegas - eps1 - Omega + 1j * eta))
    return Omega, w, sig


def one_transition_sigma_derivative(eps0, eps1, b, B00, B11, eta, omegas):
    """d Sigma_mm / d omega of the one-transition closed form above, term by
    term: d/dw [c / (w - e + Om - i eta)] = -c / (w - e + Om - i eta)^2 and the
    same for the virtual pole.  Returns [2][len(omegas)] complex."""
    Omega, w, _ = one_transition_closed_form(eps0, eps1, b, B00, B11, eta, [0.0])
    omegas = np.asarray(omegas, dtype=np.complex128)
    out = np.zeros((2, omegas.size), dtype=np.complex128)
    for m in range(2):
        out[m] = (-w[m, 0] ** 2 / (omegas - eps0 + Omega - 1j * eta) ** 2
                  - w[m, 1] ** 2 / (omegas - eps1 - Omega + 1j * eta) ** 2)
    return out


# ------------------------------------------------------------ helpers ----
def mo_eri(B_mo):
    n = B_mo.shape[1]
    flat = B_mo.reshape(B_mo.shape[0], -1)
    return np.einsum("pi,pj->ij", flat, flat).reshape(n, n, n, n)


def _pairs(nbf, nocc):
    return [(i, a) for i in range(nocc) for a in range(nocc, nbf)]


# ------------------------------------------------------------ P2 ---------
def casida_nonhermitian(B_mo, eps, nocc):
    """Diagonalise the full 2n x 2n matrix [[A, B], [-B, -A]] of Eq. (12).

    A and B are the singlet blocks built element by element from four-index
    MO integrals.  Returns positive eigenvalues Omega (ascending) and X+Y
    normalised with X^T X - Y^T Y = 1, columns in the order of Omega.
    """
    eri = mo_eri(B_mo)
    pr = _pairs(eps.size, nocc)
    n = len(pr)
    A = np.zeros((n, n))
    B = np.zeros((n, n))
    for t, (i, a) in enumerate(pr):
        for u, (j, b) in enumerate(pr):
            A[t, u] = (eps[a] - eps[i]) * (t == u) + 2.0 * eri[i, a, j, b]
            B[t, u] = 2.0 * eri[i, a, b, j]
    big = np.block([[A, B], [-B, -A]])
    lam, vec = np.linalg.eig(big)
    lam = lam.real
    vec = vec.real
    pos = np.where(lam > 0)[0]
    pos = pos[np.argsort(lam[pos])]
    Om = lam[pos]
    X = vec[:n, pos]
    Y = vec[n:, pos]
    norm = np.einsum("ts,ts->s", X, X) - np.einsum("ts,ts->s", Y, Y)
    XpY = (X + Y) / np.sqrt(norm)[None, :]
    return Om, XpY


# ------------------------------------------------------------ P3 ---------
def spin_orbital_gw(B_mo, eps, nocc, eta, omegas, m, n):
    """Eqs. (12)-(18) literally with spin labels sigma, sigma'.

    Transitions are (i, a, sigma) with both spins; (ia sigma|jb sigma') is the
    spatial integral for every spin pair.  Solves the 2n_tr Casida problem in
    its Hermitian form (A - B is diagonal), builds w^s_{mk sigma} by Eq. (18)
    with the explicit sum over sigma', and evaluates Eq. (17) for spin up.
    Returns (all Omega ascending, Sigma_mn(omega) for spin up).
    """
    eri = mo_eri(B_mo)
    pr = [(i, a, s) for s in (0, 1) for (i, a) in _pairs(eps.size, nocc)]
    n2 = len(pr)
    A = np.zeros((n2, n2))
    B = np.zeros((n2, n2))
    d = np.zeros(n2)
    for t, (i, a, s) in enumerate(pr):
        d[t] = eps[a] - eps[i]
        for u, (j, b, s2) in enumerate(pr):
            A[t, u] = d[t] * (t == u) + eri[i, a, j, b]
            B[t, u] = eri[i, a, b, j]
    sq = np.sqrt(d)
    Mh = sq[:, None] * (A + B) * sq[None, :]
    lam, Z = np.linalg.eigh(Mh)
    Om = np.sqrt(lam)
    XpY = sq[:, None] * Z / np.sqrt(Om)[None, :]
    nb = eps.size
    # w^s_{pq sigma} = sum_{ia sigma'} (pq|ia) (X+Y)^s_{ia sigma'}
    eri_pq_t = np.array([[[eri[p, q, i, a] for (i, a, s) in pr] for q in range(nb)]
                         for p in range(nb)])
    w = np.einsum("pqt,ts->pqs", eri_pq_t, XpY)
    sig = np.zeros(len(omegas), dtype=np.complex128)
    for j, om in enumerate(omegas):
        tot = 0.0 + 0.0j
        for k in range(nb):
            for s in range(n2):
                if k < nocc:
                    den = om - eps[k] + Om[s] - 1j * eta
                else:
                    den = om - eps[k] - Om[s] + 1j * eta
                tot += w[m, k, s] * w[n, k, s] / den
        sig[j] = tot
    return Om, sig


# ------------------------------------------------------------ P4 ---------
def screened_dyson(B_mo, eps, nocc, nu):
    """W_c = v chi v on the imaginary axis from the Dyson equation in the RI basis.

    Pi_PQ(i nu) = -4 sum_t B_Pt B_Qt Delta_t / (nu^2 + Delta_t^2) (two spins,
    two time orderings); W_c[mk, nl] = sum_PQ B^P_mk [(1 - Pi)^-1 Pi]_PQ B^Q_nl.
    Returns W_c as [m][k][n][l].
    """
    naux, nb, _ = B_mo.shape
    Bia = B_mo[:, :nocc, nocc:].reshape(naux, -1)
    delta = (eps[None, nocc:] - eps[:nocc, None]).reshape(-1)
    chi0 = -4.0 * delta / (nu * nu + delta * delta)
    Pi = (Bia * chi0[None, :]) @ Bia.T
    core = np.linalg.solve(np.eye(naux) - Pi, Pi)
    flat = B_mo.reshape(naux, nb * nb)
    return (flat.T @ core @ flat).reshape(nb, nb, nb, nb)


def screened_spectral(w, Omega, nu):
    """-sum_s w_mks w_nls 2 Omega_s / (nu^2 + Omega_s^2), as [m][k][n][l]."""
    f = -2.0 * Omega / (nu * nu + Omega * Omega)
    return np.einsum("mks,nls,s->mknl", w, w, f)


# ------------------------------------------------------------ P5 ---------
def sigma_frequency_integral(B_mo, eps, nocc, z, m, n, npts=2000, nu0=2.0):
    """Sigma_mn(z) = -(1/2pi) int dnu sum_k W_c[mk, nk](i nu) / (z + i nu - eps_k).

    W_c comes from the Dyson route (screened_dyson), never from the Casida
    eigenvectors.  nu = nu0 tan(theta) maps the real line onto (-pi/2, pi/2),
    integrated with Gauss-Legendre.  Valid for Re z between the highest
    occupied and the lowest empty level.
    """
    x, wt = np.polynomial.legendre.leggauss(npts)
    theta = 0.5 * np.pi * x
    wtheta = 0.5 * np.pi * wt
    nus = nu0 * np.tan(theta)
    jac = nu0 / np.cos(theta) ** 2
    total = 0.0 + 0.0j
    for nu, wq, jq in zip(nus, wtheta, jac):
        W = screened_dyson(B_mo, eps, nocc, nu)
        wk = np.array([W[m, k, n, k] for k in range(eps.size)])
        total += wq * jq * np.sum(wk / (z + 1j * nu - eps))
    return -total / (2.0 * np.pi)


# ------------------------------------------------------------ P6 ---------
def sigma_mp2_direct(B_mo, eps, nocc, eta, omega, m, n):
    """First (direct, second-order Coulomb) sum of the MP2 self-energy, Eq. (20).

    sum_{i a p sigma'} (mp|ia)(pn|ai) [f_p / (omega + eps_a - eps_i - eps_p - i eta)
                                        + (1 - f_p) / (omega + eps_i - eps_a - eps_p + i eta)]
    with the spin sum over sigma' giving a factor 2.
    """
    eri = mo_eri(B_mo)
    nb = eps.size
    tot = 0.0 + 0.0j
    for i in range(nocc):
        for a in range(nocc, nb):
            for p in range(nb):
                num = 2.0 * eri[m, p, i, a] * eri[p, n, a, i]
                if p < nocc:
                    tot += num / (omega + eps[a] - eps[i] - eps[p] - 1j * eta)
                else:
                    tot += num / (omega + eps[i] - eps[a] - eps[p] + 1j * eta)
    return tot


# ------------------------------------------------------------ P9 ---------
def jk_four_index(B_ao, D):
    """Eqs. (7) and (10) with explicit four-index (mu nu|lambda tau) = sum_P B B."""
    eri = mo_eri(B_ao)
    J = np.einsum("mnlt,lt->mn", eri, 2.0 * D)
    K = np.einsum("lt,mltn->mn", D, eri)
    return J, K


# ------------------------------------------------------------ P12 --------
def sigma2_spin_orbital(B_mo, eps, nocc, eta, omega):
    """Second-order (MP2) self-energy from antisymmetrised spin-orbital integrals.

    Spin orbital q = 2 k + spin has energy eps_k; <pq||rs> = <pq|rs> - <pq|sr>
    with <pq|rs> = (pr|qs) delta(spin p, spin r) delta(spin q, spin s).  With
    i, j occupied and a, b virtual spin orbitals:
      Sigma_pq(omega) = 1/2 sum_{ija} <pa||ij><ij||qa> / (omega + e_a - e_i - e_j - i eta)
                      + 1/2 sum_{iab} <pi||ab><ab||qi> / (omega + e_i - e_a - e_b + i eta).
    Returns the spatial matrix (spin-up block) at one frequency.
    """
    nb = eps.size
    eri = mo_eri(B_mo)                          # chemist (kl|rs)
    ns = 2 * nb
    orb = np.arange(ns) // 2
    spin = np.arange(ns) % 2
    # <pq|rs> = (pr|qs) with spin deltas
    chem = eri[np.ix_(orb, orb, orb, orb)]      # (pr|qs) indexed [p][r][q][s]
    same_pr = spin[:, None] == spin[None, :]
    phys = np.einsum("prqs->pqrs", chem) * same_pr[:, None, :, None] * same_pr[None, :, None, :]
    anti = phys - np.swapaxes(phys, 2, 3)
    e = eps[orb]
    O_ = np.where(orb < nocc)[0]
    V_ = np.where(orb >= nocc)[0]
    d2h = omega + e[V_][None, None, :] - e[O_][:, None, None] - e[O_][None, :, None] - 1j * eta
    d2p = omega + e[O_][:, None, None] - e[V_][None, :, None] - e[V_][None, None, :] + 1j * eta
    up = np.arange(0, ns, 2)
    t1 = 0.5 * np.einsum("pAij,ijqA,ijA->pq", anti[np.ix_(up, V_, O_, O_)],
                         anti[np.ix_(O_, O_, up, V_)], 1.0 / d2h)
    t2 = 0.5 * np.einsum("piab,abqi,iab->pq", anti[np.ix_(up, O_, V_, V_)],
                         anti[np.ix_(V_, V_, up, O_)], 1.0 / d2p)
    return t1 + t2


# ------------------------------------------------------------ P13 --------
def mp2_two_level_closed_form(B, eps0, eps1, eta, omega):
    """N_b = 2, n_occ = 1, N_aux = 1 with B = [[B00, b], [b, B11]]: every
    integral is (mk|rs) = B_mk B_rs and the direct and exchange terms of the
    second-order self-energy combine to
      Sigma_mn = b^2 [B_m0 B_n0 / (omega + eps1 - 2 eps0 - i eta)
                      + B_m1 B_n1 / (omega + eps0 - 2 eps1 + i eta)].
    """
    b = B[0, 1]
    return b * b * (np.outer(B[:, 0], B[:, 0]) / (omega + eps1 - 2 * eps0 - 1j * eta)
                    + np.outer(B[:, 1], B[:, 1]) / (omega + eps0 - 2 * eps1 + 1j * eta))


# ------------------------------------------------------------ P15 --------
def ao2mo_brute_force(eri_ao, C):
    """Eq. (16) as the literal eight-fold sum (tiny N only)."""
    n = C.shape[0]
    out = np.zeros((n, n, n, n))
    for m in range(n):
        for q in range(n):
            for k in range(n):
                for l in range(n):
                    acc = 0.0
                    for a in range(n):
                        for b in range(n):
                            for c in range(n):
                                for d in range(n):
                                    acc += C[a, m] * C[b, q] * C[c, k] * C[d, l] * eri_ao[a, b, c, d]
                    out[m, q, k, l] = acc
    return out


def ri_four_index(B, C):
    """(mn|kl) of an RI tensor: transform each B^P to the MO basis with explicit
    loops over the AO pair, then sum_P B^P_mn B^P_kl."""
    naux, n, _ = B.shape
    Bm = np.zeros((naux, n, n))
    for P in range(naux):
        for a in range(n):
            for b in range(n):
                Bm[P] += B[P, a, b] * np.outer(C[a], C[b])
    return np.einsum("Pmn,Pkl->mnkl", Bm, Bm)


# ------------------------------------------------------------ P17 --------
def casida_spin_blocks_eig(B_mo_s, eps_s, nocc_s):
    """Open-shell direct RPA from the full non-Hermitian problem
    [[A, B], [-B, -A]] (X, Y) = Omega (X, Y) over transitions (i, a, sigma),
    with (ia sigma|jb sigma') built element by element from the two spins' RI
    factors.  Returns (positive Omega ascending, X+Y normalised so that
    X^T X - Y^T Y = 1, columns in the order of Omega)."""
    pr = []
    for s, (e, no) in enumerate(zip(eps_s, nocc_s)):
        pr += [(i, a, s) for i in range(no) for a in range(no, e.size)]
    n = len(pr)
    A = np.zeros((n, n))
    B = np.zeros((n, n))
    for t, (i, a, s) in enumerate(pr):
        for u, (j, b, s2) in enumerate(pr):
            v = float(np.dot(B_mo_s[s][:, i, a], B_mo_s[s2][:, j, b]))
            A[t, u] = (eps_s[s][a] - eps_s[s][i]) * (t == u) + v
            B[t, u] = float(np.dot(B_mo_s[s][:, i, a], B_mo_s[s2][:, b, j]))
    H = np.block([[A, B], [-B, -A]])
    lam, vec = np.linalg.eig(H)
    keep = np.where(lam.real > 0)[0]
    order = keep[np.argsort(lam.real[keep])]
    Om = lam.real[order]
    X = vec[:n, order].real
    Y = vec[n:, order].real
    norm = np.sqrt(np.einsum("ts,ts->s", X, X) - np.einsum("ts,ts->s", Y, Y))
    return Om, (X + Y) / norm[None, :], pr


def gw_unrestricted_spin_sums(B_mo_s, eps_s, nocc_s, eta, spin):
    """Eqs. (17)-(19) for one spin from P17's excitations: residues
    w^s_{mk} = sum_{(i, a, sigma')} (mk sigma|ia sigma') (X+Y)^s, summed term by
    term, and V = 1/2 Re[Sigma(eps_m) + Sigma(eps_n)] element by element."""
    Om, XpY, pr = casida_spin_blocks_eig(B_mo_s, eps_s, nocc_s)
    Bs, es, no = B_mo_s[spin], eps_s[spin], nocc_s[spin]
    nb = es.size
    w = np.zeros((nb, nb, Om.size))
    for t, (i, a, s2) in enumerate(pr):
        integ = np.einsum("P,Pmk->mk", B_mo_s[s2][:, i, a], Bs)
        w += integ[:, :, None] * XpY[t][None, None, :]
    V = np.zeros((nb, nb))
    for m in range(nb):
        for q in range(nb):
            tot = 0.0
            for om in (es[m], es[q]):
                for k in range(nb):
                    den = (om - es[k] + Om - 1j * eta) if k < no else (om - es[k] - Om + 1j * eta)
                    tot += np.sum(w[m, k] * w[q, k] / den).real
            V[m, q] = 0.5 * tot
    return V, Om
