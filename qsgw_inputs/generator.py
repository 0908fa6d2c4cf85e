"""Seeded synthetic RI tensors shaped like molecular qsGW workloads.

The paper's workloads are alkanes in cc-pVTZ (section "Benchmark", Table III),
whose geometries, basis sets and integrals are not available here.  This
module synthesises inputs with the same shapes and structure instead:

* RI tensor  B^P_{mu nu} = sum_r L_{P r} U_{r mu} U_{r nu}   (symmetric in mu nu)
  with U ~ N(0, 1) of shape (R, N_b) and L = Q diag(s), Q the orthonormal
  factor of an N_aux x R Gaussian, s_r = s0 * d**r.  s0 is fixed so that the
  mean diagonal Coulomb integral (mu mu|mu mu) = sum_r s_r^2 U_{r mu}^4 has
  expectation 0.5 Ha (E[U^4] = 3), times an optional coupling scale.
* orbital energies: occupied uniform in [-30, -0.3] Ha, virtual uniform in
  [0.05, 20] Ha, each sorted ascending.
* C: a Haar-orthogonal N_b x N_b matrix (QR of a Gaussian, columns signed by
  sign(diag R)), so the synthetic AO basis is orthonormal (S = I).

Draw order from ``numpy.random.default_rng(seed)``: U, the Gaussian behind L,
eps_occ, eps_virt, the Gaussian behind C.

Because Q has orthonormal columns, sum_P B^P_{ab} B^P_{cd} = sum_r s_r^2 U_ra
U_rb U_rc U_rd is symmetric under every permutation of (a, b, c, d): more
symmetry than molecular integrals have (those are symmetric within each pair
and under the exchange of the two pairs only).  ``make_mo_tensor`` draws a
general symmetric RI tensor instead, for the terms whose index pairing that
extra symmetry would hide (the exchange term of the MP2 self-energy):

* B^P_{mn} = g (G^P_{mn} + G^P_{nm}) / 2 with G ~ N(0, 1), g fixed so that
  the mean (m m|m m) = sum_P (B^P_{mm})^2 is 0.5 Ha times the coupling scale;
  orbital energies drawn as above.  Draw order: G, eps_occ, eps_virt.  Nothing here evaluates any
equation of the method; the core Hamiltonian that makes (eps, C) a
Hartree-Fock fixed point is built by each implementation on its own.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# One coupling scale for every workload.  At scale 1 (mean (mu mu|mu mu) =
# 0.5 Ha) the self-consistent iteration at eta = 1e-3 Ha is chaotic: a 1e-11
# Ha perturbation of the start grows to 1e-4 Ha within 8 iterations and
# HOMO/LUMO corrections reach several Ha.  At 0.1 the HOMO/LUMO corrections
# of the N_b = 150..300 workloads fall in 0.01..0.5 Ha.
COUPLING = 0.1


@dataclass
class Problem:
    nbf: int
    naux: int
    nocc: int
    B_ao: np.ndarray  # [naux][nbf][nbf], float64, symmetric in the last two
    C0: np.ndarray  # [nbf][nbf], float64, orthogonal, column m = MO m
    eps0: np.ndarray  # [nbf], float64, ascending
    meta: dict = field(default_factory=dict)

    @property
    def nvirt(self) -> int:
        return self.nbf - self.nocc

    @property
    def ntr(self) -> int:
        return self.nocc * (self.nbf - self.nocc)


def _coupling_s0(rank: int, decay: float, coupling: float) -> float:
    geo = float(np.sum(decay ** (2.0 * np.arange(rank))))
    return float(np.sqrt(coupling * 0.5 / (3.0 * geo)))


def make_problem(nbf: int, naux: int, nocc: int, rank: int, decay: float,
                 seed: int, coupling: float = COUPLING) -> Problem:
    """Draw one synthetic instance.  See the module docstring for the recipe."""
    if not (0 < nocc < nbf):
        raise ValueError("need 0 < nocc < nbf")
    if rank < 1 or naux < 1:
        raise ValueError("need rank >= 1 and naux >= 1")
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((rank, nbf))
    GL = rng.standard_normal((naux, rank))
    eps_occ = np.sort(rng.uniform(-30.0, -0.3, nocc))
    eps_virt = np.sort(rng.uniform(0.05, 20.0, nbf - nocc))
    GC = rng.standard_normal((nbf, nbf))

    # L = Q diag(s); reduced QR keeps min(naux, rank) orthonormal columns.
    Q, _ = np.linalg.qr(GL)
    r_eff = Q.shape[1]
    s0 = _coupling_s0(rank, decay, coupling)
    s = s0 * decay ** np.arange(r_eff)
    L = Q * s[None, :]
    UU = (U[:r_eff, :, None] * U[:r_eff, None, :]).reshape(r_eff, nbf * nbf)
    B = (L @ UU).reshape(naux, nbf, nbf)
    B = 0.5 * (B + B.transpose(0, 2, 1))  # exact symmetry in (mu, nu)

    QC, RC = np.linalg.qr(GC)
    C = QC * np.sign(np.diag(RC))[None, :]

    eps = np.concatenate([eps_occ, eps_virt])
    meta = dict(nbf=nbf, naux=naux, nocc=nocc, rank=rank, decay=decay,
                seed=seed, coupling=coupling, s0=s0)
    return Problem(nbf, naux, nocc, np.ascontiguousarray(B),
                   np.ascontiguousarray(C), eps, meta)



def make_mo_tensor(nbf: int, naux: int, nocc: int, seed: int,
                   coupling: float = COUPLING):
    """General symmetric RI tensor in the MO basis and sorted orbital energies.

    Returns (B_mo [naux][nbf][nbf], eps [nbf]); see the module docstring.
    """
    if not (0 < nocc < nbf) or naux < 1:
        raise ValueError("need 0 < nocc < nbf and naux >= 1")
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((naux, nbf, nbf))
    eps_occ = np.sort(rng.uniform(-30.0, -0.3, nocc))
    eps_virt = np.sort(rng.uniform(0.05, 20.0, nbf - nocc))
    g = np.sqrt(coupling * 0.5 / naux)
    B = g * 0.5 * (G + G.transpose(0, 2, 1))
    return np.ascontiguousarray(B), np.concatenate([eps_occ, eps_virt])


# The workloads of the benchmark configurations.  cfg1..cfg3 are single
# instances; the batched and learned workloads draw many small instances
# (see batch_shapes).
CONFIGS = {
    "cfg1": dict(nbf=24, naux=96, nocc=5, rank=48, decay=0.5, seed=0, eta=1e-3),
    "cfg2": dict(nbf=300, naux=1200, nocc=40, rank=600, decay=0.99, seed=0,
                 eta=1e-3, tol=1e-6, max_iter=5),
    "cfg3": dict(nbf=600, naux=2400, nocc=80, rank=1200, decay=0.99, seed=0,
                 eta=1e-3, near_pole=0.05),
}


def make_config(name: str, coupling: float = COUPLING) -> Problem:
    c = CONFIGS[name]
    return make_problem(c["nbf"], c["naux"], c["nocc"], c["rank"], c["decay"],
                        c["seed"], coupling)


def cfg1_omega_grid() -> np.ndarray:
    """201 frequencies -2 + 0.02 j Ha, j = 0..200."""
    return -2.0 + 0.02 * np.arange(201, dtype=np.float64)


def batch_shapes(nmol: int = 256, seed: int = 4, base_seed: int = 1000):
    """Shapes of a batch of uneven molecules.

    N_b is a uniform integer in [20, 120] (drawn from default_rng(seed)),
    N_aux = 4 N_b, n_occ = floor(N_b / 6 + 1/2) (round half up), rank
    R = N_aux / 2, decay 0.99 and instance seed base_seed + i.
    """
    rng = np.random.default_rng(seed)
    nbfs = rng.integers(20, 121, size=nmol)
    out = []
    for i, nb in enumerate(nbfs):
        nb = int(nb)
        out.append(dict(nbf=nb, naux=4 * nb, nocc=int(np.floor(nb / 6.0 + 0.5)),
                        rank=2 * nb, decay=0.99, seed=base_seed + i))
    return out
