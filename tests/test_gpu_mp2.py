"""Parity of the qsMP2 potential (Eqs. 20-21) on the GPU with the FP64 oracle.

Inputs are general symmetric RI tensors from the seeded generator (the qsGW
workload tensor has integrals symmetric under every index permutation, which
would let a mistake in the pairing of the exchange integrals pass).  Small
and ragged sizes compare every element, with one and several blocks of
transitions; the N_b = 300, N_aux = 1200, n_occ = 40 size compares sampled
elements computed one by one.  The bound for each element is the sum of the
absolute values of its terms times (K + N_aux + 8) unit roundoffs, K = N_b n_tr
the length of the final contraction (8 for the rounding of the pole weight).
"""
import numpy as np
import pytest

import oracle as O
import oracle.qsgw_oracle as OM
from qsgw_inputs import make_mo_tensor, make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53
ETA = 1e-3


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2210_17093_amd.qsgw as q
    return q


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context()
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def log(*a):
    print(*a, flush=True)


def abs_bound(B_mo, eps, nocc, eta):
    """Sum of |terms| of each element of V (oracle integrals, absolute values)."""
    L, R, X = OM._mp2_integrals(B_mo, nocc)
    nb = eps.size
    S = np.empty((nb, nb))
    for n in range(nb):
        g = np.abs(OM._mp2_denominators(eps[n], eps, nocc, eta))
        S[:, n] = np.einsum("mpia,pia->m", np.abs(L), np.abs(2.0 * R[n] - X[n]) * g)
    return 0.5 * (S + S.T)


SHAPES = [  # nbf, naux, nocc, seed
    (2, 1, 1, 0),
    (5, 7, 2, 1),
    (24, 96, 5, 2),
    (37, 53, 9, 3),
    (70, 150, 11, 4),
    (6, 8, 5, 5),  # one empty state
]


@pytest.mark.parametrize("nbf,naux,nocc,seed", SHAPES)
def test_mp2_potential_matches_oracle(q, ctx, nbf, naux, nocc, seed):
    log(f"[mp2] nbf={nbf} naux={naux} nocc={nocc} seed={seed}")
    B_mo, eps = make_mo_tensor(nbf, naux, nocc, seed)
    ref = O.qsmp2_potential(B_mo, eps, nocc, ETA)
    tol = (nbf * nocc * (nbf - nocc) + naux + 8) * U * abs_bound(B_mo, eps, nocc, ETA)
    Bd, ed = dev(B_mo), dev(eps)
    blocks = sorted({0, 1, max(1, nocc // 2), nocc})
    for ob in blocks:
        V = host(q.qsgw_mp2_sigma(ctx, Bd, ed, nocc, ETA, occ_block=ob))
        np.testing.assert_array_equal(V, V.T)
        err = np.abs(V - ref)
        assert np.all(err <= tol), (ob, float(err.max()), float(tol.min()))
        assert err.max() < 1e-8


def test_mp2_accumulate_and_ragged_blocks(q, ctx):
    nbf, naux, nocc = 41, 64, 7
    B_mo, eps = make_mo_tensor(nbf, naux, nocc, 9)
    ref = O.qsmp2_potential(B_mo, eps, nocc, ETA)
    tol = (nbf * nocc * (nbf - nocc) + naux + 8) * U * abs_bound(B_mo, eps, nocc, ETA)
    Bd, ed = dev(B_mo), dev(eps)
    base = np.random.default_rng(5).standard_normal((nbf, nbf))
    base = base + base.T
    for ob in (3, 4):  # 3 + 3 + 1 and 4 + 3 occupied states per block
        out = dev(base)
        q.qsgw_mp2_sigma(ctx, Bd, ed, nocc, ETA, out=out, occ_block=ob, accumulate=True)
        got = host(out) - base
        assert np.all(np.abs(got - ref) <= tol + 4 * U * np.abs(base)), ob


def test_mp2_sampled_at_full_size(q, ctx):
    nbf, naux, nocc = 300, 1200, 40
    log(f"[mp2] sampled nbf={nbf} naux={naux} nocc={nocc}")
    B_mo, eps = make_mo_tensor(nbf, naux, nocc, 0)
    V = host(q.qsgw_mp2_sigma(ctx, dev(B_mo), dev(eps), nocc, ETA))
    assert np.all(np.isfinite(V))
    np.testing.assert_array_equal(V, V.T)
    scale = np.abs(V).max()
    for m, n in ((0, 0), (3, 257), (39, 40), (120, 299)):
        ref = O.qsmp2_entry(B_mo, eps, nocc, ETA, m, n)
        assert abs(V[m, n] - ref) < 1e-11 * scale + 1e-13, (m, n, V[m, n], ref)


def test_mp2_errors(q, ctx):
    B_mo, eps = make_mo_tensor(6, 5, 2, 0)
    Bd, ed = dev(B_mo), dev(eps)
    with pytest.raises(q.QsgwError) as e:
        q.qsgw_mp2_sigma(ctx, Bd, ed, 2, ETA, precision=q.PREC_FP32)
    assert e.value.code == q.ERR_UNSUPPORTED
    for kw in (dict(nocc=0, eta=ETA), dict(nocc=6, eta=ETA), dict(nocc=2, eta=0.0),
               dict(nocc=2, eta=ETA, occ_block=-1)):
        with pytest.raises(q.QsgwError) as e:
            q.qsgw_mp2_sigma(ctx, Bd, ed, **kw)
        assert e.value.code == q.ERR_INVALID_ARG


@pytest.mark.parametrize("nbf,naux,nocc", [(7, 9, 3), (24, 60, 5), (37, 53, 9)])
def test_qsmp2_iteration_matches_oracle(q, ctx, nbf, naux, nocc):
    """Two qsMP2 iterations through qsgw_iterate (QSGW_OPT_QSMP2) against the
    oracle's steps, on general RI factors in the AO basis."""
    log(f"[qsmp2-iter] nbf={nbf} naux={naux} nocc={nocc}")
    B_ao, eps0 = make_mo_tensor(nbf, naux, nocc, nbf)
    C0 = make_problem(nbf, 2, nocc, 1, 0.5, nbf).C0
    h = O.hf_core(B_ao, C0, eps0, nocc)
    e_ref, C_ref = eps0, C0
    for _ in range(2):
        e_ref, C_ref = O.qsmp2_step(B_ao, h, C_ref, e_ref, nocc, ETA)
    e, C = dev(eps0), dev(C0)
    rc, rep, it = q.qsgw_iterate(ctx, dev(B_ao), dev(h), nocc, e, C, ETA, tol=0.0, max_iter=2,
                                 qsmp2=True)
    assert it == 2 and rep["iterations"] == 2
    np.testing.assert_allclose(host(e), e_ref, rtol=0, atol=1e-8)
    with pytest.raises(q.QsgwError) as x:
        q.qsgw_iterate(ctx, dev(B_ao), dev(h), nocc, dev(eps0), dev(C0), ETA, tol=0.0,
                       max_iter=1, qsmp2=True, precision=q.PREC_FP32)
    assert x.value.code == q.ERR_UNSUPPORTED
