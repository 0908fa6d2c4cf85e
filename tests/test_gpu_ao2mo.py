"""Parity of the four-index AO->MO transform (Eq. 16) on the GPU with the oracle.

The AO integrals are (mu nu|lambda tau) = sum_P B^P_{mu nu} B^P_{lambda tau}
of a general symmetric RI tensor from the seeded generator, so the result also
has the RI form sum_P B'^P_mn B'^P_kl with B' = C^T B C; small and ragged
sizes and slabs compare every element with the oracle, the N_b = 300 slab
(the benchmark's launch) compares sampled elements with the RI form.  Bound:
the same contraction on absolute values times (4 N_b + 8) unit roundoffs.
"""
import numpy as np
import pytest

import oracle as O
from qsgw_inputs import make_mo_tensor, make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53


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


def inputs(nbf, naux, seed):
    B = make_mo_tensor(nbf, naux, 1, seed)[0]
    flat = B.reshape(naux, nbf * nbf)
    eri = (flat.T @ flat).reshape(nbf, nbf, nbf, nbf)
    C = make_problem(nbf, 2, 1, 1, 0.5, seed).C0
    return B, eri, C


@pytest.mark.parametrize("nbf,naux,m0,mc", [(2, 1, 1, 1), (5, 4, 0, 5), (24, 30, 3, 7),
                                            (37, 20, 0, 37), (70, 40, 10, 33)])
def test_ao2mo_slab_matches_oracle(q, ctx, nbf, naux, m0, mc):
    log(f"[ao2mo] nbf={nbf} slab=[{m0}, {m0 + mc})")
    B, eri, C = inputs(nbf, naux, nbf)
    rows = np.arange(m0, m0 + mc)
    ref = O.ao2mo_4center(eri, C, rows)
    bound = (4 * nbf + 8) * U * O.ao2mo_4center(np.abs(eri), np.abs(C), rows)
    got = host(q.qsgw_ao2mo_4center(ctx, dev(eri), dev(C), m0, mc))
    assert np.all(np.abs(got - ref) <= bound), float(np.abs(got - ref).max())


def test_ao2mo_full_size_slab_sampled(q, ctx):
    nbf, naux, m0, mc = 300, 400, 100, 64
    log(f"[ao2mo] nbf={nbf} slab=[{m0}, {m0 + mc}) sampled")
    B = make_mo_tensor(nbf, naux, 1, 3)[0]
    C = make_problem(nbf, 2, 1, 1, 0.5, 3).C0
    Bd = dev(B.reshape(naux, nbf * nbf))
    eri = (Bd.T @ Bd).reshape(nbf, nbf, nbf, nbf)       # synthetic AO integrals
    out = q.qsgw_ao2mo_4center(ctx, eri, dev(C), m0, mc)
    Bm = O.mo_transform(B, C)
    eri_max = float(eri.abs().max())
    rng = np.random.default_rng(1)
    idx = [(0, 0, 0, 0), (mc - 1, 299, 150, 7), (17, 5, 5, 17)]
    idx += [tuple(int(v) for v in rng.integers(0, [mc, nbf, nbf, nbf])) for _ in range(40)]
    got = host(out)
    for m, n, k, l in idx:
        ref = float(np.dot(Bm[:, m0 + m, n], Bm[:, k, l]))
        # sum over the four AO indices of |C||C||C||C||eri| <= (max_m sum_a |C_am|)^4 max|eri|
        scale = float(np.sum(np.abs(Bm[:, m0 + m, n]) * np.abs(Bm[:, k, l]))) + \
            float(np.abs(C).sum(0).max() ** 4 * eri_max)
        assert abs(got[m, n, k, l] - ref) <= (4 * nbf + naux + 8) * U * scale, (m, n, k, l)
    del eri, out, Bd
    torch.cuda.empty_cache()


def test_ao2mo_errors(q, ctx):
    _, eri, C = inputs(4, 3, 0)
    e, c = dev(eri), dev(C)
    with pytest.raises(q.QsgwError) as x:
        q.qsgw_ao2mo_4center(ctx, e, c, 0, 4, precision=q.PREC_FP32)
    assert x.value.code == q.ERR_UNSUPPORTED
    for m0, mc in ((-1, 2), (3, 2), (0, 0)):
        with pytest.raises(q.QsgwError) as x:
            q.qsgw_ao2mo_4center(ctx, e, c, m0, mc, out=torch.empty((mc, 4, 4, 4),
                                                                   dtype=torch.float64,
                                                                   device="cuda"))
        assert x.value.code == q.ERR_INVALID_ARG
