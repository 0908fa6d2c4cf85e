"""The allocation-free qsGW matrix product (qsgw_sigma_qs_noalloc) against the
allocating entry point (qsgw_sigma, QSGW_SIGMA_QS_MATRIX) on the same inputs,
through the C-ABI: two calls in a row, the second with a smaller input (the
static scratch keeps the first call's contents), with and without the
pole-weighted copy, overwrite and accumulate, plus the error paths.  Inputs
are residues the oracle computes from the seeded generator; the bound is the
FP64 rounding bound of the product (sum of absolute terms) used for qsgw_sigma.
"""
import ctypes as ct

import numpy as np
import pytest

import oracle as O
from qsgw_inputs import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2210_17093_amd.qsgw as q
    return q


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def abs_bound(w, eps, Om, nocc, eta):
    nbf = eps.size
    aw = np.abs(w)
    G = np.empty((nbf, nbf))
    for m in range(nbf):
        x = np.empty((nbf, Om.size))
        x[:nocc] = eps[m] - eps[:nocc, None] + Om[None, :]
        x[nocc:] = eps[m] - eps[nocc:, None] - Om[None, :]
        G[m] = np.tensordot(aw, aw[m] * np.abs(x / (x * x + eta * eta)), axes=([1, 2], [0, 1]))
    return 0.5 * (G + G.T)


def residues(shape, seed):
    nbf, naux, nocc = shape
    p = make_problem(nbf, naux, nocc, max(1, naux // 2), 0.99, seed)
    B_mo = O.mo_transform(p.B_ao, p.C0)
    M, sq = O.rpa_hermitian(B_mo, p.eps0, nocc)
    Om, XpY = O.rpa_solve(M, sq)
    return O.residues(B_mo, XpY, nocc), p.eps0, Om


@pytest.mark.parametrize("eta", [1e-3, 0.05])
def test_noalloc_matches_allocating_entry_point(q, eta):
    print("sigma_qs_noalloc", eta, flush=True)
    with q.Context() as ctx:
        # the shipped large-workload table asks for many K slices; the
        # allocation-free call caps them at what the scratch holds
        ctx.set_tiles("sigma=64x64,sigma_target=32768")
        for shape, seed in (((70, 200, 11), 1), ((37, 53, 9), 2)):  # the second call is smaller
            nbf, _, nocc = shape
            w, eps, Om = residues(shape, seed)
            dw, de, dO = dev(w), dev(eps), dev(Om)
            ref = host(q.qsgw_sigma_qs(ctx, dw, de, dO, nocc, eta))
            out = torch.full((nbf, nbf), np.nan, dtype=torch.float64, device="cuda")
            got = host(q.qsgw_sigma_qs_noalloc(ctx, dw, de, dO, nocc, eta, out))
            np.testing.assert_array_equal(got, got.T)
            bound = 2e-12 * abs_bound(w, eps, Om, nocc, eta) + 1e-300
            assert np.all(np.abs(got - ref) <= bound), shape
            # pole-weighted copy from the residue entry point, and accumulation
            wh = w * 0.0
            for m in range(nbf):
                x = np.empty((nbf, Om.size))
                x[:nocc] = eps[m] - eps[:nocc, None] + Om[None, :]
                x[nocc:] = eps[m] - eps[nocc:, None] - Om[None, :]
                wh[m] = w[m] * x / (x * x + eta * eta)
            dwh = dev(wh)
            ref2 = host(q.qsgw_sigma_qs(ctx, dw, de, dO, nocc, eta, wh=dwh))
            got2 = host(q.qsgw_sigma_qs_noalloc(ctx, dw, de, dO, nocc, eta, out, wh=dwh))
            assert np.all(np.abs(got2 - ref2) <= bound), shape
            got3 = host(q.qsgw_sigma_qs_noalloc(ctx, dw, de, dO, nocc, eta, out, accumulate=True))
            assert np.all(np.abs(got3 - (ref2 + ref)) <= 2 * bound), shape


def test_noalloc_errors(q):
    print("sigma_qs_noalloc errors", flush=True)
    with q.Context() as ctx:
        w, eps, Om = residues((24, 40, 5), 3)
        dw, de, dO = dev(w), dev(eps), dev(Om)
        out = torch.zeros((24, 24), dtype=torch.float64, device="cuda")
        bad = w.copy()
        bad[3, 4, 5] = np.nan
        with pytest.raises(q.QsgwError) as e:
            q.qsgw_sigma_qs_noalloc(ctx, dev(bad), de, dO, 5, 1e-3, out)
        assert e.value.code == q.ERR_NONFINITE
        # the scratch holds no partial sum of a 3000 x 3000 matrix: refused
        # from the sizes alone, before any array is read
        rc = q.lib().qsgw_sigma_qs_noalloc(ctx.handle, 3000, 5, 1, ct.c_void_p(dw.data_ptr()),
                                           None, ct.c_void_p(de.data_ptr()),
                                           ct.c_void_p(dO.data_ptr()), 1e-3,
                                           ct.c_void_p(out.data_ptr()), 0)
        assert rc == q.ERR_INVALID_ARG
        # still usable afterwards
        ref = host(q.qsgw_sigma_qs(ctx, dw, de, dO, 5, 1e-3))
        got = host(q.qsgw_sigma_qs_noalloc(ctx, dw, de, dO, 5, 1e-3, out))
        assert np.all(np.abs(got - ref) <= 2e-12 * abs_bound(w, eps, Om, 5, 1e-3) + 1e-300)
