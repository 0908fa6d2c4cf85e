"""Parity of the open-shell (spin-unrestricted) GW potential on the GPU.

Each spin has its own orbitals (two seeded orthogonal matrices applied to one
synthetic AO tensor), energies and occupation.  The GPU call builds and solves
the shared Casida problem and the potential of each spin; it is compared with
the FP64 oracle element by element, and with the restricted GPU chain when
both spins are equal.  The eigensolvers differ (rocSOLVER dsyevd, LAPACK
dsyevr), so V is compared at 1e-10 of its largest element (eta well above the
level spacing of the poles it weights); Omega at 1e-11 relative.
"""
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


def two_spins(nbf, naux, nocc_a, nocc_b, seed):
    pa = make_problem(nbf, naux, nocc_a, max(1, naux // 2), 0.99, seed, coupling=0.1)
    pb = make_problem(nbf, naux, nocc_b, max(1, naux // 2), 0.99, seed + 100, coupling=0.1)
    return ([O.mo_transform(pa.B_ao, pa.C0), O.mo_transform(pa.B_ao, pb.C0)],
            [pa.eps0, pb.eps0], [nocc_a, nocc_b])


CASES = [  # nbf, naux, nocc_a, nocc_b, eta
    (2, 1, 1, 1, 0.05),
    (6, 9, 3, 2, 0.05),
    (5, 7, 1, 3, 0.02),
    (24, 96, 5, 4, 0.05),
    (37, 53, 9, 8, 0.02),
    (70, 150, 11, 10, 0.05),
    (6, 8, 5, 4, 0.05),  # one empty alpha state
]


@pytest.mark.parametrize("nbf,naux,na,nb,eta", CASES)
def test_unrestricted_matches_oracle(q, ctx, nbf, naux, na, nb, eta):
    print(f"[uhf] nbf={nbf} naux={naux} nocc=({na}, {nb}) eta={eta}", flush=True)
    B_s, e_s, n_s = two_spins(nbf, naux, na, nb, nbf)
    V_ref, Om_ref = O.gw_unrestricted(B_s, e_s, n_s, eta)
    Va, Vb, Om = q.qsgw_gw_unrestricted(ctx, dev(B_s[0]), dev(B_s[1]), dev(e_s[0]), dev(e_s[1]),
                                        na, nb, eta)
    np.testing.assert_allclose(host(Om), Om_ref, rtol=1e-11)
    for V, R in ((host(Va), V_ref[0]), (host(Vb), V_ref[1])):
        np.testing.assert_array_equal(V, V.T)
        assert np.abs(V - R).max() <= 1e-10 * np.abs(R).max() + 1e-15


def test_unrestricted_equal_spins_is_restricted_chain(q, ctx):
    p = make_problem(30, 80, 6, 40, 0.99, 4, coupling=0.1)
    eta = 0.05
    B_mo = q.qsgw_mo_transform(ctx, dev(p.B_ao), dev(p.C0))
    e = dev(p.eps0)
    M, sq = q.qsgw_rpa_build(ctx, B_mo, e, 6)
    Z, Om_r = q.qsgw_rpa_solve(ctx, M)
    w, wh = q.qsgw_residues(ctx, B_mo, sq, Z, Om_r, 6, weighted=True, eps=e, eta=eta)
    Vr = host(q.qsgw_sigma_qs(ctx, w, e, Om_r, 6, eta, wh=wh))
    Va, Vb, Om = q.qsgw_gw_unrestricted(ctx, B_mo, B_mo, e, e, 6, 6, eta)
    scale = np.abs(Vr).max()
    assert np.abs(host(Va) - Vr).max() <= 1e-10 * scale
    np.testing.assert_array_equal(host(Va), host(Vb))
    both = np.sort(np.concatenate([host(Om_r), O.transition_energies(p.eps0, 6)]))
    np.testing.assert_allclose(host(Om), both, rtol=1e-11)


def test_unrestricted_errors(q, ctx):
    B_s, e_s, n_s = two_spins(6, 5, 2, 2, 0)
    args = [dev(B_s[0]), dev(B_s[1]), dev(e_s[0]), dev(e_s[1])]
    with pytest.raises(q.QsgwError) as x:
        q.qsgw_gw_unrestricted(ctx, *args, 2, 2, 0.05, precision=q.PREC_FP32)
    assert x.value.code == q.ERR_UNSUPPORTED
    for na, nb, eta in ((0, 2, 0.05), (2, 6, 0.05), (2, 2, 0.0)):
        with pytest.raises(q.QsgwError) as x:
            q.qsgw_gw_unrestricted(ctx, *args, na, nb, eta)
        assert x.value.code == q.ERR_INVALID_ARG


@pytest.mark.parametrize("nbf,naux,na,nb", [(6, 9, 3, 2), (24, 96, 5, 4), (37, 53, 9, 8)])
def test_unrestricted_step_matches_oracle(q, ctx, nbf, naux, na, nb):
    """One open-shell step through the C-ABI (MO transform of each spin, the
    open-shell GW potential, the open-shell Fock update) against the oracle's."""
    print(f"[uhf-step] nbf={nbf} naux={naux} nocc=({na}, {nb})", flush=True)
    eta = 0.05
    pa = make_problem(nbf, naux, na, max(1, naux // 2), 0.99, nbf, coupling=0.1)
    pb = make_problem(nbf, naux, nb, max(1, naux // 2), 0.99, nbf + 100, coupling=0.1)
    h = O.hf_core(pa.B_ao, pa.C0, pa.eps0, na)
    e_ref, C_ref = O.unrestricted_step(pa.B_ao, h, [pa.C0, pb.C0], [pa.eps0, pb.eps0], [na, nb],
                                       eta)
    Bd = dev(pa.B_ao)
    Ca, Cb = dev(pa.C0), dev(pb.C0)
    ea, eb = dev(pa.eps0), dev(pb.eps0)
    Ba = q.qsgw_mo_transform(ctx, Bd, Ca)
    Bb = q.qsgw_mo_transform(ctx, Bd, Cb)
    Va, Vb, _ = q.qsgw_gw_unrestricted(ctx, Ba, Bb, ea, eb, na, nb, eta)
    ea2, eb2 = torch.empty_like(ea), torch.empty_like(eb)
    q.qsgw_fock_unrestricted(ctx, Ba, Bb, dev(h), Va, Vb, na, nb, ea2, eb2, Ca, Cb)
    V_ref, _ = O.gw_unrestricted([O.mo_transform(pa.B_ao, pa.C0), O.mo_transform(pa.B_ao, pb.C0)],
                                 [pa.eps0, pb.eps0], [na, nb], eta)
    F_ref = O.fock_unrestricted(h, pa.B_ao, [pa.C0, pb.C0], [na, nb], V_ref)
    for e, C, er, F in ((ea2, Ca, e_ref[0], F_ref[0]), (eb2, Cb, e_ref[1], F_ref[1])):
        e, C = host(e), host(C)
        np.testing.assert_allclose(e, er, rtol=0, atol=1e-8)
        np.testing.assert_allclose(C.T @ C, np.eye(nbf), rtol=0, atol=1e-11)
        np.testing.assert_allclose(C.T @ F @ C, np.diag(er), rtol=0, atol=1e-8)


def test_unrestricted_step_equal_spins_is_iterate(q, ctx):
    p = make_problem(30, 80, 6, 40, 0.99, 4, coupling=0.1)
    eta = 0.05
    Bd, e0, C0 = dev(p.B_ao), dev(p.eps0), dev(p.C0)
    h = q.qsgw_hf_core(ctx, Bd, C0, e0, 6)
    e_it, C_it = e0.clone(), C0.clone()
    q.qsgw_iterate(ctx, Bd, h, 6, e_it, C_it, eta, tol=0.0, max_iter=1)
    B_mo = q.qsgw_mo_transform(ctx, Bd, C0)
    Va, Vb, _ = q.qsgw_gw_unrestricted(ctx, B_mo, B_mo, e0, e0, 6, 6, eta)
    Ca, Cb = C0.clone(), C0.clone()
    ea, eb = torch.empty_like(e0), torch.empty_like(e0)
    q.qsgw_fock_unrestricted(ctx, B_mo, B_mo, h, Va, Vb, 6, 6, ea, eb, Ca, Cb)
    np.testing.assert_allclose(host(ea), host(e_it), rtol=0, atol=1e-10)
    np.testing.assert_array_equal(host(ea), host(eb))


def test_unrestricted_full_size_equal_spins(q, ctx):
    """N_b = 300, N_aux = 1200, 40 + 40 electrons on the workload's orbitals:
    20,800 transitions, so the residues run in two excitation blocks as in the
    benchmark's doublet.  Equal spins must give the restricted chain's V for
    both spins and Omega = singlets plus triplets at Delta."""
    from qsgw_inputs import make_config
    p = make_config("cfg2")
    eta = 0.05
    print("[uhf] full size, equal spins", flush=True)
    B_mo = q.qsgw_mo_transform(ctx, dev(p.B_ao), dev(p.C0))
    e = dev(p.eps0)
    M, sq = q.qsgw_rpa_build(ctx, B_mo, e, p.nocc)
    Z, Om_r = q.qsgw_rpa_solve(ctx, M)
    w, wh = q.qsgw_residues(ctx, B_mo, sq, Z, Om_r, p.nocc, weighted=True, eps=e, eta=eta)
    Vr = host(q.qsgw_sigma_qs(ctx, w, e, Om_r, p.nocc, eta, wh=wh))
    om_r = host(Om_r)
    del M, Z, w, wh
    torch.cuda.empty_cache()
    Va, Vb, Om = q.qsgw_gw_unrestricted(ctx, B_mo, B_mo, e, e, p.nocc, p.nocc, eta)
    Va, Vb = host(Va), host(Vb)
    np.testing.assert_array_equal(Va, Vb)
    assert np.abs(Va - Vr).max() <= 1e-9 * np.abs(Vr).max()
    both = np.sort(np.concatenate([om_r, O.transition_energies(p.eps0, p.nocc)]))
    np.testing.assert_allclose(host(Om), both, rtol=1e-10)


@pytest.mark.parametrize("nbf,naux,na,nb", [(24, 96, 5, 4), (37, 53, 9, 8), (30, 80, 3, 1)])
def test_unrestricted_iterations_match_oracle(q, ctx, nbf, naux, na, nb):
    """Open-shell iterations through qsgw_iterate_unrestricted against the
    oracle's open-shell steps chained: every iteration's orbital energies of
    both spins to 1e-8 Ha, max|d eps| as the oracle's, one call of three
    iterations equal to three calls of one, and the convergence exit."""
    print(f"[uhf-iterate] nbf={nbf} naux={naux} nocc=({na}, {nb})", flush=True)
    eta, iters = 0.05, 3
    pa = make_problem(nbf, naux, na, max(1, naux // 2), 0.99, nbf, coupling=0.1)
    pb = make_problem(nbf, naux, nb, max(1, naux // 2), 0.99, nbf + 100, coupling=0.1)
    h = O.hf_core(pa.B_ao, pa.C0, pa.eps0, na)
    es, Cs = [pa.eps0, pb.eps0], [pa.C0, pb.C0]
    refs, deps = [], []
    for _ in range(iters):
        new_e, Cs = O.unrestricted_step(pa.B_ao, h, Cs, es, [na, nb], eta)
        deps.append(max(np.max(np.abs(a - b)) for a, b in zip(new_e, es)))
        es = new_e
        refs.append([e.copy() for e in es])
    Bd, hd = dev(pa.B_ao), dev(h)
    ea, eb, Ca, Cb = dev(pa.eps0), dev(pb.eps0), dev(pa.C0), dev(pb.C0)
    it = 0
    for j in range(iters):
        rc, rep, it = q.qsgw_iterate_unrestricted(ctx, Bd, hd, na, nb, ea, Ca, eb, Cb, eta,
                                                  tol=0.0, max_iter=1, iteration=it)
        assert rc == q.NOT_CONVERGED and rep["iterations"] == 1 and it == j + 1
        np.testing.assert_allclose(host(ea), refs[j][0], rtol=0, atol=1e-8)
        np.testing.assert_allclose(host(eb), refs[j][1], rtol=0, atol=1e-8)
        assert abs(rep["max_deps"][0] - deps[j]) <= 1e-8
    ea3, eb3, Ca3, Cb3 = dev(pa.eps0), dev(pb.eps0), dev(pa.C0), dev(pb.C0)
    rc, rep, it = q.qsgw_iterate_unrestricted(ctx, Bd, hd, na, nb, ea3, Ca3, eb3, Cb3, eta,
                                              tol=0.0, max_iter=iters)
    assert rep["iterations"] == iters and it == iters
    np.testing.assert_array_equal(host(ea3), host(ea))
    np.testing.assert_array_equal(host(eb3), host(eb))
    np.testing.assert_allclose(rep["max_deps"][:iters], deps, rtol=0, atol=1e-8)
    # a tolerance above the first change stops after one iteration
    ea4, eb4, Ca4, Cb4 = dev(pa.eps0), dev(pb.eps0), dev(pa.C0), dev(pb.C0)
    rc, rep, it = q.qsgw_iterate_unrestricted(ctx, Bd, hd, na, nb, ea4, Ca4, eb4, Cb4, eta,
                                              tol=deps[0] * 1.5 + 1e-12, max_iter=iters)
    assert rc == q.OK and rep["converged"] == 1 and rep["iterations"] == 1
    with pytest.raises(q.QsgwError) as x:
        q.qsgw_iterate_unrestricted(ctx, Bd, hd, na, nbf, ea4, Ca4, eb4, Cb4, eta)
    assert x.value.code == q.ERR_INVALID_ARG


@pytest.mark.parametrize("nbf,naux,na,nb", [(24, 96, 5, 4), (70, 150, 11, 10)])
def test_unrestricted_two_stage_projection_matches_oracle(q, nbf, naux, na, nb):
    """With the two-stage solver the open-shell step takes rho' of every
    excitation from the eigensolver's projection of the spin-stacked Bt (the
    eigenvectors never formed; at 20,579 transitions this is the default):
    V of both spins and Omega against the oracle as above."""
    print(f"[uhf two-stage] nbf={nbf} naux={naux} nocc=({na}, {nb})", flush=True)
    B_s, e_s, n_s = two_spins(nbf, naux, na, nb, nbf)
    V_ref, Om_ref = O.gw_unrestricted(B_s, e_s, n_s, 0.05)
    with q.Context() as c:
        c.set_eigensolver(q.EIG_TWO_STAGE)
        Va, Vb, Om = q.qsgw_gw_unrestricted(c, dev(B_s[0]), dev(B_s[1]), dev(e_s[0]), dev(e_s[1]),
                                            na, nb, 0.05)
        np.testing.assert_allclose(host(Om), Om_ref, rtol=1e-11)
        for V, R in ((host(Va), V_ref[0]), (host(Vb), V_ref[1])):
            np.testing.assert_array_equal(V, V.T)
            assert np.abs(V - R).max() <= 1e-10 * np.abs(R).max() + 1e-15
