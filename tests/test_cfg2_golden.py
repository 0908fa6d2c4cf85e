"""Full-size parity: five plain qsGW iterations at N_b = 300, N_aux = 1200,
n_occ = 40 (10,400 transitions) through the C-ABI, against the oracle
trajectory stored in tests/golden/cfg2_oracle.json (written by
tests/golden/make_golden.py, which calls only the oracle).

The inputs are regenerated from the seeded generator; their fingerprint is
checked against the stored one first.  Every iteration's orbital energies are
compared; so are the excitation energies and the qsGW potential of the first
iteration (sampled entries), which the GPU path exposes through the same
entry points the iteration uses.

Conditioning.  At eta = 1e-3 Ha this workload does not converge in five
iterations and its trajectory amplifies any rounding difference ~30x per
iteration (near-pole terms of Eq. (17)).  The stored file records the
oracle's own spread: the distance between two oracle runs that differ only by
a permutation of the auxiliary index (an exact symmetry of the method, so only
the rounding order of every P-sum changes).  Iteration j is held to 1e-8 Ha
where that spread is far below it, and otherwise to 10x the spread: no FP64
evaluation order can be expected to do better than the oracle agrees with
itself.
"""
import json
import os

import numpy as np
import pytest

from qsgw_inputs import CONFIGS, make_config

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "cfg2_oracle.json")
QP_TOL = 1e-8  # Ha


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2210_17093_amd.qsgw as q
    with open(GOLD) as f:
        gold = json.load(f)
    p = make_config("cfg2")
    fp = gold["fingerprint"]
    assert abs(p.B_ao.sum() - fp["B_sum"]) <= 1e-9 * fp["B_abs"]
    assert abs(np.abs(p.B_ao).sum() - fp["B_abs"]) <= 1e-12 * fp["B_abs"]
    assert abs(p.eps0.sum() - fp["eps_sum"]) <= 1e-12 * np.abs(p.eps0).sum()
    ctx = q.Context()
    dev = torch.device("cuda:0")
    B = torch.from_numpy(p.B_ao).to(dev)
    C0 = torch.from_numpy(p.C0.copy()).to(dev)
    e0 = torch.from_numpy(p.eps0.copy()).to(dev)
    h = q.qsgw_hf_core(ctx, B, C0, e0, p.nocc)
    yield q, ctx, p, gold, B, C0, e0, h
    ctx.close()


def test_cfg2_first_iteration_intermediates(setup):
    q, ctx, p, gold, B, C0, e0, h = setup
    print("cfg2 intermediates", flush=True)
    g1 = gold["iterations"][0]
    eta = gold["eta"]
    B_mo = q.qsgw_mo_transform(ctx, B, C0)
    M, sq = q.qsgw_rpa_build(ctx, B_mo, e0, p.nocc)
    Z, Om = q.qsgw_rpa_solve(ctx, M)
    Omh = Om.cpu().numpy()
    np.testing.assert_allclose(Omh[:32], g1["Omega_low"], rtol=1e-11)
    np.testing.assert_allclose(Omh[-8:], g1["Omega_high"], rtol=1e-11)
    assert abs(Omh.sum() - g1["Omega_sum"]) <= 1e-11 * g1["Omega_sum"]
    w = q.qsgw_residues(ctx, B_mo, sq, Z, Om, p.nocc)
    V = q.qsgw_sigma_qs(ctx, w, e0, Om, p.nocc, eta).cpu().numpy()
    del w
    torch.cuda.empty_cache()
    Vd = np.asarray(g1["V_diag"])
    scale = np.abs(Vd).max()
    assert np.max(np.abs(np.diag(V) - Vd)) <= 1e-9 * scale
    for m, n, v in g1["V_samples"]:
        assert abs(V[m, n] - v) <= 1e-9 * scale, (m, n, V[m, n], v)
    assert abs(np.linalg.norm(V) - g1["V_fro"]) <= 1e-9 * g1["V_fro"]


def test_cfg2_five_iterations(setup):
    q, ctx, p, gold, B, C0, e0, h = setup
    eta = gold["eta"]
    e = e0.clone()
    C = C0.clone()
    it = 0
    errs = []
    for j, g in enumerate(gold["iterations"]):
        rc, rep, it = q.qsgw_iterate(ctx, B, h, p.nocc, e, C, eta, tol=gold["tol"], max_iter=1,
                                     iteration=it)
        err = float(np.max(np.abs(e.cpu().numpy() - np.asarray(g["eps"]))))
        errs.append(err)
        print(f"cfg2 iteration {j + 1}: max|eps - oracle| = {err:.3e} Ha, "
              f"max|d eps| = {rep['max_deps'][0]:.3e}", flush=True)
        assert abs(rep["max_deps"][0] - g["max_deps"]) <= QP_TOL + err
    spread = gold["reorder_spread"]
    for j, (err, sp) in enumerate(zip(errs, spread)):
        tol = QP_TOL if 10.0 * sp < QP_TOL else 10.0 * sp
        assert err <= tol, (j + 1, err, tol)
    # the first three iterations meet the 1e-8 Ha gate outright
    assert all(x <= QP_TOL for x in errs[:3]), errs


def _shipped_tables():
    path = os.path.join(os.path.dirname(HERE), "paper_2210_17093_amd", "tiles.json")
    with open(path) as f:
        table = json.load(f)
    return [(k, v["spec"]) for k, v in table.items() if k.startswith("cfg2")]


@pytest.mark.parametrize("key,spec", _shipped_tables())
def test_cfg2_first_iteration_under_shipped_tiles(setup, key, spec):
    """The tile tables the benchmark ships for this workload (the FP64 one
    splits the qsGW product into ~1,300 K slices) against the stored oracle
    iteration: FP64 at 1e-8 Ha, the reduced-precision variants at 1 meV."""
    q, ctx, p, gold, B, C0, e0, h = setup
    prec = {"cfg2": q.PREC_FP64, "cfg2:fp32": q.PREC_FP32,
            "cfg2:bf16x3": q.PREC_SPLIT_BF16}[key]
    ctx.set_tiles(spec)
    try:
        e, C = e0.clone(), C0.clone()
        q.qsgw_iterate(ctx, B, h, p.nocc, e, C, gold["eta"], tol=0.0, max_iter=1, precision=prec)
        err = float(np.max(np.abs(e.cpu().numpy() - np.asarray(gold["iterations"][0]["eps"]))))
    finally:
        ctx.set_tiles(None)
    print(f"cfg2 {key} ({spec}): max|eps - oracle| = {err:.3e} Ha", flush=True)
    assert err <= (QP_TOL if prec == q.PREC_FP64 else 1.0 / 27211.386)

