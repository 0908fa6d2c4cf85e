"""The reduced-precision gate at the headline workload (N_b = 600,
N_aux = 2400, n_occ = 80, 41,600 transitions): one qsGW iteration from the
same start in FP64, with FP32 matrix-core products and with split-BF16
products (each variant solving its own Casida matrix with the two-stage
solver and streaming 14 residue blocks); every one of the 600 quasiparticle
energies of the reduced variants within 1 meV of the FP64 iteration."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MEV = 1.0 / 27211.386


def test_reduced_precision_within_1meV_at_600_basis_functions():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2210_17093_amd.qsgw as q
    from qsgw_inputs import make_config
    print("N_b = 600 precision gate: generating inputs", flush=True)
    p = make_config("cfg3")
    d = torch.device("cuda:0")
    B = torch.from_numpy(p.B_ao).to(d)
    C0 = torch.from_numpy(p.C0.copy()).to(d)
    e0 = torch.from_numpy(p.eps0.copy()).to(d)
    out = {}
    with q.Context() as ctx:
        h = q.qsgw_hf_core(ctx, B, C0, e0, p.nocc)
        for name, prec in (("fp64", q.PREC_FP64), ("fp32", q.PREC_FP32),
                           ("bf16x3", q.PREC_SPLIT_BF16)):
            print(f"  one iteration, {name}", flush=True)
            e, C = e0.clone(), C0.clone()
            q.qsgw_iterate(ctx, B, h, p.nocc, e, C, 1e-3, tol=0.0, max_iter=1, precision=prec)
            out[name] = e.cpu().numpy()
    for name in ("fp32", "bf16x3"):
        err = np.abs(out[name] - out["fp64"])
        print(f"  {name}: max {err.max() / MEV:.3f} meV, median {np.median(err) / MEV:.4f} meV",
              flush=True)
        assert err.max() <= MEV, name
