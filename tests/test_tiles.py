"""The tile table (qsgw_set_tiles, chosen by the autotuner): every shape
variant keeps parity with the oracle and the batched path matches the
single-instance path under the same table."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _shipped():
    """Every table the autotuner wrote to tiles.json (the ones bench.py runs)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2210_17093_amd", "tiles.json")
    with open(path) as f:
        return sorted({v["spec"] for v in json.load(f).values()})


TABLES = [
    "mo1=64x64,mo2=128x128,casida=64x64,rho=64x64,sigma=128x128,exchange=128x128,"
    "sigma_target=2048,rho_target=1024",
    "mo1=128x128,rho=128x64,sigma=128x64,sigma_target=8192,rho_target=4096,exchange_target=512",
    "persistent=1,mo1=64x64,sigma_target=1024",
] + _shipped()


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle as O
    import paper_2210_17093_amd.qsgw as q
    from qsgw_inputs import make_problem
    p = make_problem(70, 280, 12, 140, 0.99, 77)
    h = O.hf_core(p.B_ao, p.C0, p.eps0, p.nocc)
    eps1, _, _ = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0, p.nocc, 1e-3, 0.0, 1)
    stream = torch.cuda.Stream()
    ctx = q.Context(stream)
    dev = torch.device("cuda:0")
    with torch.cuda.stream(stream):
        B = torch.from_numpy(p.B_ao).to(dev)
        C0 = torch.from_numpy(p.C0.copy()).to(dev)
        e0 = torch.from_numpy(p.eps0.copy()).to(dev)
        hd = q.qsgw_hf_core(ctx, B, C0, e0, p.nocc)
    stream.synchronize()
    yield q, ctx, stream, p, B, C0, e0, hd, eps1
    ctx.close()


def test_table_roundtrip_and_errors(env):
    q, ctx, *_ = env
    ctx.set_tiles(None)
    default = ctx.get_tiles()
    assert "mo1=128x64" in default and "sigma_target=4096" in default
    ctx.set_tiles(TABLES[0])
    got = dict(kv.split("=") for kv in ctx.get_tiles().split(","))
    assert got["sigma"] == "128x128" and got["rho_target"] == "1024" and got["mo2"] == "128x128"
    assert got["dc_leaf"] == "6144"
    ctx.set_tiles("dc_leaf=512")
    assert "dc_leaf=512" in ctx.get_tiles()
    for bad in ("casida=128x64", "sigma=32x32", "nope=64x64", "sigma_target=7", "mo1",
                "persistent=9", "dc_leaf=8", "dc_leaf=50000", "panel_coop=2"):
        with pytest.raises(q.QsgwError):
            ctx.set_tiles(bad)
    ctx.set_tiles("")
    assert ctx.get_tiles() == default


@pytest.mark.parametrize("spec", TABLES)
@pytest.mark.parametrize("precision", [0, 1])
def test_tables_keep_parity(env, spec, precision):
    q, ctx, stream, p, B, C0, e0, hd, eps1 = env
    ctx.set_tiles(spec)
    try:
        with torch.cuda.stream(stream):
            e, C = e0.clone(), C0.clone()
            q.qsgw_iterate(ctx, B, hd, p.nocc, e, C, 1e-3, tol=0.0, max_iter=1, precision=precision)
            mols = [dict(B_ao=B, h=hd, nocc=p.nocc, eps=e0.clone(), C=C0.clone())]
            q.qsgw_iterate_batched(ctx, mols, 1e-3, tol=0.0, max_iter=1, precision=precision)
        stream.synchronize()
    finally:
        ctx.set_tiles(None)
    err = np.max(np.abs(e.cpu().numpy() - eps1))
    errb = np.max(np.abs(mols[0]["eps"].cpu().numpy() - e.cpu().numpy()))
    print(f"{spec} precision {precision}: oracle {err:.2e}, batched {errb:.2e}", flush=True)
    if precision == 0:
        assert err <= 1e-8
    else:
        assert err <= 1.0 / 27211.386  # FP32 products: the 1 meV gate
    assert errb <= 1e-8
