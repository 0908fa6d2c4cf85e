"""Tile-shape autotuner for the products of one qsGW iteration.

For a workload it times each tunable product (libqsgw's tile table, see
qsgw_set_tiles) under every shape the product allows, and the K-split targets
of the split products, by coordinate descent from the default table: one key
at a time, every candidate value with the other keys at their best so far,
the median of `reps` iterations of that product's own HIP-event time.  A
candidate whose orbital energies leave those of the default table by more
than a rounding-order difference (1e-10 Ha for FP64, a tenth of the 1 meV
gate for the reduced precisions) is dropped.  The fastest table per workload
goes to tiles.json next to this file, which bench.py applies to its workload.

    python -m paper_2210_17093_amd.tune cfg2 cfg2:fp32 cfg2:bf16x3 cfg3 cfg4 [--reps 3]

A workload name may carry the variant (":fp32" for the FP32 matrix-core
products, ":bf16x3" for the split-BF16 ones); the batched workload is tuned
in its FP32 variant.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import qsgw as q

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tiles.json")

# key -> (candidate values, kernels whose time decides)
CANDIDATES = {
    "mo1": (["128x64", "64x64", "128x128"], ["mo_transform_1"]),
    "mo2": (["64x64", "128x128"], ["mo_transform_2"]),
    "casida": (["128x128", "64x64"], ["casida"]),
    "rho": (["128x128", "128x64", "64x64"], ["residue_rho"]),
    "rho_target": ([2048, 1024, 4096], ["residue_rho"]),
    # the qsGW product's tile shape and K-split target interact (small tiles
    # pay off only with many splits): they are searched jointly
    "sigma+sigma_target": ([f"{sh}+{tg}" for sh in ("64x64", "128x64", "128x128")
                            for tg in (4096, 16384, 32768, 65536, 131072)],
                           ["sigma_qs_gemm", "sigma_qs_reduce"]),
    "exchange": (["64x64", "128x128"], ["fock"]),
    "persistent": ([0, 2, 4], ["mo_transform_1", "mo_transform_2", "casida", "residue_rho",
                               "residue_w", "sigma_qs_gemm", "fock"]),
}
DEFAULTS = {"mo1": "128x64", "mo2": "64x64", "casida": "128x128", "rho": "128x128",
            "rho_target": 2048, "sigma": "64x64", "sigma_target": 4096, "exchange": "64x64",
            "persistent": 0}


def spec_of(table):
    return ",".join(f"{k}={v}" for k, v in table.items())


def assign(table, key, value):
    """Set one candidate: a joint key "a+b" takes a value "x+y"."""
    if "+" in key:
        for k, v in zip(key.split("+"), str(value).split("+")):
            table[k] = v
    else:
        table[key] = value


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def single_timer(name, precision):
    """Per-kernel times of one iteration of a single-instance workload."""
    from qsgw_inputs import CONFIGS, make_config
    p = make_config(name)
    eta = CONFIGS[name]["eta"]
    dev = torch.device("cuda:0")
    ctx = q.Context()
    B = torch.from_numpy(p.B_ao).to(dev)
    C0 = torch.from_numpy(p.C0.copy()).to(dev)
    e0 = torch.from_numpy(p.eps0.copy()).to(dev)
    h = q.qsgw_hf_core(ctx, B, C0, e0, p.nocc)
    e, C = torch.empty_like(e0), torch.empty_like(C0)
    solved = [False]

    def once(replay):
        e.copy_(e0)
        C.copy_(C0)
        torch.cuda.synchronize()
        _, rep, _ = q.qsgw_iterate(ctx, B, h, p.nocc, e, C, eta, tol=0.0, max_iter=1,
                                   precision=precision, replay_eig=replay)
        return rep

    def run(spec):
        # The Casida eigensolve is not among the tuned products: after the
        # first solve, iterations replay its eigenpairs (the library checks
        # that the rebuilt Casida matrix is bitwise the solved one; a table
        # whose Casida product rounds differently gets a fresh solve first).
        ctx.set_tiles(spec)
        if solved[0]:
            try:
                rep = once(True)
                return rep["kernel_ms"], e.cpu().numpy()
            except q.QsgwError:
                pass
        once(False)
        solved[0] = True
        rep = once(True)
        return rep["kernel_ms"], e.cpu().numpy()
    return ctx, run


def batched_timer(name):
    """Per-kernel times of one eager batched iteration (the 256-molecule
    workload of bench.py --config cfg4)."""
    from qsgw_inputs import batch_shapes, make_problem
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    ctx = q.Context(stream)
    mols = []
    with torch.cuda.stream(stream):
        for s in batch_shapes():
            p = make_problem(s["nbf"], s["naux"], s["nocc"], s["rank"], s["decay"], s["seed"])
            B = torch.from_numpy(p.B_ao).to(dev)
            C0 = torch.from_numpy(p.C0.copy()).to(dev)
            e0 = torch.from_numpy(p.eps0.copy()).to(dev)
            mols.append(dict(B=B, C0=C0, e0=e0, nocc=p.nocc, h=q.qsgw_hf_core(ctx, B, C0, e0, p.nocc)))
    stream.synchronize()

    def run(spec):
        ctx.set_tiles(spec)
        with torch.cuda.stream(stream):
            runs = [dict(B_ao=m["B"], h=m["h"], nocc=m["nocc"], eps=m["e0"].clone(),
                         C=m["C0"].clone()) for m in mols]
        stream.synchronize()
        with torch.cuda.stream(stream):
            _, reps = q.qsgw_iterate_batched(ctx, runs, 1e-3, tol=0.0, max_iter=1,
                                             precision=q.PREC_FP32)
        stream.synchronize()
        return reps[0]["kernel_ms"], np.concatenate([r["eps"].cpu().numpy() for r in runs])
    return ctx, run


def tune(name, reps=3, timer=None):
    """Coordinate search over CANDIDATES from DEFAULTS for workload `name`
    ("cfg3", "cfg3:fp32", ...).  timer: None (time on the device), or a pair
    (ctx, run) with run(spec) -> (kernel_ms dict, energies) and ctx.close()."""
    base, _, variant = name.partition(":")
    prec = {"fp32": q.PREC_FP32, "bf16x3": q.PREC_SPLIT_BF16}.get(variant, q.PREC_FP64)
    if timer is None:
        timer = batched_timer(base) if base == "cfg4" else single_timer(base, prec)
    ctx, run = timer
    best = dict(DEFAULTS)
    _, eps_ref = run(spec_of(best))  # warm-up, and the default table's energies
    # a tile table changes only the rounding order of the products
    max_dev = 1e-10 if prec == q.PREC_FP64 and base != "cfg4" else 0.1 / 27211.386
    trials = []
    for key, (values, kernels) in CANDIDATES.items():
        if key == "persistent" and base != "cfg4":
            continue  # grouped (batched) products only
        scores = {}
        for v in values:
            table = dict(best)
            assign(table, key, v)
            try:
                outs = [run(spec_of(table)) for _ in range(reps)]
            except q.QsgwError as err:
                log(f"[tune] {name} {key}={v}: {err}")
                continue
            dev = max(float(np.max(np.abs(e - eps_ref))) for _, e in outs)
            if dev > max_dev:
                log(f"[tune] {name} {key}={v}: dropped, energies moved by {dev:.2e} Ha")
                continue
            ts = [sum(km[k] for k in kernels) for km, _ in outs]
            scores[v] = float(np.median(ts))
            trials.append(dict(key=key, value=v, ms=scores[v]))
            log(f"[tune] {name} {key}={v}: {scores[v]:.3f} ms")
        assign(best, key, min(scores, key=scores.get))
    kd = [run(spec_of(DEFAULTS))[0] for _ in range(reps)]
    kb = [run(spec_of(best))[0] for _ in range(reps)]
    default_ms = {k: float(np.median([x[k] for x in kd])) for k in kd[0]}
    best_ms = {k: float(np.median([x[k] for x in kb])) for k in kb[0]}
    ctx.close()
    return dict(spec=spec_of(best), kernel_ms=best_ms, default_kernel_ms=default_ms,
                trials=trials)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+",
                    choices=("cfg1", "cfg2", "cfg3", "cfg1:fp32", "cfg2:fp32", "cfg2:bf16x3",
                             "cfg3:fp32", "cfg3:bf16x3", "cfg4"))
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    table = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            table = json.load(f)
    for name in args.workloads:
        t0 = time.time()
        res = tune(name, args.reps)
        res["seconds"] = round(time.time() - t0, 1)
        res["command"] = "python -m paper_2210_17093_amd.tune " + " ".join(sys.argv[1:])
        table[name] = res
        log(f"[tune] {name}: {res['spec']}")
        with open(args.out, "w") as f:
            json.dump(table, f, indent=1)
    print(json.dumps({k: v["spec"] for k, v in table.items()}))


if __name__ == "__main__":
    main()
