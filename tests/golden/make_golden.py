"""Write the stored oracle values for the full-size plain qsGW workload.

Calls only the FP64 oracle and the seeded input generator.  Running the
oracle at N_b = 300, N_aux = 1200, n_occ = 40 (10,400 transitions) takes a
few minutes per iteration on a workstation, too long for a GPU test, so its
trajectory is stored here and the GPU tests compare against the file.

    python tests/golden/make_golden.py cfg2            # writes cfg2_oracle.json
    python tests/golden/make_golden.py cfg2 --perturb  # also records how a
                                                       # 1e-11 Ha start shift grows
    python tests/golden/make_golden.py cfg2 --spread   # also records the distance to
                                                       # the oracle run on P-permuted
                                                       # inputs (pure rounding spread)
    python tests/golden/make_golden.py cfg2 --converge # writes cfg2_converged_oracle.json:
                                                       # the same workload at the paper's
                                                       # broadening (eta = 0.05 Ha) iterated
                                                       # with DIIS to its fixed point
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from qsgw_inputs import CONFIGS, make_config  # noqa: E402

# Off-diagonal entries of V (MO basis of the iteration's input orbitals) that
# are stored for iteration 1, as (m, n) pairs.
V_SAMPLES = [(0, 1), (3, 250), (39, 40), (38, 41), (10, 200), (120, 121),
             (299, 0), (150, 298), (40, 41), (5, 5)]


def input_fingerprint(p):
    return dict(B_sum=float(p.B_ao.sum()), B_abs=float(np.abs(p.B_ao).sum()),
                C_sum=float(p.C0.sum()), eps_sum=float(p.eps0.sum()))


def run(name, perturb, spread):
    c = CONFIGS[name]
    p = make_config(name)
    t0 = time.time()
    h = O.hf_core(p.B_ao, p.C0, p.eps0, p.nocc)
    eps, C, hist = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0, p.nocc, c["eta"],
                                  c["tol"], c["max_iter"], keep=("eps", "Omega", "V"))
    out = dict(config=name, meta=p.meta, eta=c["eta"], tol=c["tol"],
               max_iter=c["max_iter"], fingerprint=input_fingerprint(p),
               h_fingerprint=dict(trace=float(np.trace(h)), fro=float(np.linalg.norm(h))),
               iterations=[])
    for j, r in enumerate(hist):
        rec = dict(max_deps=r["max_deps"], eps=r["eps"].tolist(),
                   Omega_low=r["Omega"][:32].tolist(), Omega_high=r["Omega"][-8:].tolist(),
                   Omega_sum=float(r["Omega"].sum()),
                   V_diag=np.diag(r["V"]).tolist(),
                   V_samples=[[m, n, float(r["V"][m, n])] for m, n in V_SAMPLES],
                   V_fro=float(np.linalg.norm(r["V"])))
        out["iterations"].append(rec)
        print(f"iteration {j + 1}: max|deps| = {r['max_deps']:.3e}", flush=True)
    out["oracle_seconds"] = time.time() - t0
    if spread:
        # Exact symmetry of the method: a permutation of the auxiliary index P.
        # Every P-contraction sums in a different order, so the two oracle
        # trajectories differ only by FP64 rounding: their distance is the
        # intrinsic rounding spread of this workload, iteration by iteration.
        perm = np.random.default_rng(123).permutation(p.naux)
        Bp = np.ascontiguousarray(p.B_ao[perm])
        hp = O.hf_core(Bp, p.C0, p.eps0, p.nocc)
        _, _, hist3 = O.qsgw_iterate(Bp, hp, p.C0, p.eps0, p.nocc, c["eta"], 0.0, c["max_iter"],
                                     keep=("eps",))
        out["reorder_spread"] = [float(np.max(np.abs(a["eps"] - b["eps"])))
                                 for a, b in zip(hist, hist3)]
        print("rounding spread", out["reorder_spread"], flush=True)
    if perturb:
        _, _, hist2 = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0 + 1e-11, p.nocc, c["eta"],
                                     0.0, c["max_iter"], keep=("eps",))
        out["sensitivity_1e-11"] = [float(np.max(np.abs(a["eps"] - b["eps"])))
                                    for a, b in zip(hist, hist2)]
        print("sensitivity", out["sensitivity_1e-11"], flush=True)
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


# The converged reference: eta of the paper's own qsGW runs, DIIS on the Fock
# matrix with 8 stored pairs, iterated until max|d eps| < 1e-10 Ha.
CONVERGE = dict(eta=0.05, diis=8, tol=1e-10, max_iter=40)


def run_converge(name):
    p = make_config(name)
    t0 = time.time()
    h = O.hf_core(p.B_ao, p.C0, p.eps0, p.nocc)
    cv = CONVERGE
    eps, C, hist = O.qsgw_iterate(p.B_ao, h, p.C0, p.eps0, p.nocc, cv["eta"], cv["tol"],
                                  cv["max_iter"], keep=("eps", "diis_err"), diis=cv["diis"])
    out = dict(config=name, meta=p.meta, **cv, fingerprint=input_fingerprint(p),
               iterations=[dict(max_deps=r["max_deps"], diis_err=r["diis_err"],
                                eps=r["eps"].tolist() if j < 3 else None)
                           for j, r in enumerate(hist)],
               converged=bool(hist[-1]["max_deps"] < cv["tol"]), eps=eps.tolist())
    for j, r in enumerate(hist):
        print(f"iteration {j + 1}: max|deps| = {r['max_deps']:.3e}", flush=True)
    out["oracle_seconds"] = time.time() - t0
    path = os.path.join(HERE, f"{name}_converged_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    if "--converge" in sys.argv:
        run_converge(sys.argv[1])
    else:
        run(sys.argv[1] if len(sys.argv) > 1 else "cfg2", "--perturb" in sys.argv,
            "--spread" in sys.argv)
