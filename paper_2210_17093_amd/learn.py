"""Learned warm start of the qsGW iteration: data, training and evaluation.

Every numerical step runs in libqsgw (batched iterations, per-state features,
network forward/backward/Adam, warm-start orbitals); this module only moves
tensors and keeps the books.

Protocol (one reading of the workload, stated in the design notes):
  * molecules from the batched distribution (N_b ~ U{20..120}, N_aux = 4 N_b,
    n_occ = round(N_b / 6)), training seeds from 100000, held-out test seeds
    from 200000;
  * the plain path: batched iterations from the Hartree-Fock start (eps0, C0)
    at the paper's broadening eta = 0.05 Ha, unmixed, up to MAX_ITER
    iterations; a molecule is converged at the first iteration with
    max|d eps| < TOL;
  * target of state m: eps_m(converged) - eps0_m ("hf") or
    eps_m(converged) - eps_m(after the first plain iteration) ("first");
  * features of state m: qsgw_mlp_features of the plain path's first
    iteration, standardized with training-set statistics;
  * warm start, two readings: "hf" predicts the full shift and starts from
    (eps0 + delta, C0); "first" predicts the shift still left after the plain
    first iteration (the one the features come from) and starts from that
    iteration's energies and orbitals plus delta; both re-sorted.  The
    network runs in BF16 (qsgw_mlp_forward_bf16), trained in FP32;
  * per-state fallback: the warm path's first iteration judges each
    prediction; a state that it moves by more than 10 meV has its prediction
    rejected and follows the plain iteration from there (the iteration itself
    replaces the predicted value), so a bad prediction costs iterations, not
    correctness; a molecule whose warm path does not converge within
    MAX_ITER falls back to the plain path as a whole (its cost adds the
    plain iterations);
  * reported: iterations to TOL with and without the warm start (the warm
    count includes the feature iteration), rejected states, and the
    prediction error against the converged plain result per state.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import qsgw as q

ETA = 0.05
MIX = 1.0
TOL = 1e-5
MAX_ITER = 40
HARTREE_MEV = 27211.386
FALLBACK_HA = 10.0 / HARTREE_MEV
NO_SCALE = (8, 14, 15)  # flags and the constant: not standardized


def _draw(shapes):
    """Synthetic inputs of many small molecules on host threads, one BLAS
    thread each (the small factorizations of the generator stall when every
    call spreads over all cores)."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    from qsgw_inputs import make_problem

    def one(s):
        return make_problem(s["nbf"], s["naux"], s["nocc"], s["rank"], s["decay"], s["seed"])
    with threadpool_limits(1), ThreadPoolExecutor(8) as ex:
        return list(ex.map(one, shapes))


def build_molecules(ctx, stream, shapes, probs=None):
    """Device inputs and the Hartree-Fock core h of each molecule (the
    drawn problems may be passed in when they were drawn ahead)."""
    dev = torch.device("cuda:0")
    mols = []
    if probs is None:
        probs = _draw(shapes)
    with torch.cuda.stream(stream):
        for p in probs:
            B = torch.from_numpy(p.B_ao).to(dev)
            C0 = torch.from_numpy(p.C0.copy()).to(dev)
            e0 = torch.from_numpy(p.eps0.copy()).to(dev)
            h = q.qsgw_hf_core(ctx, B, C0, e0, p.nocc)
            mols.append(dict(nbf=p.nbf, nocc=p.nocc, B=B, C0=C0, e0=e0, h=h))
    stream.synchronize()
    return mols


def iterate(ctx, stream, mols, starts, max_iter, diag=False, graph=True):
    """Batched mixed iterations from the given (eps, C) starts.  Returns the
    run dicts (final energies and orbitals, potential, iteration count, and
    optionally the first iteration's diagonal outputs) and each molecule's
    max|d eps| history."""
    with torch.cuda.stream(stream):
        runs = []
        for m, (e, C) in zip(mols, starts):
            nbf = m["nbf"]
            r = dict(B_ao=m["B"], h=m["h"], nocc=m["nocc"], eps=e.clone(), C=C.clone())
            if MIX != 1.0:
                r["Vc"] = torch.zeros((nbf, nbf), dtype=torch.float64, device=e.device)
            if diag:
                r["diag"] = torch.empty((nbf, 4), dtype=torch.float64, device=e.device)
            runs.append(r)
    stream.synchronize()
    return runs, resume(ctx, stream, runs, max_iter, graph)


CHUNK = 3  # batched iterations per call while some molecule has not met TOL


def resume(ctx, stream, runs, max_iter, graph=True):
    """More batched iterations on existing run dicts (their potential and
    iteration counts carry the mixing state), in calls of CHUNK iterations
    until every molecule has met TOL once or max_iter iterations are done;
    returns each molecule's max|d eps| history."""
    hist = [[] for _ in runs]
    done = 0
    while done < max_iter:
        k = min(CHUNK, max_iter - done)
        with torch.cuda.stream(stream):
            _, reps = q.qsgw_iterate_batched(ctx, runs, ETA, tol=TOL, max_iter=k, graph=graph,
                                             mix=MIX)
        stream.synchronize()
        for h, r in zip(hist, reps):
            h.extend(r["max_deps"])
        done += k
        if all(first_below(h) is not None for h in hist):
            break
    return hist


def first_below(hist, tol=TOL):
    for j, d in enumerate(hist):
        if d < tol:
            return j + 1
    return None


def solve_plain(ctx, stream, mols, batch=256, max_iter=MAX_ITER):
    """Plain path for every molecule: its first iteration (with the diagonal
    outputs, the features' source), the state after it, then the remaining
    iterations; converged energies and iteration counts."""
    out = []
    for b0 in range(0, len(mols), batch):
        sub = mols[b0:b0 + batch]
        runs, h1 = iterate(ctx, stream, sub, [(m["e0"], m["C0"]) for m in sub], 1, diag=True)
        first = [(r["eps"].clone(), r["C"].clone()) for r in runs]
        diags = [r.pop("diag") for r in runs]
        h2 = resume(ctx, stream, runs, max_iter - 1)
        for r, a, b, (e1, C1), d in zip(runs, h1, h2, first, diags):
            h = list(a) + list(b)
            out.append(dict(eps=r["eps"], diag=d, eps1=e1, C1=C1, hist=h, iters=first_below(h)))
    return out


def features(ctx, stream, mols, plain, mean=None, scale=None):
    with torch.cuda.stream(stream):
        X = [q.qsgw_mlp_features(ctx, m["e0"], r["diag"], m["nocc"], mean, scale)
             for m, r in zip(mols, plain)]
        X = torch.cat(X)
    stream.synchronize()
    return X


def standardization(X):
    Xh = X.double().cpu().numpy()
    mean = Xh.mean(axis=0)
    scale = Xh.std(axis=0)
    for k in NO_SCALE:
        mean[k], scale[k] = 0.0, 1.0
    scale[scale < 1e-12] = 1.0
    dev = X.device
    return (torch.tensor(mean, dtype=torch.float32, device=dev),
            torch.tensor(scale, dtype=torch.float32, device=dev))


def init_params(seed):
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (128, 16)) / math.sqrt(16)
    W2 = rng.uniform(-1, 1, (128, 128)) / math.sqrt(128)
    w3 = rng.uniform(-1, 1, 128) / math.sqrt(128)
    p = np.concatenate([W1.ravel(), np.zeros(128), W2.ravel(), np.zeros(128), w3, np.zeros(1)])
    assert p.size == q.MLP_NPARAMS
    return torch.tensor(p, dtype=torch.float32, device="cuda")


def train(ctx, stream, X, T, epochs=150, batch=4096, lr=2e-3, seed=0, log=None):
    """Adam on minibatches (reshuffled each epoch), cosine learning-rate decay.
    Targets are scaled to unit variance for training; returns (params, tscale)."""
    n = X.shape[0]
    tscale = float(T.double().std().item()) or 1.0
    Ts = (T / tscale).contiguous()
    P = init_params(seed)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    L = torch.zeros(1, dtype=torch.float64, device=X.device)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    steps = 0
    total = epochs * ((n + batch - 1) // batch)
    with torch.cuda.stream(stream):
        for ep in range(epochs):
            perm = torch.randperm(n, generator=gen).to(X.device)
            Xp, Tp = X[perm].contiguous(), Ts[perm].contiguous()
            for b0 in range(0, n, batch):
                steps += 1
                rate = 0.5 * lr * (1.0 + math.cos(math.pi * steps / total))
                q.qsgw_mlp_train_step(ctx, P, M, V, steps, rate, Xp[b0:b0 + batch].contiguous(),
                                      Tp[b0:b0 + batch].contiguous(), loss=L)
            if log and (ep % 25 == 0 or ep == epochs - 1):
                stream.synchronize()
                log(f"[learn] epoch {ep + 1}/{epochs}: batch loss {L.item():.4e} (scaled)")
    stream.synchronize()
    return P, tscale


def predict(ctx, stream, P, tscale, X, bf16=True):
    """Predicted shifts (Ha); BF16 inference unless bf16=False."""
    with torch.cuda.stream(stream):
        y = q.qsgw_mlp_forward(ctx, P, X.contiguous(), bf16=bf16) * tscale
    stream.synchronize()
    return y


def evaluate_warm(ctx, stream, name, mols, plain, dhat, sizes, max_iter):
    """Warm path of one reading for a batch of held-out molecules: the first
    warm iteration judges every state's prediction (moved by more than
    10 meV: rejected, the state follows the plain iteration from there), then
    the warm path runs to TOL.  One row per molecule: plain and warm
    iteration counts (the warm cost includes the feature iteration; a warm
    path that does not converge adds the plain path), rejected states and
    the per-state prediction error against the converged plain result."""
    starts = []
    with torch.cuda.stream(stream):
        for m, r, d in zip(mols, plain, torch.split(dhat, sizes)):
            e_base, C_base = (m["e0"], m["C0"]) if name == "hf" else (r["eps1"], r["C1"])
            starts.append(q.qsgw_warm_start(ctx, e_base, C_base, d.contiguous()))
    stream.synchronize()
    runs, h1 = iterate(ctx, stream, mols, starts, 1)
    judged = [(r["eps"] - s0[0]).abs().cpu().numpy() for r, s0 in zip(runs, starts)]
    h2 = resume(ctx, stream, runs, max_iter - 1)
    rows = []
    for m, r, d, a, b, mv, s0 in zip(mols, plain, torch.split(dhat, sizes), h1, h2, judged,
                                     starts):
        h = list(a) + list(b)
        true = None
        start_gap = base_gap = None
        if r["iters"]:
            base = m["e0"] if name == "hf" else r["eps1"]
            true = (r["eps"] - base).double().cpu().numpy()
            # distance of the warm start and of the unshifted start from the fixed point
            start_gap = (s0[0] - r["eps"]).abs().cpu().numpy()
            base_gap = (base - r["eps"]).abs().cpu().numpy()
        state_err = np.abs(d.double().cpu().numpy() - true) if true is not None else None
        rejected = mv > FALLBACK_HA
        warm = first_below(h)
        if warm is not None:
            cost = 1 + warm  # feature iteration + warm path
        elif r["iters"] is not None:
            cost = 1 + max_iter + r["iters"]  # the warm path failed: the plain path too
        else:
            cost = None
        bad = state_err > FALLBACK_HA if state_err is not None else None
        rows.append(dict(plain=r["iters"], warm=warm, cost=cost, rejected=int(rejected.sum()),
                         states=int(mv.size), err=state_err, start_gap=start_gap,
                         base_gap=base_gap,
                         bad_accepted=int((bad & ~rejected).sum()) if bad is not None else 0,
                         good_rejected=int((~bad & rejected).sum()) if bad is not None else 0))
    return rows


def _gap(rows, key, per_molecule):
    """Median over held-out molecules (per_molecule = np.max: of each
    molecule's largest state distance) or over all states (np.median), meV."""
    vals = [x[key] for x in rows if x[key] is not None]
    if not vals:
        return None
    if per_molecule is np.median:
        return float(np.median(np.concatenate(vals)) * HARTREE_MEV)
    return float(np.median([per_molecule(v) for v in vals]) * HARTREE_MEV)


def run(n_train=1024, n_test=256, epochs=150, max_iter=MAX_ITER, log=print):
    """Full protocol; returns a dict of results."""
    from qsgw_inputs import batch_shapes
    stream = torch.cuda.Stream()
    ctx = q.Context(stream)
    t0 = time.perf_counter()
    res = dict(eta=ETA, mix=MIX, tol=TOL, max_iter=max_iter, n_train=n_train, n_test=n_test)
    tr_shapes = batch_shapes(nmol=n_train, seed=5, base_seed=100000)
    te_shapes = batch_shapes(nmol=n_test, seed=6, base_seed=200000)
    # two readings of the warm start: from the Hartree-Fock start with the
    # full shift ("hf"), or from the plain first iteration's state with the
    # remaining shift ("first"); targets per state index (energies sorted)
    X_tr, T_tr = [], {"hf": [], "first": []}
    conv_tr = 0
    from concurrent.futures import ThreadPoolExecutor
    ahead = ThreadPoolExecutor(1)  # draws the next batch's inputs while this one is solved
    nxt = ahead.submit(_draw, tr_shapes[0:256])
    for b0 in range(0, n_train, 256):
        probs = nxt.result()
        if b0 + 256 < n_train:
            nxt = ahead.submit(_draw, tr_shapes[b0 + 256:b0 + 512])
        mols = build_molecules(ctx, stream, tr_shapes[b0:b0 + 256], probs)
        plain = solve_plain(ctx, stream, mols, max_iter=max_iter)
        X = features(ctx, stream, mols, plain)
        for m, r, xs in zip(mols, plain, torch.split(X, [m["nbf"] for m in mols])):
            if r["iters"] is None:
                continue
            conv_tr += 1
            X_tr.append(xs)
            T_tr["hf"].append((r["eps"] - m["e0"]).float())
            T_tr["first"].append((r["eps"] - r["eps1"]).float())
        log(f"[learn] training molecules {b0 + len(mols)}/{n_train} solved, "
            f"{conv_tr} converged ({time.perf_counter() - t0:.0f} s)")
        del mols, plain, X, probs
    ahead.shutdown()
    X_tr = torch.cat(X_tr)
    mean, scale = standardization(X_tr)
    Xs = ((X_tr - mean) / scale).contiguous()
    t1 = time.perf_counter()
    nets = {k: train(ctx, stream, Xs, torch.cat(v), epochs=epochs, log=log) for k, v in T_tr.items()}
    res["train_seconds"] = time.perf_counter() - t1
    res["train_states"] = int(X_tr.shape[0])
    res["train_molecules_converged"] = conv_tr
    # held-out molecules, in batches of 256: plain, then each warm reading
    rows_by = {name: [] for name in nets}
    bf16_dev = {name: 0.0 for name in nets}
    res["test_converged_plain"] = 0
    for b0 in range(0, n_test, 256):
        mols = build_molecules(ctx, stream, te_shapes[b0:b0 + 256])
        plain = solve_plain(ctx, stream, mols, max_iter=max_iter)
        X = features(ctx, stream, mols, plain, mean, scale)
        sizes = [m["nbf"] for m in mols]
        res["test_converged_plain"] += sum(r["iters"] is not None for r in plain)
        for name, (P, tscale) in nets.items():
            dhat = predict(ctx, stream, P, tscale, X)
            d32 = predict(ctx, stream, P, tscale, X, bf16=False)
            bf16_dev[name] = max(bf16_dev[name], float((dhat - d32).abs().max().item()))
            rows_by[name].extend(evaluate_warm(ctx, stream, name, mols, plain, dhat, sizes,
                                               max_iter))
        log(f"[learn] held-out molecules {b0 + len(mols)}/{n_test} evaluated "
            f"({time.perf_counter() - t0:.0f} s)")
        del mols, plain, X
    res["variants"] = {}
    for name, rows in rows_by.items():
        both = [x for x in rows if x["plain"] is not None and x["cost"] is not None]
        errs = [x["err"] for x in rows if x["err"] is not None]
        errs = np.concatenate(errs) if errs else np.zeros(0)
        res["variants"][name] = dict(
            compared=len(both),
            plain_mean_iterations=float(np.mean([x["plain"] for x in both])) if both else None,
            warm_mean_iterations=float(np.mean([x["cost"] for x in both])) if both else None,
            molecules_faster=sum(x["cost"] < x["plain"] for x in both),
            molecules_slower=sum(x["cost"] > x["plain"] for x in both),
            warm_not_converged=sum(x["warm"] is None for x in rows),
            states=sum(x["states"] for x in rows),
            states_rejected=sum(x["rejected"] for x in rows),
            states_bad_accepted=sum(x["bad_accepted"] for x in rows),
            states_good_rejected=sum(x["good_rejected"] for x in rows),
            prediction_err_meV_median=float(np.median(errs) * HARTREE_MEV) if errs.size else None,
            prediction_err_meV_p90=float(np.percentile(errs, 90) * HARTREE_MEV) if errs.size else None,
            prediction_within_10meV=float(np.mean(errs <= FALLBACK_HA)) if errs.size else None,
            bf16_vs_fp32_inference_max_meV=bf16_dev[name] * HARTREE_MEV,
            # distance to the converged energies of the warm start and of the
            # unshifted start (Hartree-Fock or first iteration): per state, and
            # the largest state of each molecule
            start_gap_state_meV_median=_gap(rows, "start_gap", np.median),
            unshifted_gap_state_meV_median=_gap(rows, "base_gap", np.median),
            start_gap_molecule_max_meV_median=_gap(rows, "start_gap", np.max),
            unshifted_gap_molecule_max_meV_median=_gap(rows, "base_gap", np.max))
        log(f"[learn] warm start '{name}': {res['variants'][name]}")
    best = "first"  # the reading reported as the result; both are listed
    res["reported"] = best
    res["plain_mean_iterations"] = res["variants"][best]["plain_mean_iterations"]
    res["warm_mean_iterations"] = res["variants"][best]["warm_mean_iterations"]
    res["seconds"] = time.perf_counter() - t0
    ctx.close()
    return res
