"""Exhaustive autotuner and cost-model trainer.

    python -m paper_2310_03983_amd.autotune sweep --db timings.json [--first G0 --last G1]
    python -m paper_2310_03983_amd.autotune retime --db timings.json --candidates 6 --max-n 2048
    python -m paper_2310_03983_amd.autotune train --db timings.json --model model.json
    python -m paper_2310_03983_amd.autotune evaluate --db timings.json --model model.json
    python -m paper_2310_03983_amd.autotune batch --db batch_timings.json
    python -m paper_2310_03983_amd.autotune select-joint --db timings.json --batch-db batch_timings.json
    python -m paper_2310_03983_amd.autotune train-joint --db timings.json --batch-db batch_timings.json --model m.json
    python -m paper_2310_03983_amd.autotune evaluate-joint --db timings.json --batch-db batch_timings.json --model m.json
    python -m paper_2310_03983_amd.autotune export --model model.json --out model.txt

`sweep` times every candidate plan of the library (apsp_candidate) on every
graph of the 200-graph sweep workload (n log-uniform in [64, 32768], p
log-uniform in [5e-4, 0.5], half of them chained to be weakly connected),
with HIP events around each solve on a fresh copy of the input, and appends
the medians to a JSON timing database (resumable: graphs already timed with
the same candidate table are skipped).  Every candidate's result is compared
bit for bit with the first candidate's; disagreement is recorded.

`train` fits the cost-model MLP on the GPU through apsp_costmodel_train:
inputs are the four plan features, targets the log run times of the
candidates, standardised with one global mean/deviation (so the per-row
argmin is unchanged).  `evaluate` reports, on held-out graphs, the regret
t(pick)/t(best) - 1 of the model's pick against exhaustive tuning, next to
the best single static candidate and the library's size rule.

`batch` times every batch candidate of apsp_batched (lock-step, the queue
schedule with whole tiles, sub-tiles above n = 128 or 256, 64-wide rounds
above n = 384, the persistent kernel) on the 160 batches of the batch sweep
(graph count, size range and density varied), checks that they agree, and
stores the medians; `train-joint` fits one model whose outputs score the
single-graph candidates and the batch candidates (masked targets), and
`evaluate-joint` reports both regrets on held-out graphs and batches.
`export` writes a trained model in the text format of apsp_costmodel_load.
At run time `choose` plans one graph: the installed model's pick, or
exhaustive tuning of that graph when no matching model is installed.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import graphgen as gg

DB_VERSION = 1


# ---------------------------------------------------------------------------
# plan features
# ---------------------------------------------------------------------------

def weakly_connected(W: np.ndarray, inf=gg.INF_I32, chunk_rows: int = 1024) -> bool:
    """True when the graph is connected ignoring edge directions; edges are
    merged a row chunk at a time and the scan stops once one component is
    left."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    n = W.shape[0]
    if n <= 1:
        return True
    labels = np.arange(n)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        blk = W[r0:r1]
        ii, jj = np.nonzero((blk < inf) if np.issubdtype(blk.dtype, np.integer) else np.isfinite(blk))
        a = labels[ii + r0]
        b = labels[jj]
        keep = a != b
        if not keep.any():
            continue
        a, b = a[keep], b[keep]
        g = coo_matrix((np.ones(a.size, np.int8), (a, b)), shape=(n, n))
        _, comp = connected_components(g, directed=True, connection="weak")
        labels = comp[labels]
        if np.unique(labels).size == 1:
            return True
    return np.unique(labels).size == 1


def features(W: np.ndarray, batch: int = 1) -> list[float]:
    """(log2 n, log10 density, log2 batch, weakly connected) of one graph."""
    n = W.shape[0]
    if np.issubdtype(W.dtype, np.integer):
        m = int(np.count_nonzero(W < gg.INF_I32)) - n
    else:
        m = int(np.count_nonzero(np.isfinite(W))) - n
    dens = m / max(1, n * (n - 1))
    return [math.log2(max(n, 1)), math.log10(max(dens, 1e-9)), math.log2(max(batch, 1)),
            1.0 if weakly_connected(W) else 0.0]


# ---------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------

def candidate_table(apsp):
    out = []
    for i in range(apsp.apsp_candidate_count()):
        o = apsp.apsp_candidate(i)
        out.append({"algo": o.algo, "block": o.block, "tile": o.tile, "closure": o.closure, "cutover": o.cutover,
                    "flags": o.flags})
    return out


def time_candidate(torch, apsp, Wd, opts, budget_s=0.3, max_reps=15):
    """Median seconds of apsp_solve(opts) on fresh copies of Wd; returns
    (median, result of the last run).  Small problems get one untimed
    warm-up; large ones (n >= 8192, seconds per solve) time every run."""
    D = Wd.clone()
    if Wd.shape[0] < 8192:
        apsp.apsp_solve(D, opts=opts)
        torch.cuda.synchronize()
    times = []
    while True:
        D.copy_(Wd)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        apsp.apsp_solve(D, opts=opts)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
        if len(times) >= max_reps or (len(times) >= 2 and sum(times) >= budget_s):
            break
    return float(np.median(times)), D


def load_db(path):
    if path and os.path.exists(path):
        with open(path) as f:
            db = json.load(f)
        if db.get("version") == DB_VERSION:
            return db
    return {"version": DB_VERSION, "records": {}}


def save_db(db, path):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=0)
    os.replace(tmp, path)


def sweep(db_path, first=0, last=199, progress=print):
    import torch
    from . import apsp
    dev = torch.device("cuda:0")
    db = load_db(db_path)
    cands = candidate_table(apsp)
    if db.get("candidates") not in (None, cands):
        db = {"version": DB_VERSION, "records": {}}
    db["candidates"] = cands
    db["device"] = torch.cuda.get_device_name(0)
    graphs = gg.sweep()
    for sg in graphs[first:last + 1]:
        key = str(sg.g)
        if key in db["records"]:
            continue
        t0 = time.time()
        W = gg.sweep_graph_i32(sg)
        feats = features(W)
        Wd = torch.from_numpy(W).to(dev)
        del W
        times, agree, ref = [], True, None
        for i in range(len(cands)):
            t, D = time_candidate(torch, apsp, Wd, apsp.apsp_candidate(i))
            times.append(t)
            if ref is None:
                ref = D
            else:
                agree = agree and bool(torch.equal(ref, D))
                del D
        db["records"][key] = {"g": sg.g, "n": sg.n, "p": sg.p, "chain": sg.chain, "features": feats,
                              "times": times, "agree": agree}
        save_db(db, db_path)
        best = int(np.argmin(times))
        progress(f"[autotune] graph {sg.g} n={sg.n} p={sg.p:.2e} best={best} "
                 f"t={times[best] * 1e3:.2f} ms agree={agree} ({time.time() - t0:.1f} s)")
        del Wd, ref
        torch.cuda.empty_cache()
    return db


def retime(db_path, candidates, max_n, progress=print):
    """Times the listed candidates again on every recorded sweep graph with
    n <= max_n (after a change to their kernels) and replaces their entries;
    each new result is compared bit for bit with candidate 0's."""
    import torch
    from . import apsp
    dev = torch.device("cuda:0")
    db = load_db(db_path)
    if db.get("candidates") != candidate_table(apsp):
        raise ValueError("the database was taken with another candidate table")
    graphs = {sg.g: sg for sg in gg.sweep()}
    for key, rec in sorted(db["records"].items(), key=lambda kv: int(kv[0])):
        if rec["n"] > max_n:
            continue
        W = gg.sweep_graph_i32(graphs[int(key)])
        Wd = torch.from_numpy(W).to(dev)
        _, ref = time_candidate(torch, apsp, Wd, apsp.apsp_candidate(0))
        for i in candidates:
            t, D = time_candidate(torch, apsp, Wd, apsp.apsp_candidate(i))
            rec["times"][i] = t
            rec["agree"] = bool(rec["agree"] and torch.equal(ref, D))
        save_db(db, db_path)
        progress(f"[autotune] graph {key} n={rec['n']} retimed {candidates}: "
                 f"{[round(rec['times'][i] * 1e3, 3) for i in candidates]} ms agree={rec['agree']}")
        del Wd, ref
    return db


# ---------------------------------------------------------------------------
# batched plans
# ---------------------------------------------------------------------------

# batches the joint model trains on, and the held-out ones it is scored on
BATCH_TRAIN = list(range(120)) + list(range(160, 200))
BATCH_TEST = list(range(120, 160))


def batch_candidate_table(apsp):
    out = []
    for i in range(apsp.apsp_batch_candidate_count()):
        o = apsp.apsp_batch_candidate(i)
        out.append({"flags": o.flags, "block": o.block, "tile": o.tile, "split": o.reserved[0]})
    return out


def batch_features(mats) -> list[float]:
    """The batch planner's inputs (as apsp_plan_batch computes them): log2
    of the largest n, log10 density over the batch, log2 of the count, and
    the share of the work (sum of n^3) in graphs with n > 256."""
    ns = np.array([m.shape[0] for m in mats], dtype=np.float64)
    edges = sum(int(np.count_nonzero(m < gg.INF_I32)) - m.shape[0] for m in mats)
    pairs = float((ns * np.maximum(ns - 1, 0)).sum())
    w = ns ** 3
    dens = edges / pairs if pairs > 0 else 0.0
    return [math.log2(max(ns.max(), 1)), math.log10(max(dens, 1e-9)), math.log2(max(len(mats), 1)),
            float(w[ns > 256].sum() / w.sum()) if w.sum() > 0 else 0.0]


def time_batch(torch, apsp, flat_d, off_d, sz_d, hs, opts, reps):
    """Median milliseconds of apsp_batched(opts) (HIP events around each
    call; the input restored before every call) and the last result."""
    work = flat_d.clone()
    apsp.apsp_batched(work, off_d, sz_d, hs, opts=opts)   # plan, capture
    ts = []
    for _ in range(reps):
        work.copy_(flat_d)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        apsp.apsp_batched(work, off_d, sz_d, hs, opts=opts)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), work


def sweep_batches(db_path, first=0, last=199, reps=7, progress=print):
    """Times every batch candidate of apsp_batched on the batch sweep
    (graphgen.batch_sweep) and appends the medians to a JSON database
    (resumable); every candidate's distances are compared bit for bit with
    the first candidate's."""
    import torch
    from . import apsp
    dev = torch.device("cuda:0")
    db = load_db(db_path)
    cands = batch_candidate_table(apsp)
    if db.get("candidates") not in (None, cands):
        db = {"version": DB_VERSION, "records": {}}
    db["candidates"] = cands
    db["device"] = torch.cuda.get_device_name(0)
    for spec in gg.batch_sweep()[first:last + 1]:
        key = str(spec.b)
        if key in db["records"]:
            continue
        t0 = time.time()
        mats = [gg.batch_graph_i32(g) for g in spec.graphs()]
        feats = batch_features(mats)
        flat, off, sz = gg.pack_batch(mats)
        del mats
        flat_d = torch.from_numpy(flat).to(dev)
        off_d, sz_d = torch.from_numpy(off).to(dev), torch.from_numpy(sz).to(dev)
        hs = sz.tolist()
        times, agree, ref = [], True, None
        for i in range(len(cands)):
            ms, out = time_batch(torch, apsp, flat_d, off_d, sz_d, hs, apsp.apsp_batch_candidate(i), reps)
            times.append(ms)
            if ref is None:
                ref = out
            else:
                agree = agree and bool(torch.equal(ref, out))
            if apsp.apsp_batched_status() != 0:
                agree = False
        db["records"][key] = {"b": spec.b, "count": spec.count, "n_lo": spec.n_lo, "n_hi": spec.n_hi,
                              "p_hi": spec.p_hi, "features": feats, "times": times, "agree": agree}
        save_db(db, db_path)
        best = int(np.argmin(times))
        progress(f"[autotune] batch {spec.b}: {spec.count} graphs n {spec.n_lo}-{spec.n_hi} best={best} "
                 f"({' '.join(f'{t:.3f}' for t in times)} ms) agree={agree} ({time.time() - t0:.1f} s)")
        del flat_d, ref
        torch.cuda.empty_cache()
    return db


# ---------------------------------------------------------------------------
# cost model
# ---------------------------------------------------------------------------

def dataset(db, ids):
    recs = [db["records"][str(g)] for g in ids if str(g) in db["records"]]
    X = np.array([r["features"] for r in recs], dtype=np.float32)
    L = np.log(np.array([r["times"] for r in recs], dtype=np.float64))
    return recs, X, L


def train_joint(db, ids, bdb, bids, steps=4000, lr=3e-3, seed=0):
    """One model for both planners: K = single candidates + batch
    candidates outputs; single-graph rows carry targets for the first ones
    (mask 1) and none for the batch outputs (mask 0), batch rows the other
    way round.  Log times standardised with one mean/deviation over every
    target present (so each row's argmin is unchanged)."""
    import torch
    from . import apsp
    dev = torch.device("cuda:0")
    _, Xs, Ls = dataset(db, ids)
    brecs = [bdb["records"][str(b)] for b in bids if str(b) in bdb["records"]]
    Xb = np.array([r["features"] for r in brecs], dtype=np.float32)
    Lb = np.log(np.array([r["times"] for r in brecs], dtype=np.float64))
    Ks, Kb = Ls.shape[1], Lb.shape[1]
    K = Ks + Kb
    X = np.concatenate([Xs, Xb]).astype(np.float32)
    L = np.zeros((X.shape[0], K))
    M = np.zeros((X.shape[0], K), dtype=np.float32)
    L[:len(Xs), :Ks], M[:len(Xs), :Ks] = Ls, 1.0
    L[len(Xs):, Ks:], M[len(Xs):, Ks:] = Lb, 1.0
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[sd < 1e-6] = 1.0
    present = M > 0
    lmu, lsd = float(L[present].mean()), float(L[present].std() or 1.0)
    T = np.where(present, (L - lmu) / lsd, 0.0).astype(np.float32)
    apsp.apsp_costmodel_init(K, seed)
    apsp.apsp_costmodel_set_norm(mu, sd)
    losses = torch.empty(steps, dtype=torch.float32, device=dev)
    apsp.apsp_costmodel_train(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev),
                              torch.from_numpy(M).to(dev), steps=steps, lr=lr, losses=losses)
    torch.cuda.synchronize()
    h = losses.cpu().numpy()
    return {"version": DB_VERSION, "K": K, "K_single": Ks, "K_batch": Kb, "mu": mu.tolist(), "sd": sd.tolist(),
            "log_mu": lmu, "log_sd": lsd, "params": apsp.apsp_costmodel_get_params(K).tolist(),
            "candidates": db["candidates"], "batch_candidates": bdb["candidates"], "train_ids": list(ids),
            "batch_train_ids": list(bids), "steps": steps, "lr": lr, "seed": seed,
            "loss_first": float(h[0]), "loss_last": float(h[-1])}


def select_joint(db, bdb, grid=((4000, 8000), (3e-3, 1e-3), (0, 1, 2)), progress=print):
    """Training settings of the joint model chosen by validation: each
    (steps, lr, seed) is trained on sweep graphs 0-119 and the batch
    training set without batches 100-119, and scored by the sum of the mean
    regrets on graphs 120-149 and batches 100-119; the best is returned (the
    held-out test graphs 150-199 and batches 120-159 are not looked at)."""
    btr = [b for b in BATCH_TRAIN if not (100 <= b < 120)]
    bval = list(range(100, 120))
    res = []
    for steps in grid[0]:
        for lr in grid[1]:
            for seed in grid[2]:
                m = train_joint(db, list(range(120)), bdb, btr, steps=steps, lr=lr, seed=seed)
                es = evaluate(db, m, list(range(120, 150)), list(range(120)))["mlp"]["mean_regret"]
                eb = evaluate_batches(bdb, m, bval, btr)["mlp"]["mean_regret"]
                res.append((es + eb, steps, lr, seed))
                progress(f"[autotune] steps={steps} lr={lr} seed={seed}: validation regret {es:.4f} + {eb:.4f}")
    _, steps, lr, seed = min(res)
    return {"steps": steps, "lr": lr, "seed": seed}


def forward(model, X):
    """The installed model's outputs for the rows of X (device forward pass)."""
    import torch
    from . import apsp
    install(model)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    out = torch.empty((X.shape[0], model["K"]), dtype=torch.float32, device=dev)
    apsp.apsp_costmodel_forward(Xd, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def evaluate_batches(bdb, model, test_ids, train_ids):
    """Regret on held-out batches of the model's batch pick against
    exhaustive tuning, next to the best static batch candidate, the former
    fixed plan (lock-step, candidate 0) and the library's default candidate."""
    recs = [bdb["records"][str(b)] for b in test_ids if str(b) in bdb["records"]]
    tr = [bdb["records"][str(b)] for b in train_ids if str(b) in bdb["records"]]
    X = np.array([r["features"] for r in recs], dtype=np.float32)
    T = np.array([r["times"] for r in recs], dtype=np.float64)
    Ks = model["K_single"]
    pick = np.argmin(forward(model, X)[:, Ks:], axis=1)
    best = T.min(axis=1)
    Ttr = np.array([r["times"] for r in tr], dtype=np.float64)
    static = int(np.argmin(np.exp(np.log(Ttr / Ttr.min(axis=1, keepdims=True)).mean(axis=0))))

    def stats(choice):
        t = T[np.arange(len(T)), choice]
        reg = t / best - 1.0
        return {"mean_regret": float(reg.mean()), "max_regret": float(reg.max()),
                "geomean_ratio": float(np.exp(np.log1p(reg).mean())), "total_ms": float(t.sum()),
                "exact_picks": int((reg == 0).sum())}

    return {"batches": len(recs), "mlp": stats(pick), "static_best": {"candidate": static, **stats(
        np.full(len(T), static))}, "lockstep": stats(np.zeros(len(T), dtype=int)),
        "default": stats(np.full(len(T), 2)), "exhaustive_total_ms": float(best.sum())}


def train(db, ids, steps=3000, lr=3e-3, seed=0):
    import torch
    from . import apsp
    dev = torch.device("cuda:0")
    recs, X, L = dataset(db, ids)
    K = L.shape[1]
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[sd < 1e-6] = 1.0
    lmu, lsd = float(L.mean()), float(L.std() or 1.0)
    T = ((L - lmu) / lsd).astype(np.float32)
    M = np.ones_like(T)
    apsp.apsp_costmodel_init(K, seed)
    apsp.apsp_costmodel_set_norm(mu, sd)
    losses = torch.empty(steps, dtype=torch.float32, device=dev)
    apsp.apsp_costmodel_train(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev),
                              torch.from_numpy(M).to(dev), steps=steps, lr=lr, losses=losses)
    torch.cuda.synchronize()
    h = losses.cpu().numpy()
    return {"version": DB_VERSION, "K": K, "mu": mu.tolist(), "sd": sd.tolist(), "log_mu": lmu, "log_sd": lsd,
            "params": apsp.apsp_costmodel_get_params(K).tolist(), "candidates": db["candidates"],
            "train_ids": list(ids), "steps": steps, "lr": lr, "seed": seed,
            "loss_first": float(h[0]), "loss_last": float(h[-1])}


def install(model):
    """Loads a trained model into the library context (used by apsp_plan)."""
    from . import apsp
    apsp.apsp_costmodel_init(model["K"], 0)
    apsp.apsp_costmodel_set_norm(model["mu"], model["sd"])
    apsp.apsp_costmodel_set_params(np.asarray(model["params"], dtype=np.float32))


def export_text(model, path):
    """Writes a trained model (the JSON dict of `train`) in the text format
    apsp_costmodel_load reads, so C callers can plan without Python."""
    f32 = lambda v: "%.9g" % float(np.float32(v))
    params = np.asarray(model["params"], dtype=np.float32)
    lines = ["apsp-costmodel 1", f"K {model['K']}", "in 4", "hidden 64",
             "mu " + " ".join(f32(v) for v in model["mu"]), "sd " + " ".join(f32(v) for v in model["sd"]),
             f"params {params.size}"] + [f32(v) for v in params]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def predict(model, X):
    import torch
    from . import apsp
    install(model)
    dev = torch.device("cuda:0")
    ch = torch.empty(X.shape[0], dtype=torch.int32, device=dev)
    apsp.apsp_costmodel_predict(torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev), ch)
    torch.cuda.synchronize()
    return ch.cpu().numpy()


def choose(Wd, exhaustive: bool = False, budget_s: float = 0.3):
    """The plan for one graph already in device memory (square int32 or
    float32 tensor): the installed cost model's pick (apsp_plan on the
    graph's features) unless no model matching the candidate table is
    installed or `exhaustive` is set; then exhaustive tuning, the model's
    fallback: every candidate the dtype can run is timed on copies of the
    graph and the fastest is kept.  Returns (opts, candidate index,
    "model" or "exhaustive", {index: median seconds} or None)."""
    import torch
    from . import apsp
    dtype = "float32" if Wd.dtype == torch.float32 else "int32"
    f = features(Wd.cpu().numpy())
    if not exhaustive:
        o, ch = apsp.apsp_plan(Wd.shape[0], 10.0 ** f[1], 1, bool(f[3]), dtype=dtype)
        if ch >= 0:
            return o, ch, "model", None
    times = {}
    for i in range(apsp.apsp_candidate_count()):
        o = apsp.apsp_candidate(i)
        if dtype == "float32" and o.flags & apsp.FLAG_PACKED16:
            continue
        times[i] = time_candidate(torch, apsp, Wd, o, budget_s=budget_s)[0]
    best = min(times, key=times.get)
    return apsp.apsp_candidate(best), best, "exhaustive", times


def size_rule(n, cands):
    """Index of the candidate the library's size rule runs (blocked FW up to
    n = 4096, R-Kleene with a 4096 FW cutover above)."""
    if n <= 4096:
        want = {"algo": 1, "block": 128, "tile": 0, "closure": 1, "cutover": 0, "flags": 0}
    else:
        want = {"algo": 2, "block": 128, "tile": 0, "closure": 1, "cutover": 4096, "flags": 0}
    for i, c in enumerate(cands):
        if c == want:
            return i
    return 0


def evaluate(db, model, test_ids, train_ids):
    _, Xtr, Ltr = dataset(db, train_ids)
    recs, X, L = dataset(db, test_ids)
    T = np.exp(L)
    best = T.min(axis=1)
    pick = np.argmin(forward(model, X)[:, :L.shape[1]], axis=1)
    # best single static choice on the training graphs (geometric mean of t / t_best)
    tr_ratio = np.exp(Ltr - Ltr.min(axis=1, keepdims=True))
    static = int(np.argmin(np.exp(np.log(tr_ratio).mean(axis=0))))
    rule = np.array([size_rule(r["n"], db["candidates"]) for r in recs])

    def stats(choice):
        reg = T[np.arange(len(T)), choice] / best - 1.0
        tot = T[np.arange(len(T)), choice].sum()
        return {"mean_regret": float(reg.mean()), "max_regret": float(reg.max()),
                "geomean_ratio": float(np.exp(np.log1p(reg).mean())), "total_s": float(tot),
                "exact_picks": int((reg == 0).sum())}

    return {"graphs": len(recs), "mlp": stats(pick), "static_best": {"candidate": static, **stats(
        np.full(len(T), static))}, "size_rule": stats(rule), "exhaustive_total_s": float(best.sum()),
        "exhaustive_tuning_cost_s": float(T.sum())}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["sweep", "retime", "train", "evaluate", "batch", "export", "select-joint",
                                    "train-joint", "evaluate-joint"])
    ap.add_argument("--candidates", default="6", help="retime: comma-separated candidate indices")
    ap.add_argument("--max-n", type=int, default=2048, help="retime: largest n re-timed")
    ap.add_argument("--batch-db", help="batch timing database (batch, train-joint, evaluate-joint)")

    ap.add_argument("--out", help="export: path of the text model file")
    ap.add_argument("--db")
    ap.add_argument("--model")
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--last", type=int, default=199)
    ap.add_argument("--train-count", type=int, default=150)
    ap.add_argument("--steps", type=int, default=None, help="Adam steps (train: 3000; train-joint: 8000)")
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=2, help="train-joint: initialisation seed")
    a = ap.parse_args(argv)
    if a.cmd == "export":
        with open(a.model) as f:
            export_text(json.load(f), a.out)
        return 0
    if not a.db:
        ap.error("--db is required for " + a.cmd)
    if a.cmd == "sweep":
        sweep(a.db, a.first, a.last, progress=lambda m: print(m, flush=True))
        return 0
    if a.cmd == "retime":
        retime(a.db, [int(c) for c in a.candidates.split(",")], a.max_n, progress=lambda m: print(m, flush=True))
        return 0
    if a.cmd == "batch":
        sweep_batches(a.db, a.first, a.last, progress=lambda m: print(m, flush=True))
        return 0
    db = load_db(a.db)
    train_ids = list(range(a.train_count))
    test_ids = list(range(a.train_count, 200))
    if a.cmd in ("select-joint", "train-joint", "evaluate-joint"):
        bdb = load_db(a.batch_db)
        btrain, btest = BATCH_TRAIN, BATCH_TEST
        if a.cmd == "select-joint":
            print(json.dumps(select_joint(db, bdb, progress=lambda m: print(m, flush=True))))
            return 0
        if a.cmd == "train-joint":
            model = train_joint(db, train_ids, bdb, btrain, steps=a.steps or 8000, lr=a.lr, seed=a.seed)
            with open(a.model, "w") as f:
                json.dump(model, f)
            print(json.dumps({k: model[k] for k in ("K", "loss_first", "loss_last", "steps")}))
            return 0
        with open(a.model) as f:
            model = json.load(f)
        print(json.dumps({"single": evaluate(db, model, test_ids, train_ids),
                          "batch": evaluate_batches(bdb, model, btest, btrain)}, indent=1))
        return 0
    if a.cmd == "train":
        model = train(db, train_ids, steps=a.steps or 3000)
        with open(a.model, "w") as f:
            json.dump(model, f)
        print(json.dumps({k: model[k] for k in ("K", "loss_first", "loss_last", "steps")}))
        return 0
    with open(a.model) as f:
        model = json.load(f)
    print(json.dumps(evaluate(db, model, test_ids, train_ids), indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
