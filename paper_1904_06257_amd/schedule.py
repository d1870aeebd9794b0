"""Learned annealing schedule for +-J energy minimisation on random 3-regular
graphs (the optimisation use of the dynamics, section 6): tune the plain
geometric schedule, generate annealing runs with the library, train the
schedule network on the best runs, and compare learned against plain on
held-out instances at equal sweeps.

    python -m paper_1904_06257_amd.schedule train --out weights.npz
    python -m paper_1904_06257_amd.schedule eval --weights weights.npz

Everything that touches the chains or the network goes through libshaken.
Instance seeds: training [10^6, 10^6 + 10^5), validation (choice of the
training round) [5 * 10^6, ...), evaluation [9 * 10^6, 9 * 10^6 + 512) --
disjoint.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import MLP
from . import anneal

TRAIN_SEED0 = 1_000_000
EVAL_SEED0 = 9_000_000
VAL_SEED0 = 5_000_000
SIZES = (4096, 16384, 65536)


def _log(*a):
    print(*a, flush=True)


def instances(seed0, counts):
    """3-regular +-J graphs, lambda = 0; counts[k] instances of SIZES[k]."""
    import synth
    out, seeds = [], []
    s = seed0
    for n, k in zip(SIZES, counts):
        for _ in range(k):
            out.append(synth.oriented_instance(n, 3, s, lam_values=(0.0,), pm_j=True))
            seeds.append(s)
            s += 1
    return out, np.array(seeds)


def tune_geometric(insts, seeds, sweeps, chunk):
    """Grid search of (beta0, beta1, q) on training instances; returns the
    policy with the lowest mean best energy density."""
    grid = [(b0, b1, q) for b0 in (0.1, 0.3) for b1 in (2.0, 4.0, 8.0) for q in (0.5, 1.0, 2.0, 3.5)]
    ns = np.array([g.n for g in insts], dtype=np.float64)
    results = []
    # all grid points in one batch: every instance once per grid point
    big = [g for _ in grid for g in insts]
    bseeds = np.concatenate([seeds for _ in grid])
    per = len(insts)

    class GridPolicy:
        def __call__(self, F, c, n_chunks):
            lb = np.zeros(F.shape[0])
            lq = np.zeros(F.shape[0])
            for k, (b0, b1, q) in enumerate(grid):
                a, b = anneal.GeometricPolicy(b0, b1, q)(F[k * per:(k + 1) * per], c, n_chunks)
                lb[k * per:(k + 1) * per] = a
                lq[k * per:(k + 1) * per] = b
            return lb, lq

    res = anneal.run(big, bseeds, GridPolicy(), sweeps, chunk)
    for k, p in enumerate(grid):
        e = res.best[k * per:(k + 1) * per] / ns
        results.append((float(e.mean()), p))
    results.sort()
    _log("geometric tuning (best 5):", results[:5])
    b0, b1, q = results[0][1]
    return anneal.GeometricPolicy(b0, b1, q), results


def generate(insts, seeds, base, k_sched, sweeps, chunk, seed, scale=1.0, piece=8192):
    """k_sched perturbed schedules per instance, in batches of at most `piece`
    runs (one persistent batch each)."""
    big = [g for g in insts for _ in range(k_sched)]
    bseeds = np.repeat(seeds, k_sched)
    n_chunks = sweeps // chunk
    pol = anneal.PerturbedPolicy(base, len(big), n_chunks, seed, sigma_b=0.12 * scale,
                                 sigma_q=0.15 * scale, q_spread=0.6 * scale)
    t0 = time.perf_counter()
    parts = []
    for a in range(0, len(big), piece):
        b = min(a + piece, len(big))
        parts.append(anneal.run(big[a:b], bseeds[a:b], pol.piece(a, b), sweeps, chunk, replica0=a))
        _log("  runs %d..%d done (%.1f s)" % (a, b, time.perf_counter() - t0))
    res = anneal.RunResult(np.concatenate([r.best for r in parts]), np.concatenate([r.last for r in parts]),
                           [], [], np.concatenate([r.feats for r in parts], axis=1),
                           np.concatenate([r.log_beta for r in parts], axis=1),
                           np.concatenate([r.log_q for r in parts], axis=1),
                           sum(r.seconds for r in parts))
    _log("generated %d runs in %.1f s" % (len(big), time.perf_counter() - t0))
    return res


def dataset(res, insts, k_sched, elite):
    """Rows (features, (log beta, log q)) of the `elite` best schedules of
    every instance (reward-weighted regression with 0/1 weights)."""
    ns = np.repeat(np.array([g.n for g in insts], dtype=np.float64), k_sched)
    e = (res.best / ns).reshape(len(insts), k_sched)
    X, Y = [], []
    for i in range(len(insts)):
        top = np.argsort(e[i], kind="stable")[:elite]
        for j in top:
            r = i * k_sched + j
            X.append(res.feats[:, r, :])
            Y.append(np.stack([res.log_beta[:, r], res.log_q[:, r]], axis=1))
    return np.concatenate(X), np.concatenate(Y)


def train(args):
    import torch
    torch.cuda.set_device(0)
    t_start = time.perf_counter()
    counts = tuple(int(c) for c in args.train_counts.split(","))
    insts, seeds = instances(TRAIN_SEED0, counts)
    _log("training instances:", counts)
    step = max(1, len(insts) // args.tune_instances)
    base, grid_res = tune_geometric(insts[::step], seeds[::step], args.sweeps, args.chunk)
    mlp = MLP()
    mlp.set_params(anneal.init_params(args.seed))
    val_insts, val_seeds = instances(VAL_SEED0, tuple(int(c) for c in args.val_counts.split(",")))
    policy = base
    history = []
    best_params, best_gain = None, -np.inf
    for rnd in range(args.rounds):
        scale = args.noise_decay ** rnd
        res = generate(insts, seeds, policy, args.k_sched, args.sweeps, args.chunk, seed=100 + rnd,
                       scale=scale)
        X, Y = dataset(res, insts, args.k_sched, args.elite)
        _log("round %d (noise scale %.2f): %d rows" % (rnd, scale, X.shape[0]))
        losses = anneal.train_mlp(mlp, X, Y, np.ones(X.shape[0]), args.epochs, 512, args.lr,
                                  seed=rnd, log=None)
        policy = anneal.MLPPolicy(mlp, base)
        # learned vs plain on the validation instances (disjoint from training and evaluation)
        val, _, _ = compare(val_insts, val_seeds, mlp, base, args.sweeps, args.chunk)
        gain = val["all"]["gain_mean"]
        history.append(dict(round=rnd, rows=int(X.shape[0]), final_loss=losses[-1], noise=scale,
                            val_gain_mean=gain, val_win_rate=val["all"]["win_rate"]))
        _log("round %d: loss %.5f, validation gain (plain - learned) %.5f per spin, learned better "
             "on %.0f%%" % (rnd, losses[-1], gain, 100 * val["all"]["win_rate"]))
        if gain > best_gain:
            best_gain, best_params = gain, mlp.params().copy()
    mlp.set_params(best_params)
    P = mlp.params()
    meta = dict(sweeps=args.sweeps, chunk=args.chunk, train_counts=counts, k_sched=args.k_sched,
                elite=args.elite, rounds=args.rounds, epochs=args.epochs, lr=args.lr,
                geometric=dict(beta0=base.beta0, beta1=base.beta1, q=base.q),
                grid=[(e, list(p)) for e, p in grid_res], history=history,
                seconds=time.perf_counter() - t_start)
    np.savez(args.out, params=P, meta=json.dumps(meta))
    _log("saved", args.out, json.dumps(meta)[:400])
    return meta


def load(path):
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    return z["params"].astype(np.float32), meta


def threshold_6_1(inst):
    """max over the vertices of sum_{(x,y) in E^o} |J_xy| + |lambda_x| (the
    reading of Theorem 6.1's condition with the out-half of x)"""
    w = np.bincount(inst.src, weights=np.abs(inst.J.astype(np.float64)), minlength=inst.n)
    lam = np.abs(np.asarray(inst.lam_values, dtype=np.float64))[inst.cls]
    return float((w + lam).max())


def compare(insts, seeds, mlp, geo, sweeps, chunk):
    """Learned and plain schedule on the same instances with the same Philox
    seeds (common random numbers), each run by the library's chunk loop;
    paired statistics per size class."""
    from scipy import stats
    rl = anneal.run_native(insts, seeds, "mlp", sweeps, chunk, geo, mlp=mlp)
    rp = anneal.run_native(insts, seeds, "geometric", sweeps, chunk, geo)
    ns = np.array([g.n for g in insts], dtype=np.float64)
    out = {}
    for n in sorted(set(ns.astype(int))):
        k = ns == n
        el, ep = rl.best[k] / n, rp.best[k] / n
        d = ep - el
        out[str(n)] = dict(instances=int(k.sum()), plain_mean=float(ep.mean()),
                           learned_mean=float(el.mean()), plain_best=float(ep.min()),
                           learned_best=float(el.min()), gain_mean=float(d.mean()),
                           win_rate=float((d > 0).mean()),
                           t_p_one_sided=float(stats.ttest_rel(ep, el, alternative="greater").pvalue)
                           if k.sum() > 1 else None,
                           wilcoxon_p_one_sided=float(stats.wilcoxon(ep, el, alternative="greater").pvalue)
                           if k.sum() > 1 and np.any(d != 0) else None)
    # Theorem 6.1 (minimisers of the pair Hamiltonian on the diagonal) asks
    # for q > max_x (sum over the out-half of |J_xy|) + |lambda_x|: the final
    # q of each run against that threshold of its instance
    thr = np.array([threshold_6_1(g) for g in insts])
    for name, r in (("learned", rl), ("plain", rp)):
        qf = r.q[-1]
        out["theorem_6_1_" + name] = dict(
            q_final_mean=float(qf.mean()), q_final_min=float(qf.min()), q_final_max=float(qf.max()),
            threshold_mean=float(thr.mean()), feasible_fraction=float((qf > thr).mean()),
            per_size={str(n): float((qf[ns == n] > thr[ns == n]).mean()) for n in sorted(set(ns.astype(int)))})
    d_all = (rp.best - rl.best) / ns
    out["all"] = dict(instances=len(insts), gain_mean=float(d_all.mean()),
                      win_rate=float((d_all > 0).mean()),
                      plain_mean=float((rp.best / ns).mean()), learned_mean=float((rl.best / ns).mean()),
                      seconds_learned=rl.seconds, seconds_plain=rp.seconds)
    return out, rl, rp


def evaluate(args):
    import torch
    torch.cuda.set_device(0)
    P, meta = load(args.weights)
    mlp = MLP()
    mlp.set_params(P)
    g = meta["geometric"]
    geo = anneal.GeometricPolicy(g["beta0"], g["beta1"], g["q"])
    counts = tuple(int(c) for c in args.eval_counts.split(","))
    insts, seeds = instances(EVAL_SEED0, counts)
    out, _, _ = compare(insts, seeds, mlp, geo, args.sweeps, args.chunk)
    out["sweeps"] = args.sweeps
    out["geometric"] = g
    _log(json.dumps(out))
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--sweeps", type=int, default=10000)
    t.add_argument("--chunk", type=int, default=250)
    t.add_argument("--train-counts", default="64,64,16")
    t.add_argument("--tune-instances", type=int, default=36)
    t.add_argument("--k-sched", type=int, default=32)
    t.add_argument("--elite", type=int, default=4)
    t.add_argument("--rounds", type=int, default=1)
    t.add_argument("--epochs", type=int, default=150)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--val-counts", default="16,16,4")
    t.add_argument("--noise-decay", type=float, default=0.6)
    t.add_argument("--seed", type=int, default=0)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--sweeps", type=int, default=10000)
    e.add_argument("--chunk", type=int, default=250)
    e.add_argument("--eval-counts", default="171,171,170")
    e.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "train":
        train(args)
    else:
        evaluate(args)


if __name__ == "__main__":
    main()
