"""Annealing schedules for the minimisation use of shaken dynamics.

Section 6 of the paper (Theorem 6.1) uses the alternate dynamics as a parallel
minimiser of H: at low temperature the pair law concentrates on the pair
minimisers, which lie on the diagonal when q exceeds every half-neighbourhood
coupling sum.  Here a schedule lowers the temperature and moves q over the run;
the chains themselves are the library's (persistent batch, one workgroup per
graph), with the lowest H of every chain tracked on the device.

Policies map per-chain features to (beta, q) once per chunk of sweeps:
  * ``GeometricPolicy`` -- beta from beta0 to beta1 geometrically, q constant;
  * ``PerturbedPolicy`` -- a geometric base plus a random walk in (log beta,
    log q) (the runs the schedule network is trained on);
  * ``MLPPolicy``       -- the network of the library (BF16/FP32 MFMA kernels)
    maps the features to (log beta, log q).

Two drivers of the chunk loop:
  * ``run_native`` -- the library's own loop (``shaken_batch_run`` with a
    geometric or network schedule): what evaluation and users run;
  * ``run`` -- the same loop written here around any policy, for the
    perturbed schedules the network is trained on.  With ``GeometricPolicy``
    or ``MLPPolicy`` it computes exactly what the library does (same features,
    libm log and exp, same clamps and fallback), which the tests check bit
    for bit.

This module only orchestrates: sampling, thresholds, tracking and the network
all run in libshaken.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import Batch, Chain, MLP, batch_run

NFEAT = 16
# libm log, as the library's clamps
LOG_BETA_RANGE = (math.log(0.05), math.log(20.0))
LOG_Q_RANGE = (math.log(0.05), math.log(8.0))


def graph_stats(inst):
    """(log2 n / 16, mean degree / 4, std of in-degree minus out-degree / 2),
    from integer sums (the differences sum to zero over the vertices), as the
    library computes them"""
    n = inst.n
    deg_in = np.bincount(inst.dst, minlength=n).astype(np.int64)
    deg_out = np.bincount(inst.src, minlength=n).astype(np.int64)
    d = deg_in - deg_out
    return (math.log2(n) / 16.0, float(int((deg_in + deg_out).sum())) / n / 4.0,
            math.sqrt(float(int((d * d).sum())) / n) / 2.0)


def features(stats, frac, e_cur, e_best, n, log_beta, log_q):
    """Feature matrix [chains, 16]: graph statistics, elapsed fraction, current
    and best energy density, previous log beta and log q, a constant 1."""
    F = np.zeros((len(stats), NFEAT), dtype=np.float32)
    F[:, 0:3] = np.asarray(stats, dtype=np.float32)
    F[:, 3] = frac
    F[:, 4] = e_cur / n
    F[:, 5] = e_best / n
    F[:, 6] = log_beta / 3.0
    F[:, 7] = log_q / 3.0
    F[:, 8] = 1.0
    return F


@dataclasses.dataclass
class GeometricPolicy:
    beta0: float
    beta1: float
    q: float

    def at(self, c, n_chunks):
        """(log beta, log q) of chunk c of n_chunks (libm log)"""
        t = (c + 0.5) / n_chunks
        l0, l1 = math.log(self.beta0), math.log(self.beta1)
        return l0 + t * (l1 - l0), math.log(self.q)

    def __call__(self, F, c, n_chunks):
        lb, lq = self.at(c, n_chunks)
        rows = F.shape[0]
        return np.full(rows, lb), np.full(rows, lq)


class PerturbedPolicy:
    """A base policy plus a per-chain random walk in (log beta, log q) and a
    per-chain offset of log q."""

    def __init__(self, base, rows, n_chunks, seed, sigma_b=0.12, sigma_q=0.15, q_spread=0.6):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.base = base
        self.db = np.cumsum(rng.normal(0, sigma_b, (n_chunks, rows)), axis=0)
        self.dq = rng.uniform(-q_spread, q_spread, rows)[None, :] + \
            np.cumsum(rng.normal(0, sigma_q, (n_chunks, rows)), axis=0)

    def __call__(self, F, c, n_chunks):
        lb, lq = self.base(F, c, n_chunks)
        return lb + self.db[c], lq + self.dq[c]

    def piece(self, a, b):
        """The same perturbations restricted to rows [a, b)."""
        p = PerturbedPolicy.__new__(PerturbedPolicy)
        p.base = self.base
        p.db = self.db[:, a:b]
        p.dq = self.dq[:, a:b]
        return p


class MLPPolicy:
    """The network's (log beta, log q) per chain; rows whose output is not
    finite take the geometric schedule `fallback` instead (counted in
    `fallbacks`)."""

    def __init__(self, mlp: MLP, fallback: GeometricPolicy, device="cuda"):
        import torch
        self.mlp = mlp
        self.fallback = fallback
        self.torch = torch
        self.device = device
        self.fallbacks = 0

    def __call__(self, F, c, n_chunks):
        torch = self.torch
        x = torch.from_numpy(np.ascontiguousarray(F)).to(self.device)
        y = torch.empty((F.shape[0], NFEAT), dtype=torch.float32, device=self.device)
        self.mlp.forward(x, y)
        out = y[:, :2].double().cpu().numpy()
        lb, lq = out[:, 0], out[:, 1]
        bad = ~np.isfinite(lb) | ~np.isfinite(lq)
        self.fallbacks += int(bad.sum())
        glb, glq = self.fallback.at(c, n_chunks)
        lb = np.clip(np.where(bad, glb, lb), *LOG_BETA_RANGE)
        lq = np.clip(np.where(bad, glq, lq), *LOG_Q_RANGE)
        return lb, lq


def init_params(seed: int) -> np.ndarray:
    """Random initial parameters of the schedule network (He initialisation of
    the hidden layers, small output layer whose unused rows are zero); the
    output bias starts at (log 1, log 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ni, nh, no = 16, 128, 16
    parts = [rng.normal(0, np.sqrt(2.0 / ni), nh * ni), np.zeros(nh),
             rng.normal(0, np.sqrt(2.0 / nh), nh * nh), np.zeros(nh),
             rng.normal(0, np.sqrt(2.0 / nh), nh * nh), np.zeros(nh)]
    w4 = np.zeros((no, nh))
    w4[:2] = rng.normal(0, 0.1 / np.sqrt(nh), (2, nh))
    parts += [w4.reshape(-1), np.zeros(no)]
    return np.concatenate(parts).astype(np.float32)


@dataclasses.dataclass
class RunResult:
    best: np.ndarray          # lowest H per chain over the run (full-step configurations)
    last: np.ndarray          # H of the final configuration
    best_spins: list          # configuration that reached `best`, per chain
    final_spins: list
    feats: np.ndarray         # [chunks, chains, 16] (None from the library's loop)
    log_beta: np.ndarray      # [chunks, chains] (clamped; exp gives beta)
    log_q: np.ndarray
    seconds: float
    beta: np.ndarray = None   # [chunks, chains]: the beta and q the chains ran
    q: np.ndarray = None
    fallbacks: int = 0


def _exp(a):
    """libm exp elementwise (the library's)"""
    return np.array([math.exp(float(v)) for v in np.ravel(a)], dtype=np.float64).reshape(np.shape(a))


def _chains(instances, seeds, replica0):
    return [Chain.graph(inst.n, inst.src, inst.dst, J=inst.J, q=1.0, beta=0.1, seed=int(seeds[i]),
                        replica=replica0 + i) for i, inst in enumerate(instances)]


def run_native(instances, seeds, schedule, sweeps, chunk, geometric, mlp=None, replica0=0,
               keep_spins=False):
    """Anneal every instance once with the library's chunk loop
    (shaken_batch_run): schedule "geometric" (the GeometricPolicy
    `geometric`) or "mlp" (network `mlp`, `geometric` as its fallback)."""
    import time
    chains = _chains(instances, seeds, replica0)
    t0 = time.perf_counter()
    out = batch_run(chains, sweeps, schedule=schedule, chunk_sweeps=chunk, beta0=geometric.beta0,
                    beta1=geometric.beta1, q=geometric.q, mlp=mlp, strategy="persistent",
                    best_spins=keep_spins)
    secs = time.perf_counter() - t0
    final = [ch.spins() for ch in chains] if keep_spins else []
    for ch in chains:
        ch.close()
    return RunResult(out.H_best, out.H_final, out.best_spins if keep_spins else [], final, None,
                     np.log(out.beta_used), np.log(out.q_used), secs, beta=out.beta_used, q=out.q_used,
                     fallbacks=out.fallbacks)


def run(instances, seeds, policy, sweeps, chunk, replica0=0, keep_spins=False):
    """Anneal every instance (synth.Instance with lambda = 0) once under
    `policy`; chains start from the random state of their seed."""
    import time
    n_chunks = sweeps // chunk
    chains = _chains(instances, seeds, replica0)
    stats = [graph_stats(inst) for inst in instances]
    ns = np.array([inst.n for inst in instances], dtype=np.float64)
    batch = Batch(chains, strategy="persistent", track=True)
    # energy (and configuration) of the starting state: a zero-step sweep
    batch.sweep(0)
    if keep_spins:
        e_cur, e_best, sp = batch.track(best_spins=True)
        offs = np.cumsum([0] + [ch.n for ch in chains])
        best_spins = [sp[offs[i]:offs[i + 1]].copy() for i in range(len(chains))]
    else:
        e_cur, e_best = batch.track()
        best_spins = []
    e_cur = e_cur.astype(np.float64)
    e_best = e_best.astype(np.float64)
    lb_prev = np.zeros(len(chains))
    lq_prev = np.zeros(len(chains))
    feats, lbs, lqs, bs, qs = [], [], [], [], []
    t0 = time.perf_counter()
    for c in range(n_chunks):
        F = features(stats, c / n_chunks, e_cur, e_best, ns, lb_prev, lq_prev)
        lb, lq = policy(F, c, n_chunks)
        lb = np.clip(lb, *LOG_BETA_RANGE)
        lq = np.clip(lq, *LOG_Q_RANGE)
        beta, q = _exp(lb), _exp(lq)
        bs.append(beta)
        qs.append(q)
        batch.set_params(beta, q)
        batch.sweep(chunk)
        if keep_spins:
            hl, hb, sp = batch.track(best_spins=True)
            for i in np.nonzero(hb < e_best)[0]:
                best_spins[i] = sp[offs[i]:offs[i + 1]].copy()
        else:
            hl, hb = batch.track()
        e_best = np.minimum(e_best, hb)
        e_cur = hl.astype(np.float64)
        feats.append(F)
        lbs.append(lb)
        lqs.append(lq)
        lb_prev, lq_prev = lb, lq
    secs = time.perf_counter() - t0
    final = [ch.spins() for ch in chains] if keep_spins else []
    batch.close()
    for ch in chains:
        ch.close()
    return RunResult(e_best, e_cur, best_spins, final, np.array(feats), np.array(lbs),
                     np.array(lqs), secs, beta=np.array(bs), q=np.array(qs),
                     fallbacks=getattr(policy, "fallbacks", 0))


def train_mlp(mlp: MLP, X, Y, w, epochs, batch_rows, lr, seed=0, device="cuda", log=None):
    """Weighted least squares of the network outputs (first two) onto targets,
    Adam on the library's kernels; X [rows, 16], Y [rows, 2], w [rows]."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = X.shape[0]
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)
    T = np.zeros((rows, NFEAT), dtype=np.float32)
    T[:, :2] = Y
    Td = torch.from_numpy(T).to(device)
    Wd = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).to(device)
    yb = torch.empty((batch_rows, NFEAT), dtype=torch.float32, device=device)
    step = 0
    losses = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(rows)).to(device)
        tot = 0.0
        nb = 0
        for s0 in range(0, rows - batch_rows + 1, batch_rows):
            idx = perm[s0:s0 + batch_rows]
            xb = Xd[idx].contiguous()
            tb = Td[idx].contiguous()
            wb = Wd[idx].contiguous()
            mlp.forward(xb, yb)
            loss = mlp.loss_backward(tb, wb)
            step += 1
            mlp.adam(lr, step)
            tot += loss
            nb += 1
        losses.append(tot / max(nb, 1))
        if log:
            log("epoch %d loss %.5f" % (ep, losses[-1]))
    return losses
