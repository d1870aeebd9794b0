"""Metastability and tunnelling of shaken dynamics on the torus (section 3.2).

Replicas start from the all-minus configuration in a small positive field with
0 < q < lambda < J: all-minus is metastable, all-plus stable.  Theorem 3.2
bounds the tunnelling time tau_{+1} by exp(2 beta (2J + q - lambda + delta))
as beta grows, and Theorem 3.3 names the typical path: after the first spin
flip the chain moves through the set D of configurations whose up-left to
down-right diagonals D_k = {(i, j): i + j - 1 = k mod L} are each of one sign,
the plus diagonals growing one at a time until all-plus.

Every quantity is read from the exact per-full-step (E_J, M) logs of one
persistent batch (one workgroup per replica, spins in LDS), swept in chunks so
that the log space stays bounded.  On the torus the up and right neighbours of
a site of D_k both lie on D_{k+1}, so a configuration of D with diagonal signs
s_k has M = L sum_k s_k and E_J = 2 J L sum_k s_k s_{k+1} = 2 J L (L - 2w), w
the (even) number of sign changes around the ring of diagonals.  These two
congruences, M = -L^2 (mod 2L) and 2 J L^2 - E_J = 0 (mod 8 J L), are
necessary for membership of D; `in_diagonal_set` decides membership exactly
from a configuration.

``python -m paper_1904_06257_amd.metastability`` prints, for the inverse
temperatures of the paper's nucleation experiment (beta in {1.3, 2.3, 3.3,
4.0}, q = 0.1, lambda = 0.15, J = 1), the exit, crossing and tunnelling times
and the mean magnetisation at logarithmically spaced times.
"""
from __future__ import annotations

import argparse
import dataclasses
import math

import numpy as np

from . import Batch, Chain

FIG4_BETAS = (1.3, 2.3, 3.3, 4.0)
FIG4_Q = 0.1
FIG4_LAM = 0.15


def tunnelling_bound(beta, J=1.0, q=FIG4_Q, lam=FIG4_LAM, delta=0.0):
    """exp(2 beta (2J + q - lambda + delta)): Theorem 3.2's time scale"""
    return math.exp(2.0 * beta * (2.0 * J + q - lam + delta))


def diagonal_signature(EJ, M, L, J=1):
    """Per log entry: the necessary conditions for a configuration of D other
    than all-minus and all-plus (see the module docstring)."""
    EJ = np.asarray(EJ, dtype=np.int64)
    M = np.asarray(M, dtype=np.int64)
    n = L * L
    return (((2 * J * n - EJ) % (8 * J * L)) == 0) & (((M + n) % (2 * L)) == 0) & (np.abs(M) != n)


def diagonal_count(M, L):
    """number of plus diagonals of a configuration of D with magnetisation M"""
    return (np.asarray(M, dtype=np.int64) + L * L) // (2 * L)


def in_diagonal_set(spins):
    """exact membership of D: spins[r, c] (row r = j - 1 going up, column
    c = i - 1 going right) is constant on every class (r + c) mod L"""
    a = np.asarray(spins)
    L = a.shape[0]
    r, c = np.indices(a.shape)
    k = (r + c) % L
    for d in range(L):
        v = a[k == d]
        if not np.all(v == v[0]):
            return False
    return True


def make_chains(L, betas, q=FIG4_Q, lam=FIG4_LAM, J=1, seed=1, replica0=0):
    """one all-minus L x L torus chain per entry of betas (replica index =
    replica0 + position)"""
    return [Chain.torus(L, J=J, q=q, beta=float(b), lam_values=[lam], init="all_down", seed=seed,
                        replica=replica0 + r) for r, b in enumerate(betas)]


@dataclasses.dataclass
class TunnelResult:
    L: int
    betas: np.ndarray          # per replica
    steps: int                 # full steps run
    exit_t: np.ndarray         # first t with M != -L^2 (-1: never)
    cross_t: np.ndarray        # first t with M > 0
    plus_t: np.ndarray         # first t with M = +L^2
    diag_steps: np.ndarray     # full steps in [exit_t, plus_t) with the D signature
    window: np.ndarray         # plus_t - exit_t (0 if not reached)
    mid_t: np.ndarray          # first step with the D signature and L // 2 plus diagonals (-1: none)
    monotone: np.ndarray       # diagonal counts along signature steps take the values 1..L-1 in order
                               # (each equal to the previous one or one more)
    times: np.ndarray          # checkpoints of the magnetisation curve
    m_mean: np.ndarray         # [beta index, checkpoint] mean M / L^2 over the replicas of that beta
    m_final: np.ndarray        # per replica, mean M / L^2 over the last `tail` steps
    beta_values: np.ndarray    # distinct betas (rows of m_mean)

    @property
    def diag_fraction(self):
        w = np.maximum(self.window, 1)
        return self.diag_steps / w


def run(L, betas, q=FIG4_Q, lam=FIG4_LAM, J=1, max_steps=10**6, chunk=20000, seed=1,
        stop="plus", tail=1000, n_times=48):
    """Run one replica per entry of `betas` from all-minus until every replica
    has reached all-plus (stop="plus") or crossed to M > 0 (stop="cross"), or
    for max_steps full steps (stop=None or neither reached); returns a
    TunnelResult."""
    betas = np.asarray(betas, dtype=np.float64)
    R = betas.shape[0]
    n = L * L
    chains = make_chains(L, betas, q=q, lam=lam, J=J, seed=seed)
    batch = Batch(chains, strategy="auto", record=True, log_reserve=chunk)
    exit_t = np.full(R, -1, np.int64)
    cross_t = np.full(R, -1, np.int64)
    plus_t = np.full(R, -1, np.int64)
    diag_steps = np.zeros(R, np.int64)
    last_count = np.zeros(R, np.int64)     # diagonal count last seen on a signature step
    monotone = np.ones(R, bool)
    low = np.full(R, L, np.int64)          # smallest and largest count seen
    high = np.zeros(R, np.int64)
    mid_t = np.full(R, -1, np.int64)
    beta_values = np.unique(betas)
    bidx = np.searchsorted(beta_values, betas)
    times = np.unique(np.concatenate([[0], np.geomspace(1, max_steps, n_times).astype(np.int64)]))
    m_sum = np.zeros((beta_values.shape[0], times.shape[0]))
    m_cnt = np.zeros_like(m_sum)
    m_tail = [np.zeros(0) for _ in range(R)]
    t0 = 0
    try:
        while t0 < max_steps:
            steps = min(chunk, max_steps - t0)
            batch.sweep(steps)
            sel = (times >= t0) & (times <= t0 + steps)
            _, M_all, EJ_all = batch.logs()        # entries t0 .. t0 + steps of every replica
            for i in range(R):
                EJ, M = EJ_all[i], M_all[i]
                t = np.arange(t0, t0 + steps + 1)
                if exit_t[i] < 0:
                    hit = np.nonzero(M != -n)[0]
                    if hit.size:
                        exit_t[i] = t[hit[0]]
                if cross_t[i] < 0:
                    hit = np.nonzero(M > 0)[0]
                    if hit.size:
                        cross_t[i] = t[hit[0]]
                start = t0 if t0 == 0 else t0 + 1    # entry t0 was read with the last chunk
                lo = start - t0
                if exit_t[i] >= 0:
                    end = plus_t[i] if plus_t[i] >= 0 else t0 + steps + 1
                    a, b = max(lo, exit_t[i] - t0), end - t0
                    if b > a:
                        sig = diagonal_signature(EJ[a:b], M[a:b], L, J)
                        # the all-plus hit ends the window
                        hitp = np.nonzero(M[a:b] == n)[0]
                        if hitp.size:
                            b = a + hitp[0]
                            plus_t[i] = t0 + b
                            sig = sig[:hitp[0]]
                        diag_steps[i] += int(sig.sum())
                        if mid_t[i] < 0:
                            w = np.nonzero(sig & (diagonal_count(M[a:b], L) == L // 2))[0]
                            if w.size:
                                mid_t[i] = t0 + a + w[0]
                        cnt = diagonal_count(M[a:b][sig], L)
                        if cnt.size:
                            # each count equals the previous one or exceeds it by one
                            steps_up = np.diff(np.concatenate([[last_count[i]], cnt]))
                            if np.any((steps_up < 0) | (steps_up > 1)):
                                monotone[i] = False
                            last_count[i] = cnt[-1]
                            low[i] = min(low[i], int(cnt.min()))
                            high[i] = max(high[i], int(cnt.max()))
                if sel.any():
                    m_sum[bidx[i], sel] += M[times[sel] - t0] / n
                    m_cnt[bidx[i], sel] += 1
                m_tail[i] = np.concatenate([m_tail[i], M[lo:] / n])[-tail:]
            t0 += steps
            if stop == "plus" and np.all(plus_t >= 0):
                break
            if stop == "cross" and np.all(cross_t >= 0):
                break
    finally:
        batch.close()
        for c in chains:
            c.close()
    # with steps of 0 or 1 from 0, reaching L - 1 means every count 1..L-1 was taken in order
    monotone &= (low == 1) & (high == L - 1) & (plus_t >= 0)
    keep = times <= t0
    m_final = np.array([x.mean() for x in m_tail])
    window = np.where((plus_t >= 0) & (exit_t >= 0), plus_t - exit_t, 0)
    with np.errstate(invalid="ignore"):
        m_mean = m_sum[:, keep] / m_cnt[:, keep]
    return TunnelResult(L=L, betas=betas, steps=t0, exit_t=exit_t, cross_t=cross_t, plus_t=plus_t,
                        diag_steps=diag_steps, window=window, mid_t=mid_t, monotone=monotone, times=times[keep],
                        m_mean=m_mean, m_final=m_final, beta_values=beta_values)


def _main():
    ap = argparse.ArgumentParser(description="tunnelling from all-minus (section 3.2)")
    ap.add_argument("--L", type=int, default=32)
    ap.add_argument("--replicas", type=int, default=32)
    ap.add_argument("--betas", default=",".join(str(b) for b in FIG4_BETAS))
    ap.add_argument("--max-steps", type=int, default=300_000)
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    betas = [float(b) for b in args.betas.split(",")]
    print("L=%d, q=%g, lambda=%g, J=1, %d replicas per beta, at most %d full steps"
          % (args.L, FIG4_Q, FIG4_LAM, args.replicas, args.max_steps), flush=True)
    rows = []
    print("beta   steps    median exit  median cross  median +1  max +1   bound e^{2b(2J+q-l)}  "
          "in D   D increasing  m_final", flush=True)
    for b in betas:
        res = run(args.L, [b] * args.replicas, max_steps=args.max_steps, seed=args.seed)
        reached = res.plus_t >= 0
        print("%-5g  %7d  %11.0f  %12.0f  %9s  %7s  %20.3g  %5.3f  %12.3f  %.4f"
              % (b, res.steps, np.median(res.exit_t), np.median(res.cross_t),
                 "%d" % np.median(res.plus_t[reached]) if reached.all() else "-",
                 "%d" % res.plus_t.max() if reached.all() else "-", tunnelling_bound(b),
                 np.mean(res.diag_fraction[reached]) if reached.any() else float("nan"),
                 np.mean(res.monotone), np.mean(res.m_final)), flush=True)
        rows.append((b, res.times, res.m_mean[0]))
    print("mean magnetisation M/L^2 at full step t")
    for b, times, m in rows:
        print("beta %g" % b)
        print("  t " + " ".join("%8d" % t for t in times))
        print("  m " + " ".join("%8.4f" % v for v in m))


if __name__ == "__main__":
    _main()
