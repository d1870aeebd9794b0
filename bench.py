"""Benchmark of the shaken-dynamics hot path on one MI355X.

Default workload (the headline): the 24 runs of the 4096 x 4096 bit-packed
torus -- q in {0.5, 1, 2} x beta in {0.30, 0.40, 0.44, 0.50} x initial state
{all up, random} -- held as 24 chains of one grid batch.  One step is one full
step (half-step dl with the fused observables of the configuration it reads,
then half-step ur) of all 24 chains; sixteen full steps are replayed per
captured HIP graph (captured in the warm-up call), the rest of a call runs
eagerly.  Inputs are resident in device memory before the timed region, and
the timed call is checked to have captured, allocated and tuned nothing.

The default run also times, under ``secondary``, the n = 2^20 random
3-regular +-J graph (CSR, int8 spins), the 2048-chain mixed batch (one
persistent launch per call) and the latency of the schedule network's
forward and backward calls; each graph or batch line has its own roofline and
oracle baseline.

Other workloads (``--workload``, one line each): ``tri4096`` (the same 24
runs on the triangular-lattice torus of section 4), ``graph``, ``batch``,
``ea`` (1024 +-J Edwards-Anderson tori 256^2).

Prints one JSON line: metric, value (site-updates/s), roofline of the
dominant kernel (HIP-event time per launch, algorithmic bytes per launch) and
the CPU oracle timed on a bounded sample of the same workload: one sample
per host core (at most 16), run at once in processes forked before the GPU
is touched, with the single-process rate beside the aggregate.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# --------------------------------------------------------------- constants
# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 39.3e12 full-rate 32-bit
# VALU lane-cycles per second.
VALU_PEAK = 256 * 64 * 2.4e9
HBM_PEAK_GBS = 8000.0
# the share of HBM peak the bit-packed torus is asked to reach
HBM_TARGET_FRAC = 0.60

# Algorithmic ALU work of one bit-packed site-update, in VALU lane-cycles, per
# 32-site word on the folded class table (the workloads' lambda = 0):
#  * levels come in groups of four, one Philox4x32-10 call each; every word
#    takes groups 0 and 1 (levels 0..7), and group g >= 2 where some site is
#    still undecided after 4g levels, DEEP_GROUPS = 0.126 groups per word on
#    average; 40 lane-cycles per call (20 v_mad_u64_u32 + 20 three-input xors,
#    both full rate on gfx950);
#  * levels 0..7 least significant first at `level_top` lane-cycles each
#    (class select, y = tf ^ c, result, agreement); the deeper levels most
#    significant first at `level_deep` (class select, difference, result and
#    undecided);
#  * `planes` lane-cycles of class planes and output per word.
PHILOX_LC = 40.0


def _undecided(levels):
    """P(a 32-site word is still undecided after `levels` levels)."""
    return 1.0 - (1.0 - 2.0 ** -levels) ** 32


DEEP_GROUPS = sum(_undecided(4 * g) for g in range(2, 8))   # 0.126


def _alu_per_site(level_top, level_deep, planes):
    return ((2.0 + DEEP_GROUPS) * PHILOX_LC + 8 * level_top + 4 * DEEP_GROUPS * level_deep
            + planes) / 32.0


# square lattice: select 2 (rest-class words in vector registers), deeper
# levels select 3; planes `one`, `al` and the output: 4.11
BP_ALU_PER_SITE = _alu_per_site(5, 7, 3)
BP_BYTES_PER_SITE = 0.25  # read 1 bit, write 1 bit
# tori in the persistent kernel (LDS-resident): the class select takes 3 at
# every level (no vector-register class words there); +-J couplings: two more
# xors per word flip the neighbour planes by the coupling signs
BP_ALU_PER_SITE_PMJ = _alu_per_site(6, 7, 3) + 2.0 / 32.0
# triangular lattice (three neighbour planes a, b, e, four agreement classes):
# select 4; planes: the diagonal plane e (shift and insert, 2), the agreement
# parity and majority (2 each), the one-hot classes (3), the output (1): 4.85
TRI_ALU_PER_SITE = _alu_per_site(7, 8, 10)


def _code_only(text):
    """Kernel source without comments and blank space: what the hash of the
    measured kernels covers (a comment edit leaves the counters valid)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "batch.hip", "device.hpp", "shaken_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1904_06257_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def read_traffic(kernel_key, per="launch", what="bytes"):
    """HBM bytes (what="bytes") or VALU lane-instructions
    (what="valu_lane_instr") per launch (or per full step) from the committed
    rocprofv3 counter summary, or None if the kernels changed since it was
    taken."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or "=" not in line:
                continue
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():
        return None
    v = vals.get(kernel_key + "." + what + "_per_" + per)
    return float(v) if v else None


def timed_sweep(batch, steps):
    """Wall time of batch.sweep(steps) between two device synchronisations.
    The call must do no host-side set-up (graph capture, log allocation,
    autotuning): that belongs to the warm-up, and the run stops if it
    happened inside the timed region."""
    import torch
    before = batch.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.sweep(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    after = batch.counters()
    for k in ("captures", "log_allocs", "autotunes"):
        if after[k] != before[k]:
            raise SystemExit("bench: the timed call did set-up work (%s %d -> %d)"
                             % (k, before[k], after[k]))
    return wall


# ------------------------------------------------------ oracle baselines
# The oracle as it stands (single-threaded C), timed on the host cores: one
# independent sample per process, all processes at once (forked before this
# process touches the GPU); value = all site-updates / the longest process's
# run time, beside it the median single-process rate.

_BATCH_SPEC = None  # built by the parent before forking, shared by the workers

def _host_cores():
    n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, min(n, 16))


def _oracle_torus_sample(args):
    import oracle
    L, steps, triangular, J, q, beta, seed, rep = args
    if J == "ea":
        J = ea_couplings(L, 10_000 + rep)
    sp = oracle.torus_init_random(L, seed, rep)
    t0 = time.perf_counter()
    oracle.torus_run(sp, J, 0.0, q, beta, seed, rep, steps, log=False, tri=triangular)
    return 2.0 * L * L * steps, time.perf_counter() - t0


def _oracle_graph_sample(args):
    import oracle
    import synth
    kind, steps, rep = args
    if kind == "graph2e20":
        n = 1 << 20
        inst = synth.oriented_instance(n, 3, 3, lam_values=(-0.5, 0.0, 0.5), pm_j=True)
        g = oracle.Graph(n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
        q, beta, seed = 1.5, 0.8, 1 + rep
    else:  # one item of the batch spec
        it = _BATCH_SPEC[kind]
        if it.kind == "torus":
            return _oracle_torus_sample((it.size, steps, False, 1, it.q, it.beta, it.seed, kind))
        gi = it.graph
        n = gi.n
        g = oracle.Graph(gi.n, gi.src, gi.dst, gi.J)
        q, beta, seed = it.q, it.beta, it.seed
    sp = oracle.graph_init_random(n, seed, rep)
    t0 = time.perf_counter()
    oracle.graph_run(g, sp, q, beta, seed, rep, steps, log=False)
    return 2.0 * n * steps, time.perf_counter() - t0


def _run_samples(fn, tasks):
    import multiprocessing as mp
    t0 = time.perf_counter()
    if len(tasks) == 1:
        res = [fn(tasks[0])]
    else:
        with mp.get_context("fork").Pool(len(tasks)) as pool:
            res = pool.map(fn, tasks)
    wall = time.perf_counter() - t0
    work = sum(r[0] for r in res)
    single = sorted(r[0] / r[1] for r in res)[len(res) // 2]
    return work / max(r[1] for r in res), single, wall


def cpu_baseline_torus(triangular=False):
    """Five full steps of one 4096^2 chain per host core (about 10-20 s)."""
    cores = _host_cores()
    tasks = [(4096, 5, triangular, 1, 1.0, 0.44, 2, r) for r in range(cores)]
    value, single, wall = _run_samples(_oracle_torus_sample, tasks)
    lattice = "triangular-lattice torus" if triangular else "torus"
    return {"value": value, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "single_core_value": single,
            "sample": "%d processes, each 5 full steps of its own 4096^2 %s chain (q=1, beta=0.44, "
                      "random init), %.1f s wall" % (cores, lattice, wall)}


def cpu_baseline_graph():
    """100 full steps of the n = 2^20 graph chain per host core (about 10-20 s)."""
    cores = _host_cores()
    value, single, wall = _run_samples(_oracle_graph_sample, [("graph2e20", 100, r) for r in range(cores)])
    return {"value": value, "unit": "vertex-updates/s", "cores": cores, "kind": "oracle",
            "single_core_value": single,
            "sample": "%d processes, each 100 full steps of its own chain of the n=2^20 graph, %.1f s "
                      "wall" % (cores, wall)}


def cpu_baseline_batch():
    """Chains of the 2048-chain batch (lambda = 0, as the batch runs them),
    alternately tori and graphs from the front of the spec, one per host core,
    800 full steps each (about 10 s)."""
    import synth
    global _BATCH_SPEC
    cores = _host_cores()
    spec = _BATCH_SPEC = synth.batch_spec(1024, 1024, seed=4)
    tori = [i for i, it in enumerate(spec) if it.kind == "torus"]
    graphs = [i for i, it in enumerate(spec) if it.kind == "graph"]
    pick = [(tori if k % 2 == 0 else graphs)[k // 2] for k in range(cores)]
    value, single, wall = _run_samples(_oracle_graph_sample, [(i, 800, i) for i in pick])
    return {"value": value, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "single_core_value": single,
            "sample": "%d chains of the batch (tori and graphs alternately), one per process, 800 "
                      "full steps each, %.1f s wall" % (cores, wall)}


def bench_torus4096(args, sk, triangular=False):
    import synth
    L = 4096
    runs = synth.torus_runs()
    make = sk.Chain.triangular if triangular else sk.Chain.torus
    chains = []
    for i, r in enumerate(runs):
        chains.append(make(L, q=r["q"], beta=r["beta"], seed=r["seed"], replica=i, init=r["init"]))
    # log space for the longest call reserved up-front; the HIP graph and the
    # block sizes are made in the warm-up call
    batch = sk.Batch(chains, strategy="grid", use_hipgraph=True, record=True, autotune=True,
                     log_reserve=max(args.steps, args.warmup))
    batch.sweep(args.warmup)
    wall = timed_sweep(batch, args.steps)
    _, ev_ms = batch.info()   # HIP events on the batch stream around the sweep
    n_chains = len(chains)
    site_updates = 2.0 * n_chains * L * L * args.steps
    value = site_updates / wall
    # dominant kernel: the bit-packed half-step, 2 launches per step; the
    # remaining launches (one counter increment per 16 steps) are < 0.1 %
    per_launch_s = ev_ms * 1e-3 / (2 * args.steps)
    units_per_launch = n_chains * L * L
    kernel = "k_tri_bp" if triangular else "k_torus_bp"
    alu_per_site = TRI_ALU_PER_SITE if triangular else BP_ALU_PER_SITE
    achieved = units_per_launch * BP_BYTES_PER_SITE / per_launch_s / 1e9
    valu = read_traffic(kernel, per="launch", what="valu_lane_instr")
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(kernel), "kernel": kernel,
            "launch_us": per_launch_s * 1e6,
            "bytes_per_site_update": BP_BYTES_PER_SITE,
            "target_frac": HBM_TARGET_FRAC,
            "gap": "%.2f of HBM peak against the 0.60 target: at 0.25 B per site-update the "
                   "kernel is bound by VALU issue (Philox and the bit-sliced compare), not by "
                   "HBM; 0.60 would need %.1f site-updates per ns" %
                   (achieved / HBM_PEAK_GBS, HBM_TARGET_FRAC * HBM_PEAK_GBS / BP_BYTES_PER_SITE),
            "valu_issue_frac": None if valu is None else valu / (VALU_PEAK * per_launch_s),
            "valu_lane_instr_per_site_update": None if valu is None else valu / units_per_launch,
            "alu_model_frac": units_per_launch * alu_per_site / per_launch_s / VALU_PEAK}
    for c in chains:
        c.close()
    batch.close()
    lattice = "triangular-lattice torus (section 4)" if triangular else "torus"
    cfg = {"workload": "4096x4096 bit-packed %s, 24 chains (q x beta x init) batched" % lattice,
           "L": L, "chains": n_chains, "J": 1, "lambda": 0.0, "q": [0.5, 1.0, 2.0],
           "beta": [0.30, 0.40, 0.44, 0.50], "init": ["all_up", "random"],
           "strategy": "grid + hipGraph (16 full steps per replay)",
           "observables": "fused, every full step"}
    return value, wall, cfg, roof, "u1 (bit-packed spins)"


def _graph_run(sk, inst, n, steps, warmup, reps=1, fmt="int8"):
    """grid batch of `reps` chains of the graph (own seeds), HIP graph replay;
    returns (wall seconds, event seconds, workgroup size the autotuner chose)
    of the timed call"""
    chains = [sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                             lam_class=inst.cls, q=1.5, beta=0.8, seed=1 + r, replica=r, layout="csr",
                             fmt=fmt) for r in range(reps)]
    batch = sk.Batch(chains, strategy="grid", use_hipgraph=True, record=True, autotune=True,
                     log_reserve=max(steps, warmup))
    batch.sweep(warmup)
    wall = timed_sweep(batch, steps)
    _, ev_ms = batch.info()
    block = batch.launch_shape(0)
    batch.close()
    for c in chains:
        c.close()
    return wall, ev_ms * 1e-3, block


def bench_graph(args, sk):
    """One chain of the n = 2^20 random 3-regular +-J graph (CSR, int8 spins);
    the same graph with bit-packed spins and 8 replicas are reported beside."""
    import synth
    n = 1 << 20
    inst = synth.oriented_instance(n, 3, 3, lam_values=(-0.5, 0.0, 0.5), pm_j=True)
    wall, ev_s, block = _graph_run(sk, inst, n, args.steps, args.warmup)
    kernel = "k_graph_lds" if block == 1024 else "k_graph"
    value = 2.0 * n * args.steps / wall
    per_launch_s = ev_s / (2 * args.steps)
    m = inst.src.shape[0]
    # algorithmic bytes per half-step: rowptr (n+1), the edges (m; the
    # LDS-staged kernel reads index and J as one 4-byte word, the plain one
    # a 4-byte index and a 1-byte J), own spin, gathered spins (m), field
    # class, written spin
    edge_bytes = 4 if kernel == "k_graph_lds" else 5
    bytes_launch = 4 * (n + 1) + edge_bytes * m + n + m + n + n
    achieved = bytes_launch / per_launch_s / 1e9
    # the library's device layout for this graph: three slots per vertex
    # where every half-degree is at most three and every |J| is equal (the
    # algorithmic bytes above stay those of the CSR arrays)
    import numpy as np
    three_slot = (kernel == "k_graph_lds" and np.abs(inst.J.astype(np.int32)).min() == np.abs(inst.J.astype(np.int32)).max()
                  and max(np.bincount(inst.src, minlength=n).max(), np.bincount(inst.dst, minlength=n).max()) <= 3)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(kernel),
            "kernel": kernel, "block": block, "launch_us": per_launch_s * 1e6,
            "bytes_per_vertex_update": bytes_launch / n,
            "device_layout": "three slots per vertex (12 B per half-step, no row pointers)" if three_slot
            else "row pointers and edge words"}
    extra_steps = max(1, args.steps // 2)
    wall_bp, _, _ = _graph_run(sk, inst, n, extra_steps, args.warmup, fmt="bitpacked")
    wall_8, _, _ = _graph_run(sk, inst, n, extra_steps, args.warmup, reps=8)
    cfg = {"workload": "random 3-regular +-J graph, n=2^20, coin orientation, CSR int32, int8 spins",
           "n": n, "q": 1.5, "beta": 0.8, "lambda": [-0.5, 0.0, 0.5],
           "bitpacked_spins_vertex_updates_per_s": 2.0 * n * extra_steps / wall_bp,
           "int8_8_replicas_vertex_updates_per_s": 2.0 * n * 8 * extra_steps / wall_8}
    return value, wall, cfg, roof, "int8"


def bench_batch(args, sk):
    """2048 mixed chains (1024 tori L in {16..256}, 1024 3-regular +-J graphs
    n in [1024, 65536]), each with its own beta, q and seed, in one persistent
    launch; baseline: the same library driving one chain at a time."""
    import numpy as np
    import synth
    import torch
    # the same spec as the oracle baseline's (built once)
    spec = _BATCH_SPEC if _BATCH_SPEC is not None else synth.batch_spec(1024, 1024, seed=4)
    chains = []
    sites = 0
    adj_bytes_half = 0
    for i, it in enumerate(spec):
        if it.kind == "torus":
            chains.append(sk.Chain.torus(it.size, q=it.q, beta=it.beta, seed=it.seed, replica=i))
            sites += it.size * it.size
        else:
            g = it.graph
            chains.append(sk.Chain.graph(g.n, g.src, g.dst, J=g.J, q=it.q, beta=it.beta,
                                         seed=it.seed, replica=i))
            sites += g.n
            m = g.src.shape[0]
            # one half-step streams one CSR: rowptr (n+1) int32, col int32 + J int8 per entry
            # (the in-half and the out-half hold m entries together: m/2 each on average)
            adj_bytes_half += 4 * (g.n + 1) + 5 * (m / 2.0)
    # log space for the longest call is reserved up-front: no allocation in the timed call
    # one persistent launch per call, replayed from a captured HIP graph, with
    # the workgroup count autotuned on the first call (the warm-up)
    batch = sk.Batch(chains, strategy="persistent", record=True, use_hipgraph=True, autotune=True,
                     log_reserve=max(args.steps, args.warmup))
    batch.sweep(args.warmup)
    wall = timed_sweep(batch, args.steps)
    _, ev_ms = batch.info()
    value = 2.0 * sites * args.steps / wall
    batch.close()
    # baseline: one chain at a time, grid kernels replayed from a HIP graph,
    # on a random subset of 64 chains
    rng = np.random.Generator(np.random.PCG64(11))
    sub = rng.choice(len(chains), 64, replace=False)
    bsteps = max(1, args.steps // 10)
    bsites = 0
    t0 = time.perf_counter()
    for i in sub:
        b1 = sk.Batch([chains[i]], strategy="grid", use_hipgraph=True)
        b1.sweep(bsteps)
        torch.cuda.synchronize()
        b1.close()
        bsites += chains[i].n
    bwall = time.perf_counter() - t0
    base_value = 2.0 * bsites * bsteps / bwall
    for c in chains:
        c.close()
    per_launch_s = ev_ms * 1e-3  # one persistent launch per sweep
    bytes_launch = adj_bytes_half * 2 * args.steps
    achieved = bytes_launch / per_launch_s / 1e9
    # counters per full step; the timed launch covers args.steps of them
    traffic_step = read_traffic("k_persistent", per="full_step")
    traffic = traffic_step * args.steps if traffic_step is not None else None
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_per_full_step": traffic_step,
            "full_steps_per_launch": args.steps, "kernel": "k_persistent", "launch_us": per_launch_s * 1e6,
            "note": "graph adjacency streamed from HBM; tori are LDS-resident (0 B)"}
    cfg = {"workload": "2048 mixed chains in one persistent launch: 1024 tori L in {16..256}, "
                       "1024 3-regular +-J graphs n in [1024, 65536], own beta~U(0.2,1.2), "
                       "q~U(0.5,3), seed each", "chains": len(spec), "sites": int(sites),
           "baseline_site_updates_per_s": base_value, "speedup_vs_one_chain_per_launch":
           value / base_value, "baseline_sample": "64 random chains, %d full steps each, one "
           "at a time (grid kernels under a HIP graph)" % bsteps}
    return value, wall, cfg, roof, "u1 (bit-packed spins in LDS)"


def ea_couplings(L, seed):
    """+-1 couplings of an Edwards-Anderson torus: (J_up, J_right), each [L, L]"""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    return tuple(np.where(rng.integers(0, 2, (L, L)) == 1, 1, -1).astype(np.int8) for _ in range(2))


def bench_ea(args, sk):
    """The paper's benchmarked workload (section 6): 2-D Edwards-Anderson +-J
    tori, lambda = 0, q > 2, L = 256.  1024 independent spin glasses (own
    couplings, seed and beta; beta geometric from 0.5 to 2.0) in one batch
    (AUTO: the persistent kernel, every 256^2 torus fits in LDS),
    observables recorded every full step."""
    import numpy as np
    import torch
    L, n_chains, q = 256, 1024, 2.5
    betas = np.geomspace(0.5, 2.0, n_chains)
    chains = [sk.Chain.torus(L, J=ea_couplings(L, 10_000 + i), q=q, beta=float(betas[i]),
                             seed=20_000 + i, replica=i) for i in range(n_chains)]
    batch = sk.Batch(chains, strategy="auto", use_hipgraph=True, record=True, autotune=True,
                     log_reserve=max(args.steps, args.warmup))
    strategy = batch.info()[0]
    batch.sweep(args.warmup)
    wall = timed_sweep(batch, args.steps)
    _, ev_ms = batch.info()
    batch.close()
    for c in chains:
        c.close()
    sites = n_chains * L * L
    value = 2.0 * sites * args.steps / wall
    persistent = strategy == sk.SHAKEN_BATCH_PERSISTENT
    # persistent: one launch for the whole sweep; grid: one launch per half-step
    launches = 1 if persistent else 2 * args.steps
    per_launch_s = ev_ms * 1e-3 / launches
    achieved = sites * (2 * args.steps / launches) * BP_ALU_PER_SITE_PMJ / per_launch_s
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "T lane-cycles/s", "frac": achieved / VALU_PEAK, "traffic": None,
            "kernel": "k_persistent" if persistent else "k_torus_bp", "launch_us": per_launch_s * 1e6,
            "half_step_us": ev_ms * 1e3 / (2 * args.steps),
            "note": "coupling-sign planes: 2 more words read per spin word"}
    cfg = {"workload": "1024 Edwards-Anderson +-J tori 256x256 (lambda=0, q=2.5, beta geometric "
                       "0.5..2.0, own couplings and seed each), one batch",
           "L": L, "chains": n_chains, "q": q,
           "strategy": "persistent (spins in LDS)" if persistent else "grid + hipGraph",
           "observables": "every full step"}
    return value, wall, cfg, roof, "u1 (bit-packed spins)"


def cpu_baseline_ea():
    """1200 full steps of one 256^2 +-J torus per host core (about 10-20 s)."""
    cores = _host_cores()
    tasks = [(256, 1200, False, "ea", 2.5, 0.5, 20_000, r) for r in range(cores)]
    value, single, wall = _run_samples(_oracle_torus_sample, tasks)
    return {"value": value, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "single_core_value": single,
            "sample": "%d processes, each 1200 full steps of its own 256^2 +-J torus (q=2.5, beta=0.5), "
                      "%.1f s wall" % (cores, wall)}


def bench_copycal(args):
    """Plain device copy of a known size: the calibration of the FETCH_SIZE /
    WRITE_SIZE counters (bytes they report per byte copied)."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)


def _counter_rows(path, grid=None, counter=None):
    """counter values per kernel name; grid: keep only dispatches of that
    grid size (work-items); counter: keep only that counter (a pass may
    collect several)"""
    import csv
    rows = list(csv.DictReader(open(path)))
    out = {}
    for r in rows:
        if grid is not None and int(r["Grid_Size"]) != grid:
            continue
        if counter is not None and r.get("Counter_Name", counter) != counter:
            continue
        name = r["Kernel_Name"]
        out.setdefault(name, []).append(float(r["Counter_Value"]))
    return out


def summarize_traffic(cal_fetch_csv, cal_write_csv, workloads, out_path, valu_workloads=()):
    """profiles/traffic.txt from rocprofv3 --pmc counter CSVs: FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) of the 1 GiB calibration copy, then per
    workload (kernel, fetch csv, write csv, full steps per timed launch or 0,
    grid size or None, suffix of the kernel's template arguments or "").
    Only the named kernel of each workload is summarised (only its dispatches
    of that grid size and with that suffix, where given: a run may launch the
    kernel for other configurations too); a kernel whose launch covers many
    full steps (the persistent batch) is reported per full step, from its
    largest dispatch."""
    def rows(path, grid=None):
        return _counter_rows(path, grid)

    def short_name(k):
        return k.split("(")[0].replace("void ", "").replace("shaken::", "").split("<")[0]

    cf, cw = rows(cal_fetch_csv), rows(cal_write_csv)
    copy_k = [k for k in cf if "copy" in k.lower() or "elementwise" in k.lower()]
    ck = max(copy_k, key=lambda k: max(cf[k]))
    fetch_factor = (1 << 30) / (max(cf[ck]) * 1024.0)    # true bytes per counted byte
    write_factor = (1 << 30) / (max(cw[ck]) * 1024.0)
    lines = ["# HBM-side traffic from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per",
             "# dispatch), scaled by the factors a 1 GiB device copy gives (bytes copied /",
             "# bytes counted).  source_hash: kernels this was measured on.",
             "source_hash = %s" % kernel_source_hash(),
             "calibration_kernel = %s" % ck.split("(")[0],
             "fetch_factor = %.4f" % fetch_factor, "write_factor = %.4f" % write_factor]
    for kernel, fetch_csv, write_csv, steps, grid, suffix in workloads:
        f, w = rows(fetch_csv, grid), rows(write_csv, grid)
        fb_all, wb_all = [], []
        for k in sorted(f):
            if short_name(k) != kernel or not k.split("(")[0].endswith(suffix):
                continue
            fv = [x * 1024.0 * fetch_factor for x in f[k]]
            wv = [x * 1024.0 * write_factor for x in w.get(k, [0.0])]
            if steps:
                fv, wv = [max(fv) / steps], [max(wv) / steps]
            lines.append("# %s%s: fetch %.0f B, write %.0f B per %s (%d dispatches)"
                         % (k.split("(")[0], "" if grid is None else " grid %d" % grid,
                            sum(fv) / len(fv), sum(wv) / len(wv),
                            "full step" if steps else "launch", len(f[k])))
            fb_all += fv
            wb_all += wv
        if not fb_all:
            raise SystemExit("kernel %s not found in %s" % (kernel, fetch_csv))
        key = "bytes_per_full_step" if steps else "bytes_per_launch"
        lines.append("%s.%s = %.0f" % (kernel, key, sum(fb_all) / len(fb_all) + sum(wb_all) / len(wb_all)))
    for kernel, sq_csv, steps, grid, suffix in valu_workloads:
        v = _counter_rows(sq_csv, grid, "SQ_INSTS_VALU")
        vals = []
        for k in sorted(v):
            if short_name(k) != kernel or not k.split("(")[0].endswith(suffix):
                continue
            lv = [x * 64.0 for x in v[k]]
            if steps:
                lv = [max(lv) / steps]
            lines.append("# %s%s: %.4g VALU lane-instructions per %s (SQ_INSTS_VALU x 64, %d dispatches)"
                         % (k.split("(")[0], "" if grid is None else " grid %d" % grid, sum(lv) / len(lv),
                            "full step" if steps else "launch", len(v[k])))
            vals += lv
        if not vals:
            raise SystemExit("kernel %s not found in %s" % (kernel, sq_csv))
        key = "valu_lane_instr_per_full_step" if steps else "valu_lane_instr_per_launch"
        lines.append("%s.%s = %.0f" % (kernel, key, sum(vals) / len(vals)))
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_trace(trace_csv, stats_csv=None):
    """Markdown tables from a rocprofv3 --kernel-trace run: per kernel and
    launch shape (grid, workgroup, registers, LDS) the number of dispatches
    and their average / min / max duration, then the tool's own per-kernel
    statistics when its kernel_stats.csv is given."""
    groups = {}
    with open(trace_csv, newline="") as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"].split("(")[0]
            key = (name, int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]), int(r["Workgroup_Size_X"]),
                   int(r["VGPR_Count"]), int(r["LDS_Block_Size"]), int(r["Scratch_Size"]))
            groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["| kernel | grid x | grid y | block | VGPR | LDS B | scratch B | calls | avg us | min us | max us |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    total = sum(sum(d) for d in groups.values())
    shown = 0.0
    rest = []
    for key in sorted(groups, key=lambda k: -sum(groups[k])):
        d = groups[key]
        if sum(d) < 0.01 * total and len(out) > 2:   # shapes under 1 % each: counted below
            rest.append(key)
            continue
        shown += sum(d)
        out.append("| %s | %d | %d | %d | %d | %d | %d | %d | %.1f | %.1f | %.1f |"
                   % (key + (len(d), sum(d) / len(d), min(d), max(d))))
    if rest:
        names = sorted({k[0] for k in rest})
        out.append("| (%d more launch shapes of %s: %.2f %% of kernel time) | | | | | | | %d | | | |"
                   % (len(rest), ", ".join(names), 100.0 * (total - shown) / total,
                      sum(len(groups[k]) for k in rest)))
    if stats_csv:
        out += ["", "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
        with open(stats_csv, newline="") as fh:
            for r in csv.DictReader(fh):
                out.append("| %s | %s | %.1f | %.1f | %.1f | %.2f |"
                           % (r["Name"].split("(")[0], r["Calls"], float(r["AverageNs"]) / 1e3,
                              float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    print("\n".join(out))


def bench_mlp(sk, rows=512, reps=200):
    """Latency of the schedule network's calls at `rows` feature rows (one
    row per chain): forward; loss + backward (it returns the loss to the host,
    so each call synchronises); one Adam step.  Microseconds per call over
    `reps` calls, device synchronised before and after."""
    import numpy as np
    import torch
    from paper_1904_06257_amd import anneal
    mlp = sk.MLP(device=0)
    mlp.set_params(anneal.init_params(1))
    x = torch.randn(rows, sk.MLP_IN, device="cuda")
    y = torch.empty(rows, sk.MLP_OUT, device="cuda")
    t = torch.randn(rows, sk.MLP_OUT, device="cuda")
    out = {"rows": rows, "calls": reps}
    for name, fn in (("forward_us", lambda: mlp.forward(x, y)),
                     ("loss_backward_us", lambda: mlp.loss_backward(t)),
                     ("adam_us", lambda: mlp.adam(1e-4, 1))):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) / reps * 1e6
    # forward FLOPs per row: 2 x (16*128 + 128*128 + 128*128 + 128*16)
    flops = 2.0 * rows * (16 * 128 + 2 * 128 * 128 + 128 * 16)
    out["forward_tflops"] = flops / (out["forward_us"] * 1e-6) / 1e12
    out["note"] = ("latency-bound: %.1f MFLOP per forward call, far below what the matrix cores "
                   "need to be busy; the figure that matters is microseconds per call" % (flops / 1e6))
    mlp.close()
    return out


def _line(metric, unit, value, steps, warmup, wall, cfg, roof, cpu, dtype):
    return {"metric": metric, "value": value, "unit": unit, "steps": steps, "warmup": warmup,
            "ms_per_step": wall * 1e3 / steps, "dtype": dtype, "config": cfg, "roofline": roof,
            "cpu_baseline": cpu}


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-trace":
        # bench.py --summarize-trace KERNEL_TRACE_CSV [KERNEL_STATS_CSV]
        summarize_trace(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else None)
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-traffic":
        # bench.py --summarize-traffic CAL_FETCH CAL_WRITE KERNEL[@STEPS][#GRID][~SUFFIX]=FETCH,WRITE ...
        #          [valu:KERNEL[@STEPS][#GRID][~SUFFIX]=SQ_CSV ...]
        wl, vl = [], []
        for arg in sys.argv[4:]:
            name, files = arg.split("=", 1)
            is_valu = name.startswith("valu:")
            name = name[5:] if is_valu else name
            name, _, suffix = name.partition("~")
            name, _, grid = name.partition("#")
            kernel, _, steps = name.partition("@")
            if is_valu:
                vl.append((kernel, files, int(steps or 0), int(grid) if grid else None, suffix))
            else:
                fetch, write = files.split(",")
                wl.append((kernel, fetch, write, int(steps or 0), int(grid) if grid else None, suffix))
        summarize_traffic(sys.argv[2], sys.argv[3], wl, os.path.join(ROOT, "profiles", "traffic.txt"), vl)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="torus4096",
                    choices=["torus4096", "tri4096", "graph", "batch", "ea", "copycal"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="default workload only: skip the graph, batch and network lines")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(chains are independent: the work would shard by chain, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)
    secondary = args.workload == "torus4096" and not args.no_secondary
    # secondary lines: enough steps for the timed region to dwarf the
    # synchronisation around it (a 2^20 graph half-step is ~15 us)
    sec_args = {"graph": argparse.Namespace(steps=max(args.steps, 500), warmup=max(args.warmup, 5)),
                "batch": argparse.Namespace(steps=max(args.steps, 200), warmup=max(args.warmup, 5))}
    # the oracle baselines run first, in processes forked before this process
    # initialises the GPU
    baselines = {"torus4096": cpu_baseline_torus, "tri4096": lambda: cpu_baseline_torus(triangular=True),
                 "graph": cpu_baseline_graph, "ea": cpu_baseline_ea, "batch": cpu_baseline_batch}
    cpu = None
    cpu_sec = {}
    if not args.no_cpu_baseline:
        if args.workload in baselines:
            cpu = baselines[args.workload]()
        if secondary:
            cpu_sec = {"graph": cpu_baseline_graph(), "batch": cpu_baseline_batch()}
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.workload == "copycal":
        bench_copycal(args)
        return
    import paper_1904_06257_amd as sk

    if args.workload == "torus4096":
        value, wall, cfg, roof, dtype = bench_torus4096(args, sk)
        metric = "spin-site updates/s (4096^2 torus, batched)"
    elif args.workload == "tri4096":
        value, wall, cfg, roof, dtype = bench_torus4096(args, sk, triangular=True)
        metric = "spin-site updates/s (4096^2 triangular-lattice torus, batched)"
    elif args.workload == "graph":
        value, wall, cfg, roof, dtype = bench_graph(args, sk)
        metric = "vertex updates/s (3-regular graph, n=2^20)"
    elif args.workload == "ea":
        value, wall, cfg, roof, dtype = bench_ea(args, sk)
        metric = "spin-site updates/s (1024 +-J Edwards-Anderson tori 256^2, batched)"
    else:
        value, wall, cfg, roof, dtype = bench_batch(args, sk)
        metric = "aggregate site updates/s (2048 mixed chains, persistent batch)"
    unit = "vertex-updates/s" if args.workload == "graph" else "site-updates/s"
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": cfg, "roofline": roof, "cpu_baseline": cpu}
    if secondary:
        sec = {}
        ga = sec_args["graph"]
        v, w, c, r, d = bench_graph(ga, sk)
        sec["graph_2e20"] = _line("vertex updates/s (3-regular graph, n=2^20)", "vertex-updates/s",
                                  v, ga.steps, ga.warmup, w, c, r, cpu_sec.get("graph"), d)
        ba = sec_args["batch"]
        v, w, c, r, d = bench_batch(ba, sk)
        sec["batch_2048"] = _line("aggregate site updates/s (2048 mixed chains, persistent batch)",
                                  "site-updates/s", v, ba.steps, ba.warmup, w, c, r,
                                  cpu_sec.get("batch"), d)
        sec["mlp_512"] = bench_mlp(sk)
        out["secondary"] = sec
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
