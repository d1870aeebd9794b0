"""Parity with the CPU oracle at the full sizes of the benchmarked workloads,
in the launch configurations the benchmark times.

Every comparison is bit-exact: whole final configurations and every logged
H and M.  The oracle (plain single-threaded C) runs one chain per worker
thread -- ctypes releases the interpreter lock for the C call, so independent
chains run side by side on the host cores.  A long trajectory is checked in
segments: the GPU configuration at the start of a segment is the oracle's
(the previous segment proved it), so the oracle re-running the segment from
that configuration and matching the GPU at its end proves the whole run
equal, step by step, to one uninterrupted oracle run.

The torus and batch tests use the default benchmark invocation: a warm-up
call of WARMUP full steps, then one call of STEPS (with 16 full steps per
captured HIP graph, that call is one graph replay plus four eager steps).
"""
import os
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

WARMUP, STEPS = 5, 20


@pytest.fixture(scope="module")
def sk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1904_06257_amd as m
    return m


def _print_case(*a):
    print("case:", *a, flush=True)


def _workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _pool_map(fn, items):
    """fn over items on the host cores (threads; each oracle call is
    single-threaded C and runs without the interpreter lock)"""
    oracle.lib()  # build / load once, before the threads start
    with cf.ThreadPoolExecutor(_workers()) as ex:
        return list(ex.map(fn, items))


# ------------------------------------------------------- 4096^2 x 24 torus

def test_torus4096_bench_batch_all_chains(sk):
    """The headline workload exactly as the benchmark runs it: the 24 (q, beta,
    start) chains of the 4096^2 bit-packed torus in one grid batch with fused
    observables, HIP-graph replay and autotuned blocks.  Starts, the
    configurations after the warm-up call and after the timed call, and
    every H and M logged by both calls equal the oracle's for every chain.
    The timed call captures no graph and allocates no log space."""
    L = 4096
    runs = synth.torus_runs()
    _print_case("torus4096 x24 bench batch", WARMUP, STEPS)
    chains = [sk.Chain.torus(L, q=r["q"], beta=r["beta"], seed=r["seed"], replica=i, init=r["init"])
              for i, r in enumerate(runs)]
    starts = [c.spins() for c in chains]
    batch = sk.Batch(chains, strategy="grid", use_hipgraph=True, record=True, autotune=True,
                     log_reserve=max(STEPS, WARMUP))
    batch.sweep(WARMUP)
    H1, M1, _ = batch.logs(with_H=True, with_EJ=False)
    mid = [c.spins() for c in chains]
    c0 = batch.counters()
    batch.sweep(STEPS)
    c1 = batch.counters()
    H2, M2, _ = batch.logs(with_H=True, with_EJ=False)
    fin = [c.spins() for c in chains]
    batch.close()
    for c in chains:
        c.close()
    assert c0["captures"] == 1 and c1["captures"] == 1
    assert c1["log_allocs"] == c0["log_allocs"] and c1["autotunes"] == c0["autotunes"]

    def job(task):
        i, seg = task
        r = runs[i]
        if seg == 0:
            if r["init"] == "random":
                init = oracle.torus_init_random(L, r["seed"], i)
            else:
                init = np.ones((L, L), dtype=np.int8)
            a, ej, m = oracle.torus_run(init, 1, 0.0, r["q"], r["beta"], r["seed"], i, WARMUP, s0=0)
            return init, a, ej, m
        a, ej, m = oracle.torus_run(mid[i], 1, 0.0, r["q"], r["beta"], r["seed"], i, STEPS,
                                    s0=2 * WARMUP)
        return None, a, ej, m

    tasks = [(i, 1) for i in range(len(runs))] + [(i, 0) for i in range(len(runs))]
    res = dict(zip(tasks, _pool_map(job, tasks)))
    for i in range(len(runs)):
        init, a5, ej5, m5 = res[(i, 0)]
        _, a25, ej25, m25 = res[(i, 1)]
        assert np.array_equal(starts[i], init), "chain %d: start" % i
        assert np.array_equal(mid[i], a5), "chain %d: after the warm-up call" % i
        assert np.array_equal(H1[i], -ej5) and np.array_equal(M1[i], m5), "chain %d: warm-up logs" % i
        assert np.array_equal(fin[i], a25), "chain %d: after the timed call" % i
        assert np.array_equal(H2[i], -ej25) and np.array_equal(M2[i], m25), "chain %d: timed logs" % i


# ------------------------------------------------- 2048 mixed chains batch

def test_batch2048_bench_configuration(sk):
    """The 2048-chain mixed batch (1024 tori 16^2..256^2, 1024 3-regular +-J
    graphs of 1024..65536 vertices, own beta, q, seed each) in the persistent
    kernel with HIP-graph replay, autotuned workgroup count and recorded
    logs, as the benchmark runs it.  Every chain: start, configurations after
    the warm-up and the timed call, and both calls' H and M logs equal the
    oracle's.  Then the batch runs on to 2000 full steps; 64 sampled chains are
    compared over the whole run (final configuration and every logged H, M)."""
    LONG = 2000
    _print_case("batch2048 spec")
    spec = synth.batch_spec(1024, 1024, seed=4)
    _print_case("batch2048 persistent", WARMUP, STEPS, LONG)
    chains = []
    for i, it in enumerate(spec):
        if it.kind == "torus":
            chains.append(sk.Chain.torus(it.size, q=it.q, beta=it.beta, seed=it.seed, replica=i))
        else:
            g = it.graph
            chains.append(sk.Chain.graph(g.n, g.src, g.dst, J=g.J, q=it.q, beta=it.beta, seed=it.seed,
                                         replica=i))
    starts = [c.spins() for c in chains]
    batch = sk.Batch(chains, strategy="persistent", record=True, use_hipgraph=True, autotune=True,
                     log_reserve=max(STEPS, WARMUP))
    batch.sweep(WARMUP)
    H1, M1, _ = batch.logs(with_H=True, with_EJ=False)
    mid = [c.spins() for c in chains]
    c0 = batch.counters()
    batch.sweep(STEPS)
    c1 = batch.counters()
    H2, M2, _ = batch.logs(with_H=True, with_EJ=False)
    fin = [c.spins() for c in chains]
    batch.sweep(LONG - WARMUP - STEPS)
    H3, M3, _ = batch.logs(with_H=True, with_EJ=False)
    rng = np.random.Generator(np.random.PCG64(2024))
    sample = sorted(int(i) for i in rng.choice(len(spec), 64, replace=False))
    fin_long = {i: chains[i].spins() for i in sample}
    batch.close()
    for c in chains:
        c.close()
    assert c1["log_allocs"] == c0["log_allocs"] and c1["autotunes"] == c0["autotunes"]

    def run(i, sp, steps, s0):
        it = spec[i]
        if it.kind == "torus":
            a, ej, m = oracle.torus_run(sp, 1, 0.0, it.q, it.beta, it.seed, i, steps, s0=s0)
            return a, -ej, m
        g = it.graph
        og = oracle.Graph(g.n, g.src, g.dst, g.J)
        a, ej, plus = oracle.graph_run(og, sp, it.q, it.beta, it.seed, i, steps, s0=s0)
        return a, -ej, 2 * plus[:, 0] - g.n

    def job(task):
        i, seg = task
        it = spec[i]
        if seg == 0:
            if it.kind == "torus":
                init = oracle.torus_init_random(it.size, it.seed, i)
            else:
                init = oracle.graph_init_random(it.graph.n, it.seed, i)
            return (init,) + run(i, init, WARMUP, 0)
        if seg == 1:
            return (None,) + run(i, mid[i], STEPS, 2 * WARMUP)
        return (None,) + run(i, fin[i], LONG - WARMUP - STEPS, 2 * (WARMUP + STEPS))

    def cost(task):
        i, seg = task
        sites = spec[i].size ** 2 if spec[i].kind == "torus" else spec[i].size
        return sites * (WARMUP, STEPS, LONG)[seg]

    tasks = [(i, 0) for i in range(len(spec))] + [(i, 1) for i in range(len(spec))] + \
        [(i, 2) for i in sample]
    tasks.sort(key=cost, reverse=True)
    res = dict(zip(tasks, _pool_map(job, tasks)))
    for i in range(len(spec)):
        shape = starts[i].shape
        init, a5, h5, m5 = res[(i, 0)]
        _, a25, h25, m25 = res[(i, 1)]
        assert np.array_equal(starts[i].reshape(-1), init.reshape(-1)), "chain %d: start" % i
        assert np.array_equal(mid[i].reshape(-1), a5.reshape(-1)), "chain %d: after the warm-up call" % i
        assert np.array_equal(H1[i], h5) and np.array_equal(M1[i], m5), "chain %d: warm-up logs" % i
        assert np.array_equal(fin[i].reshape(-1), a25.reshape(-1)), "chain %d: after the timed call" % i
        assert np.array_equal(H2[i], h25) and np.array_equal(M2[i], m25), "chain %d: timed logs" % i
        assert shape == mid[i].shape
    for i in sample:
        _, a, h, m = res[(i, 2)]
        assert np.array_equal(fin_long[i].reshape(-1), a.reshape(-1)), "chain %d: after %d steps" % (i, LONG)
        assert np.array_equal(H3[i], h) and np.array_equal(M3[i], m), "chain %d: long logs" % i


# -------------------------------------------- graph n = 2^20, 5000 steps

def _graph_case(n, seed, lam=(-0.5, 0.0, 0.5)):
    inst = synth.oriented_instance(n, 3, seed, lam_values=lam, pm_j=True)
    g = oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    return inst, g


def test_graph2e20_full_length_bench_configuration(sk):
    """The n = 2^20 random 3-regular +-J graph (lambda in {-1/2, 0, 1/2},
    q = 1.5, beta = 0.8) for its whole 5000 full steps in the benchmark's
    launch configuration (CSR, int8 spins, grid batch, HIP graph, autotuned
    blocks, recorded observables): ten calls of 500 full steps, each checked
    against the oracle re-running it from the configuration the call
    started from -- every H and M of all 5000 steps and the configuration
    after every call bit-exact."""
    n, T, SEG, q, beta, seed = 1 << 20, 5000, 500, 1.5, 0.8, 1
    _print_case("graph 2^20 full length", T)
    inst, g = _graph_case(n, 3)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values, lam_class=inst.cls,
                        q=q, beta=beta, seed=seed, replica=0, layout="csr", fmt="int8")
    b = sk.Batch([ch], strategy="grid", use_hipgraph=True, record=True, autotune=True, log_reserve=SEG)
    states = [ch.spins()]
    logs = []
    for k in range(T // SEG):
        b.sweep(SEG)
        logs.append(b.log(0))
        states.append(ch.spins())
    cnt = b.counters()
    b.close()
    ch.close()
    assert cnt["captures"] == 1 and cnt["log_allocs"] == 1
    assert np.array_equal(states[0], oracle.graph_init_random(n, seed, 0))
    ncls = np.bincount(inst.cls, minlength=len(inst.lam_values))
    lam2 = (2 * inst.lam_values).astype(np.int64)

    def job(k):
        return oracle.graph_run(g, states[k], q, beta, seed, 0, SEG, s0=2 * SEG * k)

    res = _pool_map(job, list(range(T // SEG)))
    for k, (a, ej, plus) in enumerate(res):
        Mk = (2 * plus - ncls[None, :])
        assert np.array_equal(states[k + 1], a), "configuration after full step %d" % (SEG * (k + 1))
        assert np.array_equal(logs[k][0], -ej - (Mk * lam2[None, :]).sum(axis=1)), "H, call %d" % k
        assert np.array_equal(logs[k][1], Mk.sum(axis=1)), "M, call %d" % k


# ------------------------------------------ 256^2 torus, 10^4 full steps

@pytest.mark.parametrize("init", ["all_up", "random"])
def test_torus256_full_length(sk, init):
    """One 256^2 torus (q = 2, beta = 0.5) for the workload's full length of
    10^4 full steps, in ten calls of 1000 with logs, each segment checked
    against the oracle run from the configuration it started from."""
    L, T, SEG, q, beta, seed = 256, 10_000, 1000, 2.0, 0.5, 2
    _print_case("torus256 full length", init)
    ch = sk.Chain.torus(L, q=q, beta=beta, seed=seed, replica=7, init=init)
    states = [ch.spins()]
    logs = []
    for k in range(T // SEG):
        logs.append(ch.sweep(SEG, log=True))
        states.append(ch.spins())
    ch.close()
    if init == "random":
        assert np.array_equal(states[0], oracle.torus_init_random(L, seed, 7))
    else:
        assert np.all(states[0] == 1)

    def job(k):
        return oracle.torus_run(states[k], 1, 0.0, q, beta, seed, 7, SEG, s0=2 * SEG * k)

    for k, (a, ej, m) in enumerate(_pool_map(job, list(range(T // SEG)))):
        assert np.array_equal(states[k + 1], a), "after full step %d" % (SEG * (k + 1))
        assert np.array_equal(logs[k][0], -ej) and np.array_equal(logs[k][1], m), "logs, call %d" % k
