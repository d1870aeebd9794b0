"""Bit-packed spins on graphs (one bit per vertex): every kernel that reads or
writes a graph configuration -- CSR and ELL half-steps, the observation
kernel, random / constant / user starts, the persistent batch -- against the
oracle, bit-exact, including sizes that leave a partial last word."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1904_06257_amd as m
    return m


def _h(inst, ej, plus):
    ncls = np.bincount(inst.cls, minlength=len(inst.lam_values))
    lam2 = (2 * inst.lam_values).astype(np.int64)
    return -ej - ((2 * plus - ncls[None, :]) * lam2[None, :]).sum(axis=1)


@pytest.mark.parametrize("n,deg,layout", [(4, 3, "csr"), (10, 3, "ell"), (33, 2, "csr"),
                                          (1002, 3, "csr"), (1002, 3, "ell"), (4096, 4, "ell"),
                                          (65537, 2, "csr"), (65539, 4, "csr")])
def test_single_chain(sk, n, deg, layout):
    T = 50
    print("case: bitpacked graph", n, deg, layout, flush=True)
    inst = synth.oriented_instance(n, deg, 700 + n, lam_values=(-0.5, 0.0, 0.5), pm_j=True)
    g = oracle.Graph(n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    sp0 = oracle.graph_init_random(n, 12, 3)
    want, ej, plus = oracle.graph_run(g, sp0, 1.5, 0.8, 12, 3, T)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values, lam_class=inst.cls,
                        q=1.5, beta=0.8, seed=12, replica=3, fmt="bitpacked", layout=layout)
    assert np.array_equal(ch.spins(), sp0)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(H, _h(inst, ej, plus))
    ob = ch.observables()
    assert ob.E_J == ej[-1]
    ch.close()


def test_full_size_prefix_and_formats_agree(sk):
    """n = 2^20 (the graph workload): 20 full steps, bit-packed = int8 = oracle."""
    n, T = 1 << 20, 20
    inst = synth.oriented_instance(n, 3, 3, lam_values=(-0.5, 0.0, 0.5), pm_j=True)
    g = oracle.Graph(n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    want, ej, plus = oracle.graph_run(g, oracle.graph_init_random(n, 1, 0), 1.5, 0.8, 1, 0, T)
    for fmt in ("bitpacked", "int8"):
        print("case: 2^20 graph", fmt, flush=True)
        ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                            lam_class=inst.cls, q=1.5, beta=0.8, seed=1, fmt=fmt, layout="csr")
        H, _ = ch.sweep(T, log=True)
        assert np.array_equal(ch.spins(), want)
        assert np.array_equal(H, _h(inst, ej, plus))
        ch.close()


@pytest.mark.parametrize("init", ["all_up", "all_down", "user"])
def test_starts_and_spin_round_trip(sk, init):
    n = 77
    inst = synth.oriented_instance(n + 1, 3, 9, lam_values=(0.0,), pm_j=True)   # n + 1 even
    rng = np.random.Generator(np.random.PCG64(4))
    user = np.where(rng.integers(0, 2, n + 1) == 1, 1, -1).astype(np.int8)
    kw = dict(init_spins=user) if init == "user" else dict(init=init)
    ch = sk.Chain.graph(n + 1, inst.src, inst.dst, J=inst.J, q=1.0, beta=0.5, seed=2,
                        fmt="bitpacked", **kw)
    start = user if init == "user" else np.full(n + 1, 1 if init == "all_up" else -1, np.int8)
    assert np.array_equal(ch.spins(), start)
    g = oracle.Graph(n + 1, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    want, _, _ = oracle.graph_run(g, start, 1.0, 0.5, 2, 0, 7)
    ch.sweep(7)
    assert np.array_equal(ch.spins(), want)
    ch.set_spins(user)
    assert np.array_equal(ch.spins(), user)
    ch.close()


@pytest.mark.parametrize("strategy", ["grid", "persistent"])
def test_batches_mixing_formats(sk, strategy):
    """bit-packed and int8 graphs (and a torus) in one batch: every chain
    bit-exact with its logs."""
    T = 30
    print("case: bitpacked batch", strategy, flush=True)
    specs = []
    for i, (n, fmt, layout) in enumerate([(1000, "bitpacked", "auto"), (2050, "int8", "auto"),
                                         (4096, "bitpacked", "csr"), (66, "bitpacked", "ell"),
                                         (30000, "bitpacked", "auto")]):
        inst = synth.oriented_instance(n, 3, 40 + i, lam_values=(-0.5, 0.5), pm_j=True)
        g = oracle.Graph(n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
        want, ej, plus = oracle.graph_run(g, oracle.graph_init_random(n, 50 + i, i), 1.2, 0.6 + 0.1 * i,
                                          50 + i, i, T)
        ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                            lam_class=inst.cls, q=1.2, beta=0.6 + 0.1 * i, seed=50 + i, replica=i,
                            fmt=fmt, layout=layout)
        specs.append((ch, inst, want, ej, plus))
    chains = [sp[0] for sp in specs]
    b = sk.Batch(chains, strategy=strategy, record=True, use_hipgraph=(strategy == "grid"))
    b.sweep(T)
    for i, (ch, inst, want, ej, plus) in enumerate(specs):
        h, _ = b.log(i)
        assert np.array_equal(ch.spins(), want), i
        assert np.array_equal(h, _h(inst, ej, plus)), i
    b.close()
    for ch in chains:
        ch.close()
