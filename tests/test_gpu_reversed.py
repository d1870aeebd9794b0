"""Reversed order P^{sh'} = P^{2->1} P^{1->2} (section 3) on every path: the
torus against the oracle's reversed half-steps, graphs against the forward
oracle on the reversed edge set (the uniforms are keyed by vertex and
half-step only).  Bit-exact configurations and H logs."""
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


@pytest.mark.parametrize("L,fmt,pm", [(33, "bitpacked", False), (64, "int8", False), (100, "bitpacked", True),
                                      (31, "int8", True)])
def test_reversed_torus(sk, L, fmt, pm):
    T, seed, lam = 40, 800 + L, 0.5
    print("case: reversed torus", L, fmt, pm, flush=True)
    rng = np.random.Generator(np.random.PCG64(L))
    J = tuple(np.where(rng.integers(0, 2, (L, L)) == 1, 1, -1).astype(np.int8) for _ in range(2)) if pm else 1
    init = oracle.torus_init_random(L, seed, 1)
    want, ej, mm = oracle.torus_run(init, J, lam, 1.3, 0.7, seed, 1, T, rev=True)
    fwd, _, _ = oracle.torus_run(init, J, lam, 1.3, 0.7, seed, 1, T)
    assert not np.array_equal(want, fwd)
    ch = sk.Chain.torus(L, J=J if pm else None, lam_values=[lam], q=1.3, beta=0.7, seed=seed, replica=1,
                        fmt=fmt, reversed=True)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(M, mm)
    assert np.array_equal(H, -ej - np.round(2 * lam * mm).astype(np.int64))
    ch.close()


@pytest.mark.parametrize("layout,fmt,strategy", [("csr", "int8", "grid"), ("ell", "bitpacked", "grid"),
                                                 ("auto", "int8", "persistent"), ("csr", "bitpacked", "persistent"),
                                                 ("ell", "int8", "persistent")])
def test_reversed_graph(sk, layout, fmt, strategy):
    n, T = 3000, 40
    print("case: reversed graph", layout, fmt, strategy, flush=True)
    inst = synth.oriented_instance(n, 3, 91, lam_values=(-0.5, 0.5), pm_j=True)
    back = oracle.Graph(n, inst.dst, inst.src, inst.J, inst.cls, inst.lam_values)
    want, ej, plus = oracle.graph_run(back, oracle.graph_init_random(n, 4, 2), 1.1, 0.9, 4, 2, T)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values, lam_class=inst.cls,
                        q=1.1, beta=0.9, seed=4, replica=2, fmt=fmt, layout=layout, reversed=True)
    b = sk.Batch([ch], strategy=strategy, record=True, use_hipgraph=(strategy == "grid"))
    b.sweep(T)
    h, _ = b.log(0)
    assert np.array_equal(ch.spins(), want)
    ncls = np.bincount(inst.cls, minlength=2)
    lam2 = (2 * inst.lam_values).astype(np.int64)
    assert np.array_equal(h, -ej - ((2 * plus - ncls[None, :]) * lam2[None, :]).sum(axis=1))
    b.close()
    ch.close()


def test_reversed_torus_in_persistent_batch(sk):
    T = 25
    chains, wants = [], []
    for i, (L, rev) in enumerate([(48, True), (48, False), (200, True)]):
        init = oracle.torus_init_random(L, 60 + i, i)
        wants.append(oracle.torus_run(init, 1, 0.0, 0.9, 0.5, 60 + i, i, T, rev=rev)[0])
        chains.append(sk.Chain.torus(L, q=0.9, beta=0.5, seed=60 + i, replica=i, reversed=rev))
    b = sk.Batch(chains, strategy="persistent")
    b.sweep(T)
    for ch, w in zip(chains, wants):
        assert np.array_equal(ch.spins(), w)
    b.close()
    for ch in chains:
        ch.close()
