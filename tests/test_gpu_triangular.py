"""Bit-packed (and int8) triangular-lattice torus (section 4) against the
oracle's triangular half-steps: ragged widths, fields that break the sign
symmetry (eight thresholds) and lambda = 0 (four), the reversed order, a
frozen set, grid and persistent batches mixing square and triangular tori.
Bit-exact configurations and H / M logs."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1904_06257_amd as m
    return m


@pytest.mark.parametrize("L,fmt,lam,q,beta,J,rev", [(3, "bitpacked", 0.0, 1.0, 0.3, 1, False),
                                                    (5, "int8", 0.5, 0.4, 0.7, 1, False),
                                                    (31, "bitpacked", 0.5, 2.0, 0.35, 1, False),
                                                    (33, "bitpacked", 0.0, 0.3, 0.5, 2, True),
                                                    (64, "int8", 0.0, 1.0, 0.28, -1, False),
                                                    (100, "bitpacked", -0.5, 1.5, 0.6, 1, True),
                                                    (256, "bitpacked", 0.0, 1.0, 0.27, 1, False)])
def test_triangular_single_chain(sk, L, fmt, lam, q, beta, J, rev):
    T, seed = 50, 1100 + L
    print("case: triangular", L, fmt, lam, q, beta, J, rev, flush=True)
    init = oracle.torus_init_random(L, seed, 3)
    want, ej, mm = oracle.torus_run(init, J, lam, q, beta, seed, 3, T, rev=rev, tri=True)
    ch = sk.Chain.triangular(L, J=np.full(3 * L * L, J, np.int8), lam_values=[lam], q=q, beta=beta,
                             seed=seed, replica=3, fmt=fmt, reversed=rev)
    assert np.array_equal(ch.spins(), init)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(M, mm)
    assert np.array_equal(H, -ej - np.round(2 * lam * mm).astype(np.int64))
    assert ch.observables().E_J == ej[-1]
    ch.close()


def test_triangular_formats_agree_at_1024(sk):
    L, T, seed = 1024, 8, 5
    init = oracle.torus_init_random(L, seed, 0)
    want, ej, _ = oracle.torus_run(init, 1, 0.0, 1.0, 0.27, seed, 0, T, tri=True)
    for fmt in ("bitpacked", "int8"):
        print("case: triangular 1024", fmt, flush=True)
        ch = sk.Chain.triangular(L, q=1.0, beta=0.27, seed=seed, fmt=fmt)
        H, _ = ch.sweep(T, log=True)
        assert np.array_equal(ch.spins(), want)
        assert np.array_equal(H, -ej)
        ch.close()


def test_triangular_frozen(sk):
    L, T, seed = 40, 30, 9
    rng = np.random.Generator(np.random.PCG64(1))
    fz = (rng.random((L, L)) < 0.1)
    start = -np.ones((L, L), np.int8)
    a = start.copy()
    a[fz] = 1
    for t in range(T):
        for k in range(2):
            a = oracle.torus_half_step(a, 1, 0.0, 0.2, 1.1, seed, 0, 2 * t + k, tri=True)
            a[fz] = 1
    ch = sk.Chain.triangular(L, q=0.2, beta=1.1, seed=seed, init="all_down", frozen=fz)
    ch.sweep(T)
    assert np.array_equal(ch.spins(), a)
    ch.close()


@pytest.mark.parametrize("strategy", ["grid", "persistent"])
def test_square_and_triangular_in_one_batch(sk, strategy):
    T = 30
    print("case: triangular batch", strategy, flush=True)
    specs = []
    for i, (L, tri, lam) in enumerate([(48, True, 0.0), (48, False, 0.0), (100, True, 0.5), (16, True, 0.0),
                                       (64, False, 0.5)]):
        seed, q, b = 300 + i, 0.5 + 0.3 * i, 0.3 + 0.05 * i
        init = oracle.torus_init_random(L, seed, i)
        want, ej, mm = oracle.torus_run(init, 1, lam, q, b, seed, i, T, tri=tri)
        make = sk.Chain.triangular if tri else sk.Chain.torus
        specs.append((make(L, q=q, beta=b, lam_values=[lam], seed=seed, replica=i), want, ej, mm, lam))
    chains = [sp[0] for sp in specs]
    bt = sk.Batch(chains, strategy=strategy, record=True, use_hipgraph=(strategy == "grid"))
    bt.sweep(T)
    for i, (ch, want, ej, mm, lam) in enumerate(specs):
        h, m = bt.log(i)
        assert np.array_equal(ch.spins(), want), i
        assert np.array_equal(m, mm), i
        assert np.array_equal(h, -ej - np.round(2 * lam * mm).astype(np.int64)), i
    bt.close()
    for ch in chains:
        ch.close()
