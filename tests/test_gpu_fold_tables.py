"""Folded class tables whose classes include fields h = 0 (T = 2^31), on the
bit-packed kernels: the grid half-step of a single chain and the persistent
batch, square and triangular lattice, against the oracle bit for bit.

At lambda = 0 the bit-packed kernels fold mirror classes (the neighbour count
reversed, the site flipped) into one class word whose sign is the site's spin
xor a per-class bit; a class with h = 0 decides alike with either sign and is
given the one opposite to its mirror's.  The cases: q = 2J on the square
lattice (classes n_plus = 2, -1 and n_plus = 0, +1), q = 0 (the one-neighbour
classes), beta = 0 (every class), J < 0, and q = 3J on the triangular lattice
(classes n_plus = 3, -1 and n_plus = 0, +1); ragged sides (L not a multiple
of 32) throughout.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

CASES = [  # L, q, beta, J
    (40, 2.0, 0.44, 1),
    (40, 0.0, 0.5, 1),
    (70, 1.0, 0.0, 1),
    (70, 2.0, 0.4, -1),
    (96, 3.0, 0.7, 1),
]


@pytest.fixture(scope="module")
def sk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1904_06257_amd as m
    return m


def _make(sk, tri, L, q, beta, J, seed, replica):
    make = sk.Chain.triangular if tri else sk.Chain.torus
    nedge = (3 if tri else 2) * L * L
    return make(L, J=np.full(nedge, J, np.int8), lam_values=[0.0], q=q, beta=beta, seed=seed,
                replica=replica, fmt="bitpacked")


@pytest.mark.parametrize("tri", [False, True])
@pytest.mark.parametrize("L,q,beta,J", CASES)
def test_single_chain(sk, tri, L, q, beta, J):
    T, seed = 40, 7000 + L
    print("case: folded table, single chain", tri, L, q, beta, J, flush=True)
    init = oracle.torus_init_random(L, seed, 1)
    want, ej, mm = oracle.torus_run(init, J, 0.0, q, beta, seed, 1, T, tri=tri)
    ch = _make(sk, tri, L, q, beta, J, seed, 1)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(M, mm)
    assert np.array_equal(H, -ej)
    ch.close()


@pytest.mark.parametrize("strategy", ["grid", "persistent"])
def test_batch(sk, strategy):
    T = 30
    print("case: folded tables, batch", strategy, flush=True)
    specs = []
    for i, (L, q, beta, J) in enumerate(CASES):
        for tri in (False, True):
            seed, rep = 7100 + 2 * i + tri, 2 * i + tri
            init = oracle.torus_init_random(L, seed, rep)
            want, ej, mm = oracle.torus_run(init, J, 0.0, q, beta, seed, rep, T, tri=tri)
            specs.append((_make(sk, tri, L, q, beta, J, seed, rep), want, ej, mm))
    chains = [sp[0] for sp in specs]
    bt = sk.Batch(chains, strategy=strategy, record=True)
    bt.sweep(T)
    for i, (ch, want, ej, mm) in enumerate(specs):
        h, m = bt.log(i)
        assert np.array_equal(ch.spins(), want), i
        assert np.array_equal(m, mm), i
        assert np.array_equal(h, -ej), i
    bt.close()
    for ch in chains:
        ch.close()
