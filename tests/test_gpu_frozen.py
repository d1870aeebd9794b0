"""Frozen set B (section 3.1): sites of B stay +1 from the start on, on every
path, and the rest of the configuration follows the oracle's restricted
half-steps bit for bit (logs included)."""
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


def _mask(n, seed, frac=0.1):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(n) < frac


@pytest.mark.parametrize("L,fmt,pm,rev,init", [(33, "bitpacked", False, False, "random"),
                                               (64, "int8", False, True, "all_down"),
                                               (100, "bitpacked", True, False, "all_down"),
                                               (31, "int8", True, True, "random")])
def test_frozen_torus(sk, L, fmt, pm, rev, init):
    T, seed, lam = 30, 900 + L, 0.5
    print("case: frozen torus", L, fmt, pm, rev, init, flush=True)
    fz = _mask(L * L, L).reshape(L, L)
    rng = np.random.Generator(np.random.PCG64(L + 1))
    J = tuple(np.where(rng.integers(0, 2, (L, L)) == 1, 1, -1).astype(np.int8) for _ in range(2)) if pm else 1
    start = oracle.torus_init_random(L, seed, 0) if init == "random" else -np.ones((L, L), np.int8)
    want, ej, mm = oracle.torus_run_frozen(start, fz, J, lam, 0.3, 1.2, seed, 0, T, rev=rev)
    ch = sk.Chain.torus(L, J=J if pm else None, lam_values=[lam], q=0.3, beta=1.2, seed=seed, fmt=fmt,
                        init=init, reversed=rev, frozen=fz)
    assert np.all(ch.spins()[fz] == 1)
    H, M = ch.sweep(T, log=True)
    got = ch.spins()
    assert np.all(got[fz] == 1)
    assert np.array_equal(got, want)
    assert np.array_equal(M, mm)
    assert np.array_equal(H, -ej - np.round(2 * lam * mm).astype(np.int64))
    ch.close()


@pytest.mark.parametrize("layout,fmt,strategy", [("csr", "int8", "grid"), ("ell", "bitpacked", "grid"),
                                                 ("auto", "int8", "persistent"),
                                                 ("csr", "bitpacked", "persistent")])
def test_frozen_graph(sk, layout, fmt, strategy):
    n, T = 2000, 30
    print("case: frozen graph", layout, fmt, strategy, flush=True)
    inst = synth.oriented_instance(n, 3, 33, lam_values=(-0.5, 0.5), pm_j=True)
    fz = _mask(n, 5, 0.05)
    g = oracle.Graph(n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    want, ej, plus = oracle.graph_run_frozen(g, oracle.graph_init_random(n, 6, 1), fz, 1.2, 0.9, 6, 1, T)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values, lam_class=inst.cls,
                        q=1.2, beta=0.9, seed=6, replica=1, fmt=fmt, layout=layout, frozen=fz)
    b = sk.Batch([ch], strategy=strategy, record=True, use_hipgraph=(strategy == "grid"))
    b.sweep(T)
    h, _ = b.log(0)
    got = ch.spins()
    assert np.all(got[fz] == 1)
    assert np.array_equal(got, want)
    ncls = np.bincount(inst.cls, minlength=2)
    lam2 = (2 * inst.lam_values).astype(np.int64)
    assert np.array_equal(h, -ej - ((2 * plus - ncls[None, :]) * lam2[None, :]).sum(axis=1))
    b.close()
    ch.close()


def test_user_start_and_set_spins_respect_b(sk):
    L = 40
    fz = _mask(L * L, 9).reshape(L, L)
    ch = sk.Chain.torus(L, q=1.0, beta=0.5, seed=1, init_spins=-np.ones((L, L), np.int8), frozen=fz)
    sp = ch.spins()
    assert np.all(sp[fz] == 1) and np.all(sp[~fz] == -1)
    ch.set_spins(-np.ones((L, L), np.int8))
    assert np.all(ch.spins()[fz] == 1)
    ch.close()
