"""Parity of the +-J torus (Edwards-Anderson couplings, section 6) with the
oracle: couplings of one magnitude with random signs on every oriented edge,
both spin formats, the grid and persistent batches, ragged widths.  Bit-exact
final configurations and H / M logs."""
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


def _couplings(L, mag, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ju = np.where(rng.integers(0, 2, (L, L)) == 1, mag, -mag).astype(np.int8)
    jr = np.where(rng.integers(0, 2, (L, L)) == 1, mag, -mag).astype(np.int8)
    return ju, jr


def _h(ej, mm, lam):
    return -ej - np.round(2 * lam * mm).astype(np.int64)


@pytest.mark.parametrize("L,fmt,lam,q,beta,mag", [
    (3, "bitpacked", 0.0, 2.5, 0.8, 1),
    (5, "int8", 0.5, 0.3, 1.1, 1),
    (31, "bitpacked", 0.5, 2.5, 1.3, 1),
    (33, "bitpacked", 0.0, 0.7, 0.9, 2),
    (64, "int8", 0.0, 2.5, 0.6, 1),
    (100, "bitpacked", -0.5, 3.0, 2.0, 1),
    (256, "bitpacked", 0.0, 2.5, 1.5, 1),
])
def test_pm_j_torus_single_chain(sk, L, fmt, lam, q, beta, mag):
    seed, T = 4000 + L, 60
    print("case: +-J torus", L, fmt, lam, q, beta, mag, flush=True)
    J = _couplings(L, mag, seed)
    init = oracle.torus_init_random(L, seed, 2)
    want, ej, mm = oracle.torus_run(init, J, lam, q, beta, seed, 2, T)
    ch = sk.Chain.torus(L, J=J, lam_values=[lam], q=q, beta=beta, seed=seed, replica=2, fmt=fmt)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(M, mm)
    assert np.array_equal(H, _h(ej, mm, lam))
    assert ch.observables().E_J == ej[-1]
    ch.close()


def test_pm_j_torus_formats_agree_at_1024(sk):
    """1024 x 1024 +-J torus for 10 full steps: both formats equal the oracle."""
    L, T, seed = 1024, 10, 77
    J = _couplings(L, 1, seed)
    init = oracle.torus_init_random(L, seed, 0)
    want, ej, mm = oracle.torus_run(init, J, 0.0, 2.5, 1.0, seed, 0, T)
    for fmt in ("bitpacked", "int8"):
        print("case: +-J torus 1024", fmt, flush=True)
        ch = sk.Chain.torus(L, J=J, q=2.5, beta=1.0, seed=seed, fmt=fmt)
        H, M = ch.sweep(T, log=True)
        assert np.array_equal(ch.spins(), want)
        assert np.array_equal(H, -ej) and np.array_equal(M, mm)
        ch.close()


@pytest.mark.parametrize("strategy", ["grid", "persistent"])
def test_pm_j_and_uniform_tori_in_one_batch(sk, strategy):
    """+-J tori and uniform tori in the same batch (one launch group): every
    chain bit-exact, logs included."""
    T = 30
    print("case: +-J batch", strategy, flush=True)
    specs = []
    for i, (L, pm) in enumerate([(16, True), (48, False), (100, True), (256, True), (64, False)]):
        seed = 900 + i
        J = _couplings(L, 1, seed) if pm else 1
        q, beta = 2.0 + 0.25 * i, 0.5 + 0.2 * i
        init = oracle.torus_init_random(L, seed, i)
        want, ej, mm = oracle.torus_run(init, J, 0.0, q, beta, seed, i, T)
        ch = sk.Chain.torus(L, J=J if pm else None, q=q, beta=beta, seed=seed, replica=i)
        specs.append((ch, want, ej, mm))
    chains = [sp[0] for sp in specs]
    b = sk.Batch(chains, strategy=strategy, record=True, use_hipgraph=(strategy == "grid"))
    b.sweep(T)
    for i, (ch, want, ej, mm) in enumerate(specs):
        h, m = b.log(i)
        assert np.array_equal(ch.spins(), want), i
        assert np.array_equal(h, -ej), i
        assert np.array_equal(m, mm), i
    b.close()
    for ch in chains:
        ch.close()
