"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact on every integer output: final configurations, per-step H and M,
threshold tables.  Sizes span several tiles and ragged tails; the full-size
workloads are checked on sampled sites, or over a short prefix the oracle can
run.  All tests need an MI355X.
"""
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


def _print_case(*a):
    print("case:", *a, flush=True)


# --------------------------------------------------------------- torus

@pytest.mark.parametrize("fmt", ["bitpacked", "int8"])
def test_torus_64_full_config(sk, fmt):
    """64 x 64, J=1, lambda=0, q=1, beta=0.4, 1000 full steps, Philox seed 1:
    final spins and the H, M logs of every step equal the oracle's."""
    L, q, beta, seed, T = 64, 1.0, 0.40, 1, 1000
    _print_case("torus64", fmt)
    init = oracle.torus_init_random(L, seed)
    want, ej, mm = oracle.torus_run(init, 1, 0.0, q, beta, seed, 0, T)
    ch = sk.Chain.torus(L, q=q, beta=beta, seed=seed, fmt=fmt)
    assert np.array_equal(ch.spins(), init)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(H, -ej)
    assert np.array_equal(M, mm)
    ob = ch.observables()
    assert ob.half_step == 2 * T and ob.H == -ej[-1] and ob.M == mm[-1]


@pytest.mark.parametrize("L,fmt,lam,q,beta,J", [
    (3, "bitpacked", 0.0, 1.0, 0.4, 1),
    (5, "int8", 0.15, 0.1, 1.3, 1),
    (31, "bitpacked", 0.15, 0.1, 2.3, 1),
    (33, "bitpacked", -0.3, 0.7, 0.9, 2),
    (37, "int8", 0.0, 0.0, 0.6, 1),
    (64, "bitpacked", 0.25, 2.0, 0.44, -1),
    (101, "bitpacked", 0.0, 0.5, 0.3, 1),
    (101, "int8", 0.0, 0.5, 0.3, 1),
    (200, "bitpacked", 0.05, 3.0, 0.5, 1),
])
def test_torus_ragged_and_parameters(sk, L, fmt, lam, q, beta, J):
    """Ragged widths (L not a multiple of 32), fields that break the sign
    symmetry, q = 0, antiferromagnetic J; M log and final spins bit-exact,
    E_J through the observables."""
    seed, T = 12345 + L, 40
    _print_case("torus", L, fmt, lam, q, beta, J)
    init = oracle.torus_init_random(L, seed, 3)
    want, ej, mm = oracle.torus_run(init, J, lam, q, beta, seed, 3, T)
    Jarr = np.full(2 * L * L, J, dtype=np.int8)
    ch = sk.Chain.torus(L, J=Jarr, lam_values=[lam], q=q, beta=beta, seed=seed, replica=3, fmt=fmt)
    M = ch.sweep_m(T)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(M, mm)
    ob = ch.observables()
    assert ob.E_J == ej[-1]


@pytest.mark.parametrize("tri", [False, True])
@pytest.mark.parametrize("sizes,autotune", [
    ((256,), False),          # every lane of the grid a strip of the chain
    ((512, 512), True),       # the same for two chains, blocks autotuned
    ((256, 512), False),      # aligned sides of two sizes: the smaller leaves lanes idle
    ((96, 32), False),        # aligned sides whose strips do not fill a block
])
def test_torus_aligned_full_and_partial_grids(sk, sizes, autotune, tri):
    """Sides that are multiples of 32 in grid batches with fused
    observables, square and triangular lattices: grids where every lane is
    a strip of every chain (all chains one size, strips a multiple of the
    block) and grids with idle lanes; every chain's configuration and H, M
    logs bit-exact."""
    T, q, beta = 6, 1.0, 0.44
    _print_case("torus aligned grid", sizes, autotune, tri)
    make = sk.Chain.triangular if tri else sk.Chain.torus
    chains = [make(L, q=q, beta=beta, seed=70 + i, replica=i) for i, L in enumerate(sizes)]
    starts = [c.spins() for c in chains]
    b = sk.Batch(chains, strategy="grid", use_hipgraph=True, record=True, autotune=autotune, log_reserve=T)
    b.sweep(T)
    H, M, _ = b.logs(with_H=True, with_EJ=False)
    got = [c.spins() for c in chains]
    b.close()
    for c in chains:
        c.close()
    for i, L in enumerate(sizes):
        init = oracle.torus_init_random(L, 70 + i, i)
        assert np.array_equal(starts[i], init)
        want, ej, mm = oracle.torus_run(init, 1, 0.0, q, beta, 70 + i, i, T, tri=tri)
        assert np.array_equal(got[i], want), "chain %d (L = %d)" % (i, L)
        assert np.array_equal(H[i], -ej) and np.array_equal(M[i], mm), "chain %d logs" % i


def test_torus_bitpacked_equals_int8(sk):
    L, T = 77, 60
    a = sk.Chain.torus(L, q=0.8, beta=0.5, seed=9, fmt="bitpacked", lam_values=[0.1])
    b = sk.Chain.torus(L, q=0.8, beta=0.5, seed=9, fmt="int8", lam_values=[0.1])
    a.sweep(T)
    b.sweep(T)
    assert np.array_equal(a.spins(), b.spins())


def test_torus_half_steps_and_parity(sk):
    """Odd numbers of half-steps, checkpoint restore of the counter."""
    L, q, beta, seed = 40, 0.9, 0.45, 4
    init = oracle.torus_init_random(L, seed)
    x = init.copy()
    for s in range(7):
        x = oracle.torus_half_step(x, 1, 0.0, q, beta, seed, 0, s)
    ch = sk.Chain.torus(L, q=q, beta=beta, seed=seed)
    ch.half_step(3)
    ch.half_step(4)
    assert np.array_equal(ch.spins(), x)
    # restore: set spins and counter, continue
    y = oracle.torus_half_step(x, 1, 0.0, q, beta, seed, 0, 7)
    c2 = sk.Chain.torus(L, q=q, beta=beta, seed=seed, init_spins=x)
    c2.set_half_step(7)
    c2.half_step(1)
    assert np.array_equal(c2.spins(), y)
    with pytest.raises(sk.ShakenError):
        c2.set_half_step(7)
        c2.sweep(1)


def test_torus_zero_temperature_diagonal(sk):
    """The printed zero-temperature growth (proof of Theorem 3.3) on the GPU."""
    L, r0, c0 = 16, 5, 11
    sp = -np.ones((L, L), dtype=np.int8)
    sp[r0, c0] = 1
    for fmt in ("bitpacked", "int8"):
        ch = sk.Chain.torus(L, q=0.1, lam_values=[0.15], beta=1000.0, seed=1, init_spins=sp, fmt=fmt)
        ch.half_step(1)
        got = set(map(tuple, np.argwhere(ch.spins() > 0)))
        assert got == {(r0 + 1, c0), (r0, c0 + 1)}
        ch.half_step(2 * (L // 2) - 1)
        got = set(map(tuple, np.argwhere(ch.spins() > 0)))
        assert got == {(r, c) for r in range(L) for c in range(L) if (r + c - r0 - c0) % L == 0}


def test_torus_lut_matches_oracle(sk):
    for q, beta, lam, J in [(1.0, 0.4, 0.0, 1), (0.1, 2.3, 0.15, 1), (2.5, 0.9, -0.2, 3)]:
        ch = sk.Chain.torus(8, J=np.full(128, J, dtype=np.int8), q=q, beta=beta, lam_values=[lam])
        lut, smax = ch.lut()
        assert smax == 2 * abs(J)
        for S in range(-smax, smax + 1):
            for sb in (0, 1):
                want = oracle.threshold_of(S, 1 if sb else -1, q, lam, beta)
                assert int(lut[(S + smax) * 2 + sb]) == want


def test_torus_4096_sampled_sites(sk):
    """Full size: one dl and one ur half-step of a 4096^2 bit-packed torus,
    16384 sampled sites recomputed one by one by the oracle."""
    L, q, beta, seed = 4096, 1.0, 0.44, 2
    _print_case("torus4096 sampled")
    ch = sk.Chain.torus(L, q=q, beta=beta, seed=seed, replica=5)
    s0 = ch.spins()
    init = oracle.torus_init_random(L, seed, 5)
    rng = np.random.Generator(np.random.PCG64(3))
    rows = rng.integers(0, L, 64)
    assert np.array_equal(s0[rows], init[rows])
    ch.half_step(1)
    s1 = ch.spins()
    ch.half_step(1)
    s2 = ch.spins()
    idx = rng.integers(0, L, size=(16384, 2))
    idx[:64, 1] = 0
    idx[64:128, 1] = L - 1
    for (r, c) in idx[:8192]:
        assert s1[r, c] == oracle.torus_site(s0, 1, 0.0, q, beta, seed, 5, 0, r, c)
    for (r, c) in idx[8192:]:
        assert s2[r, c] == oracle.torus_site(s1, 1, 0.0, q, beta, seed, 5, 1, r, c)


def test_torus_256_long_prefix(sk):
    L, q, beta, T = 256, 2.0, 0.5, 200
    init = np.ones((L, L), dtype=np.int8)
    want, ej, mm = oracle.torus_run(init, 1, 0.0, q, beta, 2, 0, T)
    ch = sk.Chain.torus(L, q=q, beta=beta, seed=2, init="all_up")
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(H, -ej) and np.array_equal(M, mm)


# ---------------------------------------------------------------- graph

def _graph_case(n, seed, lam=(-0.5, 0.0, 0.5)):
    inst = synth.oriented_instance(n, 3, seed, lam_values=lam, pm_j=True)
    g = oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    return inst, g


def _h_from_plus(inst, ej, plus):
    ncls = np.bincount(inst.cls, minlength=len(inst.lam_values))
    lam2 = (2 * inst.lam_values).astype(np.int64)
    return -ej - ((2 * plus - ncls[None, :]) * lam2[None, :]).sum(axis=1)


@pytest.mark.parametrize("n", [4, 10, 1002, 4096])
def test_graph_3regular(sk, n):
    """3-regular +-J graph, coin orientation, lambda in {-1/2, 0, 1/2},
    q = 1.5, beta = 0.8: spins and H, M logs bit-exact over 200 full steps."""
    T = 200
    _print_case("graph3reg", n)
    inst, g = _graph_case(n, 100 + n)
    sp0 = oracle.graph_init_random(n, 1)
    want, ej, plus = oracle.graph_run(g, sp0, 1.5, 0.8, 1, 0, T)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                        lam_class=inst.cls, q=1.5, beta=0.8, seed=1)
    assert np.array_equal(ch.spins(), sp0)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(H, _h_from_plus(inst, ej, plus))
    ncls = np.bincount(inst.cls, minlength=3)
    assert np.array_equal(M, (2 * plus - ncls[None, :]).sum(axis=1))


@pytest.mark.parametrize("n,p,jmax,ncls", [(1, 0.0, 1, 1), (7, 0.0, 1, 2), (333, 0.05, 3, 4),
                                            (1001, 0.01, 5, 7)])
def test_graph_general(sk, n, p, jmax, ncls):
    """Erdos-Renyi graphs (no edges, isolated vertices, larger couplings, many
    field classes, n not a multiple of 4)."""
    T = 50
    _print_case("graphER", n, p, jmax, ncls)
    inst = synth.random_oriented_graph(n, p, 7 + n, jmax=jmax, n_classes=ncls, lam_scale=0.3)
    g = oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    sp0 = oracle.graph_init_random(n, 3, 2)
    want, ej, plus = oracle.graph_run(g, sp0, 0.6, 0.7, 3, 2, T)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                        lam_class=inst.cls, q=0.6, beta=0.7, seed=3, replica=2)
    M = ch.sweep_m(T)
    assert np.array_equal(ch.spins(), want)
    ncls_cnt = np.bincount(inst.cls, minlength=ncls)
    assert np.array_equal(M, (2 * plus - ncls_cnt[None, :]).sum(axis=1))
    assert ch.observables().E_J == ej[-1]


def test_graph_full_size_prefix(sk):
    """N = 2^20 3-regular +-J graph: 6 full steps bit-exact (whole configuration)."""
    n, T = 1 << 20, 6
    _print_case("graph 2^20")
    inst, g = _graph_case(n, 3)
    sp0 = oracle.graph_init_random(n, 1)
    want, ej, plus = oracle.graph_run(g, sp0, 1.5, 0.8, 1, 0, T)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                        lam_class=inst.cls, q=1.5, beta=0.8, seed=1)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(H, _h_from_plus(inst, ej, plus))


def test_graph_full_size_bench_configuration(sk):
    """The n = 2^20 graph workload as the bench runs it: CSR, int8 spins, a grid
    batch replayed from a captured HIP graph with autotuned blocks; 100 full
    steps, every H and M and the final configuration bit-exact."""
    n, T = 1 << 20, 100
    _print_case("graph 2^20 bench configuration", T)
    inst, g = _graph_case(n, 3)
    sp0 = oracle.graph_init_random(n, 1, 0)
    want, ej, plus = oracle.graph_run(g, sp0, 1.5, 0.8, 1, 0, T)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                        lam_class=inst.cls, q=1.5, beta=0.8, seed=1, replica=0, layout="csr", fmt="int8")
    b = sk.Batch([ch], strategy="grid", use_hipgraph=True, record=True, autotune=True, log_reserve=T)
    b.sweep(T)
    H, M = b.log(0)
    assert np.array_equal(ch.spins(), want)
    assert np.array_equal(H, _h_from_plus(inst, ej, plus))
    ncls = np.bincount(inst.cls, minlength=len(inst.lam_values))
    assert np.array_equal(M, (2 * plus - ncls[None, :]).sum(axis=1))
    b.close()
    ch.close()


def _acceptance_z(keys, up, probs):
    """binomial z-score of the +1 frequency per key (keys with >= 1000 sites)"""
    zs = []
    for k in np.unique(keys):
        sel = keys == k
        nk = int(sel.sum())
        p = probs[k]
        if nk < 1000 or p <= 0.0 or p >= 1.0:
            if p <= 0.0:
                assert not np.any(up[sel]), k
            if p >= 1.0:
                assert np.all(up[sel]), k
            continue
        zs.append((int(up[sel].sum()) - nk * p) / np.sqrt(nk * p * (1 - p)))
    return np.array(zs)


def test_per_class_acceptance_torus(sk):
    """One half-step of a 1024^2 torus from a random configuration: for every
    (neighbour sum, own spin) class the frequency of +1 matches the threshold
    probability T/2^32 of the contract (binomial z-scores)."""
    L, q, beta, lam = 1024, 1.0, 0.44, 0.0
    _print_case("acceptance torus", L)
    ch = sk.Chain.torus(L, q=q, beta=beta, seed=17, replica=3)
    before = ch.spins().astype(np.int64)
    ch.half_step(1)
    after = ch.spins()
    # half-step 1 (dl): down and left neighbours; row r + 1 is up, column c + 1 right
    S = np.roll(before, 1, axis=0) + np.roll(before, 1, axis=1)
    keys = ((S + 2) * 2 + (before > 0)).reshape(-1)
    probs = {}
    for Sv in (-2, 0, 2):
        for sg in (-1, 1):
            probs[(Sv + 2) * 2 + (sg > 0)] = oracle.threshold_of(Sv, sg, q, lam, beta) / 2.0 ** 32
    z = _acceptance_z(keys, (after > 0).reshape(-1), probs)
    print("torus z:", np.round(z, 2), flush=True)
    assert len(z) == 6 and np.all(np.abs(z) < 5)
    ch.close()


def test_per_class_acceptance_graph(sk):
    """One half-step of the n = 2^20 graph: +1 frequency per (field sum, own
    spin, field class) against the threshold probability of the contract."""
    n, q, beta = 1 << 20, 1.5, 0.8
    _print_case("acceptance graph", n)
    inst, g = _graph_case(n, 3)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                        lam_class=inst.cls, q=q, beta=beta, seed=5, replica=1)
    before = ch.spins().astype(np.int64)
    ch.half_step(1)
    after = ch.spins()
    # half-step 1: the in-half, sum over edges (y, x) of J sigma_y
    S = np.zeros(n, np.int64)
    np.add.at(S, inst.dst, inst.J.astype(np.int64) * before[inst.src])
    smax = 3
    nc = len(inst.lam_values)
    keys = ((S + smax) * 2 + (before > 0)) * nc + inst.cls
    probs = {}
    for Sv in range(-smax, smax + 1):
        for sg in (-1, 1):
            for k in range(nc):
                probs[((Sv + smax) * 2 + (sg > 0)) * nc + k] = oracle.threshold_of(
                    Sv, sg, q, float(inst.lam_values[k]), beta) / 2.0 ** 32
    z = _acceptance_z(keys, after > 0, probs)
    print("graph z:", np.round(z, 2), flush=True)
    assert len(z) >= 12 and np.all(np.abs(z) < 5)
    ch.close()


def test_graph_lut_matches_oracle(sk):
    inst, g = _graph_case(64, 8)
    ch = sk.Chain.graph(64, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                        lam_class=inst.cls, q=1.5, beta=0.8, seed=1)
    lut, smax = ch.lut()
    nc = len(inst.lam_values)
    for S in range(-smax, smax + 1):
        for sb in (0, 1):
            for k in range(nc):
                want = oracle.threshold_of(S, 1 if sb else -1, 1.5, inst.lam_values[k], 0.8)
                assert int(lut[((S + smax) * 2 + sb) * nc + k]) == want


def test_set_params_changes_law(sk):
    L, T = 48, 10
    init = oracle.torus_init_random(L, 5)
    x, _, _ = oracle.torus_run(init, 1, 0.0, 1.0, 0.4, 5, 0, T)
    y, _, _ = oracle.torus_run(x, 1, 0.0, 2.0, 0.7, 5, 0, T, s0=2 * T)
    ch = sk.Chain.torus(L, q=1.0, beta=0.4, seed=5)
    ch.sweep(T)
    ch.set_params(0.7, 2.0)
    ch.sweep(T)
    assert np.array_equal(ch.spins(), y)


# ---------------------------------------------------------------- batches

@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_grid_mixed(sk, use_graph):
    """A grid batch of tori (both formats, several sizes) and graphs, each
    with its own beta, q, seed and replica, advanced together."""
    T = 37
    specs = []
    chains = []
    for i, (L, fmt) in enumerate([(64, "bitpacked"), (96, "bitpacked"), (50, "int8"), (33, "bitpacked")]):
        q, b, seed = 0.5 + 0.3 * i, 0.3 + 0.1 * i, 1000 + i
        init = oracle.torus_init_random(L, seed, i)
        want, ej, mm = oracle.torus_run(init, 1, 0.0, q, b, seed, i, T)
        specs.append(("t", want, -ej, mm))
        chains.append(sk.Chain.torus(L, q=q, beta=b, seed=seed, replica=i, fmt=fmt))
    for i, n in enumerate([500, 2048]):
        inst, g = _graph_case(n, 50 + i)
        sp0 = oracle.graph_init_random(n, 77 + i, i)
        want, ej, plus = oracle.graph_run(g, sp0, 1.2, 0.6, 77 + i, i, T)
        ncls = np.bincount(inst.cls, minlength=3)
        specs.append(("g", want, _h_from_plus(inst, ej, plus), (2 * plus - ncls[None, :]).sum(axis=1)))
        chains.append(sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                                     lam_class=inst.cls, q=1.2, beta=0.6, seed=77 + i, replica=i))
    b = sk.Batch(chains, strategy="grid", use_hipgraph=use_graph, record=True, autotune=True)
    b.sweep(T)
    for i, (kind, want, H, M) in enumerate(specs):
        assert np.array_equal(chains[i].spins(), want), i
        h, m = b.log(i)
        assert np.array_equal(h, H), i
        assert np.array_equal(m, M), i
    # a second sweep continues the same chains
    b.sweep(3)
    st, ms = b.info()
    assert st == sk.SHAKEN_BATCH_GRID and ms > 0


def test_batch_rejects_mismatched_counters(sk):
    a = sk.Chain.torus(16, seed=1)
    c = sk.Chain.torus(16, seed=2)
    c.half_step(2)
    with pytest.raises(sk.ShakenError):
        sk.Batch([a, c], strategy="grid")


def _mixed_specs(T, torus_sizes, graph_sizes, seed0=0):
    specs = []
    for i, L in enumerate(torus_sizes):
        q, b, seed = 0.5 + 0.25 * i, 0.25 + 0.15 * i, 5000 + i + seed0
        lam = 0.0 if i % 2 == 0 else 0.2
        init = oracle.torus_init_random(L, seed, i)
        want, ej, mm = oracle.torus_run(init, 1, lam, q, b, seed, i, T)
        specs.append(dict(kind="torus", L=L, q=q, beta=b, seed=seed, rep=i, lam=lam,
                          want=want, H=(-ej - (2 * lam * mm).round().astype(np.int64)) if lam == 0 else None,
                          M=mm, EJ=ej))
    for i, n in enumerate(graph_sizes):
        inst, g = _graph_case(n, 900 + i + seed0)
        seed = 7000 + i + seed0
        sp0 = oracle.graph_init_random(n, seed, 40 + i)
        want, ej, plus = oracle.graph_run(g, sp0, 1.1 + 0.3 * i, 0.5 + 0.2 * i, seed, 40 + i, T)
        ncls = np.bincount(inst.cls, minlength=3)
        specs.append(dict(kind="graph", inst=inst, n=n, q=1.1 + 0.3 * i, beta=0.5 + 0.2 * i,
                          seed=seed, rep=40 + i, want=want, H=_h_from_plus(inst, ej, plus),
                          M=(2 * plus - ncls[None, :]).sum(axis=1), EJ=ej))
    return specs


def _make(sk, sp):
    if sp["kind"] == "torus":
        return sk.Chain.torus(sp["L"], q=sp["q"], beta=sp["beta"], seed=sp["seed"], replica=sp["rep"],
                              lam_values=[sp["lam"]])
    inst = sp["inst"]
    return sk.Chain.graph(sp["n"], inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                          lam_class=inst.cls, q=sp["q"], beta=sp["beta"], seed=sp["seed"],
                          replica=sp["rep"])


def test_batch_persistent_mixed(sk):
    """Persistent strategy: tori (ragged and full 256) and graphs (ragged, up to
    65536 vertices), spins in LDS for all steps; every chain bit-exact, logs
    included, and the same as the grid strategy."""
    T = 30
    _print_case("persistent mixed")
    specs = _mixed_specs(T, [16, 48, 100, 256], [1024, 2050, 65536])
    chains = [_make(sk, sp) for sp in specs]
    b = sk.Batch(chains, strategy="auto", record=True)
    st, _ = b.info()
    assert st == sk.SHAKEN_BATCH_PERSISTENT
    b.sweep(T)
    for i, sp in enumerate(specs):
        assert np.array_equal(chains[i].spins().reshape(sp["want"].shape), sp["want"]), i
        h, m = b.log(i, with_H=sp["H"] is not None)
        assert np.array_equal(m, sp["M"]), i
        if sp["H"] is not None:
            assert np.array_equal(h, sp["H"]), i
        assert chains[i].observables().E_J == sp["EJ"][-1]
    # the chains continue on their own from where the batch left them
    sp = specs[0]
    x, _, _ = oracle.torus_run(sp["want"], 1, sp["lam"], sp["q"], sp["beta"], sp["seed"], sp["rep"], 3, s0=2 * T)
    chains[0].sweep(3)
    assert np.array_equal(chains[0].spins(), x)


@pytest.mark.parametrize("strategy", ["grid", "persistent"])
def test_batch_log_reserve_and_growth(sk, strategy):
    """Logs of consecutive sweeps of different lengths, within the reserved log
    space and beyond it (the batch then grows it), against the oracle's
    trajectory cut at the same points."""
    lengths = [7, 20, 3, 33]
    T = sum(lengths)
    _print_case("log reserve", strategy)
    specs = _mixed_specs(T, [16, 100], [1024, 2050], seed0=11)
    chains = [_make(sk, sp) for sp in specs]
    with pytest.raises(sk.ShakenError):
        sk.Batch(chains, strategy=strategy, record=True, log_reserve=-1)
    b = sk.Batch(chains, strategy=strategy, record=True, use_hipgraph=(strategy == "grid"),
                 log_reserve=20)
    t0 = 0
    for n_full in lengths:
        b.sweep(n_full)
        _, M_all, EJ_all = b.logs()           # every chain with one device copy
        for i, sp in enumerate(specs):
            h, m = b.log(i, with_H=sp["H"] is not None)
            assert np.array_equal(m, sp["M"][t0:t0 + n_full + 1]), (i, n_full)
            if sp["H"] is not None:
                assert np.array_equal(h, sp["H"][t0:t0 + n_full + 1]), (i, n_full)
            ej, m2 = b.log_ej(i)
            assert np.array_equal(ej, sp["EJ"][t0:t0 + n_full + 1]), (i, n_full)
            assert np.array_equal(m2, m) and np.array_equal(M_all[i], m), (i, n_full)
            assert np.array_equal(EJ_all[i], ej), (i, n_full)
        t0 += n_full
    for i, sp in enumerate(specs):
        assert np.array_equal(chains[i].spins().reshape(sp["want"].shape), sp["want"]), i
    b.close()
    for c in chains:
        c.close()


def test_batch_persistent_equals_grid(sk):
    T = 12
    specs = _mixed_specs(T, [32, 80], [4096], seed0=3)
    a = [_make(sk, sp) for sp in specs]
    c = [_make(sk, sp) for sp in specs]
    ba = sk.Batch(a, strategy="persistent")
    bc = sk.Batch(c, strategy="grid", use_hipgraph=True)
    ba.sweep(T)
    bc.sweep(T)
    for x, y, sp in zip(a, c, specs):
        assert np.array_equal(x.spins(), y.spins())
        assert np.array_equal(x.spins().reshape(sp["want"].shape), sp["want"])


@pytest.mark.parametrize("n,deg", [(1002, 3), (4096, 4), (37, 2), (65536, 3)])
def test_graph_ell_equals_csr_equals_oracle(sk, n, deg):
    """The CSR, ELL and packed layouts give the same trajectory as the oracle
    (grid and persistent strategies; the grid kernels read ELL where the packed
    record is given)."""
    T = 40
    _print_case("ell vs csr", n, deg)
    inst = synth.oriented_instance(n, deg, 300 + n, lam_values=(-0.5, 0.5), pm_j=True)
    g = oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    sp0 = oracle.graph_init_random(n, 4, 1)
    want, ej, plus = oracle.graph_run(g, sp0, 0.9, 0.6, 4, 1, T)
    layouts = ("csr", "ell", "packed", "auto") if deg <= 3 else ("csr", "ell", "auto")
    for layout in layouts:
        for strat in ("grid", "persistent"):
            ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                                lam_class=inst.cls, q=0.9, beta=0.6, seed=4, replica=1, layout=layout)
            b = sk.Batch([ch], strategy=strat, record=True)
            b.sweep(T)
            h, m = b.log(0)
            assert np.array_equal(ch.spins(), want), (layout, strat)
            assert np.array_equal(h, _h_from_plus(inst, ej, plus)), (layout, strat)
            b.close()
            ch.close()


def test_batch_auto_strategy_choice(sk):
    """AUTO: persistent when every chain fits in LDS (tori up to 256^2), grid as
    soon as one does not; both give the oracle's trajectory."""
    tori = [sk.Chain.torus(L, q=1.0, beta=0.4, seed=60 + L, replica=L) for L in (16, 40)]
    b = sk.Batch(tori)
    assert b.info()[0] == sk.SHAKEN_BATCH_PERSISTENT
    b.close()
    # 300^2 needs 3000 words of LDS per buffer: the whole batch runs on the grid
    small = sk.Chain.torus(24, q=1.0, beta=0.4, seed=324, replica=24)
    big = sk.Chain.torus(300, q=1.0, beta=0.4, seed=600, replica=300)
    b = sk.Batch([small, big])
    assert b.info()[0] == sk.SHAKEN_BATCH_GRID
    b.sweep(5)
    b.close()
    for ch, L in ((small, 24), (big, 300)):
        want, _, _ = oracle.torus_run(oracle.torus_init_random(L, 300 + L, L), 1, 0.0, 1.0, 0.4,
                                      300 + L, L, 5)
        assert np.array_equal(ch.spins(), want)
    with pytest.raises(sk.ShakenError):
        sk.Batch([small, big], track=True)
    small.close()
    big.close()
    inst = synth.oriented_instance(100, 3, 61, lam_values=(0.0,), pm_j=True)
    g = sk.Chain.graph(inst.n, inst.src, inst.dst, J=inst.J, q=1.0, beta=0.4, seed=61, replica=7)
    b = sk.Batch(tori + [g])
    assert b.info()[0] == sk.SHAKEN_BATCH_PERSISTENT
    b.sweep(5)
    b.close()
    for ch, L in zip(tori, (16, 40)):
        want, _, _ = oracle.torus_run(oracle.torus_init_random(L, 60 + L, L), 1, 0.0, 1.0, 0.4, 60 + L, L, 5)
        assert np.array_equal(ch.spins(), want)
        ch.close()
    og = oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    want, _, _ = oracle.graph_run(og, oracle.graph_init_random(inst.n, 61, 7), 1.0, 0.4, 61, 7, 5)
    assert np.array_equal(g.spins(), want)
    g.close()


@pytest.mark.parametrize("n,deg,strategy", [(1000, 3, "grid"), (1000, 3, "persistent"),
                                             (2002, 2, "grid"), (2002, 2, "persistent")])
def test_split_graph_parity(sk, n, deg, strategy):
    """Generalised split (section 5): every edge of a random regular graph given
    in both orientations with independent +-1 couplings (degree 2: the ELL
    layout applies); bit-exact with the oracle, logs included."""
    T = 40
    _print_case("split graph", n, deg, strategy)
    inst = synth.oriented_instance(n, deg, 500 + n + deg, lam_values=(-0.5, 0.5), pm_j=True)
    rng = np.random.Generator(np.random.PCG64(n + deg))
    src = np.concatenate([inst.src, inst.dst]).astype(np.int32)
    dst = np.concatenate([inst.dst, inst.src]).astype(np.int32)
    J = np.where(rng.integers(0, 2, src.shape[0]) == 1, 1, -1).astype(np.int8)
    g = oracle.Graph(n, src, dst, J, inst.cls, inst.lam_values)
    sp0 = oracle.graph_init_random(n, 8, 2)
    want, ej, plus = oracle.graph_run(g, sp0, 1.3, 0.7, 8, 2, T)
    ch = sk.Chain.graph(n, src, dst, J=J, lam_values=inst.lam_values, lam_class=inst.cls, q=1.3,
                        beta=0.7, seed=8, replica=2, split=True)
    b = sk.Batch([ch], strategy=strategy, record=True)
    b.sweep(T)
    h, m = b.log(0)
    assert np.array_equal(ch.spins(), want)
    ncls = np.bincount(inst.cls, minlength=2)
    assert np.array_equal(m, (2 * plus - ncls[None, :]).sum(axis=1))
    assert np.array_equal(h, _h_from_plus(inst, ej, plus))
    b.close()
    ch.close()


def test_batch_run_one_call(sk):
    """shaken_batch_run: create, sweep, read the final H, free -- in one call
    through the C ABI; chains continue on their own afterwards."""
    T = 20
    L = 40
    inst = synth.oriented_instance(1002, 3, 71, lam_values=(-0.5, 0.5), pm_j=True)
    tor = sk.Chain.torus(L, q=0.9, beta=0.45, seed=71, replica=1, lam_values=[0.5])
    gr = sk.Chain.graph(inst.n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                        lam_class=inst.cls, q=1.2, beta=0.7, seed=72, replica=2)
    o = sk.shaken_batch_opts(sk.SHAKEN_BATCH_AUTO, 0, 0, 0, None, 0, 0)
    H = np.zeros(2, dtype=np.int64)
    Hb = np.zeros(2, dtype=np.int64)
    res = sk.shaken_run_result(H_final=H.ctypes.data_as(sk._i64p), H_best=Hb.ctypes.data_as(sk._i64p))
    sk.shaken_batch_run([tor.handle, gr.handle], T, o, None, res)
    assert res.chunks == 1 and res.fallbacks == 0
    wt, ejt, mmt = oracle.torus_run(oracle.torus_init_random(L, 71, 1), 1, 0.5, 0.9, 0.45, 71, 1, T)
    og = oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    wg, ejg, plg = oracle.graph_run(og, oracle.graph_init_random(inst.n, 72, 2), 1.2, 0.7, 72, 2, T)
    assert np.array_equal(tor.spins(), wt) and np.array_equal(gr.spins(), wg)
    assert H[0] == -ejt[-1] - mmt[-1]
    assert H[1] == _h_from_plus(inst, ejg, plg)[-1]
    assert Hb[0] == (-ejt - mmt).min()
    assert Hb[1] == _h_from_plus(inst, ejg, plg).min()
    tor.sweep(2)
    wt2, _, _ = oracle.torus_run(wt, 1, 0.5, 0.9, 0.45, 71, 1, 2, s0=2 * T)
    assert np.array_equal(tor.spins(), wt2)
    tor.close()
    gr.close()


def test_persistent_hipgraph_and_autotune_equal_eager(sk):
    """Persistent strategy under a captured HIP graph with the workgroup count
    autotuned: replays of one capture (5 full steps), a re-capture at another
    length and back, with log reads (eager copies and synchronisations)
    between the replays; every call equals the eager batch and the oracle."""
    calls = [5, 5, 5, 8, 5, 5]
    T = sum(calls)
    _print_case("persistent hipgraph", calls)
    specs = _mixed_specs(T, [16, 100, 256], [1024, 2050], seed0=21)
    a = [_make(sk, sp) for sp in specs]
    c = [_make(sk, sp) for sp in specs]
    ba = sk.Batch(a, strategy="persistent", record=True)
    bc = sk.Batch(c, strategy="persistent", record=True, use_hipgraph=True, autotune=True)
    assert bc.info()[0] == sk.SHAKEN_BATCH_PERSISTENT
    t0 = 0
    for n_full in calls:
        ba.sweep(n_full)
        bc.sweep(n_full)
        _, Ma, EJa = ba.logs()
        _, Mc, EJc = bc.logs()
        assert np.array_equal(Ma, Mc) and np.array_equal(EJa, EJc), n_full
        for i, sp in enumerate(specs):
            assert np.array_equal(Mc[i], sp["M"][t0:t0 + n_full + 1]), (i, t0)
            assert np.array_equal(EJc[i], sp["EJ"][t0:t0 + n_full + 1]), (i, t0)
        t0 += n_full
    for i, sp in enumerate(specs):
        assert np.array_equal(c[i].spins().reshape(sp["want"].shape), sp["want"]), i
        assert np.array_equal(a[i].spins(), c[i].spins()), i
    ba.close()
    bc.close()
    for x in a + c:
        x.close()


@pytest.mark.parametrize("strategy", ["grid", "persistent"])
def test_autotune_cached_shapes(sk, strategy):
    """autotune="cached": the first batch of a shape measures, a second batch
    of the same shape (fresh chains, same seeds) reuses the result without
    measuring and runs bit for bit like the first and the oracle; a batch of
    another shape measures again; autotune values other than 0, 1, 2 are
    rejected."""
    T = 6
    _print_case("autotune cached", strategy)
    specs = _mixed_specs(T, [16, 100], [1024], seed0=91)
    a = [_make(sk, sp) for sp in specs]
    c = [_make(sk, sp) for sp in specs]
    ba = sk.Batch(a, strategy=strategy, record=True, use_hipgraph=True, autotune="cached")
    ba.sweep(T)
    bc = sk.Batch(c, strategy=strategy, record=True, use_hipgraph=True, autotune="cached")
    bc.sweep(T)
    assert ba.counters()["autotunes"] <= 1 and bc.counters()["autotunes"] == 0
    assert ba.launch_shape(0) == bc.launch_shape(0)
    _, Ma, EJa = ba.logs()
    _, Mc, EJc = bc.logs()
    assert np.array_equal(Ma, Mc) and np.array_equal(EJa, EJc)
    for i, sp in enumerate(specs):
        assert np.array_equal(c[i].spins().reshape(sp["want"].shape), sp["want"]), i
        assert np.array_equal(Mc[i], sp["M"]) and np.array_equal(EJc[i], sp["EJ"]), i
    # another shape measures
    specs2 = _mixed_specs(2, [48], [1030], seed0=93)
    d = [_make(sk, sp) for sp in specs2]
    bd = sk.Batch(d, strategy=strategy, record=True, use_hipgraph=True, autotune="cached")
    bd.sweep(2)
    assert bd.counters()["autotunes"] == 1
    for b in (ba, bc, bd):
        b.close()
    import ctypes
    o = sk.shaken_batch_opts(sk._STRAT[strategy], 0, 3, 0, None, 0, 0)
    arr = (ctypes.c_void_p * len(a))(*[x.handle.value for x in a])
    h = ctypes.c_void_p()
    assert sk._lib.shaken_batch_create(ctypes.byref(h), arr, len(a), ctypes.byref(o)) == sk.SHAKEN_EINVAL
    assert not h.value
    with pytest.raises(ValueError):
        sk.Batch(a, autotune="sometimes")
    for x in a + c + d:
        x.close()
