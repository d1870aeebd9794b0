"""The LDS-staged graph kernel (the configuration copied bit-packed into LDS,
every neighbour gather an LDS read) against the oracle, bit-exact: final
configurations and the H / M logs of every full step.

Forced with graph_kernel="lds" on sizes the default would give to the plain
kernel too: one vertex, ragged n (not a multiple of 4 or 32), the largest n
it takes (1,179,648) and one beyond (which falls back), both spin formats,
many field classes, the reversed order, the frozen set, split couplings,
single half-steps from odd counters with configurations set in between (the
int8 chains' packed mirror is rebuilt at every call), grid batches of mixed
sizes (a chain smaller than the grid leaves its surplus workgroups), and the
sweep that allocates nothing."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

LDS_MAX = 1_179_648


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


def _instance(n, seed):
    if n >= 4 and n % 2 == 0:
        return synth.oriented_instance(n, 3, seed, lam_values=(-0.5, 0.0, 0.5), pm_j=True)
    p = min(1.0, 3.0 / max(n - 1, 1))
    return synth.random_oriented_graph(n, p, seed, jmax=2, n_classes=3, lam_scale=0.5)


def _oracle_graph(inst):
    return oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)


def _H_M(inst, ej, plus):
    ncls = np.bincount(inst.cls, minlength=len(inst.lam_values))
    lam2 = np.rint(2 * inst.lam_values).astype(np.int64)
    Mk = 2 * plus - ncls[None, :]
    return -ej - (Mk * lam2[None, :]).sum(axis=1), Mk.sum(axis=1)


def _chain(sk, inst, seed, replica=0, **kw):
    return sk.Chain.graph(inst.n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                          lam_class=inst.cls, q=1.5, beta=0.8, seed=seed, replica=replica, **kw)


@pytest.mark.parametrize("fmt", ["int8", "bitpacked"])
@pytest.mark.parametrize("n", [1, 5, 37, 1002, 4099, 65538, 131072, 200002, LDS_MAX, LDS_MAX + 2])
def test_lds_kernel_sizes(sk, n, fmt):
    T = 30 if n < 100_000 else 8
    _print_case("graph lds", n, fmt)
    inst = _instance(n, 500 + n % 1000)
    g = _oracle_graph(inst)
    ch = _chain(sk, inst, 11, replica=3, fmt=fmt, graph_kernel="lds")
    sp0 = oracle.graph_init_random(n, 11, 3)
    assert np.array_equal(ch.spins(), sp0)
    want, ej, plus = oracle.graph_run(g, sp0, 1.5, 0.8, 11, 3, T)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    Hw, Mw = _H_M(inst, ej, plus)
    assert np.array_equal(H, Hw) and np.array_equal(M, Mw)
    ch.close()


def test_lds_kernel_many_classes_and_couplings(sk):
    """Erdos-Renyi graph with couplings up to +-5 and seven field classes."""
    n, T = 3001, 40
    inst = synth.random_oriented_graph(n, 0.002, 77, jmax=5, n_classes=7, lam_scale=0.5)
    g = _oracle_graph(inst)
    ch = sk.Chain.graph(n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values, lam_class=inst.cls,
                        q=0.6, beta=0.7, seed=3, replica=2, graph_kernel="lds")
    want, ej, plus = oracle.graph_run(g, oracle.graph_init_random(n, 3, 2), 0.6, 0.7, 3, 2, T)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    Hw, Mw = _H_M(inst, ej, plus)
    assert np.array_equal(H, Hw) and np.array_equal(M, Mw)
    ch.close()


@pytest.mark.parametrize("fmt", ["int8", "bitpacked"])
def test_lds_kernel_single_half_steps_and_set_spins(sk, fmt):
    """Calls of one and three half-steps, starting at odd counters, a
    configuration set between calls and a checkpoint restore to an odd
    counter: each call packs the configuration it reads."""
    n = 200_002
    inst = _instance(n, 91)
    g = _oracle_graph(inst)
    ch = _chain(sk, inst, 5, fmt=fmt, graph_kernel="lds")
    x = oracle.graph_init_random(n, 5, 0)
    s = 0
    rng = np.random.Generator(np.random.PCG64(4))
    for k, steps in enumerate([1, 3, 1, 2, 1]):
        ch.half_step(steps)
        for _ in range(steps):
            x = oracle.graph_half_step(g, x, 1.5, 0.8, 5, 0, s)
            s += 1
        assert np.array_equal(ch.spins(), x), (k, s)
        if k == 2:
            x = np.where(rng.integers(0, 2, n) == 1, 1, -1).astype(np.int8)
            ch.set_spins(x)
    ch.set_half_step(s + 1)   # restore: the same configuration read at s + 1
    s += 1
    ch.half_step(2)
    for _ in range(2):
        x = oracle.graph_half_step(g, x, 1.5, 0.8, 5, 0, s)
        s += 1
    assert np.array_equal(ch.spins(), x)
    ch.close()


def test_lds_kernel_reversed_frozen_split(sk):
    n, T = 150_000, 6
    inst = _instance(n, 33)
    g = _oracle_graph(inst)
    # reversed order = the forward order on the reversed edge set
    ch = _chain(sk, inst, 8, reversed=True, graph_kernel="lds")
    gr = oracle.Graph(n, inst.dst, inst.src, inst.J, inst.cls, inst.lam_values)
    want, _, _ = oracle.graph_run(gr, oracle.graph_init_random(n, 8, 0), 1.5, 0.8, 8, 0, T, log=False)
    ch.sweep(T)
    assert np.array_equal(ch.spins(), want)
    ch.close()
    # frozen set B: every 7th vertex stays +1
    fz = (np.arange(n) % 7) == 0
    ch = _chain(sk, inst, 9, frozen=fz, graph_kernel="lds")
    want, ej, plus = oracle.graph_run_frozen(g, oracle.graph_init_random(n, 9, 0), fz, 1.5, 0.8, 9, 0, T)
    H, M = ch.sweep(T, log=True)
    assert np.array_equal(ch.spins(), want)
    Hw, Mw = _H_M(inst, ej, plus)
    assert np.array_equal(H, Hw) and np.array_equal(M, Mw)
    ch.close()
    # generalised split: every edge in both orientations
    src = np.concatenate([inst.src, inst.dst])
    dst = np.concatenate([inst.dst, inst.src])
    J = np.concatenate([inst.J, inst.J])
    gs = oracle.Graph(n, src, dst, J, inst.cls, inst.lam_values)
    ch = sk.Chain.graph(n, src, dst, J=J, lam_values=inst.lam_values, lam_class=inst.cls, q=1.5, beta=0.8,
                        seed=10, split=True, graph_kernel="lds")
    want, _, _ = oracle.graph_run(gs, oracle.graph_init_random(n, 10, 0), 1.5, 0.8, 10, 0, T, log=False)
    ch.sweep(T)
    assert np.array_equal(ch.spins(), want)
    ch.close()


@pytest.mark.parametrize("fmt", ["int8", "bitpacked"])
def test_lds_kernel_grid_batch_mixed_sizes(sk, fmt):
    """One grid batch (HIP graph replay, recorded logs) of graphs of 1002,
    70002 and 300000 vertices on the staged kernel: the small chains leave
    their surplus workgroups; every chain equal to the oracle."""
    T = 20
    sizes = [1002, 70002, 300000]
    insts = [_instance(n, 700 + i) for i, n in enumerate(sizes)]
    chains = [_chain(sk, x, 20 + i, replica=i, fmt=fmt, graph_kernel="lds") for i, x in enumerate(insts)]
    b = sk.Batch(chains, strategy="grid", use_hipgraph=True, record=True)
    b.sweep(T)
    for i, x in enumerate(insts):
        want, ej, plus = oracle.graph_run(_oracle_graph(x), oracle.graph_init_random(x.n, 20 + i, i), 1.5, 0.8,
                                          20 + i, i, T)
        assert np.array_equal(chains[i].spins(), want), i
        H, M = b.log(i)
        Hw, Mw = _H_M(x, ej, plus)
        assert np.array_equal(H, Hw) and np.array_equal(M, Mw), i
    b.close()
    for c in chains:
        c.close()


def test_lds_kernel_noalloc_sweep(sk):
    import torch
    n, T = 140_000, 12
    inst = _instance(n, 55)
    a = _chain(sk, inst, 4, graph_kernel="lds")
    b = _chain(sk, inst, 4, graph_kernel="plain")
    H = torch.empty(T + 1, dtype=torch.int64, device="cuda")
    M = torch.empty(T + 1, dtype=torch.int64, device="cuda")
    a.sweep_noalloc(T, H, M)
    torch.cuda.synchronize()
    Hb, Mb = b.sweep(T, log=True)
    assert np.array_equal(H.cpu().numpy(), Hb) and np.array_equal(M.cpu().numpy(), Mb)
    assert np.array_equal(a.spins(), b.spins())
    a.close()
    b.close()


@pytest.mark.parametrize("fmt", ["int8", "bitpacked"])
def test_lds_kernel_extreme_couplings(sk, fmt):
    """Couplings at the ends of the int8 range (-128 and 127 included) on a
    3-regular graph (every lane's edges in one window: the packed per-vertex
    sums) and on an Erdos-Renyi graph of mean degree 12 (lanes with more
    edges than one window); the threshold table is then too large for LDS."""
    rng = np.random.Generator(np.random.PCG64(17))
    vals = np.array([-128, -127, -64, -1, 1, 63, 126, 127], dtype=np.int8)
    for inst, T in [(_instance(100_002, 41), 8),
                    (synth.random_oriented_graph(2001, 0.006, 43, jmax=1, n_classes=3, lam_scale=0.5), 12)]:
        _print_case("graph lds extreme J", inst.n, fmt)
        J = rng.choice(vals, size=inst.J.shape[0]).astype(np.int8)
        g = oracle.Graph(inst.n, inst.src, inst.dst, J, inst.cls, inst.lam_values)
        ch = sk.Chain.graph(inst.n, inst.src, inst.dst, J=J, lam_values=inst.lam_values, lam_class=inst.cls,
                            q=2.0, beta=0.01, seed=6, replica=1, fmt=fmt, graph_kernel="lds")
        want, ej, plus = oracle.graph_run(g, oracle.graph_init_random(inst.n, 6, 1), 2.0, 0.01, 6, 1, T)
        H, M = ch.sweep(T, log=True)
        assert np.array_equal(ch.spins(), want)
        Hw, Mw = _H_M(inst, ej, plus)
        assert np.array_equal(H, Hw) and np.array_equal(M, Mw)
        ch.close()


def _max_half_degree(inst):
    return max(np.bincount(inst.dst, minlength=inst.n).max(), np.bincount(inst.src, minlength=inst.n).max())


@pytest.mark.parametrize("fmt", ["int8", "bitpacked"])
def test_lds_kernel_three_slot_layout(sk, fmt):
    """Graphs whose half-degrees are at most three and whose couplings share
    one magnitude run on the three-slot layout (twelve slots per lane, empty
    slots reading a zero word, the field j0 (2 count - degree)): magnitudes
    2, 127 and 128 with both signs, ragged n, reversed order and a frozen
    set; then grid batches where every chain has the layout and where one
    chain lacks it (the launch then takes the row-bound layout for all)."""
    rng = np.random.Generator(np.random.PCG64(23))
    base = synth.oriented_instance(100_002, 3, 61, lam_values=(-0.5, 0.0, 0.5), pm_j=True)
    assert _max_half_degree(base) <= 3
    m = base.J.shape[0]
    cases = [(2 * base.J).astype(np.int8),
             np.where(rng.integers(0, 2, m) == 1, 127, -127).astype(np.int8),
             np.full(m, -128, dtype=np.int8)]
    for k, J in enumerate(cases):
        _print_case("graph lds three-slot", k, fmt)
        g = oracle.Graph(base.n, base.src, base.dst, J, base.cls, base.lam_values)
        ch = sk.Chain.graph(base.n, base.src, base.dst, J=J, lam_values=base.lam_values, lam_class=base.cls,
                            q=1.5, beta=0.05 if k else 0.4, seed=30 + k, replica=k, fmt=fmt, graph_kernel="lds")
        T = 12
        want, ej, plus = oracle.graph_run(g, oracle.graph_init_random(base.n, 30 + k, k), 1.5,
                                          0.05 if k else 0.4, 30 + k, k, T)
        H, M = ch.sweep(T, log=True)
        assert np.array_equal(ch.spins(), want), k
        Hw, Mw = _H_M(base, ej, plus)
        assert np.array_equal(H, Hw) and np.array_equal(M, Mw), k
        ch.close()
    J = cases[0]
    # reversed order and a frozen set on the same layout
    _print_case("graph lds three-slot reversed/frozen", fmt)
    gr = oracle.Graph(base.n, base.dst, base.src, J, base.cls, base.lam_values)
    ch = sk.Chain.graph(base.n, base.src, base.dst, J=J, lam_values=base.lam_values, lam_class=base.cls,
                        q=1.5, beta=0.4, seed=40, reversed=True, fmt=fmt, graph_kernel="lds")
    want, _, _ = oracle.graph_run(gr, oracle.graph_init_random(base.n, 40, 0), 1.5, 0.4, 40, 0, 8, log=False)
    ch.sweep(8)
    assert np.array_equal(ch.spins(), want)
    ch.close()
    fz = (np.arange(base.n) % 5) == 2
    g = oracle.Graph(base.n, base.src, base.dst, J, base.cls, base.lam_values)
    ch = sk.Chain.graph(base.n, base.src, base.dst, J=J, lam_values=base.lam_values, lam_class=base.cls,
                        q=1.5, beta=0.4, seed=41, frozen=fz, fmt=fmt, graph_kernel="lds")
    want, ej, plus = oracle.graph_run_frozen(g, oracle.graph_init_random(base.n, 41, 0), fz, 1.5, 0.4, 41, 0, 8)
    H, M = ch.sweep(8, log=True)
    assert np.array_equal(ch.spins(), want)
    Hw, Mw = _H_M(base, ej, plus)
    assert np.array_equal(H, Hw) and np.array_equal(M, Mw)
    ch.close()
    # grid batches: all on the three-slot layout, then mixed with a graph of
    # mean degree 6 (half-degrees above three)
    other = synth.random_oriented_graph(3001, 0.002, 45, jmax=1, n_classes=3, lam_scale=0.5)
    assert _max_half_degree(other) > 3
    small = synth.oriented_instance(2_050, 3, 62, lam_values=(-0.5, 0.0, 0.5), pm_j=True)
    for members in ([base, small], [base, other, small]):
        _print_case("graph lds three-slot batch", len(members), fmt)
        chains = [_chain(sk, x, 50 + i, replica=i, fmt=fmt, graph_kernel="lds") for i, x in enumerate(members)]
        b = sk.Batch(chains, strategy="grid", use_hipgraph=True, record=True)
        b.sweep(10)
        for i, x in enumerate(members):
            want, ej, plus = oracle.graph_run(_oracle_graph(x), oracle.graph_init_random(x.n, 50 + i, i), 1.5,
                                              0.8, 50 + i, i, 10)
            assert np.array_equal(chains[i].spins(), want), i
            H, M = b.log(i)
            Hw, Mw = _H_M(x, ej, plus)
            assert np.array_equal(H, Hw) and np.array_equal(M, Mw), i
        b.close()
        for c in chains:
            c.close()


@pytest.mark.parametrize("fmt", ["int8", "bitpacked"])
def test_lds_kernel_three_slot_degenerate(sk, fmt):
    """The three-slot layout with every slot empty (graphs without edges, n = 1
    and a ragged n) and with half-degrees of at most one (a perfect matching,
    each pair one coin-oriented edge of coupling +-2): the field is q sigma +
    lambda alone, or one neighbour's."""
    rng = np.random.Generator(np.random.PCG64(29))
    cases = []
    for n in (1, 4099):
        cases.append(synth.random_oriented_graph(n, 0.0, 30 + n, jmax=1, n_classes=3, lam_scale=0.5))
    n = 10_002
    perm = rng.permutation(n).astype(np.int32)
    u, v = perm[0::2], perm[1::2]
    flip = rng.integers(0, 2, n // 2).astype(bool)
    src, dst = np.where(flip, v, u).astype(np.int32), np.where(flip, u, v).astype(np.int32)
    J = np.where(rng.integers(0, 2, n // 2) == 1, 2, -2).astype(np.int8)
    cls = rng.integers(0, 3, n).astype(np.uint8)
    cases.append(synth.Instance(n, src, dst, J, cls, np.array([-0.5, 0.0, 0.5])))
    for k, inst in enumerate(cases):
        _print_case("graph lds three-slot degenerate", inst.n, inst.src.shape[0], fmt)
        assert inst.src.shape[0] == 0 or _max_half_degree(inst) <= 1
        g = _oracle_graph(inst)
        ch = _chain(sk, inst, 70 + k, replica=k, fmt=fmt, graph_kernel="lds")
        T = 15
        want, ej, plus = oracle.graph_run(g, oracle.graph_init_random(inst.n, 70 + k, k), 1.5, 0.8, 70 + k, k, T)
        H, M = ch.sweep(T, log=True)
        assert np.array_equal(ch.spins(), want), k
        Hw, Mw = _H_M(inst, ej, plus)
        assert np.array_equal(H, Hw) and np.array_equal(M, Mw), k
        ch.close()
