"""Pins of the C trajectory oracle against the paper: the worked
zero-temperature example (proof of Theorem 3.3), the zero-temperature sign
law read off the pair Hamiltonian, chi^2 of one-step and long-run laws against
exact enumeration (Theorem 2.3), the first-exit law from the all-minus state,
and the energy observable against equation ham1.  CPU only."""
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import enumeration as en
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "zero_temperature_diagonal.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *rest = line.split()
            vals[k] = rest
    return vals


def _plus_sites(sp):
    return set(map(tuple, np.argwhere(sp > 0)))


@pytest.mark.parametrize("L,r0,c0", [(8, 3, 2), (9, 0, 0), (10, 7, 9), (16, 5, 11)])
def test_zero_temperature_diagonal_growth(L, r0, c0):
    g = _golden()
    J = int(g["J"][0]); q = float(g["q"][0]); lam = float(g["lambda"][0]); b = float(g["beta"][0])
    # paper (i, j) = (col, row)
    def to_rc(off):
        di, dj = map(int, off.split(","))
        return ((r0 + dj) % L, (c0 + di) % L)
    sp = -np.ones((L, L), dtype=np.int8)
    sp[r0, c0] = 1
    a = oracle.torus_half_step(sp, J, lam, q, b, seed=1, replica=0, s=0)
    assert _plus_sites(a) == {to_rc(o) for o in g["after_dl"]}
    bb = oracle.torus_half_step(a, J, lam, q, b, seed=1, replica=0, s=1)
    assert _plus_sites(bb) == {to_rc(o) for o in g["after_ur"]}
    diag = {(r, c) for r in range(L) for c in range(L) if (r + c - r0 - c0) % L == 0}
    fin, _, _ = oracle.torus_run(sp, J, lam, q, b, seed=1, replica=0, n_full=L // 2)
    assert _plus_sites(fin) == diag
    early, _, _ = oracle.torus_run(sp, J, lam, q, b, seed=1, replica=0, n_full=L // 2 - 1)
    assert _plus_sites(early) != diag


def _rand_spins(rng, n):
    return np.where(rng.integers(0, 2, n) == 1, 1, -1).astype(np.int8)


@pytest.mark.parametrize("L", [3, 4, 5])
def test_zero_temperature_torus_follows_pair_hamiltonian_fields(L):
    """At beta -> infinity each half-step sets every spin to the sign of its
    field; the fields come from the pair Hamiltonian of ham2 (enumeration
    model with E^o = {(x,x_up),(x,x_right)}), dl first, then ur."""
    q, lam = 0.5, 0.25     # fields never vanish
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, lam=np.full(L * L, lam), q=q, beta=1.0)
    rng = np.random.Generator(np.random.PCG64(L))
    for _ in range(20):
        sp = _rand_spins(rng, L * L)
        want1 = np.sign(m.field12_of(sp)).astype(np.int8)
        got1 = oracle.torus_half_step(sp.reshape(L, L), 1, lam, q, 1000.0, 5, 0, 0).reshape(-1)
        assert np.array_equal(got1, want1)
        want2 = np.sign(m.field21_of(got1)).astype(np.int8)
        got2 = oracle.torus_half_step(got1.reshape(L, L), 1, lam, q, 1000.0, 5, 0, 1).reshape(-1)
        assert np.array_equal(got2, want2)


def _small_graph(seed=3, n=6):
    inst = synth.random_oriented_graph(n, 0.6, seed, jmax=2, n_classes=3, lam_scale=0.25)
    g = oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    return inst, g


def test_zero_temperature_graph_follows_pair_hamiltonian_fields():
    inst, g = _small_graph(seed=4, n=8)
    q = 0.5
    lam = inst.lam_values[inst.cls]
    m = en.Model(inst.n, inst.src, inst.dst, J=inst.J.astype(float), lam=lam, q=q, beta=1.0)
    assert np.all(np.abs(m.fields12()) > 1e-9) and np.all(np.abs(m.fields21()) > 1e-9)
    rng = np.random.Generator(np.random.PCG64(9))
    for _ in range(30):
        sp = _rand_spins(rng, inst.n)
        i = en.index_of(sp)
        got1 = oracle.graph_half_step(g, sp, q, 1000.0, 1, 0, 0)
        assert np.array_equal(got1, np.sign(m.fields12()[i]).astype(np.int8))
        got2 = oracle.graph_half_step(g, got1, q, 1000.0, 1, 0, 1)
        assert np.array_equal(got2, np.sign(m.fields21()[en.index_of(got1)]).astype(np.int8))


def _chi2_p(counts, probs):
    probs = np.asarray(probs)
    keep = probs * counts.sum() >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(probs[keep], probs[~keep].sum()) * counts.sum()
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    return stats.chisquare(obs, exp).pvalue


def test_graph_one_step_law_chi2():
    """Empirical law of one half-step and of one full step from a fixed
    configuration, over replicas, against P^{1->2} and P^sh rows."""
    inst, g = _small_graph(seed=3, n=6)
    q, b = 0.7, 0.6
    lam = inst.lam_values[inst.cls]
    m = en.Model(inst.n, inst.src, inst.dst, J=inst.J.astype(float), lam=lam, q=q, beta=b)
    sp = np.array([1, -1, -1, 1, 1, -1], dtype=np.int8)
    i0 = en.index_of(sp)
    n = 20000
    half = np.zeros(2 ** inst.n)
    full = np.zeros(2 ** inst.n)
    for r in range(n):
        a = oracle.graph_half_step(g, sp, q, b, 77, r, 0)
        half[en.index_of(a)] += 1
        c = oracle.graph_half_step(g, a, q, b, 77, r, 1)
        full[en.index_of(c)] += 1
    assert _chi2_p(half, m.P12()[i0]) > 1e-4
    assert _chi2_p(full, m.Psh()[i0]) > 1e-4


def test_torus_one_step_law_chi2():
    L, q, lam, b = 3, 0.6, 0.2, 0.5
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, lam=np.full(L * L, lam), q=q, beta=b)
    sp = np.array([1, -1, 1, 1, 1, -1, -1, -1, 1], dtype=np.int8).reshape(L, L)
    i0 = en.index_of(sp.reshape(-1))
    n = 30000
    full = np.zeros(2 ** (L * L))
    for r in range(n):
        a = oracle.torus_half_step(sp, 1, lam, q, b, 5, r, 0)
        c = oracle.torus_half_step(a, 1, lam, q, b, 5, r, 1)
        full[en.index_of(c.reshape(-1))] += 1
    assert _chi2_p(full, m.Psh()[i0]) > 1e-4


def test_graph_long_run_law_chi2():
    """States after many full steps, over independent replicas, against the
    stationary law pi of Theorem 2.3 (parameters where 25 steps mix)."""
    inst = synth.random_oriented_graph(6, 0.6, 3, jmax=1, n_classes=3, lam_scale=0.25)
    g = oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    q, b = 0.7, 0.3
    lam = inst.lam_values[inst.cls]
    m = en.Model(inst.n, inst.src, inst.dst, J=inst.J.astype(float), lam=lam, q=q, beta=b)
    n = 20000
    cnt = np.zeros(2 ** inst.n)
    for r in range(n):
        sp0 = oracle.graph_init_random(inst.n, 99, r)
        fin, _, _ = oracle.graph_run(g, sp0, q, b, 99, r, n_full=25, log=False)
        cnt[en.index_of(fin)] += 1
    assert _chi2_p(cnt, m.pi()) > 1e-4
    # and it is not the Gibbs law of H at this q (the two differ here)
    assert 0.5 * np.abs(m.pi() - m.gibbs()).sum() > 0.02
    assert _chi2_p(cnt, m.gibbs()) < 1e-6


def test_graph_finite_time_law_chi2():
    """A slowly mixing instance: the law after t full steps from the fair-coin
    initial state is mu_0 (P^sh)^t exactly."""
    inst, g = _small_graph(seed=3, n=6)
    q, b, t = 0.7, 0.6, 6
    lam = inst.lam_values[inst.cls]
    m = en.Model(inst.n, inst.src, inst.dst, J=inst.J.astype(float), lam=lam, q=q, beta=b)
    mu = np.full(2 ** inst.n, 2.0 ** -inst.n)
    P = m.Psh()
    for _ in range(t):
        mu = mu @ P
    cnt = np.zeros(2 ** inst.n)
    for r in range(20000):
        sp0 = oracle.graph_init_random(inst.n, 31, r)
        fin, _, _ = oracle.graph_run(g, sp0, q, b, 31, r, n_full=t, log=False)
        cnt[en.index_of(fin)] += 1
    assert _chi2_p(cnt, mu) > 1e-4


def test_first_exit_from_all_minus_is_geometric():
    """From -1 each half-step leaves -1 with probability 1-(1-p)^N where
    p = P(+1 | h = -(2J + q - lambda)) (first move of the proof of Theorem 3.3)."""
    L, J, q, lam, b = 4, 1, 0.1, 0.15, 1.0
    N = L * L
    T = oracle.threshold(oracle.field(-2 * J, -1, q, lam), b)
    p = T / 2 ** 32
    stay = (1 - p) ** N
    times = []
    for r in range(3000):
        sp = -np.ones((L, L), dtype=np.int8)
        s = 0
        while True:
            sp = oracle.torus_half_step(sp, J, lam, q, b, 21, r, s)
            s += 1
            if (sp > 0).any():
                break
        times.append(s)
    times = np.array(times)
    kmax = 12
    counts = np.array([(times == k).sum() for k in range(1, kmax)] + [(times >= kmax).sum()])
    probs = np.array([stay ** (k - 1) * (1 - stay) for k in range(1, kmax)] + [stay ** (kmax - 1)])
    assert stats.chisquare(counts, probs * len(times)).pvalue > 1e-4


def test_energy_observable_matches_ham1():
    inst, g = _small_graph(seed=5, n=8)
    lam = inst.lam_values[inst.cls]
    m = en.Model(inst.n, inst.src, inst.dst, J=inst.J.astype(float), lam=lam, q=1.0, beta=1.0)
    HG = m.gibbs_H()
    rng = np.random.Generator(np.random.PCG64(1))
    for _ in range(50):
        sp = _rand_spins(rng, inst.n)
        EJ, plus = oracle.graph_observe(g, sp)
        # sum_x 2 lam_x s_x from the per-class plus counts
        ncls = np.bincount(inst.cls, minlength=len(inst.lam_values))
        lam2 = float((2 * inst.lam_values * (2 * plus - ncls)).sum())
        assert abs(oracle.energy(EJ, lam2) - HG[en.index_of(sp)]) < 1e-12
        assert abs(m.gibbs_H_of(sp) - HG[en.index_of(sp)]) < 1e-12
    L = 5
    s, d = en.torus_edges(L)
    mt = en.Model(L * L, s, d, lam=np.full(L * L, 0.0), q=1.0, beta=1.0)
    for _ in range(20):
        sp = _rand_spins(rng, L * L)
        EJ, M = oracle.torus_observe(sp.reshape(L, L))
        assert -EJ == mt.gibbs_H_of(sp)
        assert M == sp.sum()


def test_beta_zero_gives_fair_coins():
    L = 32
    sp = oracle.torus_init_random(L, 1)
    out = oracle.torus_half_step(sp, 1, 0.0, 1.0, 0.0, 4, 0, 0)
    k = int((out > 0).sum())
    assert abs(k - L * L / 2) < 4 * np.sqrt(L * L / 4)


def test_run_equals_repeated_half_steps():
    L, J, q, lam, b = 7, 1, 0.9, 0.0, 0.45
    sp = oracle.torus_init_random(L, 8, 2)
    fin, ej, mm = oracle.torus_run(sp, J, lam, q, b, 8, 2, n_full=5)
    x = sp.copy()
    for s in range(10):
        x = oracle.torus_half_step(x, J, lam, q, b, 8, 2, s)
    assert np.array_equal(fin, x)
    assert ej.shape == (6,) and mm[0] == sp.sum() and mm[-1] == fin.sum()
