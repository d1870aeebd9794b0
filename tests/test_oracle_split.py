"""Pins of the generalised split (section 5): an undirected pair may carry both
orientations, J = J^o + J^o^T.  The enumeration model takes the oriented
coupling matrix as given; the oracle sums whatever oriented edges it gets.

* Theorem 2.3 holds for any J^o: pi = Zfwd / Z is stationary and P^sh is
  reversible with respect to it.
* The symmetric split J^o = J / 2 makes the pair Hamiltonian symmetric, so the
  two half-step kernels coincide: P^{1->2} = P^{2->1} (the kernel of a
  probabilistic cellular automaton).
* The oracle's one-step law on a split graph matches P^{1->2} and P^sh, and its
  energy is the Ising energy with the summed couplings (equation ham1)."""
import numpy as np
from scipy import stats

import oracle
from oracle import enumeration as en


def _split_graph(seed=5, n=6):
    """a random simple graph, every edge given in both orientations with
    couplings that sum to an even J (so J/2 splits are integers)"""
    rng = np.random.Generator(np.random.PCG64(seed))
    src, dst, J = [], [], []
    for x in range(n):
        for y in range(x + 1, n):
            if rng.random() < 0.6:
                a = int(rng.integers(-2, 3))
                b = int(rng.integers(-2, 3))
                src += [x, y]
                dst += [y, x]
                J += [a, b]
    return np.array(src), np.array(dst), np.array(J, dtype=np.int8)


def test_theorem_2_3_for_a_general_split():
    src, dst, J = _split_graph()
    lam = np.linspace(-0.5, 0.5, 6)
    m = en.Model(6, src, dst, J=J.astype(float), lam=lam, q=0.6, beta=0.7)
    P, pi = m.Psh(), m.pi()
    assert np.allclose(pi @ P, pi, atol=1e-13, rtol=0)
    D = pi[:, None] * P
    assert np.allclose(D, D.T, atol=1e-15, rtol=0)


def test_symmetric_split_half_steps_coincide():
    rng = np.random.Generator(np.random.PCG64(2))
    n = 5
    src, dst, J = [], [], []
    for x in range(n):
        for y in range(x + 1, n):
            j = int(rng.choice([-2, 2]))
            src += [x, y]
            dst += [y, x]
            J += [j // 2, j // 2]
    m = en.Model(n, np.array(src), np.array(dst), J=np.array(J, float), lam=np.full(n, 0.3),
                 q=0.4, beta=0.9)
    assert np.allclose(m.P12(), m.P21(), atol=1e-14, rtol=0)
    # and a one-way orientation of the same graph does not have this property
    one = en.Model(n, np.array(src[0::2]), np.array(dst[0::2]), J=np.array(J[0::2], float) * 2,
                   lam=np.full(n, 0.3), q=0.4, beta=0.9)
    assert not np.allclose(one.P12(), one.P21(), atol=1e-3)


def _chi2_p(counts, probs):
    probs = np.asarray(probs)
    keep = probs * counts.sum() >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(probs[keep], probs[~keep].sum()) * counts.sum()
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    return stats.chisquare(obs, exp).pvalue


def test_oracle_one_step_law_on_a_split_graph():
    src, dst, J = _split_graph(seed=7)
    cls = np.array([0, 1, 2, 0, 1, 2], dtype=np.uint8)
    lamv = np.array([-0.5, 0.0, 0.5])
    g = oracle.Graph(6, src, dst, J, cls, lamv)
    q, b = 0.8, 0.5
    m = en.Model(6, src, dst, J=J.astype(float), lam=lamv[cls], q=q, beta=b)
    sp = np.array([1, -1, 1, -1, -1, 1], dtype=np.int8)
    i0 = en.index_of(sp)
    half = np.zeros(64)
    full = np.zeros(64)
    for r in range(20000):
        a = oracle.graph_half_step(g, sp, q, b, 31, r, 0)
        half[en.index_of(a)] += 1
        full[en.index_of(oracle.graph_half_step(g, a, q, b, 31, r, 1))] += 1
    assert _chi2_p(half, m.P12()[i0]) > 1e-4
    assert _chi2_p(full, m.Psh()[i0]) > 1e-4
    for _ in range(10):
        x = np.where(np.random.default_rng(_).integers(0, 2, 6) == 1, 1, -1).astype(np.int8)
        ej = oracle.graph_observe(g, x)[0]
        assert -ej - float((2 * lamv[cls] * x).sum()) == m.gibbs_H_of(x)
