"""Pins of the float64 enumeration oracle against what the paper and the
mathematics fix (section 2, Theorem 2.3 and its proof; section 3 identities;
Theorem 3.1 limit; Theorem 6.1).  CPU only."""
import itertools

import numpy as np
import pytest

from oracle import enumeration as en

TOL = 1e-12


def _zoo():
    rng = np.random.Generator(np.random.PCG64(7))
    out = []
    # path, oriented left to right, with a field
    out.append(("path5", en.Model(5, [0, 1, 2, 3], [1, 2, 3, 4], lam=[0.3] * 5, q=0.7, beta=0.9)))
    # cycle with mixed orientation and signs
    out.append(("cycle5", en.Model(5, [0, 2, 2, 4, 0], [1, 1, 3, 3, 4], J=[1, -1, 2, 1, -1],
                                   lam=[0.1, -0.2, 0.0, 0.5, 0.25], q=0.4, beta=1.1)))
    # K4 with an arbitrary orientation
    src, dst = zip(*[(0, 1), (2, 0), (0, 3), (1, 2), (3, 1), (2, 3)])
    out.append(("K4", en.Model(4, src, dst, J=[1, 1, -1, 1, 2, -1], lam=[0.2, 0, -0.4, 0.1],
                               q=1.3, beta=0.6)))
    # Petersen graph, orientation by a coin
    edges = [(i, (i + 1) % 5) for i in range(5)] + [(i, i + 5) for i in range(5)] + \
            [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    flips = rng.integers(0, 2, len(edges))
    src = [a if f == 0 else b for (a, b), f in zip(edges, flips)]
    dst = [b if f == 0 else a for (a, b), f in zip(edges, flips)]
    out.append(("petersen", en.Model(10, src, dst, lam=np.full(10, 0.15), q=0.8, beta=0.7)))
    # 3 x 3 torus (the square-lattice orientation up/right)
    s, d = en.torus_edges(3)
    out.append(("torus3", en.Model(9, s, d, lam=np.full(9, 0.3), q=0.8, beta=0.7)))
    # random +-J graph with field classes
    n = 7
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < 0.5
    a, b = iu[keep], ju[keep]
    f = rng.integers(0, 2, a.shape[0]).astype(bool)
    out.append(("random7", en.Model(n, np.where(f, b, a), np.where(f, a, b),
                                    J=rng.choice([-1.0, 1.0], a.shape[0]),
                                    lam=rng.choice([-0.5, 0.0, 0.5], n), q=1.5, beta=0.8)))
    return out


ZOO = _zoo()
IDS = [z[0] for z in ZOO]


@pytest.mark.parametrize("name,m", ZOO, ids=IDS)
def test_half_step_kernels_are_products_of_site_factors(name, m):
    """P^{1->2}, built as normalised exp(-b H(s, s')), factorises over sites
    with the in-half field h^{1->2}; P^{2->1} with the out-half field h^{2->1}
    (the product formulas that follow ham21).  Swapping the halves fails."""
    assert np.allclose(m.P12(), m.product_form(m.fields12()), rtol=0, atol=TOL)
    assert np.allclose(m.P21(), m.product_form(m.fields21()), rtol=0, atol=TOL)
    if name in ("path5", "cycle5", "K4", "torus3"):
        assert not np.allclose(m.P12(), m.product_form(m.fields21()), atol=1e-6)


@pytest.mark.parametrize("name,m", ZOO, ids=IDS)
def test_rows_sum_to_one(name, m):
    for P in (m.P12(), m.P21(), m.Psh()):
        assert np.abs(P.sum(axis=1) - 1).max() < TOL


@pytest.mark.parametrize("name,m", ZOO, ids=IDS)
def test_theorem_2_3_stationary_and_reversible(name, m):
    """pi = Zfwd/Z is stationary for P^sh and satisfies detailed balance."""
    pi = m.pi()
    P = m.Psh()
    assert np.abs(pi @ P - pi).max() < TOL
    F = pi[:, None] * P
    assert np.abs(F - F.T).max() < TOL


@pytest.mark.parametrize("name,m", [z for z in ZOO if z[0] in ("path5", "cycle5", "torus3")],
                         ids=["path5", "cycle5", "torus3"])
def test_reversed_order_has_the_other_marginal(name, m):
    """P^{sh'} = P^{2->1} P^{1->2} (section 3) is stationary for the sigma^(2)
    marginal of pi^b, which differs from pi when the orientation matters."""
    Prev = m.P21() @ m.P12()
    pib = m.pib()
    pi2 = pib.sum(axis=0)
    assert np.abs(pi2 @ Prev - pi2).max() < TOL
    pi = m.pi()
    assert np.abs(pi - pi2).max() > 1e-6
    assert np.abs(pi @ Prev - pi).max() > 1e-6


@pytest.mark.parametrize("name,m", [z for z in ZOO if z[1].n <= 5], ids=["path5", "cycle5", "K4"])
def test_alternate_dynamics(name, m):
    """pi^b is stationary for P^alt, and P^sh is the sigma^(1) marginal of
    P^alt (equations eqshalt, Palt, stmeasalt)."""
    Pa = m.Palt()
    N = 2 ** m.n
    pib = m.pib().reshape(-1)  # pair index i1 * N + i2
    assert np.abs(pib @ Pa - pib).max() < TOL
    Psh = m.Psh()
    # P^sh(s1, t1) = sum_{t2} P^alt((s1, any), (t1, t2))
    marg = Pa.reshape(N, N, N, N)[:, 0, :, :].sum(axis=2)
    assert np.abs(marg - Psh).max() < TOL
    # pi is the sigma^(1) marginal of pi^b
    assert np.abs(m.pib().sum(axis=1) - m.pi()).max() < TOL


def test_alternate_dynamics_not_reversible_on_Knn():
    """K_{n,n} with equal weights, (s1,s2) = (+1,+1) and (t1,t2) = (+1,-1):
    pi^b(s) P^alt(s,t) != pi^b(t) P^alt(t,s) (counterexample after the proof
    of Theorem 2.3).  K_{n,n} as a doubling graph puts x^(1)-y^(2) edges in
    both directions, i.e. Jo has every off-diagonal entry (section 5 split)."""
    n, w = 3, 0.7
    src, dst = zip(*[(x, y) for x in range(n) for y in range(n) if x != y])
    m = en.Model(n, src, dst, J=[w] * len(src), q=w, beta=0.9)
    N = 2 ** n
    Pa = m.Palt()
    pib = m.pib().reshape(-1)
    up = N - 1  # all +1
    dn = 0      # all -1
    s = up * N + up
    t = up * N + dn
    lhs = pib[s] * Pa[s, t]
    rhs = pib[t] * Pa[t, s]
    assert abs(lhs - rhs) > 1e-3 * max(lhs, rhs)


@pytest.mark.parametrize("name,m", ZOO, ids=IDS)
def test_diagonal_identity(name, m):
    """H(s, s) = H(s) - q |V|  (section 2, after the matrix form; eq. HGibbs)."""
    d = np.diag(m.pair_H())
    assert np.abs(d - (m.gibbs_H() - m.q * m.n)).max() < 1e-12


def test_isolated_vertex_closed_form():
    """One vertex, no edges: Zfwd_s = sum_t exp(b(q s t + lam s + lam t)) =
    exp(b lam s) 2 cosh(b (q s + lam)); the chain is the 2-state chain with
    that stationary law (Theorem 2.3 on a single site)."""
    q, lam, b = 0.9, 0.35, 1.3
    m = en.Model(1, [], [], lam=[lam], q=q, beta=b)
    w = np.array([np.exp(b * lam * s) * 2 * np.cosh(b * (q * s + lam)) for s in (-1.0, 1.0)])
    assert np.abs(m.pi() - w / w.sum()).max() < TOL
    p_up = 1.0 / (1.0 + np.exp(-2 * b * (q * 1 + lam)))   # from +1
    assert abs(m.P12()[1, 1] - p_up) < TOL


def test_pi_on_torus_needs_the_field_factor():
    """On Z^2 the stationary law of Theorem 2.3 is
    pi(s) ~ exp(b lam sum s) prod_x 2 cosh(b h^dl_x(s)); the shorter form
    printed in section 3.2 without exp(b lam sum s) is not stationary when
    lam != 0 (reading A4)."""
    L, q, lam, b = 3, 0.8, 0.3, 0.7
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, lam=np.full(L * L, lam), q=q, beta=b)
    H = m.fields12()
    logw = b * lam * m.S.sum(axis=1) + np.log(2 * np.cosh(b * H)).sum(axis=1)
    w = np.exp(logw - logw.max())
    w /= w.sum()
    P = m.Psh()
    assert np.abs(w - m.pi()).max() < TOL
    assert np.abs(w @ P - w).max() < TOL
    logw2 = np.log(2 * np.cosh(b * H)).sum(axis=1)
    w2 = np.exp(logw2 - logw2.max())
    w2 /= w2.sum()
    assert np.abs(w2 @ P - w2).max() > 1e-3


def test_gibbs_limit_large_q():
    """Theorem 3.1 mechanism: as q grows the shaken law approaches the Gibbs
    law of H (the tau = sigma term dominates Zfwd); TV shrinks with q."""
    L, lam, b = 3, 0.1, 0.6
    s, d = en.torus_edges(L)
    tvs = []
    for q in (1.0, 2.0, 4.0, 8.0):
        m = en.Model(L * L, s, d, lam=np.full(L * L, lam), q=q, beta=b)
        tvs.append(0.5 * np.abs(m.pi() - m.gibbs()).sum())
    assert all(tvs[i + 1] < tvs[i] for i in range(3))
    assert tvs[-1] < 1e-3


def _brute(m):
    HP = m.pair_H()
    HG = m.gibbs_H()
    return HP, HG


@pytest.mark.parametrize("seed", range(6))
def test_theorem_6_1(seed):
    """(1) if q > max_x (sum over the out-neighbours y of |J_xy| + |lam_x|)
    every minimiser of H(s, t) has s = t, so min H(s,t) = min H(s) - q|V|;
    (2) for any q > 0, min H(s, t) <= min H(s) - q|V|.  Brute force."""
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    n = 6
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < 0.6
    a, b = iu[keep], ju[keep]
    f = rng.integers(0, 2, a.shape[0]).astype(bool)
    src, dst = np.where(f, b, a), np.where(f, a, b)
    J = rng.choice([-1.0, 1.0], a.shape[0])
    lam = rng.choice([-0.5, 0.0, 0.5], n)
    out_sum = np.zeros(n)
    for e in range(len(src)):
        out_sum[src[e]] += abs(J[e])
    qmin = (out_sum + np.abs(lam)).max()
    m = en.Model(n, src, dst, J=J, lam=lam, q=qmin + 0.01, beta=1.0)
    HP, HG = _brute(m)
    mn = HP.min()
    arg = np.argwhere(np.abs(HP - mn) < 1e-9)
    assert np.all(arg[:, 0] == arg[:, 1])
    assert abs(mn - (HG.min() - m.q * n)) < 1e-9
    for q in (0.05, 0.5, 1.0):
        m2 = en.Model(n, src, dst, J=J, lam=lam, q=q, beta=1.0)
        HP2, HG2 = _brute(m2)
        assert HP2.min() <= HG2.min() - q * n + 1e-12


def test_theorem_6_1_small_q_can_be_strict():
    """Below the threshold the pair minimum can undercut the diagonal: a
    frustrated triangle with q small."""
    m = en.Model(3, [0, 1, 2], [1, 2, 0], J=[-1.0, -1.0, -1.0], q=0.1, beta=1.0)
    HP, HG = _brute(m)
    assert HP.min() < HG.min() - m.q * 3 - 1e-9
