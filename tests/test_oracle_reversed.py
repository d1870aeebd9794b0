"""Pins of the reversed order P^{sh'} = P^{2->1} P^{1->2} on the torus
(section 3: P^{ur} first, then P^{dl}); the oracle's half read at half-step s
is (s & 1) ^ 1.  The enumeration model gives the half-step kernels from the pair
Hamiltonian, so the oracle must follow the out-half fields first at zero
temperature, and its one-step law must be the P21 P12 row; on graphs the
reversed order is the forward order on the reversed edge set (pathwise, the
uniforms being keyed by vertex and half-step only), which the library relies
on and the model confirms."""
import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import enumeration as en


def _rand_spins(rng, n):
    return np.where(rng.integers(0, 2, n) == 1, 1, -1).astype(np.int8)


@pytest.mark.parametrize("L", [3, 4])
def test_zero_temperature_reversed_follows_out_half_first(L):
    q, lam = 0.5, 0.25
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, lam=np.full(L * L, lam), q=q, beta=1.0)
    rng = np.random.Generator(np.random.PCG64(70 + L))
    for _ in range(20):
        sp = _rand_spins(rng, L * L)
        g1 = oracle.torus_half_step(sp.reshape(L, L), 1, lam, q, 1000.0, 5, 0, 0, rev=True).reshape(-1)
        assert np.array_equal(g1, np.sign(m.field21_of(sp)).astype(np.int8))
        g2 = oracle.torus_half_step(g1.reshape(L, L), 1, lam, q, 1000.0, 5, 0, 1, rev=True).reshape(-1)
        assert np.array_equal(g2, np.sign(m.field12_of(g1)).astype(np.int8))


def _chi2_p(counts, probs):
    probs = np.asarray(probs)
    keep = probs * counts.sum() >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(probs[keep], probs[~keep].sum()) * counts.sum()
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    return stats.chisquare(obs, exp).pvalue


def test_reversed_one_step_law_and_stationarity():
    L, q, lam, b = 3, 0.6, 0.2, 0.5
    rng = np.random.Generator(np.random.PCG64(13))
    ju, jr = (np.where(rng.integers(0, 2, (L, L)) == 1, 1, -1).astype(np.int8) for _ in range(2))
    s, d = en.torus_edges(L)
    Je = np.stack([ju.reshape(-1), jr.reshape(-1)], axis=1).reshape(-1).astype(float)
    m = en.Model(L * L, s, d, J=Je, lam=np.full(L * L, lam), q=q, beta=b)
    Prev = m.P21() @ m.P12()
    # its stationary law is the sigma^2-marginal of pi^b
    pib = m.pib()
    pi2 = pib.sum(axis=0)
    assert np.allclose(pi2 @ Prev, pi2, atol=1e-13, rtol=0)
    sp = np.array([1, -1, 1, 1, 1, -1, -1, -1, 1], dtype=np.int8).reshape(L, L)
    i0 = en.index_of(sp.reshape(-1))
    full = np.zeros(2 ** (L * L))
    for r in range(30000):
        a = oracle.torus_half_step(sp, (ju, jr), lam, q, b, 6, r, 0, rev=True)
        c = oracle.torus_half_step(a, (ju, jr), lam, q, b, 6, r, 1, rev=True)
        full[en.index_of(c.reshape(-1))] += 1
    assert _chi2_p(full, Prev[i0]) > 1e-4


def test_graph_reversed_order_is_the_reversed_edge_set():
    rng = np.random.Generator(np.random.PCG64(3))
    n = 6
    src, dst = [], []
    for x in range(n):
        for y in range(x + 1, n):
            if rng.random() < 0.6:
                if rng.random() < 0.5:
                    src.append(x); dst.append(y)
                else:
                    src.append(y); dst.append(x)
    src, dst = np.array(src), np.array(dst)
    J = rng.integers(-2, 3, src.shape[0]).astype(float)
    fwd = en.Model(n, src, dst, J=J, lam=np.full(n, 0.1), q=0.5, beta=0.8)
    back = en.Model(n, dst, src, J=J, lam=np.full(n, 0.1), q=0.5, beta=0.8)
    assert np.allclose(back.P12(), fwd.P21(), atol=1e-14, rtol=0)
    assert np.allclose(back.P21(), fwd.P12(), atol=1e-14, rtol=0)
