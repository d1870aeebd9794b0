"""Pins of the frozen set B (section 3.1, state space X_{Lambda,B}: spins on B
fixed at +1).  The half-step kernels factorise over sites, so on X_{Lambda,B}
they are the full kernels conditioned on sigma'_B = +1; the oracle's one-step
law must be the restricted P^sh row, B must stay +1, and the restricted chain
keeps the reversibility of Theorem 2.3 with pi_B(sigma) proportional to the
sum of exp(-beta H(sigma, tau)) over tau in X_{Lambda,B}."""
import numpy as np
from scipy import stats

import oracle
from oracle import enumeration as en


def _restricted(P, ok):
    R = P[np.ix_(ok, ok)]
    return R / R.sum(axis=1, keepdims=True)


def test_restricted_chain_is_reversible():
    L, q, lam, b = 3, 0.6, 0.2, 0.7
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, lam=np.full(L * L, lam), q=q, beta=b)
    B = [0, 4]
    S = m.S
    ok = np.all(S[:, B] > 0, axis=1)
    P = _restricted(m.P12(), ok) @ _restricted(m.P21(), ok)
    A = -b * m.pair_H()[np.ix_(ok, ok)]
    pi = np.exp(A - A.max()).sum(axis=1)
    pi /= pi.sum()
    assert np.allclose(pi @ P, pi, atol=1e-14, rtol=0)
    D = pi[:, None] * P
    assert np.allclose(D, D.T, atol=1e-15, rtol=0)


def _chi2_p(counts, probs):
    probs = np.asarray(probs)
    keep = probs * counts.sum() >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(probs[keep], probs[~keep].sum()) * counts.sum()
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    return stats.chisquare(obs, exp).pvalue


def test_oracle_one_step_law_on_the_frozen_torus():
    L, q, lam, b = 3, 0.6, 0.2, 0.5
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, lam=np.full(L * L, lam), q=q, beta=b)
    frozen = np.zeros((L, L), dtype=bool)
    frozen[0, 1] = frozen[2, 2] = True
    B = np.nonzero(frozen.reshape(-1))[0]
    ok = np.all(m.S[:, B] > 0, axis=1)
    Psh = _restricted(m.P12(), ok) @ _restricted(m.P21(), ok)
    idx = np.nonzero(ok)[0]
    pos = {int(i): k for k, i in enumerate(idx)}
    sp = np.array([1, 1, -1, -1, 1, -1, 1, -1, 1], dtype=np.int8).reshape(L, L)
    i0 = pos[en.index_of(sp.reshape(-1))]
    counts = np.zeros(len(idx))
    for r in range(20000):
        out, _, _ = oracle.torus_run_frozen(sp, frozen, 1, lam, q, b, 17, r, 1)
        assert np.all(out[frozen] == 1)
        counts[pos[en.index_of(out.reshape(-1))]] += 1
    assert _chi2_p(counts, Psh[i0]) > 1e-4


def test_no_frozen_sites_is_the_plain_run():
    L = 20
    sp = oracle.torus_init_random(L, 3, 1)
    a, ea, ma = oracle.torus_run_frozen(sp, np.zeros((L, L), bool), 1, 0.1, 0.7, 0.5, 3, 1, 15)
    b, eb, mb = oracle.torus_run(sp, 1, 0.1, 0.7, 0.5, 3, 1, 15)
    assert np.array_equal(a, b) and np.array_equal(ea, eb) and np.array_equal(ma, mb)
