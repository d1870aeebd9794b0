"""Metastability helpers (section 3.2) on the CPU: the D signature read from
the (E_J, M) logs against exact membership of the diagonal set D, and
Theorem 3.3's path (plus diagonals growing one at a time from the first flip
to all-plus) on the oracle's own trajectories."""
import numpy as np
import pytest

import oracle
from paper_1904_06257_amd import metastability as ms


def _diag_config(signs):
    L = len(signs)
    r, c = np.indices((L, L))
    return np.asarray(signs, dtype=np.int8)[(r + c) % L]


@pytest.mark.parametrize("L", [4, 7, 16])
def test_signature_holds_on_diagonal_configurations(L):
    """every configuration of D (random diagonal signs) satisfies the
    congruences; E_J = 2 J L (L - 2w) with w the sign changes; the count of
    plus diagonals is recovered from M"""
    rng = np.random.default_rng(L)
    for _ in range(50):
        s = rng.choice([-1, 1], L)
        if abs(s.sum()) == L:
            continue
        x = _diag_config(s)
        assert ms.in_diagonal_set(x)
        ej, m = oracle.torus_observe(x, 1)
        w = int(np.sum(s != np.roll(s, -1)))
        assert ej == 2 * L * (L - 2 * w)
        assert m == int(x.sum())
        assert ms.diagonal_signature([ej], [m], L)[0]
        assert ms.diagonal_count([m], L)[0] == int(np.sum(s > 0))


@pytest.mark.parametrize("L", [5, 8])
def test_signature_rejects_one_site_off_D(L):
    """one spin flipped away from a configuration of D breaks the
    magnetisation congruence; diagonals of the other direction are not in D"""
    rng = np.random.default_rng(100 + L)
    for _ in range(40):
        s = rng.choice([-1, 1], L)
        x = _diag_config(s)
        i, j = rng.integers(0, L, 2)
        x[i, j] = -x[i, j]
        assert not ms.in_diagonal_set(x)
        ej, m = oracle.torus_observe(x, 1)
        assert not ms.diagonal_signature([ej], [m], L)[0]
    # anti-diagonals (r - c constant) with two sign changes: not in D
    r, c = np.indices((L, L))
    y = np.where((r - c) % L < 2, 1, -1).astype(np.int8)
    assert not ms.in_diagonal_set(y)


def test_theorem_3_3_path_on_the_oracle():
    """L = 8, beta = 3.3, q = 0.1, lambda = 0.15, J = 1 from all-minus
    (Theorem 3.3's regime 0 < q < lambda < J): between the first flip and
    all-plus, the signature and exact membership of D agree at every full
    step, the chain is in D most of the time, the number of plus diagonals
    runs through 1, 2, ..., L-1 one at a time, and all-plus comes well
    before exp(2 beta (2J + q - lambda))."""
    L, beta, q, lam = 8, 3.3, ms.FIG4_Q, ms.FIG4_LAM
    n = L * L
    start = -np.ones((L, L), np.int8)
    T = 70000
    _, ej, m = oracle.torus_run(start, 1, lam, q, beta, 5, 2, T)
    t_exit = int(np.nonzero(m != -n)[0][0])
    t_plus = int(np.nonzero(m == n)[0][0])
    assert t_plus < ms.tunnelling_bound(beta)
    sig = ms.diagonal_signature(ej[t_exit:t_plus], m[t_exit:t_plus], L)
    assert sig.mean() > 0.8
    counts = ms.diagonal_count(m[t_exit:t_plus][sig], L)
    steps = np.diff(np.concatenate([[0], counts]))
    assert np.all((steps == 0) | (steps == 1))
    assert counts[0] == 1 and counts[-1] == L - 1
    # exact membership along the window, one full step at a time
    x, _, _ = oracle.torus_run(start, 1, lam, q, beta, 5, 2, t_exit, log=False)
    for t in range(t_exit, t_plus):
        exact = ms.in_diagonal_set(x) and abs(int(x.sum())) != n
        assert exact == bool(sig[t - t_exit]), t
        x, _, _ = oracle.torus_run(x, 1, lam, q, beta, 5, 2, 1, s0=2 * t, log=False)


@pytest.mark.parametrize("beta,q,lam", [(0.7, 0.1, 0.15), (1.3, 0.1, 0.15), (0.5, 0.4, 0.6), (1.0, 0.8, 0.3)])
def test_stationary_law_concentrates_on_all_plus(beta, q, lam):
    """Section 3.2: for 0 < lambda < J and q > 0 the stationary law of the
    shaken dynamics puts every configuration other than +1 below
    exp(-2 beta q) pi(+1).  Exact enumeration of Theorem 2.3's pi on the 3 x 3
    torus, against the closed form of the ratio: the product over sites of
    cosh(beta h^dl_x(sigma)) / cosh(beta (2J + q + lambda)) times Theorem 2.3's
    field factor exp(beta lambda (sum sigma - N))."""
    from oracle import enumeration as en
    L, J = 3, 1.0
    n = L * L
    src, dst = en.torus_edges(L)
    m = en.Model(n, src, dst, lam=np.full(n, lam), q=q, beta=beta)
    pi = m.pi()
    S = en.states(n)
    plus = 2 ** n - 1
    ratio = pi / pi[plus]
    others = np.arange(2 ** n) != plus
    assert np.all(ratio[others] <= np.exp(-2 * beta * q) * (1 + 1e-12))
    # closed form: the dl field collects the tails of the edges pointing at x
    h = np.zeros_like(S)
    for a, b in zip(src, dst):
        h[:, b] += J * S[:, a]
    h += q * S + lam
    closed = np.exp(beta * lam * (S.sum(axis=1) - n)) * np.prod(
        np.cosh(beta * h) / np.cosh(beta * (2 * J + q + lam)), axis=1)
    assert np.allclose(ratio, closed, rtol=1e-10, atol=0)
