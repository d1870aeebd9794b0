"""Property-based pins on random small oriented graphs (hypothesis): couplings
of mixed sign and magnitude, several field classes, q >= 0.

* Theorem 2.3 for any orientation: pi(sigma) = Zfwd_sigma / Z is stationary
  for P^sh = P^{1->2} P^{2->1} and P^sh is reversible with respect to it.
* The diagonal of the pair Hamiltonian (Definition 2.2): H(sigma, sigma) =
  H(sigma) - q |V|.
* The oracle's threshold of a site equals the marginal probability of +1
  under the enumerated one-step kernel P^{1->2} within 2^-32.
* At zero temperature the oracle's half-steps take the sign of the
  pair-Hamiltonian field wherever it is not zero.
"""
import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
from oracle import enumeration as en


@st.composite
def small_graphs(draw, max_n=7):
    n = draw(st.integers(2, max_n))
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    chosen = draw(st.lists(st.sampled_from(pairs), unique=True, min_size=1, max_size=len(pairs)))
    src, dst = [], []
    for a, b in chosen:
        if draw(st.booleans()):
            a, b = b, a
        src.append(a)
        dst.append(b)
    J = draw(st.lists(st.sampled_from([-2, -1, 1, 2]), min_size=len(src), max_size=len(src)))
    ncls = draw(st.integers(1, 3))
    lam_values = draw(st.lists(st.sampled_from([-1.0, -0.5, 0.0, 0.5, 1.0]), min_size=ncls, max_size=ncls))
    cls = draw(st.lists(st.integers(0, ncls - 1), min_size=n, max_size=n))
    q = draw(st.sampled_from([0.0, 0.25, 0.5, 1.0, 2.0]))
    beta = draw(st.sampled_from([0.1, 0.3, 0.7, 1.2]))
    return (n, np.array(src, np.int32), np.array(dst, np.int32), np.array(J, np.int8),
            np.array(cls, np.uint8), np.array(lam_values, np.float64), q, beta)


def _model(gr):
    n, src, dst, J, cls, lam_values, q, beta = gr
    return en.Model(n, src, dst, J=J.astype(float), lam=lam_values[cls], q=q, beta=beta)


SETTINGS = settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(small_graphs())
def test_theorem_2_3_on_random_graphs(gr):
    m = _model(gr)
    P = m.Psh()
    pi = m.pi()
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
    assert np.max(np.abs(pi @ P - pi)) < 1e-12
    F = pi[:, None] * P
    assert np.max(np.abs(F - F.T)) < 1e-12


@SETTINGS
@given(small_graphs())
def test_pair_hamiltonian_diagonal(gr):
    m = _model(gr)
    assert np.allclose(np.diag(m.pair_H()), m.gibbs_H() - m.q * m.n, atol=1e-9)


@SETTINGS
@given(small_graphs(), st.integers(0, 2 ** 31 - 1))
def test_oracle_threshold_is_the_one_step_marginal(gr, pick):
    n, src, dst, J, cls, lam_values, q, beta = gr
    m = _model(gr)
    S = m.S
    i = pick % S.shape[0]
    P12 = m.P12()[i]
    h = m.fields12()[i]
    for x in range(n):
        marg = P12[S[:, x] > 0].sum()
        t = oracle.threshold(float(h[x]), beta)
        assert abs(t / 2.0 ** 32 - marg) <= 2.0 ** -32 + 1e-12, (x, h[x])


@SETTINGS
@given(small_graphs(), st.integers(0, 2 ** 31 - 1))
def test_zero_temperature_half_steps_follow_the_field(gr, pick):
    n, src, dst, J, cls, lam_values, q, beta = gr
    m = _model(gr)
    g = oracle.Graph(n, src, dst, J, cls, lam_values)
    sp = m.S[pick % m.S.shape[0]].astype(np.int8)
    i = en.index_of(sp)
    got = oracle.graph_half_step(g, sp, q, 1.0e6, 3, 0, 0)
    h = m.fields12()[i]
    nz = np.abs(h) > 1e-9
    assert np.array_equal(got[nz], np.sign(h[nz]).astype(np.int8))
    got2 = oracle.graph_half_step(g, got, q, 1.0e6, 3, 0, 1)
    h2 = m.fields21()[en.index_of(got)]
    nz2 = np.abs(h2) > 1e-9
    assert np.array_equal(got2[nz2], np.sign(h2[nz2]).astype(np.int8))
