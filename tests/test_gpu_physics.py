"""Statistical checks of the GPU sampler at scale against closed forms.

Theorem 3.1: for large self-interaction q (delta = exp(-2 beta q) small) the
stationary law of shaken dynamics on the square lattice approaches the Gibbs
law of H.  The energy per site and the spontaneous magnetisation measured on
batches of tori must then approach Onsager's exact energy and Yang's
magnetisation of the 2-D Ising model, with a deviation shrinking roughly like
exp(-2 beta (q - 2J)) (the weight of the tau != sigma terms in Zfwd).
Reversibility (Theorem 2.3) is checked as the time symmetry of the
(M, E_J) cross-correlation.
"""
import numpy as np
import pytest
from scipy.special import ellipk

pytestmark = pytest.mark.gpu


def onsager_u(beta):
    """Energy per site of the 2-D Ising model, J = 1 (Onsager)."""
    k = 2 * np.sinh(2 * beta) / np.cosh(2 * beta) ** 2
    return -1 / np.tanh(2 * beta) * (1 + 2 / np.pi * (2 * np.tanh(2 * beta) ** 2 - 1) * ellipk(k * k))


def yang_m(beta):
    return (1 - np.sinh(2 * beta) ** -4) ** 0.125


@pytest.fixture(scope="module")
def sk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1904_06257_amd as m
    return m


def _measure(sk, beta, q, init, L=128, reps=64, burn=2000, blocks=10, block_steps=200):
    chains = [sk.Chain.torus(L, q=q, beta=beta, seed=1000 + r, replica=r, init=init)
              for r in range(reps)]
    b = sk.Batch(chains, strategy="persistent", record=True)
    b.sweep(burn)
    es, ms = [], []
    for _ in range(blocks):
        b.sweep(block_steps)
        for i in range(reps):
            h, m = b.log(i)
            es.append(h[1:])
            ms.append(m[1:])
    b.close()
    for c in chains:
        c.close()
    N = L * L
    e = np.array(es, dtype=np.float64) / N        # H per site (lambda = 0: H = -E_J)
    m = np.abs(np.array(ms, dtype=np.float64)) / N
    # error bar from the spread of per-block means
    be = e.reshape(blocks * reps, -1).mean(axis=1)
    return e.mean(), be.std(ddof=1) / np.sqrt(be.size), m.mean()


# q values per beta: the mobility falls like eps too (a spin against its
# neighbours and q flips with probability ~ exp(-2 beta (q - 2J))), so the
# largest q is limited by what a few thousand steps equilibrate.
@pytest.mark.parametrize("beta,init,qs,burn", [(0.30, "random", (4.0, 6.0, 8.0), 2000),
                                               (0.50, "all_up", (4.0, 5.0, 6.0), 4000)])
def test_large_q_approaches_onsager(sk, beta, init, qs, burn):
    u0 = onsager_u(beta)
    devs = []
    for q in qs:
        u, err, m = _measure(sk, beta, q, init, burn=burn)
        eps = np.exp(-2 * beta * (q - 2.0))
        devs.append(abs(u - u0))
        print("beta %.2f q %.0f: u %.5f +- %.5f (Onsager %.5f, dev %.5f, eps %.4f), |m| %.4f"
              % (beta, q, u, err, u0, u - u0, eps, m), flush=True)
        # first-order correction in eps (the tau != sigma terms of Zfwd whose
        # weight is largest, exp(-2 beta (q - 2J))): |dev| <= 0.75 eps
        assert abs(u - u0) <= 0.75 * eps + 6 * err + 1e-3
        if beta > 0.44:
            assert abs(m - yang_m(beta)) <= 0.75 * eps + 2e-3
    assert devs[0] > devs[1] > devs[2]


def test_time_reversibility(sk):
    """Theorem 2.3: the chain is reversible, so in equilibrium
    E[A(s_t) B(s_{t+1})] = E[B(s_t) A(s_{t+1})] for A = M^2, B = H (full
    steps; M itself is odd under the global flip and would make the check
    trivial)."""
    L, reps, beta, q = 64, 128, 0.42, 1.0
    chains = [sk.Chain.torus(L, q=q, beta=beta, seed=77 + r, replica=r) for r in range(reps)]
    b = sk.Batch(chains, strategy="persistent", record=True)
    b.sweep(500)
    a, c = [], []
    for _ in range(4):
        b.sweep(500)
        for i in range(reps):
            h, m = b.log(i)
            h = h.astype(np.float64) - h.mean()
            m2 = m.astype(np.float64) ** 2
            m2 -= m2.mean()
            a.append((m2[:-1] * h[1:]).mean())
            c.append((h[:-1] * m2[1:]).mean())
    d = np.array(a) - np.array(c)
    z = d.mean() / (d.std(ddof=1) / np.sqrt(d.size))
    print("reversibility: mean difference %.3f, z = %.2f" % (d.mean(), z), flush=True)
    assert abs(z) < 4.5


def _chi2_p(counts, probs):
    from scipy import stats
    probs = np.asarray(probs)
    keep = probs * counts.sum() >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(probs[keep], probs[~keep].sum()) * counts.sum()
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    return stats.chisquare(obs, exp).pvalue


@pytest.mark.parametrize("case,T", [("graph6", 40), ("torus3", 150)])
def test_long_run_state_histogram_chi2(sk, case, T):
    """Sixteen thousand independent GPU chains on a tiny system: the histogram
    of their states after T full steps against the exact stationary law pi of
    Theorem 2.3 (float64 enumeration).  T is long enough that the exact law
    after T steps from the uniform start is within 1e-4 of pi in total
    variation (checked here), and the Gibbs law of H, which pi is not at this
    small q, is rejected by the same data (the test has power)."""
    import synth
    from oracle import enumeration as en
    reps = 16384
    if case == "graph6":
        inst = synth.random_oriented_graph(6, 0.6, 3, jmax=1, n_classes=3, lam_scale=0.25)
        q, beta = 0.7, 0.3
        m = en.Model(inst.n, inst.src, inst.dst, J=inst.J.astype(float),
                     lam=inst.lam_values[inst.cls], q=q, beta=beta)
        chains = [sk.Chain.graph(inst.n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                                 lam_class=inst.cls, q=q, beta=beta, seed=5, replica=r)
                  for r in range(reps)]
    else:
        L, q, beta, lam = 3, 0.8, 0.5, 0.15
        s, d = en.torus_edges(L)
        m = en.Model(L * L, s, d, lam=np.full(L * L, lam), q=q, beta=beta)
        chains = [sk.Chain.torus(L, q=q, beta=beta, lam_values=[lam], seed=6, replica=r)
                  for r in range(reps)]
    pi = m.pi()
    u = np.full(pi.size, 1.0 / pi.size)
    pT = u @ np.linalg.matrix_power(m.Psh(), T)
    assert 0.5 * np.abs(pT - pi).sum() < 1e-4
    b = sk.Batch(chains, strategy="grid", use_hipgraph=True)
    b.sweep(T)
    cnt = np.zeros(pi.size)
    for c in chains:
        cnt[en.index_of(c.spins().reshape(-1))] += 1
        c.close()
    b.close()
    p = _chi2_p(cnt, pi)
    p_gibbs = _chi2_p(cnt, m.gibbs())
    print("%s: chi2 p-value vs pi %.3g, vs Gibbs %.3g" % (case, p, p_gibbs), flush=True)
    assert p > 1e-4
    assert p_gibbs < 1e-10


def test_large_q_onsager_at_4096(sk):
    """The headline lattice: 4096^2 tori, beta = 0.30, random start, q in
    {4, 6, 8}, grid batch.  After 2000 burn-in steps the energy per site
    averaged over 1000 steps (statistical error ~1e-5 at this size) approaches
    Onsager's as q grows, within the first-order bound 0.75 eps."""
    L, beta, qs = 4096, 0.30, (4.0, 6.0, 8.0)
    chains = [sk.Chain.torus(L, q=q, beta=beta, seed=300 + k, replica=k) for k, q in enumerate(qs)]
    b = sk.Batch(chains, strategy="grid", use_hipgraph=True, record=True, log_reserve=2000)
    b.sweep(2000)
    b.sweep(1000)
    u0 = onsager_u(beta)
    devs, ratios = [], []
    for k, q in enumerate(qs):
        h, _ = b.log(k)
        u = h[1:].astype(np.float64).mean() / (L * L)
        eps = np.exp(-2 * beta * (q - 2.0))
        devs.append(abs(u - u0))
        ratios.append((u - u0) / eps)
        print("4096^2, beta %.2f q %.0f: u %.6f (Onsager %.6f, dev %.6f, eps %.4f, dev/eps %.3f)"
              % (beta, q, u, u0, u - u0, eps, (u - u0) / eps), flush=True)
        assert abs(u - u0) <= 0.75 * eps + 2e-4
    assert devs[0] > devs[1] > devs[2]
    # first order in eps: the ratio is nearly the same at every q
    assert max(ratios) - min(ratios) < 0.15
    b.close()
    for c in chains:
        c.close()


def test_first_exit_from_all_minus_is_geometric(sk):
    """Metastability set-up of section 3 (start -1, small q, lambda > 0): the
    number of full steps until the chain first leaves -1 is geometric with
    parameter 1 - P^sh(-1, -1), computed exactly by enumeration (3 x 3 torus,
    q = 0.1, lambda = 0.15, beta = 1.3; 16384 replicas, exit read from the
    magnetisation log)."""
    from scipy import stats
    from oracle import enumeration as en
    L, q, lam, beta, T, reps = 3, 0.1, 0.15, 1.3, 60, 16384
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, lam=np.full(L * L, lam), q=q, beta=beta)
    stay = m.Psh()[0, 0]                      # state index 0 = all -1
    chains = [sk.Chain.torus(L, q=q, beta=beta, lam_values=[lam], init="all_down", seed=7, replica=r)
              for r in range(reps)]
    b = sk.Batch(chains, record=True, use_hipgraph=True)
    b.sweep(T)
    times = np.full(reps, T + 1)
    for i in range(reps):
        _, mlog = b.log(i, with_H=False)
        assert mlog[0] == -L * L
        out = np.nonzero(mlog[1:] != -L * L)[0]
        if out.size:
            times[i] = out[0] + 1
    b.close()
    for c in chains:
        c.close()
    kmax = 30
    counts = np.array([(times == k).sum() for k in range(1, kmax)] + [(times >= kmax).sum()])
    probs = np.array([stay ** (k - 1) * (1 - stay) for k in range(1, kmax)] + [stay ** (kmax - 1)])
    p = stats.chisquare(counts, probs * reps).pvalue
    print("first exit: mean %.3f steps (geometric %.3f), chi2 p %.3g" % (times.mean(), 1 / (1 - stay), p),
          flush=True)
    assert p > 1e-4
