"""Metastability on the GPU (section 3.2): replicas from all-minus with
0 < q < lambda < J in one persistent batch.

* the chains of the workload are the oracle's chains (E_J and M logs, final
  spins, bit for bit);
* Theorem 3.3 at beta = 4 (the largest inverse temperature of the paper's
  nucleation experiment): from the first flip to all-plus the chain moves
  through the diagonal set D, the plus diagonals growing one at a time, and
  all-plus comes before exp(2 beta (2J + q - lambda)) (Theorem 3.2); the
  configuration half-way (L/2 plus diagonals) is checked in D exactly;
* the shaken side of the nucleation experiment (beta in {1.3, 2.3, 3.3},
  q = 0.1, lambda = 0.15): tunnelling slows down as beta grows, every
  replica tunnels before the theorem's time scale, and the magnetisation
  after tunnelling is close to, and at beta = 1.3 visibly below, +1.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1904_06257_amd as m
    return m


@pytest.fixture(scope="module")
def ms(sk):
    from paper_1904_06257_amd import metastability
    return metastability


def test_metastable_chains_match_oracle(sk, ms):
    L, beta, T, R = 16, 2.3, 3000, 4
    print("metastable parity L=%d beta=%g T=%d replicas=%d" % (L, beta, T, R), flush=True)
    chains = ms.make_chains(L, [beta] * R, seed=3)
    b = sk.Batch(chains, record=True)
    b.sweep(T)
    for r in range(R):
        x, ej, m = oracle.torus_run(-np.ones((L, L), np.int8), 1, ms.FIG4_LAM, ms.FIG4_Q, beta, 3, r, T)
        EJ, M = b.log_ej(r)
        assert np.array_equal(EJ, ej), r
        assert np.array_equal(M, m), r
        _, M_all, EJ_all = b.logs()
        assert np.array_equal(EJ_all[r], ej) and np.array_equal(M_all[r], m), r
        assert np.array_equal(chains[r].spins(), x), r
        assert m[-1] > 0, "replica %d has not tunnelled in %d steps" % (r, T)
    b.close()
    for c in chains:
        c.close()


def test_theorem_3_3_diagonal_growth(sk, ms):
    L, beta, R = 16, 4.0, 32
    print("theorem 3.3: L=%d beta=%g replicas=%d" % (L, beta, R), flush=True)
    res = ms.run(L, [beta] * R, max_steps=2_000_000, chunk=50_000, seed=11)
    bound = ms.tunnelling_bound(beta)
    print("steps %d, exit median %d, all-plus median %d max %d (bound %.3g), in D %.4f (min %.4f), "
          "increasing %d/%d" % (res.steps, np.median(res.exit_t), np.median(res.plus_t), res.plus_t.max(),
                                bound, res.diag_fraction.mean(), res.diag_fraction.min(),
                                res.monotone.sum(), R), flush=True)
    assert np.all(res.plus_t > 0)
    assert res.plus_t.max() < bound
    # a limit in probability as beta grows: at beta = 4 nearly every replica
    # follows the path (31 of 32 in a first run)
    assert res.monotone.mean() >= 0.9
    assert res.diag_fraction.mean() > 0.95
    # the half-way configuration of two replicas, recomputed from scratch, is in D
    for r in [k for k in range(R) if res.monotone[k]][:2]:
        t = int(res.mid_t[r])
        assert t > 0
        ch = ms.make_chains(L, [beta], seed=11, replica0=r)[0]
        ch.sweep(t)
        x = ch.spins()
        ch.close()
        assert ms.in_diagonal_set(x), r
        assert int(np.sum(x[0] > 0)) == L // 2     # row 0 meets every diagonal once


def test_nucleation_experiment_shaken_side(sk, ms):
    L, R, T = 32, 48, 30_000
    betas = (1.3, 2.3, 3.3)
    print("nucleation L=%d replicas=%d T=%d" % (L, R, T), flush=True)
    res = ms.run(L, np.repeat(betas, R), max_steps=T, chunk=15_000, seed=21, stop=None)
    med = []
    for b in betas:
        k = res.betas == b
        cross = res.cross_t[k]
        print("beta %g: crossing median %d max %d, bound %.3g, final m %.4f"
              % (b, np.median(cross), cross.max(), ms.tunnelling_bound(b), res.m_final[k].mean()), flush=True)
        assert np.all(cross > 0)
        assert cross.max() < ms.tunnelling_bound(b)
        med.append(np.median(cross))
    assert med[0] < med[1] < med[2]
    m13 = res.m_final[res.betas == 1.3].mean()
    assert 0.9 < m13 < 0.995           # below +1 at finite beta
    for b in betas[1:]:
        assert res.m_final[res.betas == b].mean() > 0.99
    # the mean magnetisation curve: beta = 3.3 still metastable at t = 100
    row = list(res.beta_values).index(3.3)
    t100 = np.nonzero(res.times >= 100)[0][0]
    assert res.m_mean[row, t100] < -0.9
