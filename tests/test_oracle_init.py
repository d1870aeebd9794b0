"""Pins of the oracle's random starts: the configuration model of the
workloads' "i.i.d. uniform" starts is independent fair coins, one per site.

Checked by what that law fixes, not by re-deriving the generator:
  * the number of +1 spins is Binomial(N, 1/2);
  * for every displacement (dr, dc) in a window around the origin, the
    fraction of sites that agree with the site displaced by (dr, dc) is 1/2
    (a wrong word index, e.g. rows sharing or overlapping generator words when
    L is not a multiple of 32, or a bit taken twice, makes some displacement
    agree far more often);
  * distinct replicas and distinct seeds give independent starts (agreement
    1/2 between them);
  * every 32-site word takes its 2^k patterns on k-bit windows uniformly
    (chi-squared), so the bits within a word are not tied to each other.
z-scores are checked at |z| < 6 over about 2,300 comparisons, so under the
law a false alarm has probability below 1e-5.  Planted mistakes in a copy of
the start (the row stride floor(L/32) or ceil(L/32) - 1, no row term, one
word per row, bit c & 15 for c & 31, the replica word ignored) each fail.
"""
import numpy as np
import pytest

import oracle

Z = 6.0


def _z_fair(k, n):
    """z-score of k successes in n fair trials"""
    return (k - 0.5 * n) / np.sqrt(0.25 * n)


def _agreement_z(a, b):
    return _z_fair(int(np.count_nonzero(a == b)), a.size)


def _stack(L, seeds, replicas):
    return np.stack([oracle.torus_init_random(L, s, r) for s in seeds for r in replicas])


@pytest.mark.parametrize("L,reps", [(37, 64), (100, 16), (33, 64), (64, 16)])
def test_torus_start_marginal_and_pair_agreement(L, reps):
    """Ragged and whole-word sides, many replicas pooled: fair marginal and
    agreement 1/2 at every displacement |dr| <= 3, |dc| <= 40 (which covers
    the 32-column word boundary and a whole word of shift)."""
    S = _stack(L, [2], range(reps)).astype(np.int8)
    assert set(np.unique(S)) <= {-1, 1}
    n = S.size
    assert abs(_z_fair(int(np.count_nonzero(S > 0)), n)) < Z
    for dr in range(-3, 4):
        for dc in range(-40, 41):
            if dr % L == 0 and dc % L == 0:
                continue  # the identity on the torus
            sh = np.roll(np.roll(S, dr, axis=1), dc, axis=2)
            z = _agreement_z(S, sh)
            assert abs(z) < Z, (L, dr, dc, z)


def test_torus_start_4096_band():
    """Full-size start (4096^2, the headline workload's seed 2): marginal over
    the whole torus, agreement 1/2 for the row and column neighbours and the
    displacements across a word, in a band of 256 rows and over all rows."""
    L = 4096
    S = oracle.torus_init_random(L, 2, 5)
    assert abs(_z_fair(int(np.count_nonzero(S > 0)), S.size)) < Z
    band = S[1000:1256]
    for dr, dc in [(0, 1), (1, 0), (1, 1), (0, 32), (1, -32), (0, 31), (0, 33), (2, 0), (0, 4064)]:
        assert abs(_agreement_z(S, np.roll(np.roll(S, dr, 0), dc, 1))) < Z, (dr, dc)
        assert abs(_agreement_z(band, np.roll(np.roll(band, dr, 0), dc, 1))) < Z, (dr, dc)
    # no two rows of the band equal, no row equal to its neighbour shifted by a word
    rows = {r.tobytes() for r in band}
    assert len(rows) == band.shape[0]


@pytest.mark.parametrize("L", [37, 64, 256])
def test_torus_start_word_patterns(L):
    """Each 32-site word of the start, read as bits, is a uniform random
    word: chi-squared of the 16 patterns of every aligned 4-bit window."""
    S = _stack(L, [2, 3], range(32))
    W = (L + 31) // 32
    counts = np.zeros(16, dtype=np.int64)
    for w in range(W):
        cols = range(32 * w, min(32 * w + 32, L))
        blk = (S[:, :, list(cols)] > 0).astype(np.int64)
        for c0 in range(0, blk.shape[2] - 3, 4):
            pat = blk[:, :, c0] | (blk[:, :, c0 + 1] << 1) | (blk[:, :, c0 + 2] << 2) | (blk[:, :, c0 + 3] << 3)
            counts += np.bincount(pat.reshape(-1), minlength=16)
    e = counts.sum() / 16.0
    chi2 = float(((counts - e) ** 2 / e).sum())
    # 15 degrees of freedom: P(chi2 > 60) < 1e-6
    assert chi2 < 60.0, chi2


def test_torus_start_replicas_and_seeds_independent():
    """Agreement 1/2 between the starts of distinct replicas and of distinct
    seeds, the same start for the same (seed, replica)."""
    L = 100
    base = oracle.torus_init_random(L, 2, 0)
    assert np.array_equal(base, oracle.torus_init_random(L, 2, 0))
    for seed, rep in [(2, 1), (2, 2), (2, 1000), (3, 0), (1 << 40, 0), (2 + (1 << 32), 0)]:
        other = oracle.torus_init_random(L, seed, rep)
        assert abs(_agreement_z(base, other)) < Z, (seed, rep)
    # pooled over many replicas: every pair of consecutive replicas independent
    S = _stack(L, [7], range(64))
    agree = np.count_nonzero(S[1:] == S[:-1])
    assert abs(_z_fair(int(agree), S[1:].size)) < Z


def test_graph_start_pair_agreement():
    """The graph start is pinned by the finite-time law elsewhere; here the
    same pair tests on vertex order: marginal and agreement at offsets 1..40
    (four vertices share a generator call)."""
    n = 1 << 16
    S = np.stack([oracle.graph_init_random(n, 11, r) for r in range(8)])
    assert abs(_z_fair(int(np.count_nonzero(S > 0)), S.size)) < Z
    for d in range(1, 41):
        assert abs(_agreement_z(S, np.roll(S, d, axis=1))) < Z, d
    assert abs(_agreement_z(S[0], S[1])) < Z
