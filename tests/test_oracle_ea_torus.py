"""Pins of the oracle's +-J torus (Edwards-Anderson couplings, the workload of
section 6): every oriented edge (x, x_up), (x, x_right) carries its own sign.

The enumeration model builds the pair Hamiltonian of Definition 2.2 from the
same couplings in matrix form (independent of the oracle's neighbour
arithmetic); the oracle must follow its fields at zero temperature, its
one-step law at finite temperature, equation ham1 for the energy, reduce
bit-exactly to the uniform torus when all signs agree, and respect the gauge
symmetry J_xy -> e_x J_xy e_y, sigma -> e sigma of the lambda = 0 model."""
import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import enumeration as en


def _signs(rng, L):
    return tuple(np.where(rng.integers(0, 2, (L, L)) == 1, 1, -1).astype(np.int8) for _ in range(2))


def _edge_couplings(ju, jr):
    """couplings in the order of enumeration.torus_edges: (x, up), (x, right) per x"""
    return np.stack([ju.reshape(-1), jr.reshape(-1)], axis=1).reshape(-1).astype(np.float64)


def _rand_spins(rng, n):
    return np.where(rng.integers(0, 2, n) == 1, 1, -1).astype(np.int8)


def _chi2_p(counts, probs):
    probs = np.asarray(probs)
    keep = probs * counts.sum() >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(probs[keep], probs[~keep].sum()) * counts.sum()
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    return stats.chisquare(obs, exp).pvalue


@pytest.mark.parametrize("sign", [1, -1])
def test_uniform_signs_reduce_to_the_uniform_torus(sign):
    L = 37
    rng = np.random.Generator(np.random.PCG64(2))
    sp = _rand_spins(rng, L * L).reshape(L, L)
    J = (np.full((L, L), sign, np.int8), np.full((L, L), sign, np.int8))
    a, ea, ma = oracle.torus_run(sp, J, 0.1, 0.8, 0.45, 7, 3, 25)
    b, eb, mb = oracle.torus_run(sp, sign, 0.1, 0.8, 0.45, 7, 3, 25)
    assert np.array_equal(a, b) and np.array_equal(ea, eb) and np.array_equal(ma, mb)


@pytest.mark.parametrize("L", [3, 4, 5])
def test_zero_temperature_follows_pair_hamiltonian_fields(L):
    q, lam = 0.5, 0.25     # |h| >= 0.25: fields never vanish
    rng = np.random.Generator(np.random.PCG64(40 + L))
    ju, jr = _signs(rng, L)
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, J=_edge_couplings(ju, jr), lam=np.full(L * L, lam), q=q, beta=1.0)
    for _ in range(20):
        sp = _rand_spins(rng, L * L)
        got1 = oracle.torus_half_step(sp.reshape(L, L), (ju, jr), lam, q, 1000.0, 5, 0, 0).reshape(-1)
        assert np.array_equal(got1, np.sign(m.field12_of(sp)).astype(np.int8))
        got2 = oracle.torus_half_step(got1.reshape(L, L), (ju, jr), lam, q, 1000.0, 5, 0, 1).reshape(-1)
        assert np.array_equal(got2, np.sign(m.field21_of(got1)).astype(np.int8))


def test_energy_matches_ham1():
    L = 4
    rng = np.random.Generator(np.random.PCG64(8))
    ju, jr = _signs(rng, L)
    lam = 0.5
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, J=_edge_couplings(ju, jr), lam=np.full(L * L, lam), q=1.0, beta=1.0)
    for _ in range(30):
        sp = _rand_spins(rng, L * L)
        ej, mm = oracle.torus_observe(sp.reshape(L, L), (ju, jr))
        assert mm == int(sp.sum())
        assert -ej - 2 * lam * mm == pytest.approx(m.gibbs_H_of(sp), abs=1e-12)


def test_one_step_law_chi2():
    L, q, lam, b = 3, 0.6, 0.2, 0.5
    rng = np.random.Generator(np.random.PCG64(11))
    ju, jr = _signs(rng, L)
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, J=_edge_couplings(ju, jr), lam=np.full(L * L, lam), q=q, beta=b)
    sp = np.array([1, -1, 1, 1, 1, -1, -1, -1, 1], dtype=np.int8).reshape(L, L)
    i0 = en.index_of(sp.reshape(-1))
    full = np.zeros(2 ** (L * L))
    for r in range(30000):
        a = oracle.torus_half_step(sp, (ju, jr), lam, q, b, 5, r, 0)
        c = oracle.torus_half_step(a, (ju, jr), lam, q, b, 5, r, 1)
        full[en.index_of(c.reshape(-1))] += 1
    assert _chi2_p(full, m.Psh()[i0]) > 1e-4


def test_gauge_symmetry_in_law():
    """lambda = 0: running the oracle with couplings e_x J_xy e_y from e*sigma
    and mapping the result back by e gives the one-step law of J from sigma."""
    L, q, b = 3, 0.7, 0.45
    rng = np.random.Generator(np.random.PCG64(12))
    ju, jr = _signs(rng, L)
    e = _rand_spins(rng, L * L).reshape(L, L)
    eu = (e * np.roll(e, -1, axis=0) * ju).astype(np.int8)     # e_x J(x, x_up) e_{x_up}
    er = (e * np.roll(e, -1, axis=1) * jr).astype(np.int8)     # e_x J(x, x_right) e_{x_right}
    s, d = en.torus_edges(L)
    m = en.Model(L * L, s, d, J=_edge_couplings(ju, jr), q=q, beta=b)
    sp = np.array([-1, -1, 1, 1, -1, -1, 1, 1, 1], dtype=np.int8).reshape(L, L)
    i0 = en.index_of(sp.reshape(-1))
    full = np.zeros(2 ** (L * L))
    for r in range(30000):
        a = oracle.torus_half_step(e * sp, (eu, er), 0.0, q, b, 9, r, 0)
        c = oracle.torus_half_step(a, (eu, er), 0.0, q, b, 9, r, 1)
        full[en.index_of((e * c).reshape(-1))] += 1
    assert _chi2_p(full, m.Psh()[i0]) > 1e-4
