"""Pins of the oracle's randomness contract: Philox4x32-10 against ATen's
independent implementation (compiled and run here), and the threshold rule
against 50-digit arithmetic.  CPU only."""
import os
import shutil
import subprocess

import mpmath
import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def aten_philox(tmp_path_factory):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("aten") / "aten_philox")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", inc, "-o", exe,
                           os.path.join(HERE, "aten_philox_check.cpp")])
    return exe


def test_philox_matches_aten(aten_philox):
    rng = np.random.Generator(np.random.PCG64(11))
    rows = [(0, 0, 0, 0, 0), (2 ** 64 - 1, 2 ** 32 - 1, 2 ** 32 - 1, 2 ** 32 - 1, 2 ** 32 - 1),
            (1, 5, 0xFFFFFFFF, 3, 7)]
    for _ in range(200):
        rows.append((int(rng.integers(0, 2 ** 63)),) + tuple(int(x) for x in rng.integers(0, 2 ** 32, 4)))
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([aten_philox], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(rows)
    for r, want in zip(rows, ref):
        got = oracle.philox(r[1:], r[0])
        assert list(int(x) for x in got) == want, r


def _p_plus(h, beta):
    mpmath.mp.dps = 50
    return 1 / (1 + mpmath.e ** (-2 * mpmath.mpf(beta) * mpmath.mpf(h)))


@pytest.mark.parametrize("beta", [0.0, 0.3, 0.4406868, 0.8, 2.0, 7.5])
def test_threshold_within_one_count_of_exact(beta):
    """P(+1) = exp(b h)/(2 cosh(b h)) (half-step kernels of section 2) =
    1/(1+exp(-2 b h)); the 33-bit threshold is within one count of 2^32 P."""
    for h in np.concatenate([np.arange(-6, 6.25, 0.25), [1e-9, -1e-9, 3.7, -3.7]]):
        T = oracle.threshold(float(h), beta)
        exact = _p_plus(float(h), beta) * 2 ** 32
        assert 0 <= T <= 2 ** 32
        assert abs(T - exact) <= 1, (h, beta, T, float(exact))


def test_threshold_symmetry_and_special_values():
    for beta in (0.2, 0.9, 3.0):
        for h in (0.1, 0.5, 1.0, 2.5, 4.0):
            assert oracle.threshold(h, beta) + oracle.threshold(-h, beta) == 2 ** 32
        assert oracle.threshold(0.0, beta) == 2 ** 31
    # beta = 0: every spin is a fair coin
    for h in (-3.0, -1.0, 0.0, 2.0):
        assert oracle.threshold(h, 0.0) == 2 ** 31
    # zero temperature: decisions saturate
    assert oracle.threshold(0.05, 1000.0) == 2 ** 32
    assert oracle.threshold(-0.05, 1000.0) == 0


def test_field_order_and_values():
    # h = S + q sigma + lambda
    assert oracle.field(2, 1, 1.0, 0.0) == 3.0
    assert oracle.field(-2, -1, 0.5, 0.15) == -2.5 + 0.15
    assert oracle.field(0, -1, 0.0, 0.0) == 0.0


def test_uniforms_are_uniform():
    """Top 4 bits of the torus and graph uniforms over many sites: chi^2."""
    L = 64
    top = np.array([oracle.torus_uniform(L, 3, 0, 5, r, c) >> 28
                    for r in range(0, L, 2) for c in range(L)])
    cnt = np.bincount(top, minlength=16)
    e = len(top) / 16
    assert ((cnt - e) ** 2 / e).sum() < 45   # chi^2_15, p ~ 1e-4
    topg = np.array([oracle.graph_uniform(3, 0, 5, v) >> 28 for v in range(4096)])
    cnt = np.bincount(topg, minlength=16)
    e = len(topg) / 16
    assert ((cnt - e) ** 2 / e).sum() < 45
