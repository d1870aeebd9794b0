"""Pins of the float64 network oracle: its back-propagation against central
finite differences of its own forward (pure float64, no rounding), and the
BF16 rounding helper against the definition of round-to-nearest-even.
CPU only."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_definition():
    # exact BF16 values are fixed points; halfway cases go to even
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0             # halfway, even mantissa kept
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # halfway, rounds up to even
    assert mlp.bf16(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7
    x = np.random.Generator(np.random.PCG64(0)).normal(size=1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8)
    assert np.array_equal(mlp.bf16(r), r)


def test_backprop_matches_finite_differences():
    rng = np.random.Generator(np.random.PCG64(1))
    P = mlp.init_params(3)
    P[mlp.OFF_B1:mlp.OFF_W2] = 0.1
    X = rng.normal(size=(12, 16))
    T = rng.normal(size=(12, 16))
    w = rng.uniform(0.5, 2.0, 12)

    def loss(p):
        y, _ = mlp.forward(p, X, rounding=False)
        return mlp.mse_grad(y, T, w)[0]

    y, cache = mlp.forward(P, X, rounding=False)
    _, dy = mlp.mse_grad(y, T, w)
    g = mlp.backward(cache, dy)
    idx = np.concatenate([rng.integers(a, b, 12) for a, b in
                          [(mlp.OFF_W1, mlp.OFF_B1), (mlp.OFF_B1, mlp.OFF_W2), (mlp.OFF_W2, mlp.OFF_B2),
                           (mlp.OFF_B2, mlp.OFF_W3), (mlp.OFF_W3, mlp.OFF_B3), (mlp.OFF_B3, mlp.OFF_W4),
                           (mlp.OFF_W4, mlp.OFF_W4 + 2 * 128), (mlp.OFF_B4, mlp.OFF_B4 + 2)]])
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(P)
        e[i] = eps
        fd = (loss(P + e) - loss(P - e)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])
    # unused output rows get no gradient
    assert np.all(g[mlp.OFF_W4 + 2 * 128:mlp.OFF_B4] == 0)
    assert np.all(g[mlp.OFF_B4 + 2:] == 0)


def test_rounded_network_close_to_exact():
    """The BF16 network differs from the float64 one by the rounding only."""
    rng = np.random.Generator(np.random.PCG64(2))
    P = mlp.init_params(5)
    X = rng.normal(size=(64, 16))
    y0, _ = mlp.forward(P, X, rounding=False)
    y1, _ = mlp.forward(P, X, rounding=True)
    assert np.linalg.norm(y1 - y0) / np.linalg.norm(y0) < 0.05
