"""Float64 reference of the annealing-schedule network.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The network is not in
the paper: it picks (beta_t, q_t) for the minimisation use of the dynamics
(section 6).  Its arithmetic is defined by the library's interface: a
16 -> 128 -> 128 -> 128 -> 16 perceptron with ReLU on the hidden layers; BF16
(round to nearest even, from FP32) copies of the weights, of the input, of the
hidden activations, of the output gradient and of the back-propagated
pre-activation gradients; FP32 biases; every product accumulated exactly here
(float64) and in FP32 on the device.

With ``rounding=False`` every rounding point is the identity and the code is a
plain float64 multilayer perceptron, whose gradient is pinned by central
finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

NI, NH, NO = 16, 128, 16
OFF_W1 = 0
OFF_B1 = OFF_W1 + NH * NI
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH * NH
OFF_W4 = OFF_B3 + NH
OFF_B4 = OFF_W4 + NO * NH
NPARAM = OFF_B4 + NO


def bf16(x) -> np.ndarray:
    """Round to BF16 (nearest, ties to even) through FP32, back to float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    return dict(W1=P[OFF_W1:OFF_B1].reshape(NH, NI), b1=P[OFF_B1:OFF_W2],
                W2=P[OFF_W2:OFF_B2].reshape(NH, NH), b2=P[OFF_B2:OFF_W3],
                W3=P[OFF_W3:OFF_B3].reshape(NH, NH), b3=P[OFF_B3:OFF_W4],
                W4=P[OFF_W4:OFF_B4].reshape(NO, NH), b4=P[OFF_B4:NPARAM])


def init_params(seed: int, scale: float = 1.0) -> np.ndarray:
    """He-style random initial parameters (used by the training driver too)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = np.zeros(NPARAM)
    P[OFF_W1:OFF_B1] = rng.normal(0, scale * np.sqrt(2.0 / NI), NH * NI)
    P[OFF_W2:OFF_B2] = rng.normal(0, scale * np.sqrt(2.0 / NH), NH * NH)
    P[OFF_W3:OFF_B3] = rng.normal(0, scale * np.sqrt(2.0 / NH), NH * NH)
    W4 = rng.normal(0, scale * np.sqrt(1.0 / NH), (NO, NH))
    W4[2:] = 0.0
    P[OFF_W4:OFF_B4] = W4.reshape(-1)
    return P


def forward(P, X, rounding=True):
    """y [rows, 16] and the cache for backward."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(P)
    x = r(X)
    W1, W2, W3, W4 = r(p["W1"]), r(p["W2"]), r(p["W3"]), r(p["W4"])
    h1 = r(np.maximum(x @ W1.T + p["b1"], 0.0))
    h2 = r(np.maximum(h1 @ W2.T + p["b2"], 0.0))
    h3 = r(np.maximum(h2 @ W3.T + p["b3"], 0.0))
    y = h3 @ W4.T + p["b4"]
    return y, dict(x=x, h1=h1, h2=h2, h3=h3, W2=W2, W3=W3, W4=W4, rounding=rounding)


def backward(cache, dy):
    """Parameter gradient (flat, NPARAM) for output gradient dy [rows, 16]."""
    r = bf16 if cache["rounding"] else (lambda a: np.asarray(a, dtype=np.float64))
    g = np.zeros(NPARAM)
    dz4 = r(dy)
    g[OFF_W4:OFF_B4] = (dz4.T @ cache["h3"]).reshape(-1)
    g[OFF_B4:NPARAM] = dz4.sum(axis=0)
    dz3 = r((cache["h3"] > 0) * (dz4 @ cache["W4"]))
    g[OFF_W3:OFF_B3] = (dz3.T @ cache["h2"]).reshape(-1)
    g[OFF_B3:OFF_W4] = dz3.sum(axis=0)
    dz2 = r((cache["h2"] > 0) * (dz3 @ cache["W3"]))
    g[OFF_W2:OFF_B2] = (dz2.T @ cache["h1"]).reshape(-1)
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    dz1 = r((cache["h1"] > 0) * (dz2 @ cache["W2"]))
    g[OFF_W1:OFF_B1] = (dz1.T @ cache["x"]).reshape(-1)
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    return g


def mse_grad(y, target, w=None):
    """Loss sum_r w_r sum_{c<2} (y - t)^2 / sum_r w_r and its gradient in y."""
    rows = y.shape[0]
    w = np.ones(rows) if w is None else np.asarray(w, dtype=np.float64)
    W = w.sum()
    d = np.zeros_like(y)
    d[:, :2] = y[:, :2] - target[:, :2]
    loss = float((w[:, None] * d ** 2).sum() / W)
    return loss, 2.0 * w[:, None] * d / W
