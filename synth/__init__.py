"""Seeded synthetic inputs for shaken dynamics workloads.

This module holds no arithmetic of the method: it only draws graphs,
orientations, couplings, field classes and per-instance parameters.  Both the
oracle-side tests and the GPU-side tests and benchmark take their inputs from
here.  Draws use numpy's PCG64 ``Generator`` seeded explicitly.

Workloads (shapes and distributions of the paper's settings, section 2 for
arbitrary graphs and section 6 for the +-J optimisation experiment):
  * ``regular_graph``  -- uniform simple d-regular graph by the configuration
    model, the whole pairing redrawn whenever it has a self-loop or a repeated
    edge;
  * ``oriented_instance`` -- each undirected edge oriented by a fair coin
    (the arbitrary orientation of Definition 2.1), couplings +-1 i.i.d. fair,
    field classes drawn uniformly from a value table;
  * ``batch_spec`` -- mixed batch of tori and 3-regular +-J graphs with
    per-instance (beta, q, seed).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def regular_graph(n: int, d: int, seed: int, max_tries: int = 10000):
    """Undirected simple d-regular graph on n vertices; returns (u, v) arrays with
    u < v, one row per edge, sorted."""
    if (n * d) % 2 or d >= n:
        raise ValueError("need n*d even and d < n")
    rng = np.random.Generator(np.random.PCG64(seed))
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    for _ in range(max_tries):
        p = rng.permutation(stubs)
        a, b = p[0::2], p[1::2]
        if np.any(a == b):
            continue
        u = np.minimum(a, b)
        v = np.maximum(a, b)
        key = u * n + v
        key.sort()
        if np.any(key[1:] == key[:-1]):
            continue
        return (key // n).astype(np.int32), (key % n).astype(np.int32)
    raise RuntimeError("configuration model did not produce a simple graph")


@dataclasses.dataclass
class Instance:
    n: int
    src: np.ndarray          # oriented edges (src[e], dst[e]) in E^o
    dst: np.ndarray
    J: np.ndarray            # int8 per oriented edge
    cls: np.ndarray          # uint8 field class per vertex
    lam_values: np.ndarray   # float64 value per class


def oriented_instance(n: int, d: int, seed: int, lam_values=(0.0,), pm_j: bool = True):
    """d-regular graph with coin orientation, +-1 couplings (or all +1) and
    uniform field classes."""
    u, v = regular_graph(n, d, seed)
    rng = np.random.Generator(np.random.PCG64([seed, 0x5EED]))
    flip = rng.integers(0, 2, size=u.shape[0]).astype(bool)
    src = np.where(flip, v, u).astype(np.int32)
    dst = np.where(flip, u, v).astype(np.int32)
    if pm_j:
        J = np.where(rng.integers(0, 2, size=u.shape[0]) == 1, 1, -1).astype(np.int8)
    else:
        J = np.ones(u.shape[0], dtype=np.int8)
    lam_values = np.asarray(lam_values, dtype=np.float64)
    cls = rng.integers(0, len(lam_values), size=n).astype(np.uint8)
    return Instance(n, src, dst, J, cls, lam_values)


def random_oriented_graph(n: int, p: float, seed: int, jmax: int = 1, n_classes: int = 1,
                          lam_scale: float = 0.5):
    """Erdos-Renyi G(n, p) with coin orientation, integer couplings uniform in
    [-jmax, jmax] without 0, and field values k * lam_scale for classes k-1..."""
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    u, v = iu[keep], ju[keep]
    flip = rng.integers(0, 2, size=u.shape[0]).astype(bool)
    src = np.where(flip, v, u).astype(np.int32)
    dst = np.where(flip, u, v).astype(np.int32)
    mag = rng.integers(1, jmax + 1, size=u.shape[0])
    sgn = np.where(rng.integers(0, 2, size=u.shape[0]) == 1, 1, -1)
    J = (mag * sgn).astype(np.int8)
    lam_values = (np.arange(n_classes) - (n_classes - 1) / 2.0) * lam_scale
    cls = rng.integers(0, n_classes, size=n).astype(np.uint8)
    return Instance(n, src, dst, J, cls, np.asarray(lam_values, dtype=np.float64))


# --------------------------------------------------------------- workloads --

#: 4096^2 torus runs: q x beta x initial state (all-up / random), J=+1, lambda=0
TORUS_Q = (0.5, 1.0, 2.0)
TORUS_BETA = (0.30, 0.40, 0.44, 0.50)
TORUS_INIT = ("all_up", "random")


def torus_runs():
    """The 24 (q, beta, init) combinations of the 4096^2 torus workload."""
    runs = []
    for q in TORUS_Q:
        for b in TORUS_BETA:
            for init in TORUS_INIT:
                runs.append(dict(q=q, beta=b, init=init, seed=2))
    return runs


@dataclasses.dataclass
class BatchItem:
    kind: str        # "torus" or "graph"
    size: int        # L for tori, n for graphs
    beta: float
    q: float
    seed: int
    graph: Instance | None = None


def batch_spec(n_tori: int, n_graphs: int, seed: int, l_max: int = 256, n_min: int = 1024,
               n_max: int = 65536, with_graphs: bool = True):
    """Mixed batch: tori with L uniform in {16, 32, ..., l_max} (J=+1, lambda=0)
    and 3-regular +-J graphs with n uniform in [n_min, n_max] rounded to even
    (lambda=0); beta ~ U(0.2, 1.2), q ~ U(0.5, 3.0), own seed each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    items = []
    for i in range(n_tori):
        L = 16 * int(rng.integers(1, l_max // 16 + 1))
        items.append(BatchItem("torus", L, float(rng.uniform(0.2, 1.2)),
                               float(rng.uniform(0.5, 3.0)), int(rng.integers(1, 2 ** 62))))
    for i in range(n_graphs):
        n = int(rng.integers(n_min, n_max + 1)) & ~1
        gseed = int(rng.integers(1, 2 ** 62))
        it = BatchItem("graph", n, float(rng.uniform(0.2, 1.2)), float(rng.uniform(0.5, 3.0)),
                       int(rng.integers(1, 2 ** 62)))
        if with_graphs:
            it.graph = oriented_instance(n, 3, gseed, lam_values=(0.0,), pm_j=True)
        items.append(it)
    return items


def triangular_torus_edges(L: int):
    """Triangular lattice on an L x L torus in skewed coordinates (site
    x = row * L + col): every site has the six neighbours x +- e1, x +- e2,
    x +- (e1 + e2) with e1 = one column, e2 = one row.  Oriented edges
    (x, x + e1), (x, x + e2), (x, x + e1 + e2): the in-half of x (its three
    "left" neighbours) is {x - e1, x - e2, x - e1 - e2}, the out-half the
    other three (section 4, shaken dynamics on the triangular lattice).
    Returns (src, dst) int32 arrays of 3 L^2 edges."""
    r, c = np.divmod(np.arange(L * L), L)
    x = r * L + c
    right = r * L + (c + 1) % L
    up = ((r + 1) % L) * L + c
    diag = ((r + 1) % L) * L + (c + 1) % L
    src = np.concatenate([x, x, x]).astype(np.int32)
    dst = np.concatenate([right, up, diag]).astype(np.int32)
    return src, dst
