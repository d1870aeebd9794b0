"""CPU oracle of shaken dynamics (arXiv:1904.06257).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP implementation.

Two parts:
  * ``shaken_oracle.c`` -- plain single-threaded C trajectories (torus and
    arbitrary oriented graph), the Philox4x32-10 generator and the threshold
    rule of the randomness contract; wrapped here through ctypes.
  * ``enumeration`` -- float64 exact enumeration of the transition matrices and
    stationary measures on small graphs (section 2, Theorem 2.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "shaken_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i8p = ctypes.POINTER(ctypes.c_int8)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)

GRAPH_STREAM = 0x80000000
INIT_STEP = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        L.oracle_philox4x32_10.argtypes = [_u32p, ctypes.c_uint64, _u32p]
        L.oracle_threshold.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_threshold.restype = ctypes.c_uint64
        L.oracle_field.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.oracle_field.restype = ctypes.c_double
        L.oracle_torus_uniform.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                           ctypes.c_uint32, ctypes.c_int, ctypes.c_int]
        L.oracle_torus_uniform.restype = ctypes.c_uint32
        L.oracle_torus_init_random.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, _i8p]
        L.oracle_torus_site.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_uint32, _i8p, ctypes.c_int, ctypes.c_int]
        L.oracle_torus_site.restype = ctypes.c_int
        L.oracle_torus_half_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                             ctypes.c_uint32, ctypes.c_uint32, _i8p, _i8p]
        L.oracle_torus_observe.argtypes = [ctypes.c_int, ctypes.c_int, _i8p, _i64p, _i64p]
        L.oracle_torus_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_uint32, _i8p, ctypes.c_int64, _i64p, _i64p]
        L.oracle_torus_run.restype = ctypes.c_int
        L.oracle_torus_site_j.argtypes = [ctypes.c_int, ctypes.c_int, _i8p, _i8p, ctypes.c_int,
                                          ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                          ctypes.c_uint32, ctypes.c_uint32, _i8p, ctypes.c_int,
                                          ctypes.c_int]
        L.oracle_torus_site_j.restype = ctypes.c_int
        L.oracle_torus_half_step_j.argtypes = [ctypes.c_int, ctypes.c_int, _i8p, _i8p, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                               _i8p, _i8p]
        L.oracle_torus_observe_j.argtypes = [ctypes.c_int, ctypes.c_int, _i8p, _i8p, ctypes.c_int,
                                             _i8p, _i64p, _i64p]
        L.oracle_torus_run_j.argtypes = [ctypes.c_int, ctypes.c_int, _i8p, _i8p, ctypes.c_int,
                                         ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_uint32, _i8p, ctypes.c_int64,
                                         _i64p, _i64p]
        L.oracle_torus_run_j.restype = ctypes.c_int
        L.oracle_graph_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint32]
        L.oracle_graph_uniform.restype = ctypes.c_uint32
        L.oracle_graph_init_random.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, _i8p]
        L.oracle_graph_half_step.argtypes = [ctypes.c_int, ctypes.c_int64, _i32p, _i32p, _i8p, _u8p,
                                             _f64p, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                             _i8p, _i8p]
        L.oracle_graph_half_step.restype = ctypes.c_int
        L.oracle_graph_observe.argtypes = [ctypes.c_int, ctypes.c_int64, _i32p, _i32p, _i8p, _u8p,
                                           ctypes.c_int, _i8p, _i64p, _i64p]
        L.oracle_graph_run.argtypes = [ctypes.c_int, ctypes.c_int64, _i32p, _i32p, _i8p, _u8p,
                                       ctypes.c_int, _f64p, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _i8p,
                                       ctypes.c_int64, _i64p, _i64p]
        L.oracle_graph_run.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


# ------------------------------------------------------------------ helpers --

def philox(ctr, seed: int) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c, _u32p), ctypes.c_uint64(seed), _p(out, _u32p))
    return out


def threshold(h: float, beta: float) -> int:
    return int(lib().oracle_threshold(float(h), float(beta)))


def field(S: int, sigma: int, q: float, lam: float) -> float:
    return float(lib().oracle_field(int(S), int(sigma), float(q), float(lam)))


def threshold_of(S: int, sigma: int, q: float, lam: float, beta: float) -> int:
    return threshold(field(S, sigma, q, lam), beta)


# -------------------------------------------------------------------- torus --

def torus_init_random(L: int, seed: int, replica: int = 0) -> np.ndarray:
    sp = np.zeros(L * L, dtype=np.int8)
    lib().oracle_torus_init_random(L, ctypes.c_uint64(seed), replica, _p(sp, _i8p))
    return sp.reshape(L, L)


def torus_uniform(L, seed, replica, s, r, c) -> int:
    return int(lib().oracle_torus_uniform(L, ctypes.c_uint64(seed), replica, s, r, c))


def _couplings(J, L):
    """J as an int (uniform coupling) or a pair (Jup, Jright) of int8 [L, L]
    arrays: Jup[r, c] couples (r, c) to (r+1, c), Jright[r, c] to (r, c+1)."""
    if np.isscalar(J):
        return int(J), None, None
    ju = np.ascontiguousarray(J[0], dtype=np.int8).reshape(L * L)
    jr = np.ascontiguousarray(J[1], dtype=np.int8).reshape(L * L)
    return 0, ju, jr


def _mode(rev, tri):
    return (1 if rev else 0) | (2 if tri else 0)


def torus_half_step(spins, J, lam, q, beta, seed, replica, s, rev=False, tri=False) -> np.ndarray:
    """rev: the reversed order P^{sh'} (out-half, ur, read at even s);
    tri: the triangular lattice (uniform J)"""
    L = spins.shape[0]
    a = np.ascontiguousarray(spins, dtype=np.int8)
    out = np.zeros_like(a)
    j, ju, jr = _couplings(J, L)
    lib().oracle_torus_half_step_j(L, j, _p(ju, _i8p), _p(jr, _i8p), _mode(rev, tri), float(lam), float(q),
                                   float(beta), ctypes.c_uint64(seed), replica, s & 0xFFFFFFFF,
                                   _p(a, _i8p), _p(out, _i8p))
    return out


def torus_site(spins, J, lam, q, beta, seed, replica, s, r, c, rev=False, tri=False) -> int:
    a = np.ascontiguousarray(spins, dtype=np.int8)
    j, ju, jr = _couplings(J, a.shape[0])
    return int(lib().oracle_torus_site_j(a.shape[0], j, _p(ju, _i8p), _p(jr, _i8p), _mode(rev, tri), float(lam),
                                         float(q), float(beta), ctypes.c_uint64(seed), replica,
                                         s & 0xFFFFFFFF, _p(a, _i8p), int(r), int(c)))


def torus_observe(spins, J=1, tri=False):
    a = np.ascontiguousarray(spins, dtype=np.int8)
    e = ctypes.c_int64()
    m = ctypes.c_int64()
    j, ju, jr = _couplings(J, a.shape[0])
    lib().oracle_torus_observe_j(a.shape[0], j, _p(ju, _i8p), _p(jr, _i8p), _mode(False, tri), _p(a, _i8p),
                                 ctypes.byref(e), ctypes.byref(m))
    return e.value, m.value


def torus_run(spins, J, lam, q, beta, seed, replica, n_full, s0=0, log=True, rev=False, tri=False):
    """Returns (final spins, E_J log, M log); logs have n_full+1 entries.  J is
    an int or a pair (Jup, Jright) of [L, L] int8 arrays."""
    a = np.ascontiguousarray(spins, dtype=np.int8).copy()
    L = a.shape[0]
    ej = np.zeros(n_full + 1, dtype=np.int64) if log else None
    m = np.zeros(n_full + 1, dtype=np.int64) if log else None
    j, ju, jr = _couplings(J, L)
    rc = lib().oracle_torus_run_j(L, j, _p(ju, _i8p), _p(jr, _i8p), _mode(rev, tri), float(lam), float(q),
                                  float(beta), ctypes.c_uint64(seed), replica, s0, _p(a, _i8p),
                                  n_full, _p(ej, _i64p), _p(m, _i64p))
    if rc != 0:
        raise RuntimeError("oracle_torus_run failed")
    return a, ej, m


# -------------------------------------------------------------------- graph --

class Graph:
    """Oriented graph: edges (src[e], dst[e]) form E^o; J per edge (int8);
    lambda given as a class per vertex and a value per class."""

    def __init__(self, n, src, dst, J=None, cls=None, lam_values=(0.0,)):
        self.n = int(n)
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.J = None if J is None else np.ascontiguousarray(J, dtype=np.int8)
        self.cls = None if cls is None else np.ascontiguousarray(cls, dtype=np.uint8)
        self.lam = np.ascontiguousarray(lam_values, dtype=np.float64)

    @property
    def m(self):
        return int(self.src.shape[0])

    def lam_of_vertex(self):
        c = np.zeros(self.n, dtype=np.int64) if self.cls is None else self.cls.astype(np.int64)
        return self.lam[c]


def graph_init_random(n, seed, replica=0) -> np.ndarray:
    sp = np.zeros(n, dtype=np.int8)
    lib().oracle_graph_init_random(n, ctypes.c_uint64(seed), replica, _p(sp, _i8p))
    return sp


def graph_uniform(seed, replica, s, v) -> int:
    return int(lib().oracle_graph_uniform(ctypes.c_uint64(seed), replica, s & 0xFFFFFFFF, v))


def graph_half_step(g: Graph, spins, q, beta, seed, replica, s) -> np.ndarray:
    a = np.ascontiguousarray(spins, dtype=np.int8)
    out = np.zeros_like(a)
    rc = lib().oracle_graph_half_step(g.n, g.m, _p(g.src, _i32p), _p(g.dst, _i32p),
                                      _p(g.J, _i8p), _p(g.cls, _u8p), _p(g.lam, _f64p),
                                      float(q), float(beta), ctypes.c_uint64(seed), replica,
                                      s & 0xFFFFFFFF, _p(a, _i8p), _p(out, _i8p))
    if rc != 0:
        raise RuntimeError("oracle_graph_half_step failed")
    return out


def graph_observe(g: Graph, spins):
    a = np.ascontiguousarray(spins, dtype=np.int8)
    e = ctypes.c_int64()
    nc = len(g.lam)
    plus = np.zeros(nc, dtype=np.int64)
    lib().oracle_graph_observe(g.n, g.m, _p(g.src, _i32p), _p(g.dst, _i32p), _p(g.J, _i8p),
                               _p(g.cls, _u8p), nc, _p(a, _i8p), ctypes.byref(e),
                               _p(plus, _i64p))
    return e.value, plus


def graph_run(g: Graph, spins, q, beta, seed, replica, n_full, s0=0, log=True):
    """Returns (final spins, E_J log [n_full+1], plus-count log [n_full+1, classes])."""
    a = np.ascontiguousarray(spins, dtype=np.int8).copy()
    nc = len(g.lam)
    ej = np.zeros(n_full + 1, dtype=np.int64) if log else None
    pl = np.zeros((n_full + 1, nc), dtype=np.int64) if log else None
    rc = lib().oracle_graph_run(g.n, g.m, _p(g.src, _i32p), _p(g.dst, _i32p), _p(g.J, _i8p),
                                _p(g.cls, _u8p), nc, _p(g.lam, _f64p), float(q), float(beta),
                                ctypes.c_uint64(seed), replica, s0, _p(a, _i8p), n_full,
                                _p(ej, _i64p), _p(pl, _i64p))
    if rc != 0:
        raise RuntimeError("oracle_graph_run failed")
    return a, ej, pl


def energy(EJ, lam2_dot_sigma):
    """H(sigma) = -E_J - sum_x 2 lambda_x sigma_x (equation ham1)."""
    return -EJ - lam2_dot_sigma


# ------------------------------------------------------------- frozen set B --
# Section 3.1: the state space X_{Lambda,B} keeps the spins of a set B at +1.
# The dynamics restricted to it redraws every other spin from its field (the
# frozen +1 spins enter the fields like any other) and leaves B at +1; the
# uniforms stay keyed by site and half-step, so a half-step on X_{Lambda,B} is
# the plain half-step followed by sigma_B := +1.

def torus_run_frozen(spins, frozen, J, lam, q, beta, seed, replica, n_full, s0=0, rev=False):
    """frozen: bool [L, L].  Returns (final spins, E_J log, M log)."""
    a = np.ascontiguousarray(spins, dtype=np.int8).copy()
    fz = np.asarray(frozen, dtype=bool)
    a[fz] = 1
    ej = np.zeros(n_full + 1, dtype=np.int64)
    m = np.zeros(n_full + 1, dtype=np.int64)
    s = s0
    for t in range(n_full + 1):
        ej[t], m[t] = torus_observe(a, J)
        if t == n_full:
            break
        for k in range(2):
            a = torus_half_step(a, J, lam, q, beta, seed, replica, s + k, rev=rev)
            a[fz] = 1
        s += 2
    return a, ej, m


def graph_run_frozen(g: Graph, spins, frozen, q, beta, seed, replica, n_full, s0=0):
    """frozen: bool [n].  Returns (final spins, E_J log, plus-count log)."""
    a = np.ascontiguousarray(spins, dtype=np.int8).copy()
    fz = np.asarray(frozen, dtype=bool)
    a[fz] = 1
    ej = np.zeros(n_full + 1, dtype=np.int64)
    pl = np.zeros((n_full + 1, len(g.lam)), dtype=np.int64)
    s = s0
    for t in range(n_full + 1):
        ej[t], pl[t] = graph_observe(g, a)
        if t == n_full:
            break
        for k in range(2):
            a = graph_half_step(g, a, q, beta, seed, replica, s + k)
            a[fz] = 1
        s += 2
    return a, ej, pl
