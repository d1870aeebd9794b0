"""Python binding of libshaken: shaken dynamics (arXiv:1904.06257) on MI355X.

Argument marshalling only.  Every half-step, observable and batch runs in the
HIP kernels of ``libshaken.so`` behind the C ABI declared in
``include/shaken.h``; this module converts numpy arrays and torch streams to
the plain pointers and sizes of that ABI.  There is no Python or CPU fallback:
importing the package fails if the library has not been built.

The functions keep the C names (``shaken_init``, ``shaken_half_step``,
``shaken_sweep``, ``shaken_observables``, ``shaken_batch_run`` ...).  The
classes ``Chain`` and ``Batch`` wrap a context / batch handle with the same
calls as methods.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch first: its HIP runtime (same soname as ROCm's) is then the one the
# library binds to, so the process holds a single HIP runtime whichever of the
# two the caller imports first
import torch  # noqa: E402,F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshaken.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libshaken.so is not built (run __graft_entry__.build() or "
                      "python paper_1904_06257_amd/build.py); there is no fallback")

_lib = ctypes.CDLL(LIB_PATH)

SHAKEN_OK, SHAKEN_EINVAL, SHAKEN_ENOMEM, SHAKEN_EDEVICE, SHAKEN_ESTATE = range(5)
SHAKEN_TORUS, SHAKEN_EDGES, SHAKEN_TRIANGULAR = 0, 1, 2
SHAKEN_FMT_AUTO, SHAKEN_FMT_INT8, SHAKEN_FMT_BITPACKED = 0, 1, 2
SHAKEN_INIT_RANDOM, SHAKEN_INIT_ALL_UP, SHAKEN_INIT_ALL_DOWN, SHAKEN_INIT_USER = 0, 1, 2, 3
SHAKEN_BATCH_AUTO, SHAKEN_BATCH_GRID, SHAKEN_BATCH_PERSISTENT = 0, 1, 2

_INIT = {"random": SHAKEN_INIT_RANDOM, "all_up": SHAKEN_INIT_ALL_UP,
         "all_down": SHAKEN_INIT_ALL_DOWN, "user": SHAKEN_INIT_USER}
_FMT = {"auto": SHAKEN_FMT_AUTO, "int8": SHAKEN_FMT_INT8, "bitpacked": SHAKEN_FMT_BITPACKED}
_STRAT = {"auto": SHAKEN_BATCH_AUTO, "grid": SHAKEN_BATCH_GRID,
          "persistent": SHAKEN_BATCH_PERSISTENT}
SHAKEN_LAYOUT_AUTO, SHAKEN_LAYOUT_CSR, SHAKEN_LAYOUT_ELL, SHAKEN_LAYOUT_PACKED = 0, 1, 2, 3
SHAKEN_GRAPH_SPLIT, SHAKEN_ORDER_REVERSED, SHAKEN_GRAPH_LDS, SHAKEN_GRAPH_NO_LDS = 1, 2, 4, 8
_GKERNEL = {"auto": 0, "lds": SHAKEN_GRAPH_LDS, "plain": SHAKEN_GRAPH_NO_LDS}
_LAYOUT = {"auto": SHAKEN_LAYOUT_AUTO, "csr": SHAKEN_LAYOUT_CSR, "ell": SHAKEN_LAYOUT_ELL,
           "packed": SHAKEN_LAYOUT_PACKED}


class shaken_graph(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("L", ctypes.c_int32), ("n", ctypes.c_int32),
                ("m", ctypes.c_int64), ("src", ctypes.POINTER(ctypes.c_int32)),
                ("dst", ctypes.POINTER(ctypes.c_int32))]


class shaken_field(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("value", ctypes.POINTER(ctypes.c_double)),
                ("class_of_vertex", ctypes.POINTER(ctypes.c_uint8))]


class shaken_opts(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int32), ("init", ctypes.c_int32),
                ("init_spins", ctypes.POINTER(ctypes.c_int8)), ("replica", ctypes.c_uint32),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("graph_layout", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("frozen", ctypes.POINTER(ctypes.c_uint8))]


class shaken_obs(ctypes.Structure):
    _fields_ = [("half_step", ctypes.c_int64), ("n_sites", ctypes.c_int64),
                ("M", ctypes.c_int64), ("E_J", ctypes.c_int64), ("E_lambda2", ctypes.c_int64),
                ("H", ctypes.c_double), ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class shaken_batch_opts(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int32), ("use_hipgraph", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("record", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("track", ctypes.c_int32),
                ("log_reserve", ctypes.c_int32)]


class shaken_batch_counts(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("captures", ctypes.c_int64),
                ("log_allocs", ctypes.c_int64), ("autotunes", ctypes.c_int64),
                ("uploads", ctypes.c_int64)]


_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)
_i8p = ctypes.POINTER(ctypes.c_int8)
_f64p = ctypes.POINTER(ctypes.c_double)

SHAKEN_SCHEDULE_NONE, SHAKEN_SCHEDULE_GEOMETRIC, SHAKEN_SCHEDULE_MLP = 0, 1, 2
_SCHED = {"none": SHAKEN_SCHEDULE_NONE, "geometric": SHAKEN_SCHEDULE_GEOMETRIC, "mlp": SHAKEN_SCHEDULE_MLP}


class shaken_schedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("chunk_sweeps", ctypes.c_int32), ("beta0", ctypes.c_double),
                ("beta1", ctypes.c_double), ("q", ctypes.c_double), ("mlp", ctypes.c_void_p)]


class shaken_run_result(ctypes.Structure):
    _fields_ = [("H_final", _i64p), ("H_best", _i64p), ("best_spins", _i8p), ("beta_used", _f64p),
                ("q_used", _f64p), ("chunks", ctypes.c_int64), ("fallbacks", ctypes.c_int64)]

_SIGS = {
    "shaken_init": [ctypes.POINTER(_vp), ctypes.POINTER(shaken_graph), _i8p,
                    ctypes.POINTER(shaken_field), ctypes.c_double, ctypes.c_double,
                    ctypes.c_uint64, ctypes.POINTER(shaken_opts)],
    "shaken_free": [_vp],
    "shaken_half_step": [_vp, ctypes.c_int64],
    "shaken_sweep": [_vp, ctypes.c_int64, _i64p, _i64p],
    "shaken_sweep_noalloc": [_vp, ctypes.c_int64, _vp, _vp],
    "shaken_observables": [_vp, ctypes.POINTER(shaken_obs)],
    "shaken_set_params": [_vp, ctypes.c_double, ctypes.c_double],
    "shaken_get_spins": [_vp, _i8p],
    "shaken_set_spins": [_vp, _i8p],
    "shaken_set_half_step": [_vp, ctypes.c_int64],
    "shaken_get_lut": [_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_size_t),
                       ctypes.POINTER(ctypes.c_int32)],
    "shaken_spins_device": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int32)],
    "shaken_synchronize": [_vp],
    "shaken_batch_create": [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int32,
                            ctypes.POINTER(shaken_batch_opts)],
    "shaken_batch_sweep": [_vp, ctypes.c_int64],
    "shaken_batch_get_log": [_vp, ctypes.c_int32, _i64p, _i64p, ctypes.c_int64],
    "shaken_batch_get_log_ej": [_vp, ctypes.c_int32, _i64p, _i64p, ctypes.c_int64],
    "shaken_batch_get_logs": [_vp, _i64p, _i64p, _i64p, ctypes.c_int64],
    "shaken_batch_info": [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
    "shaken_batch_counters": [_vp, ctypes.POINTER(shaken_batch_counts)],
    "shaken_batch_launch_shape": [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "shaken_batch_free": [_vp],
    "shaken_batch_run": [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.c_int64,
                         ctypes.POINTER(shaken_batch_opts), ctypes.POINTER(shaken_schedule),
                         ctypes.POINTER(shaken_run_result)],
    "shaken_batch_set_params": [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "shaken_batch_get_track": [_vp, _i64p, _i64p, _i8p],
    "shaken_mlp_create": [ctypes.POINTER(_vp), ctypes.c_int32, _vp],
    "shaken_mlp_free": [_vp],
    "shaken_mlp_set_params": [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t],
    "shaken_mlp_get_params": [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t],
    "shaken_mlp_forward": [_vp, _vp, ctypes.c_int32, _vp],
    "shaken_mlp_loss_backward": [_vp, _vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)],
    "shaken_mlp_backward": [_vp, _vp, ctypes.c_int32],
    "shaken_mlp_get_grads": [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t],
    "shaken_mlp_adam": [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                        ctypes.c_int32],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.shaken_strerror.argtypes = [ctypes.c_int]
_lib.shaken_strerror.restype = ctypes.c_char_p
_lib.shaken_last_error.argtypes = []
_lib.shaken_last_error.restype = ctypes.c_char_p
_lib.shaken_version.argtypes = []
_lib.shaken_version.restype = ctypes.c_int32

EXPORTED = sorted(list(_SIGS) + ["shaken_strerror", "shaken_last_error", "shaken_version"])


class ShakenError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_lib.shaken_strerror(status).decode(), msg))
        self.status = status


def _check(st):
    if st != SHAKEN_OK:
        raise ShakenError(st, _lib.shaken_last_error().decode())


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(t))


def _stream_handle(stream):
    """torch stream, raw handle (int) or None -> void*"""
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


# ------------------------------------------------------------- raw functions

def shaken_version():
    return int(_lib.shaken_version())


def shaken_init(graph, J, lam, q, beta, seed, opts):
    """Returns a context handle (c_void_p).  graph, lam, opts are the ctypes
    structs above (lam may be None); J a contiguous int8 array or None."""
    h = _vp()
    _check(_lib.shaken_init(ctypes.byref(h), ctypes.byref(graph), _ptr(J, ctypes.c_int8),
                            None if lam is None else ctypes.byref(lam), float(q), float(beta),
                            ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ctypes.byref(opts)))
    return h


def shaken_free(ctx):
    _check(_lib.shaken_free(ctx))


def shaken_half_step(ctx, n):
    _check(_lib.shaken_half_step(ctx, int(n)))


def shaken_sweep(ctx, n_full, H_out=None, M_out=None):
    for a in (H_out, M_out):
        if a is not None and (a.dtype != np.int64 or not a.flags.c_contiguous or a.size < int(n_full) + 1):
            raise ValueError("log outputs must be contiguous int64 arrays of n_full + 1 entries")
    _check(_lib.shaken_sweep(ctx, int(n_full), _ptr(H_out, ctypes.c_int64), _ptr(M_out, ctypes.c_int64)))


def shaken_observables(ctx):
    o = shaken_obs()
    _check(_lib.shaken_observables(ctx, ctypes.byref(o)))
    return o


def shaken_batch_run(ctxs, n_full, opts=None, sched=None, res=None):
    """raw call: ctxs are context handles, opts / sched / res ctypes structs
    or None (res arrays are filled in place)"""
    arr = (_vp * len(ctxs))(*[c.value for c in ctxs])
    _check(_lib.shaken_batch_run(arr, len(ctxs), int(n_full), None if opts is None else ctypes.byref(opts),
                                 None if sched is None else ctypes.byref(sched),
                                 None if res is None else ctypes.byref(res)))


# ------------------------------------------------------------------ classes

class Chain:
    """One shaken-dynamics chain (a libshaken context)."""

    def __init__(self, kind, *, L=0, n=0, src=None, dst=None, J=None, lam_values=None,
                 lam_class=None, q=1.0, beta=1.0, seed=0, replica=0, init="random",
                 init_spins=None, fmt="auto", device=-1, stream=None, layout="auto", split=False,
                 reversed=False, frozen=None, graph_kernel="auto"):
        g = shaken_graph()
        self._keep = []
        if kind in ("torus", "triangular"):
            g.kind, g.L = (SHAKEN_TORUS if kind == "torus" else SHAKEN_TRIANGULAR), int(L)
            self.shape = (int(L), int(L))
            self.n = int(L) * int(L)
        elif kind == "graph":
            src = np.ascontiguousarray(src, dtype=np.int32).reshape(-1)
            dst = np.ascontiguousarray(dst, dtype=np.int32).reshape(-1)
            if src.shape != dst.shape:
                raise ValueError("src and dst must have the same length")
            self._keep += [src, dst]
            g.kind, g.n, g.m = SHAKEN_EDGES, int(n), int(src.shape[0])
            g.src, g.dst = _ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32)
            self.shape = (int(n),)
            self.n = int(n)
        else:
            raise ValueError("kind must be 'torus', 'triangular' or 'graph'")
        if kind == "torus" and isinstance(J, tuple):
            # (Jup, Jright), each [L, L]: interleave into the per-edge order
            # of the C ABI (2x = (x, x_up), 2x+1 = (x, x_right))
            ju = np.asarray(J[0], dtype=np.int8).reshape(-1)
            jr = np.asarray(J[1], dtype=np.int8).reshape(-1)
            J = np.stack([ju, jr], axis=1).reshape(-1)
        # one coupling per oriented edge: 2 L^2 (torus), 3 L^2 (triangular), m (graph)
        n_edges = {"torus": 2 * self.n, "triangular": 3 * self.n}.get(kind, g.m)
        if J is not None and np.ndim(J) == 0:
            J = np.full(n_edges, int(J), dtype=np.int8)
        Jarr = None if J is None else np.ascontiguousarray(J, dtype=np.int8).reshape(-1)
        if Jarr is not None and Jarr.shape[0] != n_edges:
            raise ValueError("J needs one coupling per oriented edge (%d), got %d" % (n_edges, Jarr.shape[0]))
        field = None
        if lam_values is not None:
            lv = np.ascontiguousarray(np.atleast_1d(lam_values), dtype=np.float64)
            lc = None if lam_class is None else np.ascontiguousarray(lam_class, dtype=np.uint8).reshape(-1)
            if lc is not None and lc.shape[0] != self.n:
                raise ValueError("lam_class needs one class per site (%d), got %d" % (self.n, lc.shape[0]))
            self._keep += [lv, lc]
            field = shaken_field(len(lv), _ptr(lv, ctypes.c_double), _ptr(lc, ctypes.c_uint8))
            self.lam_values = lv
            self.lam_class = lc
        else:
            self.lam_values = np.zeros(1)
            self.lam_class = None
        o = shaken_opts()
        o.format = _FMT[fmt]
        o.init = _INIT[init]
        sp = None
        if init_spins is not None:
            sp = np.ascontiguousarray(init_spins, dtype=np.int8).reshape(-1)
            if sp.shape[0] != self.n:
                raise ValueError("init_spins needs one spin per site (%d), got %d" % (self.n, sp.shape[0]))
            o.init = SHAKEN_INIT_USER
            o.init_spins = _ptr(sp, ctypes.c_int8)
        o.replica = int(replica)
        o.device = int(device)
        o.stream = _stream_handle(stream)
        o.graph_layout = _LAYOUT[layout]
        o.flags = (SHAKEN_GRAPH_SPLIT if split else 0) | (SHAKEN_ORDER_REVERSED if reversed else 0) | \
            _GKERNEL[graph_kernel]
        fz = None
        if frozen is not None:
            fz = np.ascontiguousarray(np.asarray(frozen).reshape(-1) != 0, dtype=np.uint8)
            if fz.shape[0] != self.n:
                raise ValueError("frozen needs one entry per site")
            o.frozen = _ptr(fz, ctypes.c_uint8)
        self.kind = kind
        self.handle = shaken_init(g, Jarr, field, q, beta, seed, o)
        self._keep = None

    @classmethod
    def torus(cls, L, **kw):
        return cls("torus", L=L, **kw)

    @classmethod
    def triangular(cls, L, **kw):
        """L x L triangular-lattice torus (section 4), skewed coordinates"""
        return cls("triangular", L=L, **kw)

    @classmethod
    def graph(cls, n, src, dst, **kw):
        return cls("graph", n=n, src=src, dst=dst, **kw)

    def close(self):
        if getattr(self, "handle", None) is not None:
            shaken_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def half_step(self, n=1):
        shaken_half_step(self.handle, n)

    def sweep(self, n_full, log=False):
        if not log:
            shaken_sweep(self.handle, n_full)
            return None
        H = np.zeros(n_full + 1, dtype=np.int64)
        M = np.zeros(n_full + 1, dtype=np.int64)
        shaken_sweep(self.handle, n_full, H, M)
        return H, M

    def sweep_noalloc(self, n_full, H=None, M=None):
        """shaken_sweep_noalloc: n_full full steps; H, M are None or int64
        device tensors of n_full + 1 entries that receive the logs (the call
        only enqueues work: synchronise before reading them)"""
        for t in (H, M):
            if t is not None and (not t.is_cuda or not t.is_contiguous() or t.numel() < n_full + 1
                                  or str(t.dtype) != "torch.int64"):
                raise ValueError("logs must be contiguous int64 device tensors of n_full + 1 entries")
        _check(_lib.shaken_sweep_noalloc(self.handle, int(n_full),
                                         None if H is None else ctypes.c_void_p(H.data_ptr()),
                                         None if M is None else ctypes.c_void_p(M.data_ptr())))

    def sweep_m(self, n_full):
        """magnetisation log only (works for any lambda)"""
        M = np.zeros(n_full + 1, dtype=np.int64)
        shaken_sweep(self.handle, n_full, None, M)
        return M

    def observables(self):
        return shaken_observables(self.handle)

    def set_params(self, beta, q):
        _check(_lib.shaken_set_params(self.handle, float(beta), float(q)))

    def spins(self):
        out = np.zeros(self.n, dtype=np.int8)
        _check(_lib.shaken_get_spins(self.handle, _ptr(out, ctypes.c_int8)))
        return out.reshape(self.shape)

    def set_spins(self, sp):
        a = np.ascontiguousarray(sp, dtype=np.int8).reshape(-1)
        if a.shape[0] != self.n:
            raise ValueError("wrong number of spins")
        _check(_lib.shaken_set_spins(self.handle, _ptr(a, ctypes.c_int8)))

    def set_half_step(self, s):
        _check(_lib.shaken_set_half_step(self.handle, int(s)))

    @property
    def half_step_index(self):
        return int(self.observables().half_step)

    def lut(self):
        n = ctypes.c_size_t(0)
        smax = ctypes.c_int32(0)
        _check(_lib.shaken_get_lut(self.handle, None, ctypes.byref(n), ctypes.byref(smax)))
        out = np.zeros(n.value, dtype=np.uint64)
        _check(_lib.shaken_get_lut(self.handle, _ptr(out, ctypes.c_uint64), ctypes.byref(n),
                                   ctypes.byref(smax)))
        return out, int(smax.value)

    def device_spins(self):
        p = _vp()
        f = ctypes.c_int32()
        _check(_lib.shaken_spins_device(self.handle, ctypes.byref(p), ctypes.byref(f)))
        return p.value, int(f.value)

    def synchronize(self):
        _check(_lib.shaken_synchronize(self.handle))


class Batch:
    """A batch of chains advanced by fused launches (libshaken batch)."""

    def __init__(self, chains, strategy="auto", use_hipgraph=False, autotune=False,
                 record=False, stream=None, track=False, log_reserve=0):
        self.chains = list(chains)
        o = shaken_batch_opts(_STRAT[strategy], int(use_hipgraph), _autotune(autotune), int(record),
                              _stream_handle(stream), int(track), int(log_reserve))
        arr = (_vp * len(self.chains))(*[c.handle.value for c in self.chains])
        h = _vp()
        _check(_lib.shaken_batch_create(ctypes.byref(h), arr, len(self.chains), ctypes.byref(o)))
        self.handle = h
        self.record = bool(record)
        self._last = None

    def sweep(self, n_full):
        _check(_lib.shaken_batch_sweep(self.handle, int(n_full)))
        self._last = int(n_full)

    def log(self, i, with_H=True):
        n = self._last + 1
        H = np.zeros(n, dtype=np.int64) if with_H else None
        M = np.zeros(n, dtype=np.int64)
        _check(_lib.shaken_batch_get_log(self.handle, int(i), _ptr(H, ctypes.c_int64),
                                         _ptr(M, ctypes.c_int64), n))
        return H, M

    def logs(self, with_H=False, with_EJ=True):
        """(H, M, E_J) of every chain, each [n_chains, n_full + 1] (None where
        not asked for), read with one device copy"""
        n = self._last + 1
        R = len(self.chains)
        H = np.zeros((R, n), dtype=np.int64) if with_H else None
        M = np.zeros((R, n), dtype=np.int64)
        EJ = np.zeros((R, n), dtype=np.int64) if with_EJ else None
        _check(_lib.shaken_batch_get_logs(self.handle, _ptr(H, ctypes.c_int64), _ptr(M, ctypes.c_int64),
                                          _ptr(EJ, ctypes.c_int64), n))
        return H, M, EJ

    def log_ej(self, i):
        """(E_J, M) logs of chain i: the coupling energy, exact for any lambda"""
        n = self._last + 1
        EJ = np.zeros(n, dtype=np.int64)
        M = np.zeros(n, dtype=np.int64)
        _check(_lib.shaken_batch_get_log_ej(self.handle, int(i), _ptr(EJ, ctypes.c_int64),
                                            _ptr(M, ctypes.c_int64), n))
        return EJ, M

    def set_params(self, beta, q):
        b = np.ascontiguousarray(beta, dtype=np.float64)
        qq = np.ascontiguousarray(q, dtype=np.float64)
        if b.shape[0] != len(self.chains) or qq.shape[0] != len(self.chains):
            raise ValueError("one beta and one q per chain")
        _check(_lib.shaken_batch_set_params(self.handle, _ptr(b, ctypes.c_double),
                                            _ptr(qq, ctypes.c_double)))

    def track(self, best_spins=False):
        """(H_last, H_best[, best configurations concatenated]) of the last sweep"""
        n = len(self.chains)
        hl = np.zeros(n, dtype=np.int64)
        hb = np.zeros(n, dtype=np.int64)
        sp = np.zeros(sum(c.n for c in self.chains), dtype=np.int8) if best_spins else None
        _check(_lib.shaken_batch_get_track(self.handle, _ptr(hl, ctypes.c_int64),
                                           _ptr(hb, ctypes.c_int64), _ptr(sp, ctypes.c_int8)))
        return (hl, hb, sp) if best_spins else (hl, hb)

    def info(self):
        st = ctypes.c_int32()
        ms = ctypes.c_double()
        _check(_lib.shaken_batch_info(self.handle, ctypes.byref(st), ctypes.byref(ms)))
        return int(st.value), float(ms.value)

    def counters(self):
        """host-side work done so far: dict of sweeps, captures, log_allocs,
        autotunes, uploads"""
        c = shaken_batch_counts()
        _check(_lib.shaken_batch_counters(self.handle, ctypes.byref(c)))
        return {k: int(getattr(c, k)) for k, _ in shaken_batch_counts._fields_}

    def launch_shape(self, i):
        """workgroup size of chain i's half-step launches (1024: the graph
        kernel with the configuration in LDS; 0: persistent strategy)"""
        v = ctypes.c_int32()
        _check(_lib.shaken_batch_launch_shape(self.handle, int(i), ctypes.byref(v)))
        return int(v.value)

    def close(self):
        if getattr(self, "handle", None) is not None:
            _check(_lib.shaken_batch_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RunOutput:
    """Results of batch_run: H_final, H_best (int64 per chain), best_spins
    (list of per-chain int8 configurations, or None), beta_used and q_used
    ([chunks, chains] or None), chunks, fallbacks."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def _autotune(a):
    """False / True / "cached" -> 0 / 1 / 2 (opts.autotune)"""
    if a == "cached":
        return 2
    if isinstance(a, str):
        raise ValueError("autotune: False, True or 'cached'")
    return int(bool(a))


def batch_run(chains, n_full, schedule="none", chunk_sweeps=0, beta0=1.0, beta1=1.0, q=1.0, mlp=None,
              strategy="auto", use_hipgraph=False, autotune=False, best_spins=False, energies=True,
              stream=None):
    """shaken_batch_run over `chains`: n_full full steps under a schedule
    ("none", "geometric", "mlp"), the chunk loop run by the library; returns a
    RunOutput (energies need every 2*lambda integer; energies=False asks for
    none of them)."""
    n = len(chains)
    kind = _SCHED[schedule]
    if n < 1:
        raise ValueError("batch_run needs at least one chain")
    o = shaken_batch_opts(_STRAT[strategy], int(use_hipgraph), _autotune(autotune), 0, _stream_handle(stream), 0, 0)
    sc = shaken_schedule(kind, int(chunk_sweeps), float(beta0), float(beta1), float(q),
                         None if mlp is None else mlp.handle)
    chunks = 0 if schedule == "none" or chunk_sweeps < 1 else int(n_full) // int(chunk_sweeps)
    hf = np.zeros(n, dtype=np.int64) if energies else None
    hb = np.zeros(n, dtype=np.int64) if energies else None
    sp = np.zeros(sum(c.n for c in chains), dtype=np.int8) if best_spins else None
    bu = np.zeros((chunks, n), dtype=np.float64) if chunks else None
    qu = np.zeros((chunks, n), dtype=np.float64) if chunks else None
    r = shaken_run_result(_ptr(hf, ctypes.c_int64), _ptr(hb, ctypes.c_int64), _ptr(sp, ctypes.c_int8),
                          _ptr(bu, ctypes.c_double), _ptr(qu, ctypes.c_double), 0, 0)
    shaken_batch_run([c.handle for c in chains], n_full, o, sc, r)
    spins = None
    if best_spins:
        off = np.cumsum([0] + [c.n for c in chains])
        spins = [sp[off[i]:off[i + 1]].reshape(chains[i].shape).copy() for i in range(n)]
    return RunOutput(H_final=hf, H_best=hb, best_spins=spins, beta_used=bu, q_used=qu,
                     chunks=int(r.chunks), fallbacks=int(r.fallbacks))


# ---------------------------------------------------------- schedule network

MLP_IN, MLP_HIDDEN, MLP_OUT = 16, 128, 16
MLP_NPARAM = 128 * 16 + 128 + 2 * (128 * 128 + 128) + 16 * 128 + 16


def _dptr(t):
    """device pointer of a torch tensor (contiguous float32 on the GPU)"""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


class MLP:
    """The annealing-schedule network (libshaken's BF16/FP32 MFMA kernels)."""

    def __init__(self, device=-1, stream=None):
        h = _vp()
        _check(_lib.shaken_mlp_create(ctypes.byref(h), int(device), _stream_handle(stream)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None:
            _check(_lib.shaken_mlp_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        _check(_lib.shaken_mlp_set_params(self.handle, _ptr(a, ctypes.c_float), a.shape[0]))

    def params(self):
        a = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(_lib.shaken_mlp_get_params(self.handle, _ptr(a, ctypes.c_float), MLP_NPARAM))
        return a

    def grads(self):
        a = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(_lib.shaken_mlp_get_grads(self.handle, _ptr(a, ctypes.c_float), MLP_NPARAM))
        return a

    def forward(self, x, y):
        """x, y: torch float32 device tensors [batch, 16]"""
        _check(_lib.shaken_mlp_forward(self.handle, _dptr(x), x.shape[0], _dptr(y)))

    def loss_backward(self, target, w=None):
        loss = ctypes.c_float()
        _check(_lib.shaken_mlp_loss_backward(self.handle, _dptr(target),
                                             None if w is None else _dptr(w), target.shape[0],
                                             ctypes.byref(loss)))
        return float(loss.value)

    def backward(self, dy):
        _check(_lib.shaken_mlp_backward(self.handle, _dptr(dy), dy.shape[0]))

    def adam(self, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(_lib.shaken_mlp_adam(self.handle, float(lr), float(beta1), float(beta2),
                                    float(eps), int(t)))
