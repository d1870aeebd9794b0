"""The C-ABI library loads, exports every symbol include/shaken.h declares,
and rejects invalid arguments before touching a device.  CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "shaken.h")).read()
    return sorted(set(re.findall(r"^\s*(?:shaken_status|const char \*|int32_t)\s*\*?\s*(shaken_\w+)\s*\(",
                                 txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    import paper_1904_06257_amd as sk
    lib = ctypes.CDLL(sk.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sk.EXPORTED)


def test_version_and_strings():
    import paper_1904_06257_amd as sk
    assert sk.shaken_version() == (0 << 16) | 1
    assert sk._lib.shaken_strerror(1) == b"invalid argument"


def _init_status(**kw):
    import paper_1904_06257_amd as sk
    try:
        sk.Chain(**kw)
    except sk.ShakenError as e:
        return e.status, str(e)
    return 0, ""


@pytest.mark.parametrize("kw,frag", [
    (dict(kind="torus", L=2), "L must be"),
    (dict(kind="torus", L=8, q=-1.0), "q must be"),
    (dict(kind="torus", L=8, beta=float("nan")), "beta must be"),
    (dict(kind="torus", L=8, lam_values=[0.1, 0.2]), "uniform"),
    (dict(kind="torus", L=4, J=np.r_[np.ones(31), 2 * np.ones(1)]), "same magnitude"),
    (dict(kind="graph", n=4, src=[0, 1], dst=[1, 1]), "self-loop"),
    (dict(kind="graph", n=4, src=[0, 1], dst=[1, 0]), "twice"),
    (dict(kind="graph", n=4, src=[0, 5], dst=[1, 2]), "out of range"),
    (dict(kind="graph", n=0, src=[], dst=[]), "n must be"),
    (dict(kind="graph", n=3, src=[0], dst=[1], lam_values=[0.0], lam_class=[0, 1, 0]), "class id"),
    (dict(kind="torus", L=3, init_spins=np.zeros(9)), "+1 or -1"),
])
def test_invalid_arguments_rejected_on_host(kw, frag):
    import paper_1904_06257_amd as sk
    st, msg = _init_status(**kw)
    assert st == sk.SHAKEN_EINVAL, msg
    assert frag in msg


def test_valid_arguments_reach_the_device_check():
    """With no GPU here a valid call fails only at the device step."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1904_06257_amd as sk
    st, msg = _init_status(kind="torus", L=8)
    assert st == sk.SHAKEN_EDEVICE


def test_ell_layout_rejected_when_it_does_not_apply():
    import paper_1904_06257_amd as sk
    st, msg = _init_status(kind="graph", n=4, src=[0, 1], dst=[1, 2], J=[2, 1], layout="ell")
    assert st == sk.SHAKEN_EINVAL and "ELL" in msg
    src = [0, 0, 0, 0, 0]
    dst = [1, 2, 3, 4, 5]
    st, msg = _init_status(kind="graph", n=6, src=src, dst=dst, layout="ell")
    assert st == sk.SHAKEN_EINVAL and "ELL" in msg


def test_packed_layout_rejected_when_it_does_not_apply():
    """The packed per-vertex record needs degree <= 3, n <= 65536 and at most
    16 field classes; AUTO falls back silently, PACKED reports why."""
    import torch
    import paper_1904_06257_amd as sk
    star4 = dict(kind="graph", n=5, src=[0, 0, 0, 0], dst=[1, 2, 3, 4])      # degree 4
    st, msg = _init_status(layout="packed", **star4)
    assert st == sk.SHAKEN_EINVAL and "packed" in msg
    big = dict(kind="graph", n=70000, src=[0, 1], dst=[1, 2])                # n > 65536
    st, msg = _init_status(layout="packed", **big)
    assert st == sk.SHAKEN_EINVAL and "packed" in msg
    cls = dict(kind="graph", n=20, src=[0, 1], dst=[1, 2], lam_values=np.zeros(17),
               lam_class=np.arange(20) % 17)                                  # 17 classes
    st, msg = _init_status(layout="packed", **cls)
    assert st == sk.SHAKEN_EINVAL and "packed" in msg
    st, msg = _init_status(layout="packed", kind="graph", n=4, src=[0, 1], dst=[1, 2], J=[2, 1])
    assert st == sk.SHAKEN_EINVAL
    if not torch.cuda.is_available():
        for kw in (star4, big, cls):
            assert _init_status(layout="auto", **kw)[0] == sk.SHAKEN_EDEVICE
        st, _ = _init_status(layout="packed", kind="graph", n=4, src=[0, 1], dst=[1, 2])
        assert st == sk.SHAKEN_EDEVICE


def test_pm_j_torus_passes_host_validation():
    """Couplings of one magnitude with mixed signs (+-J) are accepted for both
    torus formats; without a GPU the call then fails only at the device step."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1904_06257_amd as sk
    rng = np.random.Generator(np.random.PCG64(1))
    ju = np.where(rng.integers(0, 2, (5, 5)) == 1, 2, -2).astype(np.int8)
    jr = np.where(rng.integers(0, 2, (5, 5)) == 1, 2, -2).astype(np.int8)
    for fmt in ("bitpacked", "int8"):
        st, msg = _init_status(kind="torus", L=5, J=(ju, jr), fmt=fmt)
        assert st == sk.SHAKEN_EDEVICE, msg


def test_split_edges_need_the_flag():
    """Both orientations of a pair are the generalised split of section 5:
    rejected by default (Definition 2.1), accepted with split=True; the same
    oriented edge twice is rejected either way."""
    import torch
    import paper_1904_06257_amd as sk
    anti = dict(kind="graph", n=3, src=[0, 1, 1], dst=[1, 0, 2], J=[1, 1, -1])
    st, msg = _init_status(**anti)
    assert st == sk.SHAKEN_EINVAL and "both orientations" in msg
    st, msg = _init_status(split=True, kind="graph", n=3, src=[0, 0], dst=[1, 1])
    assert st == sk.SHAKEN_EINVAL and "oriented edge" in msg
    st, msg = _init_status(split=True, kind="torus", L=4)
    assert st == sk.SHAKEN_EINVAL and "graphs only" in msg
    if not torch.cuda.is_available():
        assert _init_status(reversed=True, kind="torus", L=4)[0] == sk.SHAKEN_EDEVICE
        assert _init_status(reversed=True, split=True, **anti)[0] == sk.SHAKEN_EDEVICE
    if not torch.cuda.is_available():
        assert _init_status(split=True, **anti)[0] == sk.SHAKEN_EDEVICE


def test_graph_bitpacked_passes_host_validation():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1904_06257_amd as sk
    st, msg = _init_status(kind="graph", n=70, src=[0, 5, 69], dst=[1, 6, 0], fmt="bitpacked")
    assert st == sk.SHAKEN_EDEVICE, msg


def test_scalar_and_wrong_length_couplings_in_the_binding():
    """A scalar J is one coupling for every oriented edge (2 L^2 on the torus,
    3 L^2 on the triangular lattice, m on a graph); an array of another length
    is refused before the library reads it."""
    import torch
    import paper_1904_06257_amd as sk
    for kind, kw, n_edges in (("torus", dict(L=5), 50), ("triangular", dict(L=5), 75),
                              ("graph", dict(n=4, src=[0, 1, 2], dst=[1, 2, 3]), 3)):
        with pytest.raises(ValueError):
            sk.Chain(kind, J=np.ones(n_edges - 1, np.int8), **kw)
        if not torch.cuda.is_available():
            st, msg = _init_status(kind=kind, J=2, **kw)
            assert st == sk.SHAKEN_EDEVICE, msg
            st, msg = _init_status(kind=kind, J=np.full(n_edges, -1, np.int8), **kw)
            assert st == sk.SHAKEN_EDEVICE, msg


def test_per_site_arrays_of_wrong_length_refused_in_the_binding():
    """lam_class and init_spins are read for every site by the library: the
    binding refuses other lengths before the call"""
    import paper_1904_06257_amd as sk
    with pytest.raises(ValueError):
        sk.Chain("torus", L=4, lam_values=[0.0, 0.5], lam_class=np.zeros(15, np.uint8))
    with pytest.raises(ValueError):
        sk.Chain("graph", n=5, src=[0, 1], dst=[1, 2], init_spins=np.ones(4, np.int8))
    with pytest.raises(ValueError):
        sk.Chain("torus", L=4, init_spins=np.ones((4, 3), np.int8))


def test_edge_and_output_arrays_checked_in_the_binding():
    import paper_1904_06257_amd as sk
    with pytest.raises(ValueError):
        sk.Chain("graph", n=4, src=[0, 1, 2], dst=[1, 2])
    with pytest.raises(ValueError):
        sk.shaken_sweep(None, 10, H_out=np.zeros(10, np.int64))
    with pytest.raises(ValueError):
        sk.shaken_sweep(None, 10, M_out=np.zeros(11, np.int32))
    with pytest.raises(ValueError):
        sk.batch_run([], 1)
    with pytest.raises(KeyError):
        sk.batch_run([None], 1, schedule="cosine")
