"""The seeded synthetic inputs are the ones the workloads were measured and
checked on.

synth draws from numpy's PCG64 Generator; numpy does not promise that a
Generator method keeps its bit stream across versions, so an upgrade could
silently change every seeded workload (graphs, orientations, couplings,
per-chain beta, q and seeds).  These digests make such a change fail here
instead.  They were written by hashing synth's own output (no oracle or
library arithmetic involved): the n = 2^20 graph workload, the whole
2048-chain batch spec, a sample of the annealing evaluation instances and the
24 torus runs.
"""
import hashlib

import numpy as np

import synth


def _digest(arrays):
    m = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        m.update(str(a.dtype).encode())
        m.update(str(a.shape).encode())
        m.update(a.tobytes())
    return m.hexdigest()[:32]


def test_graph_2e20_workload_digest():
    inst = synth.oriented_instance(1 << 20, 3, 3, lam_values=(-0.5, 0.0, 0.5), pm_j=True)
    assert inst.src.shape == (3 * (1 << 19),)
    assert _digest([inst.src, inst.dst, inst.J, inst.cls, inst.lam_values]) == "2f762fb50f2d379700f4c661f8e7e0ec"


def test_batch_2048_spec_digest():
    spec = synth.batch_spec(1024, 1024, seed=4)
    meta = np.array([(0 if it.kind == "torus" else 1, it.size, it.seed) for it in spec], dtype=np.int64)
    bq = np.array([(it.beta, it.q) for it in spec])
    m = hashlib.sha256()
    m.update(meta.tobytes())
    m.update(bq.tobytes())
    for it in spec:
        if it.graph is not None:
            m.update(it.graph.src.tobytes())
            m.update(it.graph.dst.tobytes())
            m.update(it.graph.J.tobytes())
    assert m.hexdigest()[:32] == "a48db8ac068819d4c0e6d9fed128eb51"
    assert sum(it.size ** 2 if it.kind == "torus" else it.size for it in spec) == 59_199_358


def test_annealing_instances_digest():
    """Three evaluation instances of each size class (seeds 9e6 + 100 k + j)."""
    m = hashlib.sha256()
    for k, n in enumerate((4096, 16384, 65536)):
        for j in range(3):
            inst = synth.oriented_instance(n, 3, 9_000_000 + 100 * k + j, lam_values=(0.0,), pm_j=True)
            m.update(inst.src.tobytes())
            m.update(inst.dst.tobytes())
            m.update(inst.J.tobytes())
    assert m.hexdigest()[:32] == "d08ce667561dd97ec994e2ec3f07a0f6"


def test_torus_runs():
    runs = synth.torus_runs()
    assert len(runs) == 24
    assert {(r["q"], r["beta"], r["init"]) for r in runs} == {
        (q, b, i) for q in (0.5, 1.0, 2.0) for b in (0.30, 0.40, 0.44, 0.50) for i in ("all_up", "random")}
    # the list order is the chains' replica index
    assert [(r["q"], r["beta"], r["init"]) for r in runs][:3] == [
        (0.5, 0.30, "all_up"), (0.5, 0.30, "random"), (0.5, 0.40, "all_up")]
    assert all(r["seed"] == 2 for r in runs)
