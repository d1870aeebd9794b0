"""Checkpoint / resume.  A run is a pure function of (inputs, seed, replica,
half-step counter s), so the state (spins, s) restored into a fresh context --
in the middle of a full step too -- continues the uninterrupted trajectory bit
for bit, on every path (bit-packed and int8 torus, +-J torus, graph)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1904_06257_amd as m
    return m


def _cases(sk):
    rng = np.random.Generator(np.random.PCG64(3))
    J = tuple(np.where(rng.integers(0, 2, (70, 70)) == 1, 1, -1).astype(np.int8) for _ in range(2))
    inst = synth.oriented_instance(3000, 3, 17, lam_values=(-0.5, 0.5), pm_j=True)
    return [
        ("torus bitpacked", lambda **kw: sk.Chain.torus(97, q=0.8, beta=0.5, lam_values=[0.1], **kw)),
        ("torus int8", lambda **kw: sk.Chain.torus(40, q=0.8, beta=0.5, fmt="int8", **kw)),
        ("torus +-J", lambda **kw: sk.Chain.torus(70, J=J, q=2.5, beta=1.2, **kw)),
        ("graph", lambda **kw: sk.Chain.graph(inst.n, inst.src, inst.dst, J=inst.J,
                                              lam_values=inst.lam_values, lam_class=inst.cls,
                                              q=1.5, beta=0.8, **kw)),
    ]


@pytest.mark.parametrize("idx", range(4))
@pytest.mark.parametrize("cut", [40, 41])   # after a full step, and in the middle of one
def test_resume_reproduces_the_uninterrupted_run(sk, idx, cut):
    name, make = _cases(sk)[idx]
    print("case: checkpoint", name, cut, flush=True)
    total = 100
    ref = make(seed=5, replica=4)
    ref.half_step(total)
    want = ref.spins()
    first = make(seed=5, replica=4)
    first.half_step(cut)
    spins, s = first.spins(), first.half_step_index
    assert s == cut
    first.close()
    resumed = make(seed=5, replica=4, init_spins=spins)
    resumed.set_half_step(s)
    resumed.half_step(total - cut)
    assert np.array_equal(resumed.spins(), want)
    # a wrong counter gives a different trajectory (the state really is (spins, s))
    other = make(seed=5, replica=4, init_spins=spins)
    other.set_half_step(s + 2)
    other.half_step(total - cut)
    assert not np.array_equal(other.spins(), want)
    for c in (ref, resumed, other):
        c.close()


@pytest.mark.parametrize("strategy", ["grid", "persistent"])
def test_batch_follows_members_restored_to_an_odd_counter(sk, strategy):
    """Batch members restored to an odd counter (shaken_set_half_step swaps a
    context's two spin buffers when the parity changes): the batch refuses to
    sweep from the odd counter, and after each member has run one half-step
    of its own the batch continues from the swapped buffers -- equal to the
    oracle's half-step at s = 7 and full steps from s = 8."""
    import oracle
    inst = synth.oriented_instance(1000, 3, 23, lam_values=(-0.5, 0.5), pm_j=True)
    og = oracle.Graph(inst.n, inst.src, inst.dst, inst.J, inst.cls, inst.lam_values)
    tor = sk.Chain.torus(40, q=0.8, beta=0.5, seed=5, replica=1)
    gr = sk.Chain.graph(inst.n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                        lam_class=inst.cls, q=1.5, beta=0.8, seed=6, replica=2)
    b = sk.Batch([tor, gr], strategy=strategy)
    b.sweep(3)
    for c in (tor, gr):
        c.set_half_step(7)
    with pytest.raises(sk.ShakenError) as ei:
        b.sweep(1)
    assert ei.value.status == sk.SHAKEN_ESTATE
    for c in (tor, gr):
        c.half_step(1)
    uploads = b.counters()["uploads"]
    b.sweep(2)
    assert b.counters()["uploads"] == uploads + 1
    t6, _, _ = oracle.torus_run(oracle.torus_init_random(40, 5, 1), 1, 0.0, 0.8, 0.5, 5, 1, 3)
    t8 = oracle.torus_half_step(t6, 1, 0.0, 0.8, 0.5, 5, 1, 7)
    t12, _, _ = oracle.torus_run(t8, 1, 0.0, 0.8, 0.5, 5, 1, 2, s0=8)
    g6, _, _ = oracle.graph_run(og, oracle.graph_init_random(inst.n, 6, 2), 1.5, 0.8, 6, 2, 3)
    g8 = oracle.graph_half_step(og, g6, 1.5, 0.8, 6, 2, 7)
    g12, _, _ = oracle.graph_run(og, g8, 1.5, 0.8, 6, 2, 2, s0=8)
    assert np.array_equal(tor.spins(), t12)
    assert np.array_equal(gr.spins(), g12)
    b.close()
    tor.close()
    gr.close()
