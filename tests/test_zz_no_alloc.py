"""shaken_sweep_noalloc, the sweep for callers that cannot allocate memory,
against shaken_sweep on twin contexts: the same logs (H, M of every full
step, bit-exact) and the same final configurations, over calls in a row that
share the device's fixed log buffer -- the second smaller than the first, so
that it runs over what the first left in the buffer."""
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


def _twins(sk, case):
    if case == "torus64":
        mk = lambda: sk.Chain.torus(64, q=1.0, beta=0.4, seed=1)
    elif case == "torus37_int8":
        mk = lambda: sk.Chain.torus(37, q=0.7, beta=0.9, seed=5, replica=3, fmt="int8", J=2,
                                    lam_values=[-0.5])
    else:  # 1001-vertex 3-regular +-J graph with three field classes
        inst = synth.oriented_instance(1002, 3, 41, lam_values=(-0.5, 0.0, 0.5), pm_j=True)
        mk = lambda: sk.Chain.graph(inst.n, inst.src, inst.dst, J=inst.J, lam_values=inst.lam_values,
                                    lam_class=inst.cls, q=1.5, beta=0.8, seed=9, replica=1)
    return mk(), mk()


def _noalloc_logs(ch, steps):
    import torch
    H = torch.full((steps + 1,), -7, dtype=torch.int64, device="cuda")
    M = torch.full((steps + 1,), -7, dtype=torch.int64, device="cuda")
    ch.sweep_noalloc(steps, H, M)
    torch.cuda.synchronize()
    return H.cpu().numpy(), M.cpu().numpy()


def test_noalloc_matches_sweep_over_calls(sk):
    """Calls in a row on the one fixed buffer: a 64^2 bit-packed torus for 300
    full steps, then a 1002-vertex graph for 100, then a 37^2 int8 torus
    (J = 2, lambda = -1/2) for 40 and, on the same context, 25 more; each equal
    to shaken_sweep on a twin context."""
    for case, calls in (("torus64", (300,)), ("graph1002", (100,)), ("torus37_int8", (40, 25))):
        a, b = _twins(sk, case)
        for steps in calls:
            print("case: noalloc", case, steps, flush=True)
            Ha, Ma = _noalloc_logs(a, steps)
            Hb, Mb = b.sweep(steps, log=True)
            assert np.array_equal(Ha, Hb), case
            assert np.array_equal(Ma, Mb), case
            assert np.array_equal(a.spins(), b.spins()), case
            assert a.half_step_index == b.half_step_index
        a.close()
        b.close()


def test_noalloc_without_logs_and_limits(sk):
    """No logs: the buffer is not needed and any length runs; with logs a call
    beyond the buffer is refused on the host with the bound in the message,
    and an odd counter is refused."""
    import torch
    a, b = _twins(sk, "torus64")
    a.sweep_noalloc(5000)
    b.sweep(5000)
    assert np.array_equal(a.spins(), b.spins())
    H = torch.empty(4097, dtype=torch.int64, device="cuda")
    with pytest.raises(sk.ShakenError) as ei:
        a.sweep_noalloc(4096, H)
    assert ei.value.status == sk.SHAKEN_EINVAL and "at most 4095" in str(ei.value)
    a.half_step(1)
    with pytest.raises(sk.ShakenError) as ei:
        a.sweep_noalloc(1)
    assert ei.value.status == sk.SHAKEN_ESTATE
    a.close()
    b.close()
