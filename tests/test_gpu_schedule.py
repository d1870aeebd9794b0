"""GPU tests of the annealing pieces: the schedule network's BF16/FP32 MFMA
kernels against the float64 oracle at the same rounding points, Adam, the
persistent batch's best-energy tracking and per-chain parameter updates, and
replay parity of a whole annealing run against the CPU oracle."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

# Tolerances (relative norm).  Products of BF16 values are exact in FP32, so
# the device and the float64 oracle differ by FP32 accumulation (<= 2^-24 *
# sqrt(K) relative, K <= 2048 here) and, rarely, by a BF16 rounding that this
# difference tips across a rounding boundary (probability ~ 2^-16 sqrt(K) per
# stored value, 2^-8 relative each): well below 1e-3.
TOL_Y = 1e-3
TOL_G = 2e-3


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1904_06257_amd as sk
    return sk, torch


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("rows", [1, 16, 100, 2048])
def test_mlp_forward_backward_parity(env, rows):
    sk, torch = env
    print("case: mlp rows", rows, flush=True)
    rng = np.random.Generator(np.random.PCG64(rows))
    P = omlp.init_params(7).astype(np.float32)
    P[omlp.OFF_B1:omlp.OFF_W2] = rng.normal(0, 0.1, 128).astype(np.float32)
    P[omlp.OFF_B4:omlp.OFF_B4 + 2] = [0.3, -0.2]
    X = rng.normal(size=(rows, 16)).astype(np.float32)
    T = rng.normal(size=(rows, 16)).astype(np.float32)
    w = rng.uniform(0.2, 2.0, rows).astype(np.float32)
    m = sk.MLP()
    m.set_params(P)
    assert np.array_equal(m.params(), P)
    x = torch.from_numpy(X).cuda()
    y = torch.empty((rows, 16), dtype=torch.float32, device="cuda")
    m.forward(x, y)
    yg = y.cpu().numpy().astype(np.float64)
    yr, cache = omlp.forward(P.astype(np.float64), X.astype(np.float64), rounding=True)
    assert _rel(yg[:, :2], yr[:, :2]) < TOL_Y
    loss = m.loss_backward(torch.from_numpy(T).cuda(), torch.from_numpy(w).cuda())
    lr_, dy = omlp.mse_grad(yr, T.astype(np.float64), w.astype(np.float64))
    assert abs(loss - lr_) <= 2e-3 * abs(lr_)
    g = m.grads().astype(np.float64)
    gr = omlp.backward(cache, dy)
    for a, b in [(omlp.OFF_W1, omlp.OFF_B1), (omlp.OFF_B1, omlp.OFF_W2), (omlp.OFF_W2, omlp.OFF_B2),
                 (omlp.OFF_W3, omlp.OFF_B3), (omlp.OFF_W4, omlp.OFF_B4), (omlp.OFF_B4, omlp.NPARAM)]:
        assert _rel(g[a:b], gr[a:b]) < TOL_G, (a, b, _rel(g[a:b], gr[a:b]))
    # an arbitrary output gradient through the same kernels
    DY = np.zeros((rows, 16), dtype=np.float32)
    DY[:, :2] = rng.normal(size=(rows, 2))
    m.backward(torch.from_numpy(DY).cuda())
    assert _rel(m.grads().astype(np.float64), omlp.backward(cache, DY.astype(np.float64))) < TOL_G
    m.close()


def test_mlp_adam_step(env):
    sk, torch = env
    rng = np.random.Generator(np.random.PCG64(3))
    P = omlp.init_params(9).astype(np.float32)
    X = rng.normal(size=(64, 16)).astype(np.float32)
    T = rng.normal(size=(64, 16)).astype(np.float32)
    m = sk.MLP()
    m.set_params(P)
    x = torch.from_numpy(X).cuda()
    y = torch.empty((64, 16), dtype=torch.float32, device="cuda")
    m.forward(x, y)
    m.loss_backward(torch.from_numpy(T).cuda())
    g = m.grads().astype(np.float64)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    m.adam(lr, 1, b1, b2, eps)
    mm = (1 - b1) * g
    vv = (1 - b2) * g * g
    want = P.astype(np.float64) - lr * (mm / (1 - b1)) / (np.sqrt(vv / (1 - b2)) + eps)
    got = m.params().astype(np.float64)
    assert np.max(np.abs(got - want)) < 1e-6
    # the unused output rows stay zero
    assert np.all(got[omlp.OFF_W4 + 2 * 128:omlp.OFF_B4] == 0)
    m.close()


def _graphs(k, n, seed):
    return [synth.oriented_instance(n, 3, seed + i, lam_values=(0.0,), pm_j=True) for i in range(k)]


def test_tracking_and_set_params(env):
    """Persistent batch with tracking: H of the last configuration, the lowest
    H over the full-step configurations of the call and that configuration,
    across a parameter change, against the oracle's trajectories."""
    sk, torch = env
    insts = _graphs(5, 1000, 40)
    seeds = [11, 12, 13, 14, 15]
    chains = [sk.Chain.graph(g.n, g.src, g.dst, J=g.J, q=1.0, beta=0.3, seed=s, replica=i)
              for i, (g, s) in enumerate(zip(insts, seeds))]
    b = sk.Batch(chains, strategy="persistent", track=True)
    betas = np.array([0.3, 0.5, 0.8, 1.2, 2.0])
    qs = np.array([0.5, 1.0, 1.5, 2.5, 3.5])
    b.set_params(betas, qs)
    T = 25
    b.sweep(T)
    hl, hb, sp = b.track(best_spins=True)
    b.set_params(betas * 2, qs / 2)
    b.sweep(T)
    hl2, hb2, sp2 = b.track(best_spins=True)
    off = 0
    for i, g in enumerate(insts):
        og = oracle.Graph(g.n, g.src, g.dst, g.J, g.cls, g.lam_values)
        x0 = oracle.graph_init_random(g.n, seeds[i], i)
        x1, ej1, _ = oracle.graph_run(og, x0, qs[i], betas[i], seeds[i], i, T)
        x2, ej2, _ = oracle.graph_run(og, x1, qs[i] / 2, betas[i] * 2, seeds[i], i, T, s0=2 * T)
        assert hl[i] == -ej1[-1] and hb[i] == (-ej1).min()
        assert hl2[i] == -ej2[-1] and hb2[i] == (-ej2).min()
        assert np.array_equal(chains[i].spins(), x2)
        e_best = oracle.graph_observe(og, sp[off:off + g.n])[0]
        assert -e_best == hb[i]
        assert -oracle.graph_observe(og, sp2[off:off + g.n])[0] == hb2[i]
        off += g.n


def test_anneal_replay_parity(env):
    """A whole annealing run under a schedule: the oracle replays the logged
    (beta_c, q_c) chunk by chunk from the same start and reaches the same final
    configuration; final and best energies re-verified from the returned
    configurations."""
    sk, torch = env
    from paper_1904_06257_amd import anneal
    insts = _graphs(6, 512, 70) + _graphs(2, 2048, 90)
    seeds = np.arange(100, 108)
    pol = anneal.PerturbedPolicy(anneal.GeometricPolicy(0.2, 3.0, 1.5), len(insts), 6, seed=5)
    res = anneal.run(insts, seeds, pol, sweeps=60, chunk=10, keep_spins=True)
    for i, g in enumerate(insts):
        og = oracle.Graph(g.n, g.src, g.dst, g.J, g.cls, g.lam_values)
        x = oracle.graph_init_random(g.n, int(seeds[i]), i)
        best = -oracle.graph_observe(og, x)[0]
        s0 = 0
        for c in range(6):
            x, ej, _ = oracle.graph_run(og, x, float(np.exp(res.log_q[c, i])),
                                        float(np.exp(res.log_beta[c, i])), int(seeds[i]), i, 10, s0=s0)
            best = min(best, (-ej).min())
            s0 += 20
        assert np.array_equal(res.final_spins[i], x)
        assert res.last[i] == -oracle.graph_observe(og, x)[0]
        assert res.best[i] == best
        assert -oracle.graph_observe(og, res.best_spins[i])[0] == best


def test_learned_schedule_beats_plain(env):
    """The committed network against the tuned geometric schedule on the 512
    held-out evaluation instances (171 / 171 / 170 graphs of n = 4096 / 16384 /
    65536; same Philox seeds for both schedules), 10^4 sweeps: every reported
    best and final energy is recomputed by the oracle from the returned
    configurations, and the learned schedule reaches lower best energies."""
    sk, torch = env
    import os
    from paper_1904_06257_amd import anneal, schedule
    P, meta = schedule.load(os.path.join(os.path.dirname(sk.__file__), "schedule_weights.npz"))
    g = meta["geometric"]
    mlp = sk.MLP()
    mlp.set_params(P)
    insts, seeds = schedule.instances(schedule.EVAL_SEED0, (171, 171, 170))
    print("case: 512 held-out instances", flush=True)
    rl = anneal.run(insts, seeds, anneal.MLPPolicy(mlp), 10000, 250, keep_spins=True)
    rp = anneal.run(insts, seeds, anneal.GeometricPolicy(g["beta0"], g["beta1"], g["q"]), 10000, 250,
                    keep_spins=True)
    ns = np.array([x.n for x in insts], dtype=np.float64)
    for res in (rl, rp):
        for i, x in enumerate(insts):
            og = oracle.Graph(x.n, x.src, x.dst, x.J, x.cls, x.lam_values)
            assert -oracle.graph_observe(og, res.best_spins[i])[0] == res.best[i]
            assert -oracle.graph_observe(og, res.final_spins[i])[0] == res.last[i]
            assert res.best[i] <= res.last[i]
    d = (rp.best - rl.best) / ns
    print("learned vs plain: mean best %.5f vs %.5f per spin, gain %.5f, learned better on %d of %d"
          % ((rl.best / ns).mean(), (rp.best / ns).mean(), d.mean(), (d > 0).sum(), len(d)), flush=True)
    assert d.mean() > 0.008
    assert (d > 0).mean() > 0.95
