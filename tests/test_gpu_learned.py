"""Learned initial assignments: HIP kernels vs the CPU FP64 oracle."""
import numpy as np
import pytest

from oracle import learned as M
from paper_2311_02101_amd import workload as wl
from tests.parity import say

pytestmark = pytest.mark.gpu


def _bits_to_float(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def _sync():
    import torch
    torch.cuda.synchronize()


def _plan(tables, ns, chains=4, seed=3):
    from paper_2311_02101_amd import hp
    K = tables[0].shape[0]
    L = wl.hidden_units_for(K)
    W, b = wl.gaussian_rbm(2, K, L, seed)
    return hp.Plan(tables, ns, W, b, chains=chains, precision="f32", seed=seed)


def _net(seed):
    from paper_2311_02101_amd import learned as Lr
    return Lr.MLP(seed=seed)


def _oracle_params(net):
    p = net.host_params()
    W1 = p[:M.F_IN * M.HIDDEN].reshape(M.F_IN, M.HIDDEN)
    b1 = p[M.F_IN * M.HIDDEN:M.F_IN * M.HIDDEN + M.HIDDEN]
    w2 = p[M.F_IN * M.HIDDEN + M.HIDDEN:M.F_IN * M.HIDDEN + 2 * M.HIDDEN]
    return W1, b1, w2, p[-1]


def test_features_match_oracle(hip):
    from paper_2311_02101_amd import learned as Lr
    for K, sizes in [(7, [100, 2048, 37]), (3, [9, 50])]:
        tables = [wl.random_formula(n, 5, k=K, lengths=[1, 2, 3] if K == 3 else wl.LENGTHS,
                                    probs=[0.2, 0.5, 0.3] if K == 3 else wl.LENGTH_PROBS, tag=f)
                  for f, n in enumerate(sizes)]
        say(f"[features] K={K} sizes={sizes}")
        plan = _plan(tables, sizes)
        x = _bits_to_float(Lr.features(plan))
        want = np.concatenate([M.bf16_round(M.features(t, n)) for t, n in zip(tables, sizes)])
        assert np.array_equal(x, want)
        plan.free()


@pytest.mark.parametrize("rows", [1, 33, 1000, 4096])
def test_forward_matches_oracle(hip, rows):
    import torch
    net = _net(11)
    rng = np.random.default_rng(rows)
    xf = M.bf16_round(rng.standard_normal((rows, M.F_IN)))
    bits = torch.tensor((xf.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16),
                        device="cuda")
    say(f"[mlp forward] rows={rows}")
    q = net.forward(bits)
    _sync()
    want, _ = M.forward(xf, *_oracle_params(net))
    assert np.max(np.abs(q.cpu().numpy() - want)) < 2e-6


def _rows(rows, seed):
    import torch
    rng = np.random.default_rng(seed)
    xf = M.bf16_round(rng.standard_normal((rows, M.F_IN)))
    y = rng.uniform(0, 1, rows)
    bits = torch.tensor((xf.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16),
                        device="cuda")
    return xf, y, bits, torch.tensor(y.astype(np.float32), device="cuda")


# 3000 rows: 24 workgroups of one tile per wave; 300 000 rows: all 1024
# workspace rows, each of the 4096 waves summing 2 or 3 tiles
@pytest.mark.parametrize("rows", [3000, 300000])
def test_backward_and_adam_match_oracle(hip, rows):
    net = _net(12)
    xf, y, bits, yt = _rows(rows, 7)
    say(f"[mlp backward] rows={rows}")
    loss = net.backward(bits, yt)
    _sync()
    W1, b1, w2, b2 = _oracle_params(net)
    g = M.gradients(xf, y.astype(np.float32).astype(np.float64), W1, b1, w2, b2)
    got = net.grad.cpu().numpy().astype(np.float64)
    parts = dict(W1=got[:M.F_IN * M.HIDDEN].reshape(M.F_IN, M.HIDDEN),
                 b1=got[M.F_IN * M.HIDDEN:M.F_IN * M.HIDDEN + M.HIDDEN],
                 w2=got[M.F_IN * M.HIDDEN + M.HIDDEN:-1], b2=got[-1:])
    errs = {k: np.max(np.abs(parts[k] - g[k])) / max(np.max(np.abs(g[k])), 1e-30) for k in parts}
    say("  grad rel err " + " ".join(f"{k}={e:.2e}" for k, e in errs.items()))
    assert all(e < 1e-4 for e in errs.values()), errs
    want_loss = M.loss(xf, y.astype(np.float32).astype(np.float64), W1, b1, w2, b2) * rows
    assert abs(float(loss.item()) - want_loss) < 1e-5 * abs(want_loss)
    # one Adam step from zero moments, FP32 on the device vs FP64 here
    p0 = net.host_params()
    gp = net.grad.cpu().numpy().astype(np.float64)
    net.adam(lr=1e-3)
    _sync()
    p1, _, _ = M.adam(p0, gp, np.zeros_like(p0), np.zeros_like(p0), 1, lr=1e-3)
    assert np.max(np.abs(net.host_params() - p1)) < 1e-6 * max(1.0, np.max(np.abs(p1)))
    # the bfloat16 copies follow the updated parameters
    wb = _bits_to_float(net.w_bf16)
    W1n = net.host_params()[:M.F_IN * M.HIDDEN].reshape(M.F_IN, M.HIDDEN)
    assert np.array_equal(wb[:M.F_IN * M.HIDDEN].reshape(M.HIDDEN, M.F_IN), M.bf16_round(W1n).T)


def test_backward_is_deterministic(hip):
    """The gradient and the loss are sums in a fixed order (per workgroup,
    then over the workgroups' rows): the same input gives the same bits, also
    after a larger call has filled more of the workspace."""
    net = _net(13)
    _, _, bits, yt = _rows(5000, 8)
    _, _, big_bits, big_yt = _rows(200000, 9)
    say("[mlp backward] determinism, rows=5000 / 200000 / 5000")
    first = (net.backward(bits, yt).clone(), net.grad.clone())
    net.backward(big_bits, big_yt)
    again = (net.backward(bits, yt).clone(), net.grad.clone())
    _sync()
    assert np.array_equal(first[0].cpu().numpy(), again[0].cpu().numpy())
    assert np.array_equal(first[1].cpu().numpy(), again[1].cpu().numpy())


def test_init_chains_and_chain_mean_match_oracle(hip):
    import torch
    from paper_2311_02101_amd import learned as Lr
    sizes = [300, 77]
    tables = [wl.random_formula(n, 6, tag=f) for f, n in enumerate(sizes)]
    plan = _plan(tables, sizes, chains=8, seed=6)
    v0 = [wl.initial_state(8, n, 6, tag=f) for f, n in enumerate(sizes)]
    st = plan.new_state(v0)
    rng = np.random.default_rng(0)
    q = torch.tensor(rng.uniform(0, 1, sum(sizes)).astype(np.float32), device="cuda")
    say("[init chains] chains 2..5 of 8")
    Lr.init_chains(plan, q, st, 2, 5)
    mean = Lr.chain_mean(plan, st.v)
    _sync()
    qh = q.cpu().numpy().astype(np.float64)
    off = np.concatenate([[0], np.cumsum(sizes)])
    for f, n in enumerate(sizes):
        v = st.formula(f)[0]
        want = M.init_assignment(qh[off[f]:off[f + 1]], 6, f, np.arange(2, 5))   # plan seed 6
        assert np.array_equal(v[2:5], want)
        assert np.array_equal(v[:2], v0[f][:2]) and np.array_equal(v[5:], v0[f][5:])
        assert np.array_equal(mean.cpu().numpy()[off[f]:off[f + 1]], v.mean(axis=0).astype(np.float32))


def test_learned_initializer_trains_and_is_judged_by_the_count(hip):
    """End to end on a small scale: labels from the sampler, training on the
    device, held-out comparison against uniform starts."""
    from paper_2311_02101_amd import learned as Lr
    say("[learned] dataset 48 formulas N=512")
    x, y = Lr.make_dataset(48, n_vars=512, seed=21, chains=16, sweeps=150, batch=48)
    assert x.shape == (48 * 512, M.F_IN) and float(y.min()) >= 0.0 and float(y.max()) <= 1.0
    net = Lr.MLP(seed=21)
    losses = Lr.train(net, x, y, epochs=30, batch_rows=4096, lr=3e-3)
    say(f"[learned] losses {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < losses[0]
    ev = Lr.evaluate(net, 16, n_vars=512, seed=21, chains=32, sweeps=(10, 50))
    say(f"[learned] evaluation {ev}")
    for s, r in ev.items():
        # paired per formula: the plain method is the fallback wherever the
        # uniform half is better
        assert r["wins"] + r["losses"] <= 16 and r["fallback_used"] == r["losses"]


def test_trained_network_gains_over_uniform_starts(hip):
    """The committed network (trained on 1e5 method-labelled formulas of
    N = 2048) on 32 held-out formulas it never saw: its predictions beat the
    best constant predictor on fresh labels, and the chains it starts beat
    the uniform starts of the same formulas (paired, same temperatures) at
    20 and 100 sweeps."""
    import torch
    from paper_2311_02101_amd import learned as Lr
    net, _ = Lr.MLP.load()
    first = 2 * 10 ** 6                   # held out: training used 0 .. 1e5, the stored evaluation 1e6 ..
    say("[learned gain] labels of 16 held-out formulas N=2048 (32 chains x 500 sweeps)")
    x, y = Lr.make_dataset(16, n_vars=2048, seed=4, chains=32, sweeps=500, batch=16, first=first)
    q = net.forward(x).double()
    yd = y.double()
    eps = 1e-7

    def bce(p):
        p = p.clamp(eps, 1 - eps)
        return float(-(yd * torch.log(p) + (1 - yd) * torch.log(1 - p)).mean())
    loss_net, loss_const = bce(q), bce(torch.full_like(yd, float(yd.mean())))
    say(f"[learned gain] held-out loss {loss_net:.5f} vs constant predictor {loss_const:.5f}")
    assert loss_net < loss_const - 0.005
    say("[learned gain] 32 held-out formulas, 64 chains (32 MLP-started, 32 uniform)")
    ev = Lr.evaluate(net, 32, n_vars=2048, seed=4, chains=64, sweeps=(20, 100), first=first + 1000)
    for s, r in ev.items():
        say(f"[learned gain] {s} sweeps: MLP half {r['mlp']:.1f}, uniform half {r['uniform']:.1f}, "
            f"gain {r['gain']:+.1f} clauses of {r['clauses']}, wins {r['wins']} / losses {r['losses']}")
    # margins: a third of the gain measured on 256 formulas (+124 at 20 sweeps),
    # and a clear majority of paired wins
    assert ev[20]["gain"] >= 40 and ev[20]["wins"] >= 28
    assert ev[100]["gain"] > 0 and ev[100]["wins"] > ev[100]["losses"]


def test_learned_form_speedup_at_equal_accuracy(hip):
    """The committed network's learned form (FP32; half the chains started
    from Bernoulli(q), 20 sweeps) against the plain method from uniform
    starts, in FP64 and in FP32, on 32 held-out formulas of N = 2048: the
    plain runs need more sweeps, and more time, to reach the same mean best
    count."""
    from paper_2311_02101_amd import learned as Lr
    net, _ = Lr.MLP.load()
    say("[learned speed-up] 32 held-out formulas, 64 chains, learned form 20 sweeps")
    r = Lr.equal_accuracy(net, 32, n_vars=2048, seed=4, chains=64, budget=20, step=5, max_sweeps=400,
                          first=2 * 10 ** 6 + 1000)
    say(f"[learned speed-up] learned form: accuracy {r['learned']['accuracy']:.1f} "
        f"in {r['learned']['seconds'] * 1e3:.2f} ms")
    for prec in ("f64", "f32"):
        p = r["plain_" + prec]
        say(f"[learned speed-up] plain {prec}: {p['sweeps_to_equal_accuracy']} sweeps "
            f"({p.get('seconds', float('nan')) * 1e3:.2f} ms), speed-up {p.get('speedup_of_learned_form')}, "
            f"per-formula median {p['per_formula_sweeps_median']} sweeps "
            f"({p['per_formula_reached']}/32 reached)")
        # measured: 45 sweeps and a speed-up of 1.99 (FP64) / 1.85 (FP32);
        # the bars are 1.5x the learned form's sweeps and a 1.4x speed-up
        assert p["sweeps_to_equal_accuracy"] is not None and p["sweeps_to_equal_accuracy"] >= 30
        assert p["accuracy"] >= r["learned"]["accuracy"]
        assert p["speedup_of_learned_form"] > 1.4
