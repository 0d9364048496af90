"""The size-clustered formula-RBM (Sec. 4) on the GPU against its oracle:
whole trajectories (teacher-forced replay on a mismatch, every difference a
flagged tie), a batch of uneven formulas, sampled chains of the 4096-variable
workload in the split launch, split vs single launch, the reduction to the
padded model when every clause has 7 literals, and replica exchange with the
clustered free energy.

Every case prints its name, sizes and seed before touching the GPU.
"""
import numpy as np
import pytest

from oracle import clustered as CL
from oracle import rbmsat as R
from oracle import tempering as PT
from paper_2311_02101_amd import hp, workload as wl
from tests.parity import NU_RTOL, TIE, say

pytestmark = pytest.mark.gpu


def _sync():
    import torch
    torch.cuda.synchronize()


def _teacher_forced(plan, st, f, ost, cp, temps, *, alpha, seed, prec, chain_ids):
    """One sweep from the oracle's state on both sides; differences in v must
    be flagged ties.  Returns the tie count; ``ost`` advances."""
    st.set_formula(f, v=ost.v, nu=ost.nu, s_max=ost.s_max, best=ost.best)
    st.set_t(ost.t)
    plan.run(st, 1)
    gv, gnu, gs, gb = st.formula(f)
    rec = CL.sweep(ost, cp, temps, alpha=alpha, seed=seed, formula_id=f, chain_ids=chain_ids)
    assert rec["hid_margin"] > TIE["f64"], "hidden-unit tie: comparison not decidable"
    assert np.array_equal(gs, ost.s_max) and np.array_equal(gb, ost.best)
    diff = gv != ost.v
    if diff.any():
        margin = np.abs(rec["u_v"] - rec["rho"])[diff]
        assert margin.max() <= TIE[prec], f"non-tie visible mismatch, margin {margin.max():.3e}"
    rel = np.abs(gnu - ost.nu) / np.maximum(np.abs(ost.nu), 1e-300)
    assert rel.max() <= NU_RTOL[prec], f"nu rel err {rel.max():.3e}"
    return int(diff.sum())


def _trajectory(tables, ns, rbms, B, S, prec, seed, label, alpha=1e-3):
    W7, b7 = rbms[max(tables[0].shape[0], 3)]     # the padded-model RBM the plan also takes
    temps = wl.default_temperatures(B, W7.shape[0])
    say(f"[{label}] clustered plan F={len(tables)} N={list(ns)} B={B} S={S} prec={prec} seed={seed}")
    plan = hp.Plan(tables, ns, W7, b7, chains=B, temps=temps, precision=prec, alpha=alpha, seed=seed,
                   size_rbms=rbms)
    v0s = [wl.initial_state(B, n, seed, tag=f) for f, n in enumerate(ns)]
    st = plan.new_state(v0s)
    plan.run(st, S)
    _sync()
    assert st.get_t() == S
    for f in range(len(tables)):
        cp = CL.ClusteredPlan(tables[f], ns[f], rbms)
        ost = CL.run(R.initial(v0s[f]), cp, temps, S, alpha=alpha, seed=seed, formula_id=f)
        gv, gnu, gs, gb = st.formula(f)
        rel = np.abs(gnu - ost.nu) / np.maximum(np.abs(ost.nu), 1e-300)
        if (np.array_equal(gv, ost.v) and np.array_equal(gs, ost.s_max) and np.array_equal(gb, ost.best)
                and rel.max() <= NU_RTOL[prec]):
            continue
        say(f"[{label}] f={f}: trajectory differs; replaying with teacher forcing")
        sub = hp.Plan([tables[f]], [ns[f]], W7, b7, chains=B, temps=temps, precision=prec, alpha=alpha,
                      seed=seed, size_rbms=rbms)
        sst = sub.new_state([v0s[f]])
        o2 = R.initial(v0s[f])
        ties = sum(_teacher_forced(sub, sst, 0, o2, cp, temps, alpha=alpha, seed=seed, prec=prec,
                                   chain_ids=np.arange(B)) for _ in range(S))
        sub.free()
        say(f"[{label}] f={f}: {ties} flagged ties over {S} sweeps")
        assert ties > 0, "trajectory mismatch without any tie"
    plan.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_trajectory_n256(hip, prec):
    n = 256
    T = wl.random_formula(n, 11)
    _trajectory([T], [n], wl.pretrained_size_rbms(), 4, 40, prec, 11, f"clust n256 {prec}")


def test_uneven_batch(hip):
    ns = [9, 130, 700, 2100]
    tables = [wl.random_formula(n, 12, tag=f) for f, n in enumerate(ns)]
    _trajectory(tables, ns, wl.pretrained_size_rbms(), 6, 12, "f64", 12, "clust uneven")


def test_gaussian_rbms_and_short_clauses(hip):
    """Random weights (every table entry distinct) and a length mix with many
    clauses of 1 and 2 literals (merged padding slots of the K = 3 group)."""
    n = 300
    T = wl.random_formula(n, 13, lengths=[1, 2, 3, 5, 7], probs=[0.2, 0.3, 0.2, 0.15, 0.15])
    rng = np.random.default_rng(13)
    rbms = {K: (0.7 * rng.standard_normal((2, K, CL.hidden_units(K))),
                0.7 * rng.standard_normal((2, CL.hidden_units(K)))) for K in range(3, 8)}
    _trajectory([T], [n], rbms, 4, 30, "f64", 13, "clust gaussian")


def test_narrow_table_needs_only_the_small_groups(hip):
    """A K = 4 table (clauses of 1..4 literals): the plan takes the K = 3 and
    K = 4 RBMs only; FP64 trajectory against the oracle."""
    n = 200
    T = wl.random_formula(n, 16, k=4, lengths=[1, 2, 3, 4], probs=[0.1, 0.4, 0.3, 0.2])
    assert T.shape[0] == 4
    full = wl.pretrained_size_rbms()
    rbms = {3: full[3], 4: full[4]}
    _trajectory([T], [n], rbms, 4, 30, "f64", 16, "clust k4")


def test_all_seven_literal_clauses_equal_the_padded_model(hip):
    n = 500
    T = wl.random_formula(n, 14, lengths=[7], probs=[1.0])
    # the unused groups scaled down so both plans pick the same fixed-point
    # scale (it follows the largest sum of |W| over the groups)
    rbms = {K: ((0.1 * W, b) if K < 7 else (W, b)) for K, (W, b) in wl.pretrained_size_rbms().items()}
    W, b = rbms[7]
    B = 8
    temps = wl.default_temperatures(B, 2)
    v0 = wl.initial_state(B, n, 14)
    say(f"[clust=padded] N={n} B={B} S=60")
    out = []
    for size_rbms in (rbms, None):
        plan = hp.Plan([T], [n], W, b, chains=B, temps=temps, seed=14, size_rbms=size_rbms)
        st = plan.new_state([v0])
        plan.run(st, 60)
        _sync()
        out.append(st.formula(0))
        plan.free()
    for a, c in zip(*out):
        assert np.array_equal(a, c)


def test_full_size_split_sampled_chains_and_single_launch(hip):
    """The 4096-variable, 64-chain workload in its split launch: two sampled
    chains against the oracle (teacher-forced), then the split state against
    the single-workgroup launch (bit-identical: integer accumulation)."""
    w = wl.config_workload("plain_n4096_b64")
    rbms = wl.pretrained_size_rbms()
    n, T, v0, B = w.n_vars[0], w.tables[0], w.v0[0], w.chains
    say(f"[clust full] N={n} B={B} seed={w.seed}")
    plan = hp.Plan([T], [n], w.W, w.b, chains=B, temps=w.temps, alpha=w.alpha, seed=w.seed, size_rbms=rbms)
    assert plan.split > 1
    st = plan.new_state([v0])
    plan.run(st, 5)
    _sync()
    cp = CL.ClusteredPlan(T, n, rbms)
    chains = np.array([3, 60])
    ost = R.initial(v0[chains])
    gv, gnu, gs, gb = st.formula(0)
    ost.v, ost.nu, ost.s_max, ost.best, ost.t = gv[chains], gnu[chains], gs[chains], gb[chains], 5
    # teacher-forced sweeps of the sampled chains: the device runs all chains
    for _ in range(3):
        gv, gnu, gs, gb = st.formula(0)
        gv[chains], gnu[chains], gs[chains], gb[chains] = ost.v, ost.nu, ost.s_max, ost.best
        st.set_formula(0, v=gv, nu=gnu, s_max=gs, best=gb)
        st.set_t(ost.t)
        plan.run(st, 1)
        g2 = st.formula(0)
        rec = CL.sweep(ost, cp, w.temps[chains], alpha=w.alpha, seed=w.seed, chain_ids=chains)
        assert rec["hid_margin"] > TIE["f64"]
        assert np.array_equal(g2[2][chains], ost.s_max) and np.array_equal(g2[3][chains], ost.best)
        diff = g2[0][chains] != ost.v
        if diff.any():
            assert np.abs(rec["u_v"] - rec["rho"])[diff].max() <= TIE["f64"]
        rel = np.abs(g2[1][chains] - ost.nu) / np.abs(ost.nu)
        assert rel.max() <= NU_RTOL["f64"]
    # split vs one workgroup per chain, from the same state
    snap = st.formula(0)
    single = hp.Plan([T], [n], w.W, w.b, chains=B, temps=w.temps, alpha=w.alpha, seed=w.seed, split=1,
                     size_rbms=rbms)
    s1 = single.new_state([v0])
    s1.set_formula(0, v=snap[0], nu=snap[1], s_max=snap[2], best=snap[3])
    s1.set_t(st.get_t())
    plan.run(st, 25)
    single.run(s1, 25)
    _sync()
    plan.check()
    for a, c in zip(st.formula(0), s1.formula(0)):
        assert np.array_equal(a, c)
    plan.free()
    single.free()


def test_replica_exchange_uses_the_clustered_free_energy(hip):
    ns = [70, 260]
    tables = [wl.random_formula(n, 15, tag=f) for f, n in enumerate(ns)]
    rbms = wl.pretrained_size_rbms(wl.FSTAR_16[:4])
    W, b = rbms[7]
    B = 12
    temps = np.array([i % 4 for i in range(B)], np.int32)
    plan = hp.Plan(tables, ns, W, b, chains=B, temps=temps, seed=15, size_rbms=rbms)
    st = plan.new_state([wl.initial_state(B, n, 15, tag=f) for f, n in enumerate(ns)])
    cps = [CL.ClusteredPlan(t, n, rbms) for t, n in zip(tables, ns)]
    say(f"[clust temper] N={ns} B={B} T=4")
    checked = 0
    for r in range(8):
        plan.run(st, 3)
        _sync()
        before = plan.current_temps()
        t = st.get_t()
        plan.temper(st, r % 2)
        _sync()
        got = plan.current_temps()
        for f in range(len(ns)):
            v = st.formula(f)[0]
            F = np.stack([CL.formula_free_energy(v, cps[f], tau) for tau in range(4)], axis=1)
            rec = []
            want = PT.swap_round(before[f], F, r % 2, t, 15, f, rec)
            if all(abs(x[3] - np.exp(min(x[2], 0.0))) > 1e-9 for x in rec):
                assert np.array_equal(got[f], want), (r, f, rec)
                checked += 1
    assert checked >= 12
    plan.free()
