"""HIP path vs the CPU FP64 oracle, through the C ABI (``libhp.so``).

Every case prints its name, sizes and seed before touching the GPU.
"""
import numpy as np
import pytest

from oracle import rbmsat as R
from paper_2311_02101_amd import workload as wl
from tests.parity import compare_state, f64_bounds, say, teacher_forced_sweep

pytestmark = pytest.mark.gpu


def _sync():
    import torch
    torch.cuda.synchronize()


def _trajectory(hip, tables, ns, W, b, B, S, prec, seed, alpha=1e-3, temps=None,
                chains=None, formulas=None, threads=0, kernel="auto", label="", check_plan=None):
    """Run S sweeps on the GPU and on the oracle (for the listed formulas and
    chains); compare final states exactly.  On a mismatch, replay with
    teacher forcing and require every difference to be a flagged tie.
    check_plan(info) may assert on the launch the plan chose."""
    from paper_2311_02101_amd import hp
    temps = wl.default_temperatures(B, W.shape[0]) if temps is None else np.asarray(temps)
    say(f"[{label}] plan F={len(tables)} N={list(ns)[:6]} B={B} S={S} prec={prec} seed={seed} "
        f"kernel={kernel}")
    plan = hp.Plan(tables, ns, W, b, chains=B, temps=temps, precision=prec, alpha=alpha,
                   seed=seed, threads=threads, kernel=kernel)
    if check_plan is not None:
        check_plan(plan.info())
    tie, nu_rtol = f64_bounds(plan, tables) if prec in ("f64", "mixed") else (None, None)
    v0s = [wl.initial_state(B, n, seed, tag=f) for f, n in enumerate(ns)]
    st = plan.new_state(v0s)
    say(f"[{label}] gpu run (tie bound {tie}, nu rtol {nu_rtol})")
    plan.run(st, S)
    _sync()
    assert st.get_t() == S
    chains = np.arange(B) if chains is None else np.asarray(chains)
    formulas = range(len(tables)) if formulas is None else formulas
    for f in formulas:
        op = R.plan(tables[f], ns[f], W, b)
        ost = R.initial(v0s[f][chains])
        R.run(ost, op, temps[chains], S, alpha=alpha, seed=seed, formula_id=f, chain_ids=chains)
        gv, gnu, gs, gbest = st.formula(f)
        got = (gv[chains], gnu[chains], gs[chains], gbest[chains])
        try:
            compare_state(got, (ost.v, ost.nu, ost.s_max, ost.best), prec, f"{label} f={f}", nu_rtol=nu_rtol)
        except AssertionError as err:
            say(f"[{label}] f={f}: trajectory mismatch ({err}); replaying with teacher forcing")
            # replay the whole run sweep by sweep in the same plan (same formula
            # id, hence the same random stream) on a second state, so every
            # differing bit of every sweep must be a flagged tie
            sst = plan.new_state(v0s)
            o2 = R.initial(v0s[f][chains])
            ties = 0
            for _ in range(S):
                ties += teacher_forced_sweep(plan, sst, f, o2, op, temps, alpha=alpha, seed=seed,
                                             prec=prec, chain_ids=chains, tie=tie, nu_rtol=nu_rtol)
            say(f"[{label}] f={f}: {ties} flagged ties over {S} sweeps")
            assert ties > 0, "trajectory mismatch without any tie"
    plan.free()
    return st


# --------------------------------------------------------------------------
# Plain method, smallest: N = 256, 1 chain, FP64, seed 0 -- 500-sweep trajectory
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", ["push", "pull"])
def test_plain_n256_b1_fp64_trajectory(hip, kernel):
    w = wl.config_workload("plain_n256_b1")
    _trajectory(hip, w.tables, w.n_vars, w.W, w.b, 1, 500, "f64", w.seed, kernel=kernel,
                label="n256 fp64")


@pytest.mark.parametrize("kernel", ["push", "pull"])
def test_plain_n256_b1_fp32_teacher_forced(hip, kernel):
    from paper_2311_02101_amd import hp
    w = wl.config_workload("plain_n256_b1")
    say(f"[n256 fp32 {kernel}] teacher forced 40 sweeps")
    plan = hp.Plan(w.tables, w.n_vars, w.W, w.b, chains=1, temps=w.temps, precision="f32",
                   seed=w.seed, kernel=kernel)
    st = plan.new_state(w.v0)
    op = R.plan(w.tables[0], 256, w.W, w.b)
    ost = R.initial(w.v0[0])
    for _ in range(40):
        teacher_forced_sweep(plan, st, 0, ost, op, w.temps, alpha=1e-3, seed=w.seed, prec="f32")


# --------------------------------------------------------------------------
# Plain method, medium: N = 4096, 64 chains, seed 1 (the benchmark's launch)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", ["push", "pull"])
def test_plain_n4096_b64_fp64_sampled_chains(hip, kernel):
    w = wl.config_workload("plain_n4096_b64")
    _trajectory(hip, w.tables, w.n_vars, w.W, w.b, 64, 40, "f64", w.seed,
                chains=[0, 1, 31, 32, 62, 63], kernel=kernel, label="n4096 fp64")


def test_push_and_pull_kernels_agree(hip):
    """The two scatter-add variants differ only in the last bits of x, so
    their trajectories coincide except at (astronomically rare) ties."""
    from paper_2311_02101_amd import hp
    w = wl.config_workload("plain_n4096_b64")
    out = []
    for kernel in ("push", "pull"):
        say(f"[push/pull] {kernel}: 64 chains x 30 sweeps")
        plan = hp.Plan(w.tables, w.n_vars, w.W, w.b, chains=64, temps=w.temps,
                       precision="f64", seed=w.seed, kernel=kernel)
        st = plan.new_state(w.v0)
        plan.run(st, 30)
        _sync()
        out.append(st.formula(0))
    for a, c in zip(out[0], out[1]):
        if a.dtype.kind == "f":
            assert np.max(np.abs(a - c) / c) < 1e-12
        else:
            assert np.array_equal(a, c)


@pytest.mark.timeout(600)
def test_plain_n4096_b64_fp32_teacher_forced_all_chains(hip):
    """The FP32 form of the 4096-variable, 64-chain workload in its own
    (split) launch: all 64 chains, 10 teacher-forced sweeps."""
    from paper_2311_02101_amd import hp
    w = wl.config_workload("plain_n4096_b64", precision="f32")
    say("[n4096 fp32] teacher forced, 64 chains x 10 sweeps")
    plan = hp.Plan(w.tables, w.n_vars, w.W, w.b, chains=64, temps=w.temps, precision="f32",
                   seed=w.seed)
    assert plan.split > 1
    st = plan.new_state(w.v0)
    plan.run(st, 25)             # move away from the initial state first
    _sync()
    v, nu, s_max, best = st.formula(0)
    op = R.plan(w.tables[0], 4096, w.W, w.b)
    ost = R.State(v, nu.astype(np.float64), s_max, best, 25)
    ties = 0
    for i in range(10):
        ties += teacher_forced_sweep(plan, st, 0, ost, op, w.temps, alpha=1e-3, seed=w.seed,
                                     prec="f32")
        say(f"[n4096 fp32] sweep {i + 1}/10, flagged ties so far: {ties}")
    plan.free()


# --------------------------------------------------------------------------
# Larger shapes of the measured configurations, on sampled chains / formulas
# --------------------------------------------------------------------------
def test_n8192_b256_fp64_sampled_chains(hip):
    w = wl.config_workload("mixed_n8192_b256", precision="f64")
    _trajectory(hip, w.tables, w.n_vars, w.W, w.b, 256, 6, "f64", w.seed,
                chains=[0, 127, 128, 255], label="n8192 fp64")


def test_uneven_batch_sampled_formulas(hip):
    sizes = wl.uneven_sizes(1024, 3)[:48]
    tables = [wl.random_formula(int(n), 3, tag=f) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    order = np.argsort(sizes)
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    _trajectory(hip, tables, [int(n) for n in sizes], W, b, 8, 12, "f64", 3,
                chains=[0, 7], formulas=pick, label="uneven fp64")


def test_uneven_batch_fp32_sampled_formulas(hip):
    from paper_2311_02101_amd import hp
    sizes = [64, 5000, 300, 16384, 77]
    tables = [wl.random_formula(int(n), 3, tag=f) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    temps = wl.default_temperatures(4, 2)
    say("[uneven fp32] teacher forced on every formula")
    plan = hp.Plan(tables, sizes, W, b, chains=4, temps=temps, precision="f32", seed=3)
    st = plan.new_state([wl.initial_state(4, n, 3, tag=f) for f, n in enumerate(sizes)])
    for f, n in enumerate(sizes):
        v, nu, s_max, best = st.formula(f)
        op = R.plan(tables[f], n, W, b)
        ost = R.State(v, nu.astype(np.float64), s_max, best, 0)
        teacher_forced_sweep(plan, st, f, ost, op, temps, alpha=1e-3, seed=3, prec="f32")


# --------------------------------------------------------------------------
# Edge cases
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", ["push", "pull"])
@pytest.mark.parametrize("threads", [64, 512, 1024])
def test_launch_shapes_agree(hip, threads, kernel):
    """Register-resident (1 or 2 groups/thread) and global-memory EMA paths."""
    n = 4096
    T = wl.random_formula(n, 21)
    W, b = wl.gaussian_rbm(2, 7, 8, 21)
    _trajectory(hip, [T], [n], W, b, 3, 8, "f64", 21, threads=threads, kernel=kernel,
                label=f"threads={threads}")


@pytest.mark.parametrize("kernel", ["push", "pull"])
def test_tiny_and_ragged_formulas(hip, kernel):
    clauses = [[[1]], [[1, -2], [2]], [[3, -1, 2], [-3]], [[-4, 1], [2, 3, 4], [-1, -2, -3]],
               [[5, -1, 2], [-3, 4], [1], [-5, 2, 3]]]
    ns = [1, 2, 3, 4, 5]
    tables = [wl.pad_clauses(cl, 3) for cl in clauses]
    W, b = wl.gaussian_rbm(1, 3, 3, 4)
    _trajectory(hip, tables, ns, W, b, 5, 30, "f64", 4, kernel=kernel, label="tiny K=3 L=3")


@pytest.mark.parametrize("kernel", ["push", "pull"])
@pytest.mark.parametrize("k,l", [(1, 2), (2, 3)])
def test_narrow_tables(hip, kernel, k, l):
    """Tables of width K = 1 (unit clauses) and K = 2 with their own RBMs."""
    n = 150
    lengths = list(range(1, k + 1))
    T = wl.random_formula(n, 20 + k, k=k, lengths=lengths, probs=[1.0 / k] * k)
    assert T.shape[0] == k
    W, b = wl.gaussian_rbm(2, k, l, 20 + k)
    _trajectory(hip, [T], [n], W, b, 6, 40, "f64", 20 + k, kernel=kernel, label=f"K={k} L={l}")


@pytest.mark.parametrize("k,l", [(7, 4), (7, 5), (5, 8), (4, 1)])
def test_hidden_unit_counts(hip, k, l):
    """Hidden-unit counts other than K + 1: one Philox block (L <= 4) or two
    with unused words (4 < L < 8), a single hidden unit."""
    n = 300
    lengths = list(range(1, k + 1))
    T = wl.random_formula(n, 30 + l, k=k, lengths=lengths, probs=[1.0 / k] * k)
    W, b = wl.gaussian_rbm(2, k, l, 30 + l)
    _trajectory(hip, [T], [n], W, b, 5, 30, "f64", 30 + l, label=f"K={k} L={l}")


def test_zero_padded_literals_are_normalised(hip):
    n = 40
    T = wl.random_formula(n, 13, ratio=3)
    Tz = T.copy()
    for c in range(T.shape[1]):
        L = len(set(T[:, c]))
        Tz[L:, c] = 0                 # trailing padding written as zeros
    W, b = wl.gaussian_rbm(2, 7, 8, 13)
    from paper_2311_02101_amd import hp
    say("[zero padding] plans from zero-padded and repeated tables")
    st = []
    for tab in (T, Tz):
        plan = hp.Plan([tab], [n], W, b, chains=4, precision="f64", seed=13)
        s = plan.new_state([wl.initial_state(4, n, 13)])
        plan.run(s, 20)
        st.append(s.formula(0))
    _sync()
    for a, c in zip(*st):
        assert np.array_equal(a, c)


def test_resume_and_count_only(hip):
    from paper_2311_02101_amd import hp
    n = 700
    T = wl.random_formula(n, 5)
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    v0 = wl.initial_state(6, n, 5)
    say("[resume] run(12) vs run(7)+run(0)+run(5)")
    p = hp.Plan([T], [n], W, b, chains=6, precision="f64", seed=5)
    a = p.new_state([v0])
    c = p.new_state([v0])
    p.run(a, 12)
    p.run(c, 7)
    p.run(c, 0)
    p.run(c, 5)
    _sync()
    for x, y in zip(a.formula(0), c.formula(0)):
        assert np.array_equal(x, y)
    assert a.get_t() == c.get_t() == 12
    # a zero-sweep run counts the current state (s_max, best) and keeps t
    d = p.new_state([v0])
    p.run(d, 0)
    _sync()
    v, nu, s_max, best = d.formula(0)
    op = R.plan(T, n, W, b)
    assert np.array_equal(s_max, R.clause_count(v0, op))
    assert np.array_equal(best, v0) and d.get_t() == 0 and np.all(nu == 0.25)


def test_split_resume_and_count_only(hip):
    """The split launch is resumable like the single one (runs of 7, 0 and 5
    sweeps equal one of 12, the best-state decisions settled inside each
    launch) and a zero-sweep run counts the current state."""
    from paper_2311_02101_amd import hp
    w = wl.config_workload("plain_n4096_b64")
    T, n, v0 = w.tables[0], w.n_vars[0], w.v0[0]
    say("[split resume] n4096 64 chains: run(12) vs run(7)+run(0)+run(5)")
    p = hp.Plan([T], [n], w.W, w.b, chains=64, temps=w.temps, seed=w.seed)
    assert p.split > 1
    a = p.new_state([v0])
    c = p.new_state([v0])
    p.run(a, 12)
    p.run(c, 7)
    p.run(c, 0)
    p.run(c, 5)
    _sync()
    p.check()
    for x, y in zip(a.formula(0), c.formula(0)):
        assert np.array_equal(x, y)
    assert a.get_t() == c.get_t() == 12
    d = p.new_state([v0])
    p.run(d, 0)
    _sync()
    v, nu, s_max, best = d.formula(0)
    op = R.plan(T, n, w.W, w.b)
    assert np.array_equal(s_max, R.clause_count(v0, op))
    assert np.array_equal(best, v0) and d.get_t() == 0
    p.free()


def test_sweep_counter_crossing_2_pow_32(hip):
    """The absolute sweep counter t addresses the random numbers through its
    low and high words: sweeps across t = 2^32 match the oracle (one
    workgroup per chain), and the split launch matches the single one there."""
    from paper_2311_02101_amd import hp
    n, B, t0 = 256, 4, (1 << 32) - 3
    T = wl.random_formula(n, 18)
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    temps = wl.default_temperatures(B, 2)
    v0 = wl.initial_state(B, n, 18)
    say(f"[t across 2^32] N={n} B={B} t0={t0}, 6 sweeps")
    plan = hp.Plan([T], [n], W, b, chains=B, temps=temps, seed=18)
    st = plan.new_state([v0])
    st.set_t(t0)
    plan.run(st, 6)
    _sync()
    assert st.get_t() == t0 + 6
    op = R.plan(T, n, W, b)
    ost = R.initial(v0)
    ost.t = t0
    R.run(ost, op, temps, 6, alpha=1e-3, seed=18)
    compare_state(st.formula(0), (ost.v, ost.nu, ost.s_max, ost.best), "f64", "t across 2^32",
                  nu_rtol=f64_bounds(plan, [T])[1])
    plan.free()
    w = wl.config_workload("plain_n4096_b64")
    out = []
    for split in (1, 4):
        say(f"[t across 2^32] n4096 64 chains split {split}")
        p2 = hp.Plan(w.tables, w.n_vars, w.W, w.b, chains=64, temps=w.temps, seed=w.seed, split=split)
        s2 = p2.new_state(w.v0)
        s2.set_t(t0)
        p2.run(s2, 6)
        _sync()
        p2.check()
        out.append(s2.formula(0))
        p2.free()
    for x, y in zip(*out):
        assert np.array_equal(x, y)


def test_largest_formulas(hip):
    """A formula too large for the push kernels' LDS (N = 19 000, C = 114 000)
    runs on the pull kernel and matches the oracle; one whose pull working
    set no longer fits either (N = 21 000) is refused with HP_EUNSUPPORTED."""
    from paper_2311_02101_amd import hp
    n, B = 19000, 2
    T = wl.random_formula(n, 19)
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    say(f"[largest] N={n} C={T.shape[1]} B={B}, 3 sweeps")
    _trajectory(hip, [T], [n], W, b, B, 3, "f64", 19, label="largest N")
    plan = hp.Plan([T], [n], W, b, chains=B, seed=19)
    assert plan.info()["bucket_kind"] == [2]
    plan.free()
    big = 21000
    with pytest.raises(hp.HpError, match="LDS"):
        hp.Plan([wl.random_formula(big, 19)], [big], W, b, chains=B, seed=19)


def test_stationary_distribution_on_gpu(hip):
    """The device sampler's long-run distribution is p(v) ~ exp(-F_f(v))."""
    from paper_2311_02101_amd import hp
    n = 5
    T = wl.pad_clauses([[1, -2], [2, 3, -4], [-5, 1, 2], [4, -1], [3, 5]], 3)
    rng = np.random.default_rng(8)
    W_c, b_c = 0.8 * rng.standard_normal((1, 3, 3)), 0.8 * rng.standard_normal((1, 3))
    op = R.plan(T, n, W_c, b_c)
    Wf, bf = R.dense_formula_rbm(op)
    V = ((np.arange(2 ** n)[:, None] >> np.arange(n)[None, :]) & 1).astype(float)
    F = R.free_energy(V, Wf, bf)
    pi = np.exp(-(F - F.min()))
    pi /= pi.sum()
    B = 8192
    say(f"[stationarity] B={B}")
    plan = hp.Plan([T], [n], W_c, b_c, chains=B, precision="f64", seed=77, threads=64)
    st = plan.new_state([wl.initial_state(B, n, 77)])
    plan.run(st, 100)
    counts = np.zeros(2 ** n)
    code = 1 << np.arange(n)
    for _ in range(60):
        plan.run(st, 5)
        v = st.formula(0)[0].astype(np.int64)
        counts += np.bincount(v @ code, minlength=2 ** n)
    tv = 0.5 * np.abs(counts / counts.sum() - pi).sum()
    say(f"[stationarity] TV = {tv:.4f}")
    assert tv < 0.01


# --------------------------------------------------------------------------
# Split launch: G workgroups per chain must reproduce the one-workgroup result
# bit for bit (exact integer partial sums, same random-number addressing)
# --------------------------------------------------------------------------
def _run_states(tables, ns, W, b, B, S, prec, seed, **kw):
    from paper_2311_02101_amd import hp
    plan = hp.Plan(tables, ns, W, b, chains=B, precision=prec, seed=seed, **kw)
    st = plan.new_state([wl.initial_state(B, n, seed, tag=f) for f, n in enumerate(ns)])
    plan.run(st, S)
    plan.run(st, 0)
    plan.check()
    out = [st.formula(f) for f in range(len(tables))]
    t = st.get_t()
    plan.free()
    return out, t


def _same(a, b):
    for fa, fb in zip(a, b):
        for x, y in zip(fa, fb):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("split,chains", [(2, 64), (4, 64), (8, 16), (16, 8)])
def test_split_matches_single_workgroup(hip, split, chains):
    w = wl.config_workload("plain_n4096_b64")
    W, b = w.W, w.b
    say(f"[split={split}] n4096 {chains} chains, 20 sweeps")
    ref, t1 = _run_states(w.tables, w.n_vars, W, b, chains, 20, "f64", w.seed, split=1)
    got, t2 = _run_states(w.tables, w.n_vars, W, b, chains, 20, "f64", w.seed, split=split)
    assert t1 == t2 == 20
    _same(ref, got)


def test_split_fp32_and_global_ema_path(hip):
    n = 4096
    T = wl.random_formula(n, 31)
    W, b = wl.gaussian_rbm(2, 7, 8, 31)
    say("[split fp32, 64 threads] 3 chains (no XCD map), split 4")
    ref, _ = _run_states([T], [n], W, b, 3, 15, "f32", 31, split=1, threads=64)
    got, _ = _run_states([T], [n], W, b, 3, 15, "f32", 31, split=4, threads=64)
    _same(ref, got)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_split_two_owned_variables_per_thread(hip, prec):
    """512 threads per member owning 1024 variables (EMA of two variables per
    thread in registers), N not a multiple of 4."""
    n = 4094
    T = wl.random_formula(n, 32)
    W, b = wl.gaussian_rbm(2, 7, 8, 32)
    say(f"[split {prec}, 512 threads] N={n} 8 chains, split 4")
    ref, _ = _run_states([T], [n], W, b, 8, 15, prec, 32, split=1, threads=512)
    got, _ = _run_states([T], [n], W, b, 8, 15, prec, 32, split=4, threads=512)
    _same(ref, got)


def test_split_wait_limit_reports_a_failed_exchange(hip):
    """The failure path of the split exchange, forced from the host: with a
    wait limit of one reload a workgroup gives up as soon as another's word
    has not arrived yet; every workgroup still exits, hp_check reports the
    void run, and a plan with the default limit is unaffected."""
    from paper_2311_02101_amd import hp
    w = wl.config_workload("plain_n4096_b64")
    say("[split wait limit] n4096 64 chains, limit 1, 200 sweeps")
    plan = hp.Plan(w.tables, w.n_vars, w.W, w.b, chains=64, temps=w.temps, seed=w.seed, split_wait_limit=1)
    assert plan.split > 1
    st = plan.new_state(w.v0)
    plan.run(st, 200)
    with pytest.raises(hp.HpError):
        plan.check()
    plan.check()                  # reported once: the flag is cleared
    plan.free()
    ok = hp.Plan(w.tables, w.n_vars, w.W, w.b, chains=64, temps=w.temps, seed=w.seed)
    st = ok.new_state(w.v0)
    ok.run(st, 20)
    ok.check()
    ok.free()


def test_split_tiny_ragged_members(hip):
    """Members that own a single variable group and members with no clauses;
    a split that would leave a member without variables is refused."""
    from paper_2311_02101_amd import hp
    clauses = [[[5, -1, 2], [-3, 4], [29, 1]], [[1, -2], [33, 2]]]
    tables = [wl.pad_clauses(cl, 3) for cl in clauses]
    W, b = wl.gaussian_rbm(1, 3, 3, 6)
    say("[split tiny] N=29,33 split 8")
    ref, _ = _run_states(tables, [29, 33], W, b, 8, 25, "f64", 6, split=1)
    got, _ = _run_states(tables, [29, 33], W, b, 8, 25, "f64", 6, split=8)
    _same(ref, got)
    with pytest.raises(hp.HpError):
        hp.Plan(tables, [29, 5], W, b, chains=8, split=8)


def test_weights_beyond_the_fixed_point_range(hip):
    """Weights so large that the push accumulators' fixed-point scale would
    drop below 2^40: the automatic choice falls back to the pull kernel (FP
    sums); the push kernel is refused with the reason."""
    from paper_2311_02101_amd import hp
    n = 64
    T = wl.random_formula(n, 17)
    W, b = wl.gaussian_rbm(1, 7, 8, 17)
    W = np.abs(W) * 2.0 ** 13          # positive: every hidden logit >= b = 0 (no underflow)
    b = b * 0.0
    say("[fixed-point range] N=64 |W| ~ 2^13")
    plan = hp.Plan([T], [n], W, b, chains=2, temps=np.zeros(2, np.int32), seed=17)
    assert plan.info()["fx_shift"] < 40
    assert plan.info()["bucket_kind"][0] == 2      # pull
    plan.free()
    with pytest.raises(hp.HpError, match="fixed-point"):
        hp.Plan([T], [n], W, b, chains=2, temps=np.zeros(2, np.int32), seed=17, kernel="push")


@pytest.mark.parametrize("split,chains", [(2, 16), (4, 8), (16, 2)])
def test_split_small_formulas_many_sweeps(hip, split, chains):
    """Small exchanges repeated over many sweeps: the exchanged lines stay in
    the CUs' vector caches unless every exchange access bypasses them."""
    sizes = [67, 64, 90, 127, 61, 80, 77, 100]     # one size class (one launch), > 4 (16 - 1) each
    tables = [wl.random_formula(n, 9, tag=f) for f, n in enumerate(sizes)]
    W, b = wl.gaussian_rbm(2, 7, 8, 9)
    say(f"[split small] sizes={sizes} split={split} chains={chains} 300 sweeps")
    ref, _ = _run_states(tables, sizes, W, b, chains, 300, "f64", 9, split=1)
    got, _ = _run_states(tables, sizes, W, b, chains, 300, "f64", 9, split=split)
    _same(ref, got)


def test_split_against_oracle(hip):
    w = wl.config_workload("plain_n4096_b64")
    _trajectory(hip, w.tables, w.n_vars, w.W, w.b, 64, 30, "f64", w.seed,
                chains=[0, 33, 63], label="n4096 fp64 auto split")


# --------------------------------------------------------------------------
# Uneven batches: size-class launches, tables in global memory for the
# largest formulas, persistent grids, hipGraph replay, autotuning
# --------------------------------------------------------------------------
def test_wide_tables_variant_against_oracle(hip):
    from paper_2311_02101_amd import hp
    sizes = [15000, 16384, 700]
    tables = [wl.random_formula(n, 9, tag=f) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    plan = hp.Plan(tables, sizes, W, b, chains=2, precision="f64", seed=9)
    info = plan.info()
    say(f"[wide] buckets {info['bucket_kind']} max_n {info['bucket_max_n']}")
    # N = 15000: contributions table in LDS, padding table in global memory;
    # N = 16384: both tables in global memory
    assert 3 in info["bucket_kind"] and 1 in info["bucket_kind"] and info["pull_items"] == 0
    plan.free()
    _trajectory(hip, tables, sizes, W, b, 2, 4, "f64", 9, label="wide tables")


def test_size_class_shares_one_launch(hip):
    """Formulas of one size class (8192 <= N < 16384) that would fit different
    table layouts (all in LDS, mid, wide) share one launch in the layout the
    largest needs, and match the oracle."""
    from paper_2311_02101_amd import hp
    sizes = [16000, 9000, 15000]
    tables = [wl.random_formula(n, 21, tag=f) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    plan = hp.Plan(tables, sizes, W, b, chains=2, precision="f64", seed=21)
    info = plan.info()
    say(f"[one class] buckets {info['bucket_kind'][:info['n_buckets']]} max_n {info['bucket_max_n'][:info['n_buckets']]}")
    assert info["n_buckets"] == 1 and info["bucket_kind"][0] == 1 and info["bucket_max_n"][0] == 16000
    plan.free()
    _trajectory(hip, tables, sizes, W, b, 2, 3, "f64", 21, label="one size class")


def test_persistent_grid_matches_small_batch(hip):
    from paper_2311_02101_amd import hp
    n_f = 300
    sizes = [64 + 3 * (f % 7) for f in range(n_f)]
    tables = [wl.random_formula(n, 12, tag=f) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    big = hp.Plan(tables, sizes, W, b, chains=64, precision="f64", seed=12)
    info = big.info()
    say(f"[persistent] buckets grid {info['bucket_grid']} items {info['bucket_items']}")
    assert any(g > 0 for g in info["bucket_grid"])
    st = big.new_state([wl.initial_state(64, n, 12, tag=f) for f, n in enumerate(sizes)])
    big.run(st, 15)
    big.check()
    small = hp.Plan(tables[:4], sizes[:4], W, b, chains=64, precision="f64", seed=12)
    st2 = small.new_state([wl.initial_state(64, n, 12, tag=f) for f, n in enumerate(sizes[:4])])
    small.run(st2, 15)
    small.check()
    # the fixed-point scale 2^-S is chosen per plan (from its largest slot
    # count), so nu may differ in the last bits between the two batches;
    # the sampled values, counts and best assignments may not
    for f in range(4):
        (v1, nu1, s1, b1), (v2, nu2, s2, b2) = st.formula(f), st2.formula(f)
        assert np.array_equal(v1, v2) and np.array_equal(s1, s2) and np.array_equal(b1, b2)
        assert np.max(np.abs(nu1 - nu2) / nu2) < 1e-12


def test_graph_replays_match_eager(hip):
    import torch
    from paper_2311_02101_amd import hp
    sizes = [300, 5000, 90, 1200]
    tables = [wl.random_formula(n, 14, tag=f) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    v0 = [wl.initial_state(8, n, 14, tag=f) for f, n in enumerate(sizes)]
    eager = hp.Plan(tables, sizes, W, b, chains=8, precision="f64", seed=14)
    graph = hp.Plan(tables, sizes, W, b, chains=8, precision="f64", seed=14, graph=True)
    # four launches of one workgroup per item: forked over side streams
    assert graph.info()["n_buckets"] == 4 and graph.info()["forked"] == 1
    se, sg = eager.new_state(v0), graph.new_state(v0)
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(4):
        say(f"[graph] replay {rep}")
        eager.run(se, 7)
        graph.run(sg, 7)
        junk.add_(1.0)                  # unrelated eager work between replays
        torch.cuda.synchronize()
        for f in range(len(sizes)):
            for x, y in zip(se.formula(f), sg.formula(f)):
                assert np.array_equal(x, y), (rep, f)
        assert se.get_t() == sg.get_t() == 7 * (rep + 1)
    graph.check()


def test_tuned_plan_reproduces_untuned_results(hip):
    from paper_2311_02101_amd import hp
    sizes = [128, 2000, 9000]
    tables = [wl.random_formula(n, 15, tag=f) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    v0 = [wl.initial_state(4, n, 15, tag=f) for f, n in enumerate(sizes)]
    ref = hp.Plan(tables, sizes, W, b, chains=4, precision="f32", seed=15)
    tuned = hp.Plan(tables, sizes, W, b, chains=4, precision="f32", seed=15)
    info = tuned.tune(n_sweeps=2)
    say(f"[tune] threads per bucket {info['bucket_threads']}")
    a, c = ref.new_state(v0), tuned.new_state(v0)
    ref.run(a, 10)
    tuned.run(c, 10)
    _sync()
    for f in range(len(sizes)):
        for x, y in zip(a.formula(f), c.formula(f)):
            assert np.array_equal(x, y)
