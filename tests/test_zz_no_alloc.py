"""hp_run_noalloc (the entry point for callers that cannot allocate) against
hp_run, through the C ABI.

The two entry points run the same kernels; only the run's scratch differs
(the plan's buffers vs the library's static device array), so every result
must be bit-identical: v, nu, s_max and best after the same sweeps from the
same state.  The calls come in a row on one device, each later one with a
smaller input than the first, so stale mailboxes and work counters left in
the shared array by an earlier call would show; a run whose scratch exceeds
the array is refused.
"""
import numpy as np
import pytest

from paper_2311_02101_amd import workload as wl
from tests.parity import say

pytestmark = pytest.mark.gpu


def _states_equal(a, b, label):
    for name, x, y in zip(("v", "nu", "s_max", "best"), a, b):
        assert np.array_equal(x, y), f"{label}: {name} differs"


def _both(tables, ns, W, b, B, sweeps, label, **kw):
    """Run `sweeps` sweeps through hp_run and hp_run_noalloc from the same
    initial states (two calls each: sweeps // 2, then the rest) and compare."""
    import torch
    from paper_2311_02101_amd import hp
    plan = hp.Plan(tables, ns, W, b, chains=B, **kw)
    info = plan.info()
    say(f"[noalloc {label}] F={len(tables)} N<={max(ns)} B={B} sweeps={sweeps} split={info['split']} "
        f"buckets={info['n_buckets']} grids={info['bucket_grid']}")
    v0 = [wl.initial_state(B, n, 7, tag=f) for f, n in enumerate(ns)]
    ref = plan.new_state(v0)
    got = plan.new_state(v0)
    half = sweeps // 2
    plan.run(ref, half)
    plan.run(ref, sweeps - half)
    plan.run_noalloc(got, half)
    plan.run_noalloc(got, sweeps - half)
    torch.cuda.synchronize()
    plan.check()
    assert got.get_t() == ref.get_t() == sweeps
    for f in range(len(tables)):
        _states_equal(got.formula(f), ref.formula(f), f"{label} f={f}")
    plan.free()
    return info


def test_noalloc_matches_run_on_calls_of_decreasing_size(hip):
    # 1: the 4096-variable, 64-chain workload in its split launch (8.7 MB of mailboxes)
    w = wl.config_workload("plain_n4096_b64")
    info = _both(w.tables, w.n_vars, w.W, w.b, 64, 30, "split n4096", temps=w.temps, seed=w.seed)
    assert info["split"] > 1
    # 2: a smaller split plan: fewer chains and variables, a different member count
    W, b = wl.gaussian_rbm(2, 7, 8, 5)
    T = wl.random_formula(700, 5)
    info = _both([T], [700], W, b, 24, 25, "split n700", seed=5)
    assert info["split"] > 1
    # 3: smaller still: persistent work queues over several size classes, a
    # plan built for graph replay (hp_run replays its graph; hp_run_noalloc
    # launches directly), FP32
    sizes = [300 + 5 * i for i in range(40)] + [70, 2000, 5000]    # 2560 items in one size class
    tables = [wl.random_formula(n, 3, tag=f) for f, n in enumerate(sizes)]
    Wp, bp, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    info = _both(tables, sizes, Wp, bp, 64, 12, "batch persistent", precision="f32", seed=3, threads=1024,
                 graph=True)
    assert info["n_buckets"] > 1 and max(info["bucket_grid"]) > 0
    # 4: the smallest: one chain, one formula, one workgroup
    w = wl.config_workload("plain_n256_b1")
    _both(w.tables, w.n_vars, w.W, w.b, 1, 20, "n256 b1", seed=w.seed)


def test_noalloc_refuses_scratch_beyond_its_array(hip):
    from paper_2311_02101_amd import hp
    n = 13000
    T = wl.random_formula(n, 9)
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    plan = hp.Plan([T], [n], W, b, chains=64, seed=9, split=4)
    say(f"[noalloc refuse] N={n} B=64 split={plan.split}: mailboxes beyond 16 MiB")
    st = plan.new_state([wl.initial_state(64, n, 9)])
    with pytest.raises(hp.HpError, match="scratch"):
        plan.run_noalloc(st, 1)
    assert st.get_t() == 0                 # nothing was enqueued
    plan.free()
