"""Parity at the launch shapes of the measured workloads, through the C ABI.

* the 4096-variable, 64-chain workload in FP64 in its benchmark launch (four
  workgroups per chain exchanging partial sums every sweep): 500-sweep
  trajectories of four chains, one per quarter of the chain range, against
  the oracle;
* the uneven batch exactly as the benchmark runs it: 1024 formulas of
  log-uniform size 64..16384, 64 chains each, FP32, size-class launches
  captured in one hipGraph, autotuned; teacher-forced sweeps of sampled
  chains of ten formulas from the smallest to the largest.

Every case prints its name, sizes and seed before touching the GPU.
"""
import numpy as np
import pytest

from oracle import rbmsat as R
from paper_2311_02101_amd import workload as wl
from tests.parity import say, teacher_forced_batch
from tests.test_gpu_parity import _sync, _trajectory

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_plain_n4096_b64_fp64_split_launch_500_sweeps(hip):
    w = wl.config_workload("plain_n4096_b64")

    def split_launch(info):
        say(f"[n4096 fp64 x500] launch: split {info['split']}, threads {info['threads']}, "
            f"fx_shift {info['fx_shift']}")
        assert info["split"] > 1

    _trajectory(hip, w.tables, w.n_vars, w.W, w.b, 64, 500, "f64", w.seed, chains=[0, 21, 42, 63],
                label="n4096 fp64 x500", check_plan=split_launch)


@pytest.fixture(scope="module")
def uneven_workload():
    say("[uneven 1024x64] generating the 1024 formulas (seed 3)")
    return wl.config_workload("uneven_1024x64", precision="f32")


@pytest.mark.timeout(900)
def test_uneven_1024x64_fp32_graph_tuned_sampled_formulas(hip, uneven_workload):
    from paper_2311_02101_amd import hp
    w = uneven_workload
    say("[uneven 1024x64] plan: FP32, graph, then tune")
    plan = hp.Plan(w.tables, w.n_vars, w.W, w.b, chains=w.chains, temps=w.temps, precision="f32",
                   alpha=w.alpha, seed=w.seed, graph=True)
    plan.tune(n_sweeps=10)
    info = plan.info()
    say(f"[uneven 1024x64] {info['n_buckets']} launches, threads {info['bucket_threads'][:info['n_buckets']]}")
    assert info["n_buckets"] > 1 and info["split"] == 1
    # every launch a persistent grid: in sequence on the caller's stream
    assert all(g > 0 for g in info["bucket_grid"]) and info["forked"] == 0
    st = plan.new_state(w.v0)
    plan.run(st, 20)                      # away from the initial states, through the graph
    _sync()
    assert st.get_t() == 20
    order = np.argsort(w.n_vars, kind="stable")
    pick = sorted({int(order[i]) for i in np.linspace(0, len(order) - 1, 10).astype(int)})
    chains = np.array([0, 1, 2, 30, 31, 32, 33, 61, 62, 63])
    cases = {}
    for f in pick:
        v, nu, s_max, best = st.formula(f, chains=chains)
        cases[f] = (R.State(v, nu.astype(np.float64), s_max, best, 20),
                    R.plan(w.tables[f], w.n_vars[f], w.W, w.b), chains)
    say(f"[uneven 1024x64] teacher forcing formulas {pick} (N = {[w.n_vars[f] for f in pick]}), "
        f"chains {list(chains)}")
    ties = 0
    for i in range(3):
        ties += teacher_forced_batch(plan, st, cases, w.temps, alpha=w.alpha, seed=w.seed, prec="f32")
        say(f"[uneven 1024x64] sweep {i + 1}/3 matches, flagged ties so far: {ties}")
    plan.check()
    plan.free()
