"""Mixed precision (hidden logits and contributions as BF16-limb MFMA
products, FP32 accumulation, FP64 recombination) against the FP64 table path
and the CPU FP64 oracle.  The appendix ("Precision") notes that the MXU
computes in bfloat16; here the weights are split into BF16 limbs so that the
products carry 64 bits, and every hidden decision that the FP32 sigmoid
cannot settle is taken from the FP64 threshold table."""
import numpy as np
import pytest

from oracle import rbmsat as R
from paper_2311_02101_amd import workload as wl
from tests.parity import compare_state, say
from tests.test_gpu_parity import _trajectory

pytestmark = pytest.mark.gpu


def _sync():
    import torch
    torch.cuda.synchronize()


def _run(tables, ns, W, b, B, S, prec, seed, temps=None, **kw):
    from paper_2311_02101_amd import hp
    temps = wl.default_temperatures(B, W.shape[0]) if temps is None else temps
    plan = hp.Plan(tables, ns, W, b, chains=B, temps=temps, precision=prec, seed=seed, **kw)
    st = plan.new_state([wl.initial_state(B, n, seed, tag=f) for f, n in enumerate(ns)])
    plan.run(st, S)
    plan.run(st, 0)
    plan.check()
    out = [st.formula(f) for f in range(len(tables))]
    info = plan.info()
    plan.free()
    return out, info


def _same_as_fp64(tables, ns, W, b, B, S, seed, label, **kw):
    say(f"[mixed {label}] B={B} S={S}")
    ref, _ = _run(tables, ns, W, b, B, S, "f64", seed, kernel="push", split=1, **kw)
    got, info = _run(tables, ns, W, b, B, S, "mixed", seed, **kw)
    for f, (a, g) in enumerate(zip(ref, got)):
        compare_state(g, a, "mixed", f"{label} f={f}")
    return info


def test_mixed_matches_fp64_path_n4096(hip):
    w = wl.config_workload("plain_n4096_b64")
    _same_as_fp64(w.tables, w.n_vars, w.W, w.b, 16, 60, w.seed, "n4096")


def test_mixed_matches_fp64_path_gaussian_weights(hip):
    """Weights ~ N(0,1): logits spread over a wide range, many draws near p."""
    tables = [wl.random_formula(n, 12, tag=f) for f, n in enumerate([300, 1001, 77])]
    W, b = wl.gaussian_rbm(2, 7, 8, 12)
    _same_as_fp64(tables, [300, 1001, 77], W, b, 8, 80, 12, "gaussian")


def test_mixed_small_clauses_K3_L3_and_ragged_tiles(hip):
    """K = 3, L = 3 (one Philox block per clause; hidden units 4..7 unused)
    and clause counts that are not multiples of the 32-clause tile."""
    sizes = [9, 50, 31]
    tables = [wl.random_formula(n, 13, k=3, lengths=[1, 2, 3], probs=[0.2, 0.5, 0.3], ratio=3, tag=f)
              for f, n in enumerate(sizes)]
    assert all(t.shape[1] % 32 for t in tables)
    W, b = wl.gaussian_rbm(2, 3, 3, 13)
    _same_as_fp64(tables, sizes, W, b, 6, 120, 13, "K3")


def test_mixed_pretrained_weights_against_oracle(hip):
    """Plain configuration n = 256 (the OR-gate weights of the benchmark),
    500-sweep trajectory against the CPU FP64 oracle."""
    w = wl.config_workload("plain_n256_b1")
    _trajectory(hip, w.tables, w.n_vars, w.W, w.b, 1, 500, "mixed", w.seed, label="mixed n256")


def test_mixed_n8192_sampled_chains_against_oracle(hip):
    w = wl.config_workload("mixed_n8192_b256")
    _trajectory(hip, w.tables, w.n_vars, w.W, w.b, 256, 6, "mixed", w.seed,
                chains=[0, 127, 128, 255], label="mixed n8192")


def test_mixed_persistent_grid_and_tuned_shapes(hip):
    """More chains than resident workgroups (persistent work queue), then an
    autotuned workgroup size: both give the FP64 path's result."""
    from paper_2311_02101_amd import hp
    sizes = [700, 64, 2000]
    tables = [wl.random_formula(n, 14, tag=f) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    B = 300                        # > 256 resident 1024-thread workgroups
    ref, _ = _run(tables, sizes, W, b, B, 12, "f64", 14, kernel="push", split=1)
    temps = wl.default_temperatures(B, 2)
    for tuned in (False, True):
        plan = hp.Plan(tables, sizes, W, b, chains=B, temps=temps, precision="mixed", seed=14)
        if tuned:
            plan.tune(n_sweeps=2)
        info = plan.info()
        say(f"[mixed tuned={tuned}] threads {info['bucket_threads']} grid {info['bucket_grid']}")
        if not tuned:
            assert any(g > 0 for g in info["bucket_grid"]), "expected a persistent launch"
        st = plan.new_state([wl.initial_state(B, n, 14, tag=f) for f, n in enumerate(sizes)])
        plan.run(st, 12)
        plan.run(st, 0)
        plan.check()
        for f in range(len(sizes)):
            compare_state(st.formula(f), ref[f], "mixed", f"tuned={tuned} f={f}")
        plan.free()
