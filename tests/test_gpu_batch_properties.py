"""Property-based GPU parity on random batches (Hypothesis, derandomized).

The single-formula property test draws the formula; this one draws the batch
around it: 1..9 random formulas (Sec. 3's length mix, 7..2100 variables, so a
batch spans up to six size classes and both sides of the one-launch-per-class
grouping), 2..6 clauses per variable, 1..40 chains over two temperatures,
1..4 sweeps, the kernel family (auto, push, pull), the precision (FP64, FP32,
mixed BF16 on the push family), eager or captured in a hipGraph, and the
launch shapes as built or autotuned first.  Whatever the plan makes of it
(buckets, persistent grids, launch order), every formula ends in the oracle's
state for a drawn subset of its chains: v, s_max and best exactly, nu within
the precision's class; a mismatch must be a flagged tie under teacher-forced
replay, as in the other parity tests.  A second test crowds the batch (40..160
formulas of 7..600 variables, 16..64 chains) past the number of workgroups the
GPU holds at once, so the push launches run persistent grids that take their
items from per-XCD queues, and checks a drawn subset of formulas and the last
one.

Every example prints its batch and seed before touching the GPU."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import rbmsat as R
from paper_2311_02101_amd import workload as wl
from tests.parity import compare_state, f64_bounds, say, teacher_forced_sweep

pytestmark = pytest.mark.gpu

# kernel family x precision pairs the plan accepts (mixed BF16 runs the push
# family only)
MODES = [("auto", "f64"), ("push", "f64"), ("pull", "f64"),
         ("auto", "f32"), ("push", "f32"), ("pull", "f32"),
         ("auto", "mixed"), ("push", "mixed")]


@st.composite
def batches(draw):
    f = draw(st.integers(1, 9))
    # log-uniform-ish sizes: a class exponent, then a size inside it
    sizes = []
    for _ in range(f):
        c = draw(st.integers(0, 5))
        lo = 7 if c == 0 else 64 << (c - 1)
        sizes.append(draw(st.integers(lo, min(2100, (64 << c) - 1))))
    ratio = draw(st.integers(2, 6))
    chains = draw(st.integers(1, 40))
    picked = draw(st.lists(st.integers(0, chains - 1), min_size=1, max_size=4, unique=True))
    return sizes, ratio, chains, sorted(picked)


def _check_batch(sizes, ratio, B, chains, seed, sweeps, mode, graph, tune, formulas=None, label="batch"):
    """Plan, run and compare the listed formulas (all by default) on the
    listed chains with the oracle."""
    from paper_2311_02101_amd import hp
    kernel, prec = mode
    tables = [wl.random_formula(n, seed, ratio=ratio, tag=f) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    temps = wl.default_temperatures(B, W.shape[0])
    formulas = range(len(sizes)) if formulas is None else formulas
    say(f"[{label}] F={len(sizes)} N={sizes[:12]} ratio={ratio} B={B} chains={chains} "
        f"checked={list(formulas)[:12]} S={sweeps} {kernel} {prec} graph={graph} tune={tune} seed={seed}")
    plan = hp.Plan(tables, sizes, W, b, chains=B, temps=temps, precision=prec, seed=seed,
                   kernel=kernel, graph=graph)
    if tune:
        plan.tune(n_sweeps=2)
    info = plan.info()
    nb = info["n_buckets"]
    grids, kinds, items = info["bucket_grid"], info["bucket_kind"], info["bucket_items"]
    say(f"[{label}] buckets={nb} items={items} threads={info['bucket_threads']} grids={grids} "
        f"split={info['split']} forked={info['forked']}")
    # every (formula, chain) item in exactly one launch; a persistent grid is
    # smaller than its launch's items; several launches fork exactly when one
    # of them runs one workgroup per item; the kernel family is the one asked
    # for
    assert info["push_items"] + info["pull_items"] == len(sizes) * B
    if nb <= 16:
        assert sum(items) == len(sizes) * B
    assert all(g == 0 or 0 < g < n for g, n in zip(grids, items))
    assert info["forked"] == int(nb > 1 and any(g == 0 for g in grids))
    if info["split"] > 1:                       # one push launch, a workgroup per member
        assert nb == 1 and grids == [0] and kinds[0] != 2 and not graph
    if kernel == "pull":
        assert all(k == 2 for k in kinds)
    elif kernel == "push":
        assert all(k != 2 for k in kinds)
    tie, nu_rtol = f64_bounds(plan, tables) if prec in ("f64", "mixed") else (None, None)
    v0s = [wl.initial_state(B, n, seed % 1000, tag=f) for f, n in enumerate(sizes)]
    gst = plan.new_state(v0s)
    plan.run(gst, sweeps)
    import torch
    torch.cuda.synchronize()
    assert gst.get_t() == sweeps
    ch = np.asarray(chains)
    for f in formulas:
        n = sizes[f]
        op = R.plan(tables[f], n, W, b)
        ost = R.run(R.initial(v0s[f][ch]), op, temps[ch], sweeps, alpha=1e-3, seed=seed,
                    formula_id=f, chain_ids=ch)
        gv, gnu, gs, gbest = gst.formula(f)
        got = (gv[ch], gnu[ch], gs[ch], gbest[ch])
        try:
            compare_state(got, (ost.v, ost.nu, ost.s_max, ost.best), prec, f"{label} f={f}",
                          nu_rtol=nu_rtol)
        except AssertionError as err:
            say(f"[{label}] f={f}: mismatch ({err}); replaying with teacher forcing")
            s2 = plan.new_state(v0s)
            o2 = R.initial(v0s[f][ch])
            ties = sum(teacher_forced_sweep(plan, s2, f, o2, op, temps, alpha=1e-3, seed=seed,
                                            prec=prec, chain_ids=ch, tie=tie, nu_rtol=nu_rtol)
                       for _ in range(sweeps))
            assert ties > 0, "trajectory mismatch without any tie"
    plan.free()
    return info


@settings(max_examples=40, deadline=None, derandomize=True, suppress_health_check=list(HealthCheck))
@given(batches(), st.integers(0, 2 ** 31 - 1), st.integers(1, 4), st.sampled_from(MODES),
       st.booleans(), st.booleans())
def test_random_batches_match_oracle(hip, batch, seed, sweeps, mode, graph, tune):
    sizes, ratio, B, chains = batch
    _check_batch(sizes, ratio, B, chains, seed, sweeps, mode, graph, tune)


@st.composite
def crowded_batches(draw):
    """More (formula, chain) items than the GPU holds workgroups at once, so
    the push launches run persistent grids over their per-XCD queues."""
    f = draw(st.integers(40, 160))
    sizes = [draw(st.integers(7, 600)) for _ in range(f)]
    B = draw(st.integers(16, 64))
    picked = draw(st.lists(st.integers(0, B - 1), min_size=1, max_size=3, unique=True))
    checked = draw(st.lists(st.integers(0, f - 1), min_size=1, max_size=5, unique=True))
    return sizes, draw(st.integers(2, 6)), B, sorted(picked), sorted(checked)


@settings(max_examples=15, deadline=None, derandomize=True, suppress_health_check=list(HealthCheck))
@given(crowded_batches(), st.integers(0, 2 ** 31 - 1), st.integers(1, 3),
       st.sampled_from([m for m in MODES if m[0] != "pull"]), st.booleans(), st.booleans())
def test_crowded_batches_match_oracle(hip, batch, seed, sweeps, mode, graph, tune):
    sizes, ratio, B, chains, checked = batch
    # the last formula too: the tail of the last queue
    _check_batch(sizes, ratio, B, chains, seed, sweeps, mode, graph, tune,
                 formulas=sorted(set(checked) | {len(sizes) - 1}), label="crowded")
