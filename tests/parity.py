"""Shared helpers for the GPU-vs-oracle parity tests.

Tolerance classes (per result):
  integer  -- clause counts, s_max, best, and every sampled bit whose margin
              |U - p| exceeds the class bound: bit-exact.
  FP64     -- a sampled bit may differ only where |U - rho_oracle| is within
              the plan's tie bound (f64_bounds): the pull kernel sums the
              logit x in the oracle's order (bit-identical x; only exp may
              differ in the last place); the push kernel sums fixed-point
              terms rounded to 2^-S, |dx| <= slots * 2^-(S+1), so
              |d rho| <= 0.25 |dx| (S = 48 and at most 101 slots on the
              4096-variable workload: 5e-14); nu relative error within
              max(1e-13, 10 x tie).  Without a plan at hand the class's worst
              case over every admitted plan (S >= 40, 200 slots) applies:
              3e-11 and 1e-12.
  mixed    -- the FP64 class: hidden draws equal the FP64 rule (an FP32
              decision is replaced by the FP64 threshold whenever U is within
              16 * 2^-24 of p), contributions are 64-bit limb products
              rounded to the same fixed-point grid.
  FP32     -- nu relative error <= 1e-5; a sampled bit may differ only where
              |U - rho_oracle| <= 2e-6 (FP32 accumulation of at most ~100
              contributions of size <= ~10 gives |dx| <= 1e-4 * 2^-24 * 100,
              far below; the bound is dominated by the FP32 sigmoid).
"""
import os
import sys

import numpy as np

from oracle import rbmsat as R

TIE = {"f64": 3e-11, "f32": 2e-6, "mixed": 3e-11}
NU_RTOL = {"f64": 1e-12, "f32": 1e-5, "mixed": 1e-12}


def max_slots(tables):
    """Largest number of clause slots on one variable over the formulas
    (every entry of the [K][C] table counted: an upper bound of the slots
    that feed its fixed-point sum after the padding merge)."""
    out = 1
    for t in tables:
        out = max(out, int(np.bincount(np.abs(np.asarray(t)).ravel()).max()))
    return out


def f64_bounds(plan, tables):
    """Tie and nu bounds of the FP64 and mixed classes for this plan: the push
    kernels round every contribution to the grid 2^-S of the plan's
    fixed-point scale, so |dx| <= slots 2^-(S+1) and |d rho| <= |dx| / 4 (the
    sigmoid's slope is at most 1/4); 1e-15 covers the last-place difference
    of exp.  Over a run nu moves by alpha |d rho| per sweep at most, and stays
    above 0.15 for alpha S <= 0.5, so 1e-13 relative covers whole trajectories
    of the tested lengths."""
    S = plan.info()["fx_shift"]
    tie = 0.25 * max_slots(tables) * 2.0 ** -(S + 1) + 1e-15
    return tie, max(1e-13, 10 * tie)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_plan(table, n, W, b):
    return R.plan(table, n, W, b)


def compare_state(gpu, orc, prec, label="", nu_rtol=None):
    """gpu/orc: (v, nu, s_max, best) tuples of host arrays."""
    gv, gnu, gs, gb = gpu
    ov, onu, os_, ob = orc
    nu_rtol = NU_RTOL[prec] if nu_rtol is None else nu_rtol
    assert np.array_equal(gs, os_), f"{label}: s_max {gs} vs {os_}"
    assert np.array_equal(gb, ob), f"{label}: best differs at {np.argwhere(gb != ob)[:5]}"
    assert np.array_equal(gv, ov), f"{label}: v differs at {np.argwhere(gv != ov)[:5]}"
    rel = np.abs(gnu - onu) / np.maximum(np.abs(onu), 1e-300)
    assert rel.max() <= nu_rtol, f"{label}: nu rel err {rel.max():.3e}"


def teacher_forced_sweep(plan, state, f, ost, op, temps, *, alpha, seed, prec, chain_ids=None,
                         tie=None, nu_rtol=None):
    """Set the device state of formula f to the oracle state, run one sweep on
    both, and check the new v (ties allowed), nu, s_max and best.  Returns the
    number of flagged ties.  ``ost`` is advanced in place.  ``tie`` and
    ``nu_rtol`` default to the precision's class bounds."""
    tie = TIE[prec] if tie is None else tie
    nu_rtol = NU_RTOL[prec] if nu_rtol is None else nu_rtol
    return teacher_forced_batch(plan, state, {f: (ost, op, chain_ids)}, temps, alpha=alpha, seed=seed,
                                prec=prec, tie=tie, nu_rtol=nu_rtol)


def teacher_forced_batch(plan, state, cases, temps, *, alpha, seed, prec, tie=None, nu_rtol=None):
    """One teacher-forced sweep of several formulas of the plan at once.
    cases: {formula: (oracle state, oracle plan, chain ids or None)}; the
    oracle states hold the listed chains (all chains if None) and share one t.
    Every listed chain of every formula is set on the device, the plan runs
    one sweep (all formulas), and each is checked as in teacher_forced_sweep.
    Returns the total number of flagged ties; the oracle states advance."""
    tie = TIE[prec] if tie is None else tie
    nu_rtol = NU_RTOL[prec] if nu_rtol is None else nu_rtol
    temps = np.asarray(temps)
    ts = {ost.t for ost, _, _ in cases.values()}
    assert len(ts) == 1, "the formulas of one teacher-forced sweep share the sweep counter"
    for f, (ost, op, ch) in cases.items():
        state.set_formula(f, v=ost.v, nu=ost.nu, s_max=ost.s_max, best=ost.best, chains=ch)
    state.set_t(ts.pop())
    plan.run(state, 1)
    ties = 0
    for f, (ost, op, ch) in cases.items():
        gv, gnu, gs, gb = state.formula(f, chains=ch)
        tf = temps if ch is None else temps[np.asarray(ch)]
        rec = R.sweep(ost, op, tf, alpha=alpha, seed=seed, formula_id=f, chain_ids=ch, record=True)
        hid_margin = np.abs(rec["u_h"] - rec["p_h"]).min()
        assert hid_margin > TIE["f64"], f"f={f}: hidden-unit tie, comparison not decidable"
        assert np.array_equal(gs, ost.s_max) and np.array_equal(gb, ost.best), f"f={f}: s_max/best"
        diff = gv != ost.v
        n_diff = int(diff.sum())
        if n_diff:
            margin = np.abs(rec["u_v"] - rec["rho"])[diff]
            assert margin.max() <= tie, f"f={f}: non-tie visible mismatch, margin {margin.max():.3e}"
        rel = np.abs(gnu - ost.nu) / np.maximum(np.abs(ost.nu), 1e-300)
        assert rel.max() <= nu_rtol, f"f={f}: nu rel err {rel.max():.3e}"
        ties += n_diff
    # the trajectory continues from the oracle's states (teacher forcing)
    return ties


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_lines(name):
    """Non-comment lines of a fixture under tests/golden/."""
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.strip() for ln in fh if ln.strip() and not ln.lstrip().startswith("#")]


def golden_fields(name):
    """``key: values`` lines of a fixture as a dict of strings."""
    out = {}
    for ln in golden_lines(name):
        if ":" in ln and "->" not in ln:
            k, v = ln.split(":", 1)
            out[k.strip()] = v.strip()
    return out
