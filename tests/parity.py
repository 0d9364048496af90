"""Shared helpers for the GPU-vs-oracle parity tests.

Tolerance classes (per result):
  integer  -- clause counts, s_max, best, and every sampled bit whose margin
              |U - p| exceeds the class bound: bit-exact.
  FP64     -- nu relative error <= 1e-12; a sampled bit may differ only where
              |U - rho_oracle| <= 3e-11 (a flagged tie).  The pull kernel sums
              the logit x in the oracle's order (bit-identical x; only exp may
              differ in the last place); the push kernel sums fixed-point
              terms rounded to 2^-S with S >= 40, |dx| <= slots * 2^-(S+1)
              <= 1e-10 even for 200 slots, so |d rho| <= 0.25 |dx|.
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_plan(table, n, W, b):
    return R.plan(table, n, W, b)


def compare_state(gpu, orc, prec, label=""):
    """gpu/orc: (v, nu, s_max, best) tuples of host arrays."""
    gv, gnu, gs, gb = gpu
    ov, onu, os_, ob = orc
    assert np.array_equal(gs, os_), f"{label}: s_max {gs} vs {os_}"
    assert np.array_equal(gb, ob), f"{label}: best differs at {np.argwhere(gb != ob)[:5]}"
    assert np.array_equal(gv, ov), f"{label}: v differs at {np.argwhere(gv != ov)[:5]}"
    rel = np.abs(gnu - onu) / np.maximum(np.abs(onu), 1e-300)
    assert rel.max() <= NU_RTOL[prec], f"{label}: nu rel err {rel.max():.3e}"


def teacher_forced_sweep(plan, state, f, ost, op, temps, *, alpha, seed, prec, chain_ids=None):
    """Set the device state of formula f to the oracle state, run one sweep on
    both, and check the new v (ties allowed), nu, s_max and best.  Returns the
    number of flagged ties.  ``ost`` is advanced in place."""
    state.set_formula(f, v=ost.v, nu=ost.nu, s_max=ost.s_max, best=ost.best)
    state.set_t(ost.t)
    plan.run(state, 1)
    gv, gnu, gs, gb = state.formula(f)
    rec = R.sweep(ost, op, temps, alpha=alpha, seed=seed, formula_id=f,
                  chain_ids=chain_ids, record=True)
    hid_margin = np.abs(rec["u_h"] - rec["p_h"]).min()
    assert hid_margin > TIE["f64"], "hidden-unit tie: comparison not decidable"
    assert np.array_equal(gs, ost.s_max) and np.array_equal(gb, ost.best)
    diff = gv != ost.v
    ties = int(diff.sum())
    if ties:
        margin = np.abs(rec["u_v"] - rec["rho"])[diff]
        assert margin.max() <= TIE[prec], f"non-tie visible mismatch, margin {margin.max():.3e}"
    rel = np.abs(gnu - ost.nu) / np.maximum(np.abs(ost.nu), 1e-300)
    assert rel.max() <= NU_RTOL[prec], f"nu rel err {rel.max():.3e}"
    # continue the trajectory from the oracle's state (teacher forcing)
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
