"""Replica exchange on the GPU (hp_temper) against the oracle: single rounds
on batches with 2 and 4 temperatures, and whole runs that alternate sweeps
and rounds."""
import numpy as np
import pytest

from oracle import rbmsat as R
from oracle import tempering as PT
from paper_2311_02101_amd import hp, workload as wl
from tests.parity import say

pytestmark = pytest.mark.gpu

TIE = 1e-9


def _sync():
    import torch
    torch.cuda.synchronize()


def _check_round(plan, st, tables, sizes, W, b, parity, seed):
    temps0 = plan.current_temps()
    t = st.get_t()
    plan.temper(st, parity)
    _sync()
    got = plan.current_temps()
    ties = 0
    for f, n in enumerate(sizes):
        v = st.formula(f)[0]
        F = PT.clause_free_energies(tables[f], n, W, b, v)
        rec = []
        want = PT.swap_round(temps0[f], F, parity, t, seed, f, rec)
        # the pairs of a round are disjoint: a near-tie acceptance draw leaves
        # only its own two chains undecided (either outcome is correct there,
        # as long as the pair keeps its two temperatures); every other chain
        # is compared exactly
        undecided = np.zeros(len(want), bool)
        for a, bb, D, u, _ in rec:
            if abs(u - np.exp(min(D, 0.0))) < TIE:
                undecided[[a, bb]] = True
                assert sorted((got[f][a], got[f][bb])) == sorted((temps0[f][a], temps0[f][bb])), (f, a, bb)
                ties += 1
        assert np.array_equal(got[f][~undecided], want[~undecided]), (f, rec)
    return ties


@pytest.mark.parametrize("n_temps", [2, 4])
def test_round_matches_oracle(hip, n_temps):
    sizes = [50, 200, 31]
    tables = [wl.random_formula(n, 7, tag=f) for f, n in enumerate(sizes)]
    if n_temps == 2:
        W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    else:
        W, b = wl.gaussian_rbm(4, 7, 8, 7)
        W, b = 0.3 * W, 0.3 * b
    B = 12
    temps = np.array([i % n_temps for i in range(B)], np.int32)
    plan = hp.Plan(tables, sizes, W, b, chains=B, temps=temps, precision="f64", seed=7)
    st = plan.new_state([wl.initial_state(B, n, 7, tag=f) for f, n in enumerate(sizes)])
    say(f"[temper] T={n_temps} B={B}")
    for r in range(6):
        plan.run(st, 3)
        _sync()
        _check_round(plan, st, tables, sizes, W, b, r % 2, 7)
    assert np.array_equal(np.sort(plan.current_temps(), axis=1), np.sort(np.tile(temps, (3, 1)), axis=1))
    plan.free()


def test_alternating_run_matches_oracle(hip):
    n = 60
    T = wl.random_formula(n, 8)
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    B = 8
    temps = np.array([0, 1] * 4, np.int32)
    v0 = wl.initial_state(B, n, 8)
    plan = hp.Plan([T], [n], W, b, chains=B, temps=temps, precision="f64", seed=8)
    st = plan.new_state([v0])
    op = R.plan(T, n, W, b)
    ost = R.initial(v0)
    otemps = temps.astype(np.int64)
    say("[temper run] 30 rounds of 2 sweeps + exchange")
    for r in range(30):
        plan.run(st, 2)
        plan.temper(st, r % 2)
        R.run(ost, op, otemps, 2, alpha=1e-3, seed=8, formula_id=0, chain_ids=np.arange(B))
        F = PT.clause_free_energies(T, n, W, b, ost.v)
        rec = []
        otemps = PT.swap_round(otemps, F, r % 2, ost.t, 8, 0, rec)
        assert all(abs(x[3] - np.exp(min(x[2], 0.0))) > TIE for x in rec)
    _sync()
    v, nu, s_max, best = st.formula(0)
    assert np.array_equal(v, ost.v) and np.array_equal(s_max, ost.s_max) and np.array_equal(best, ost.best)
    assert np.max(np.abs(nu - ost.nu) / ost.nu) < 1e-12
    assert np.array_equal(plan.current_temps()[0], otemps)
    plan.free()
