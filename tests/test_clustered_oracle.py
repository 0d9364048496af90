"""Pins of the size-clustered formula-RBM oracle (Sec. 4): reduction to the
padded model when every clause has 7 literals, conditionals against the
enumerated joint energy of the clustered RBM, its stationary distribution,
and the pretrained free energy against the satisfied-clause count."""
import itertools

import numpy as np
import pytest

from oracle import clustered as CL
from oracle import rbmsat as R
from paper_2311_02101_amd import workload as wl


def _gauss_rbms(seed, T=1, scale=0.8):
    rng = np.random.default_rng(seed)
    return {K: (scale * rng.standard_normal((T, K, CL.hidden_units(K))),
                scale * rng.standard_normal((T, CL.hidden_units(K)))) for K in range(3, 8)}


def test_all_clauses_of_seven_literals_reduce_to_the_padded_model():
    n = 30
    T = wl.random_formula(n, 3, lengths=[7], probs=[1.0])
    rbms = _gauss_rbms(1, T=2)
    W, b = rbms[7]
    cp = CL.ClusteredPlan(T, n, rbms)
    p = R.plan(T, n, W, b)
    v0 = wl.initial_state(4, n, 3)
    a, c = R.initial(v0), R.initial(v0)
    temps = np.array([0, 1, 0, 1])
    for _ in range(15):
        CL.sweep(a, cp, temps, alpha=1e-3, seed=5)
        R.sweep(c, p, temps, alpha=1e-3, seed=5)
    assert np.array_equal(a.v, c.v) and np.array_equal(a.s_max, c.s_max) and np.array_equal(a.best, c.best)
    assert np.array_equal(a.nu, c.nu)


def _tiny():
    clauses = [[1], [-2, 3], [2, -4, 5], [-1, 3, 4, -5], [5, -3]]
    T = wl.pad_clauses(clauses, 7)
    return clauses, T, 5


def _joint_energy(clauses, rbms, v, hs):
    """E(v, h) = -sum_c [b^T h_c + lit_c^T W h_c] with each clause's RBM on
    its literal values (inputs padded to 3 by the first literal)."""
    E = 0.0
    for cl, h in zip(clauses, hs):
        K = max(len(cl), 3)
        lits = [(v[abs(l) - 1] if l > 0 else 1 - v[abs(l) - 1]) for l in cl]
        lits += [lits[0]] * (K - len(lits))
        W, b = rbms[K]
        E -= b[0] @ h + np.array(lits, float) @ W[0] @ h
    return E


def test_conditionals_match_the_enumerated_joint():
    clauses, T, n = _tiny()
    rbms = _gauss_rbms(2)
    cp = CL.ClusteredPlan(T, n, rbms)
    Ls = [CL.hidden_units(max(len(c), 3)) for c in clauses]
    rng = np.random.default_rng(3)
    for _ in range(6):
        v = rng.integers(0, 2, n)
        g, _ = R.literal_truth(v[None].astype(np.uint8), cp.full)
        ph = CL.hidden_probabilities(g, cp, 0)
        # group order: clauses of K = 3 (0, 1, 2, 4), then K = 4 (3)
        order = [c for Kg, Lg, cs, sp in cp.groups for c in cs]
        flat = np.concatenate([p[0].T.reshape(-1) for p in ph])
        pos = 0
        for c in order:
            for j in range(Ls[c]):
                # p(h_cj = 1 | v) from the energy: other hidden units cancel
                hs0 = [np.zeros(L) for L in Ls]
                hs1 = [np.zeros(L) for L in Ls]
                hs1[c][j] = 1
                d = _joint_energy(clauses, rbms, v, hs0) - _joint_energy(clauses, rbms, v, hs1)
                assert abs(flat[pos] - 1 / (1 + np.exp(-d))) < 1e-12
                pos += 1
        # visible logits for a random hidden state
        hs = [rng.integers(0, 2, L) for L in Ls]
        hg = [np.stack([hs[c] for c in cs], axis=1)[None] for Kg, Lg, cs, sp in cp.groups]
        x = CL.visible_logits(hg, cp, 0)[0]
        for i in range(n):
            v1, v0_ = v.copy(), v.copy()
            v1[i], v0_[i] = 1, 0
            want = _joint_energy(clauses, rbms, v0_, hs) - _joint_energy(clauses, rbms, v1, hs)
            assert abs(x[i] - want) < 1e-12


def test_free_energy_matches_hidden_enumeration():
    clauses, T, n = _tiny()
    rbms = _gauss_rbms(4)
    cp = CL.ClusteredPlan(T, n, rbms)
    Ls = [CL.hidden_units(max(len(c), 3)) for c in clauses]
    H = list(itertools.product(*[list(itertools.product([0, 1], repeat=L)) for L in Ls]))
    for v in ([0, 1, 0, 1, 1], [1, 1, 1, 0, 0]):
        Z = sum(np.exp(-_joint_energy(clauses, rbms, np.array(v), [np.array(h) for h in hh])) for hh in H)
        assert abs(CL.formula_free_energy(np.array(v), cp, 0)[0] + np.log(Z)) < 1e-9


@pytest.mark.slow
def test_stationary_distribution():
    clauses, T, n = _tiny()
    rbms = _gauss_rbms(5, scale=0.6)
    cp = CL.ClusteredPlan(T, n, rbms)
    V = ((np.arange(32)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)
    F = CL.formula_free_energy(V, cp, 0)
    pi = np.exp(-(F - F.min()))
    pi /= pi.sum()
    st = R.initial(wl.initial_state(256, n, 6))
    temps = np.zeros(256, np.int64)
    counts = np.zeros(32)
    code = 1 << np.arange(n)
    for it in range(1200):
        CL.sweep(st, cp, temps, alpha=1e-3, seed=11)
        if it >= 100:
            counts += np.bincount(st.v.astype(np.int64) @ code, minlength=32)
    assert 0.5 * np.abs(counts / counts.sum() - pi).sum() < 0.01


def test_pretrained_free_energy_tracks_the_count():
    n = 40
    T = wl.random_formula(n, 8)
    rbms, res = {}, {}
    for K in range(3, 8):
        W, b, r = wl.pretrained_rbm(K, wl.FSTAR_PAIR)
        rbms[K], res[K] = (W, b), r
    cp = CL.ClusteredPlan(T, n, rbms)
    V = np.random.default_rng(0).integers(0, 2, (20, n)).astype(np.uint8)
    s = R.clause_count(V, cp.full)
    for tau, fstar in enumerate(wl.FSTAR_PAIR):
        F = CL.formula_free_energy(V, cp, tau)
        bound = sum(len(cs) * res[Kg][tau] for Kg, Lg, cs, sp in cp.groups)
        assert np.abs(F + fstar * s).max() <= bound + 1e-9
