"""Pins of the replica-exchange oracle: the free energies against the dense
formula-RBM definition and brute-force enumeration of the hidden units, the
acceptance rule against exact probability ratios, the random-number layout
against Philox, and the joint stationary distribution of tempering plus
Gibbs sampling against the exact product of the temperatures' marginals."""
import itertools

import numpy as np
import pytest

from oracle import philox as PH
from oracle import rbmsat as R
from oracle import tempering as PT
from paper_2311_02101_amd import workload as wl


def _small(seed=3):
    T = wl.pad_clauses([[1, -2], [2, 3, -4], [-5, 1, 2], [4, -1], [3, 5]], 3)
    rng = np.random.default_rng(seed)
    W, b = 0.9 * rng.standard_normal((2, 3, 3)), 0.9 * rng.standard_normal((2, 3))
    return T, 5, W, b


def test_free_energy_matches_dense_definition_and_brute_force():
    T, n, W, b = _small()
    V = ((np.arange(32)[:, None] >> np.arange(5)[None, :]) & 1).astype(np.uint8)
    F = PT.clause_free_energies(T, n, W, b, V)
    p = R.plan(T, n, W, b)
    for tau in range(2):
        Wf, bf = R.dense_formula_rbm(p, tau)
        assert np.allclose(F[:, tau], R.free_energy(V.astype(float), Wf, bf), rtol=0, atol=1e-12)
        # brute force over all 2^(C L) = 2^15 hidden states for two inputs
        for row in (0, 21):
            H = ((np.arange(2 ** Wf.shape[1])[:, None] >> np.arange(Wf.shape[1])[None, :]) & 1)
            e = -(V[row].astype(float) @ Wf @ H.T + H @ bf)
            assert abs(F[row, tau] + np.log(np.exp(-e).sum())) < 1e-9


def test_acceptance_is_the_exact_probability_ratio():
    T, n, W, b = _small(4)
    V = ((np.arange(32)[:, None] >> np.arange(5)[None, :]) & 1).astype(np.uint8)
    F = PT.clause_free_energies(T, n, W, b, V)
    P = np.exp(-F)                                   # unnormalised p_tau(v)
    rng = np.random.default_rng(0)
    for _ in range(20):
        a, c = rng.integers(0, 32, 2)
        rec = []
        PT.swap_round([0, 1], F[[a, c]], 0, 7, 11, record=rec)
        ratio = (P[c, 0] * P[a, 1]) / (P[a, 0] * P[c, 1])
        assert abs(np.exp(rec[0][2]) - ratio) < 1e-9 * max(1.0, ratio)


def test_swap_uniform_layout():
    seed, f, t, a = 0x12345678_9abcdef0, 3, (5 << 32) + 17, 9
    key = (seed & 0xFFFFFFFF, ((seed >> 32) ^ f) & 0xFFFFFFFF)
    w = PH.philox4x32((17, 9, (1 << 31) - 1, 5), key)[0]
    assert PT.swap_uniform(seed, f, t, a) == (int(w) >> 8) / 2.0 ** 24


def test_pairing_and_parity():
    F = np.zeros((6, 3))                             # D = 0: every proposal accepted
    temps = [2, 0, 1, 0, 1, 2]
    assert list(PT.swap_round(temps, F, 0, 1, 5)) == [2, 1, 0, 1, 0, 2]     # (0,1) pairs: 1-2, 3-4
    assert list(PT.swap_round(temps, F, 1, 1, 5)) == [1, 0, 2, 0, 2, 1]     # (1,2) pairs: 2-0, 4-5


def _tv_tempering(swap=True, sweeps=1500, burn=100):
    """Two chains per temperature pair on the tiny formula; histogram of the
    states found at each temperature vs the exact p_tau."""
    T, n, W, b = _small(5)
    p = R.plan(T, n, W, b)
    V = ((np.arange(32)[:, None] >> np.arange(5)[None, :]) & 1).astype(np.uint8)
    F = PT.clause_free_energies(T, n, W, b, V)
    exact = [np.exp(-(F[:, t] - F[:, t].min())) for t in range(2)]
    exact = [e / e.sum() for e in exact]
    B = 128
    st = R.initial(wl.initial_state(B, n, 6))
    temps = np.array([i % 2 for i in range(B)])
    code = 1 << np.arange(n)
    hist = np.zeros((2, 32))
    for it in range(sweeps):
        R.sweep(st, p, temps, alpha=1e-3, seed=9)
        if swap:
            Fc = PT.clause_free_energies(T, n, W, b, st.v)
            temps = PT.swap_round(temps, Fc, it % 2, st.t, 9)
        if it >= burn:
            idx = st.v.astype(np.int64) @ code
            for t in range(2):
                hist[t] += np.bincount(idx[temps == t], minlength=32)
    return [0.5 * np.abs(hist[t] / hist[t].sum() - exact[t]).sum() for t in range(2)]


@pytest.mark.slow
def test_tempering_keeps_every_temperature_marginal():
    tv = _tv_tempering()
    assert max(tv) < 0.02, tv


def test_planted_sign_error_in_acceptance_is_caught(monkeypatch):
    orig = PT.swap_round

    def wrong(temps, F, parity, t, seed, formula_id=0, record=None):
        return orig(temps, -F, parity, t, seed, formula_id, record)

    monkeypatch.setattr(PT, "swap_round", wrong)
    with pytest.raises(AssertionError):
        test_acceptance_is_the_exact_probability_ratio()
