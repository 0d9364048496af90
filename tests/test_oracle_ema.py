"""Pins of the oracle's variance moving average (Sec. 3.4: the priority of a
variable in prioritized unit propagation is a moving average of the variance
of its visible conditional, rho (1 - rho); the appendix program starts it at
0.25 and updates it once per Gibbs round).

The pins tie the EMA to things other than its own line:
  * alpha = 0 leaves the appendix program's initial value 0.25 untouched;
  * alpha = 1 makes nu the Bernoulli variance rho (1 - rho) of the last
    visible draw, where rho is read off the *enumerated joint* p(v, h) of a
    tiny formula at the hidden state the chain drew (not the oracle's
    scatter-add);
  * over many chains that start from one state, the mean of nu (alpha = 1)
    is the expected Bernoulli variance E_h[rho (1 - rho)] under the exact
    p(h | v), and the empirical variance of the sampled values is that plus
    Var_h(rho) (law of total variance);
  * for 0 < alpha < 1, nu after S rounds is the unrolled geometric sum
    (1 - alpha)^S nu_0 + sum_s alpha (1 - alpha)^(S-1-s) rho_s (1 - rho_s)
    over the rho of every round.
Planted mistakes (alpha and 1 - alpha swapped; rho in place of rho (1 - rho))
must each fail one of them.
"""
import numpy as np
import pytest

from oracle import clustered as CL
from oracle import rbmsat as R
from paper_2311_02101_amd import workload as wl
from tests.test_oracle_pins import joint_log_weights

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

TINY_T = wl.pad_clauses([[1, -2, 3], [-1, 2], [3, -2]], 3)     # N = 3, C = 3, K = 3
TINY_N = 3


def _tiny_rbm():
    rng = np.random.default_rng(31)
    return 1.5 * rng.standard_normal((1, 3, 3)), rng.standard_normal((1, 3))


def _enumerated(W_c, b_c, v0):
    """p(h | v0) over all hidden states and p(v_i = 1 | h) for every h, from
    the joint p(v, h) of the formula-RBM enumerated over all states."""
    V, H, lw = joint_log_weights(TINY_T, TINY_N, W_c[0], b_c[0])
    row = int(np.nonzero((V == np.asarray(v0)[None]).all(axis=1))[0][0])
    ph = np.exp(lw[row] - lw[row].max())
    ph /= ph.sum()
    w = np.exp(lw - lw.max())
    rho_h = (w.T @ V) / w.sum(axis=0)[:, None]            # [2^(CL)][N]
    return ph, rho_h


def _hidden_index(h):
    """Enumeration index of recorded hidden states h [B][L][C]: unit (c, l)
    is bit c L + l (the column order of the dense formula-RBM)."""
    B, L, C = h.shape
    flat = np.transpose(h, (0, 2, 1)).reshape(B, C * L).astype(np.int64)
    return flat @ (1 << np.arange(C * L))


def test_alpha_zero_keeps_initial_value():
    W_c, b_c = _tiny_rbm()
    p = R.plan(TINY_T, TINY_N, W_c, b_c)
    st = R.initial(wl.initial_state(16, TINY_N, 3))
    R.run(st, p, np.zeros(16, np.int64), 12, alpha=0.0, seed=4)
    assert np.all(st.nu == 0.25)


def test_alpha_one_is_bernoulli_variance_of_enumerated_conditional():
    W_c, b_c = _tiny_rbm()
    p = R.plan(TINY_T, TINY_N, W_c, b_c)
    v0 = np.array([1, 0, 1], np.uint8)
    M = 512
    st = R.initial(np.tile(v0, (M, 1)))
    rec = R.sweep(st, p, np.zeros(M, np.int64), alpha=1.0, seed=11, record=True)
    _, rho_h = _enumerated(W_c, b_c, v0)
    rho = rho_h[_hidden_index(rec["h"])]                  # [M][N], the chain's own h
    np.testing.assert_allclose(st.nu, rho * (1 - rho), rtol=1e-12, atol=0)


def test_alpha_one_mean_over_chains_is_expected_bernoulli_variance():
    W_c, b_c = _tiny_rbm()
    p = R.plan(TINY_T, TINY_N, W_c, b_c)
    v0 = np.array([0, 1, 1], np.uint8)
    M = 40000
    st = R.initial(np.tile(v0, (M, 1)))
    R.sweep(st, p, np.zeros(M, np.int64), alpha=1.0, seed=23)
    ph, rho_h = _enumerated(W_c, b_c, v0)
    e_nu = ph @ (rho_h * (1 - rho_h))                     # E_h[rho (1 - rho)]
    e_rho = ph @ rho_h
    var_rho = ph @ (rho_h - e_rho) ** 2
    se_nu = st.nu.std(axis=0) / np.sqrt(M)
    assert np.all(np.abs(st.nu.mean(axis=0) - e_nu) < 5 * se_nu + 1e-12), (st.nu.mean(axis=0), e_nu)
    # the sampled values are Bernoulli(E[rho]): variance E[nu] + Var(rho)
    var_v = st.v.astype(np.float64).var(axis=0)
    se_var = np.sqrt(e_rho * (1 - e_rho) / M)             # loose bound on the sd of a variance estimate
    assert np.all(np.abs(var_v - (e_nu + var_rho)) < 5 * se_var)
    # not vacuous: the mean, E[rho], and the initial 0.25 are all far from E[nu]
    assert np.all(np.abs(e_rho - e_nu) > 50 * se_nu) and np.all(np.abs(e_nu - 0.25) > 50 * se_nu)


def _closed_form(nu0, rhos, alpha):
    S = len(rhos)
    out = (1 - alpha) ** S * nu0
    for s, rho in enumerate(rhos):
        out = out + alpha * (1 - alpha) ** (S - 1 - s) * rho * (1 - rho)
    return out


def test_unrolled_geometric_sum():
    n = 48
    T = wl.random_formula(n, 7)
    W, b = wl.gaussian_rbm(2, 7, 8, 7)
    p = R.plan(T, n, W, b)
    st = R.initial(wl.initial_state(6, n, 7))
    alpha, rhos = 0.3, []
    for _ in range(7):
        rhos.append(R.sweep(st, p, wl.default_temperatures(6, 2), alpha=alpha, seed=2, record=True)["rho"])
    np.testing.assert_allclose(st.nu, _closed_form(0.25, rhos, alpha), rtol=1e-13, atol=0)


def test_clustered_model_uses_the_same_average():
    n = 40
    T = wl.random_formula(n, 8)
    cp = CL.ClusteredPlan(T, n, wl.pretrained_size_rbms())
    st = R.initial(wl.initial_state(4, n, 8))
    alpha, rhos = 0.3, []
    for _ in range(5):
        rhos.append(CL.sweep(st, cp, wl.default_temperatures(4, 2), alpha=alpha, seed=3)["rho"])
    np.testing.assert_allclose(st.nu, _closed_form(0.25, rhos, alpha), rtol=1e-13, atol=0)


# ---------------------------------------------------------------------------
# Planted mistakes
# ---------------------------------------------------------------------------

def test_planted_swapped_rates_are_caught(monkeypatch):
    monkeypatch.setattr(R, "variance_ema", lambda nu, rho, alpha: alpha * nu + (1 - alpha) * rho * (1 - rho))
    with pytest.raises(AssertionError):
        test_alpha_zero_keeps_initial_value()
    with pytest.raises(AssertionError):
        test_unrolled_geometric_sum()
    with pytest.raises(AssertionError):
        test_alpha_one_is_bernoulli_variance_of_enumerated_conditional()
    with pytest.raises(AssertionError):
        test_clustered_model_uses_the_same_average()


def test_planted_mean_instead_of_variance_is_caught(monkeypatch):
    monkeypatch.setattr(R, "variance_ema", lambda nu, rho, alpha: (1 - alpha) * nu + alpha * rho)
    with pytest.raises(AssertionError):
        test_alpha_one_is_bernoulli_variance_of_enumerated_conditional()
    with pytest.raises(AssertionError):
        test_alpha_one_mean_over_chains_is_expected_bernoulli_variance()
