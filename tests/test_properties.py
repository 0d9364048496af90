"""Property-based checks of the CPU oracle on tiny random formulas (Hypothesis).

Properties that hold for every formula, state and seed:
  * the satisfied-clause count equals plain clause evaluation, and does not
    change when the literals inside a clause are permuted or a clause is
    padded with copies of its first literal (Sec. 3.3);
  * after any number of sweeps: 0 <= s_max <= the brute-force optimum,
    s_max is the count of `best`, s_max never decreases, the assignment is
    binary and the variance average stays in (0, 0.25] (it starts at 0.25
    and moves towards rho (1 - rho) <= 1/4);
  * zero padding and padding by repetition give the same trajectory;
  * run(S1), run(0), run(S2) equals run(S1 + S2) for S2 >= 1 (a zero-sweep
    run counts the current state, which the next sweep counts first anyway).
"""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import rbmsat as R
from paper_2311_02101_amd import workload as wl

SETTINGS = dict(max_examples=60, deadline=None, derandomize=True,
                suppress_health_check=[HealthCheck.too_slow])


@st.composite
def tiny_formulas(draw, max_vars=7, max_clauses=9, max_k=5):
    n = draw(st.integers(1, max_vars))
    k = draw(st.integers(1, max_k))
    c = draw(st.integers(1, max_clauses))
    clauses = []
    for _ in range(c):
        ln = draw(st.integers(1, k))
        lits = draw(st.lists(st.integers(1, n), min_size=ln, max_size=ln))
        signs = draw(st.lists(st.sampled_from([1, -1]), min_size=ln, max_size=ln))
        clauses.append([s * v for s, v in zip(signs, lits)])
    return n, k, clauses


def _plain_count(clauses, v):
    return sum(any((v[abs(l) - 1] == 1) if l > 0 else (v[abs(l) - 1] == 0) for l in cl) for cl in clauses)


def _rbm(k, seed):
    L = 3 if k <= 3 else k + 1
    rng = np.random.default_rng(seed)
    return rng.standard_normal((2, k, L)), rng.standard_normal((2, L))


@settings(**SETTINGS)
@given(tiny_formulas(), st.integers(0, 2 ** 31 - 1), st.randoms(use_true_random=False))
def test_count_is_plain_clause_evaluation_and_order_free(f, seed, rnd):
    n, k, clauses = f
    T = wl.pad_clauses(clauses, k)
    W, b = _rbm(k, seed)
    p = R.plan(T, n, W, b)
    V = np.array([[(m >> i) & 1 for i in range(n)] for m in range(min(2 ** n, 64))], np.uint8)
    want = np.array([_plain_count(clauses, v) for v in V])
    assert np.array_equal(R.clause_count(V, p), want)
    perm = [rnd.sample(cl, len(cl)) for cl in clauses]
    p2 = R.plan(wl.pad_clauses(perm, k), n, W, b)
    assert np.array_equal(R.clause_count(V, p2), want)


@settings(**SETTINGS)
@given(tiny_formulas(), st.integers(0, 2 ** 31 - 1), st.integers(1, 4), st.integers(1, 12))
def test_sweep_invariants(f, seed, chains, sweeps):
    n, k, clauses = f
    T = wl.pad_clauses(clauses, k)
    W, b = _rbm(k, seed)
    p = R.plan(T, n, W, b)
    opt = R.brute_force_maxsat(T, n)
    st_ = R.initial(wl.initial_state(chains, n, seed % 1000))
    temps = wl.default_temperatures(chains, 2)
    prev = st_.s_max.copy()
    for _ in range(sweeps):
        R.sweep(st_, p, temps, alpha=0.05, seed=seed, formula_id=seed % 7)
        assert np.all(st_.s_max >= prev) and np.all(st_.s_max <= opt) and np.all(st_.s_max >= 0)
        prev = st_.s_max.copy()
        assert set(np.unique(st_.v)) <= {0, 1}
        assert np.all(st_.nu > 0.0) and np.all(st_.nu <= 0.25)
    assert np.array_equal(R.clause_count(st_.best, p), st_.s_max)


@settings(**SETTINGS)
@given(tiny_formulas(), st.integers(0, 2 ** 31 - 1), st.integers(0, 6), st.integers(1, 6))
def test_zero_padding_and_resume(f, seed, s1, s2):
    n, k, clauses = f
    T = wl.pad_clauses(clauses, k)
    Z = np.zeros_like(T)
    for j, cl in enumerate(clauses):
        Z[:len(cl), j] = cl                                  # short clauses end in zeros
    W, b = _rbm(k, seed)
    temps = wl.default_temperatures(3, 2)
    v0 = wl.initial_state(3, n, seed % 997)
    a = R.run(R.initial(v0), R.plan(T, n, W, b), temps, s1 + s2, alpha=0.01, seed=seed)
    # a zero-sweep run between the two only counts the state that the next
    # sweep counts first anyway (the count opens every sweep)
    z = R.run(R.initial(v0), R.plan(Z, n, W, b), temps, s1, alpha=0.01, seed=seed)
    R.run(z, R.plan(Z, n, W, b), temps, 0, alpha=0.01, seed=seed)
    R.run(z, R.plan(Z, n, W, b), temps, s2, alpha=0.01, seed=seed)
    for name in ("v", "nu", "s_max", "best"):
        assert np.array_equal(getattr(a, name), getattr(z, name)), name
    assert a.t == z.t == s1 + s2
