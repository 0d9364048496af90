"""The host unit-propagation engine (hp_unit_propagate, C++) against the
oracle: bit-exact on random formulas, states and variance averages,
including padded clauses, repeated literals, tautologies and ties in nu."""
import numpy as np
import pytest

from oracle import up as U
from paper_2311_02101_amd import hp, workload as wl


def _cases():
    rng = np.random.default_rng(31)
    for trial in range(40):
        n = int(rng.integers(2, 200))
        T = wl.random_formula(max(n, 7), 200 + trial, ratio=int(rng.integers(2, 7)))
        n = max(n, 7)
        B = int(rng.integers(1, 6))
        v = rng.integers(0, 2, (B, n)).astype(np.uint8)
        nu = rng.random((B, n))
        if trial % 4 == 0:
            nu = np.round(nu * 4) / 4            # many ties in the priority order
        yield T, n, v, nu


def test_native_matches_oracle_random():
    for T, n, v, nu in _cases():
        got = hp.unit_propagate([T], [n], 0, v, nu, threads=3)
        for b in range(v.shape[0]):
            assert np.array_equal(got[b], U.prioritized_up(T, n, v[b], nu[b]))


def test_native_handles_repeats_tautologies_and_zero_padding():
    T = np.array([[1, 2, -3, 4, 0],
                  [1, -2, 3, 0, 0],
                  [-1, 2, 3, -4, 0]], np.int32)
    T[:, 4] = [2, 0, 0]                       # a unit clause written with zero padding
    rng = np.random.default_rng(2)
    for _ in range(30):
        v = rng.integers(0, 2, (3, 4)).astype(np.uint8)
        nu = rng.random((3, 4))
        got = hp.unit_propagate([T], [4], 0, v, nu)
        for b in range(3):
            assert np.array_equal(got[b], U.prioritized_up(T, 4, v[b], nu[b]))


def test_native_second_formula_of_a_batch_and_thread_counts():
    ts = [wl.random_formula(n, 40 + f, tag=f) for f, n in enumerate([30, 64, 17])]
    ns = [30, 64, 17]
    rng = np.random.default_rng(9)
    v = rng.integers(0, 2, (9, 64)).astype(np.uint8)
    nu = rng.random((9, 64))
    want = np.stack([U.prioritized_up(ts[1], 64, v[b], nu[b]) for b in range(9)])
    for threads in (0, 1, 4, 16):
        assert np.array_equal(hp.unit_propagate(ts, ns, 1, v, nu, threads=threads), want)


def test_native_rejects_bad_arguments():
    import ctypes as ct
    lib = hp.load()
    T = wl.random_formula(10, 1)
    lits = np.ascontiguousarray(T, dtype=np.int32)
    vo = np.array([0, 10], np.int64)
    co = np.array([0, T.shape[1]], np.int64)
    cnf = hp.HpCnf(1, hp._ptr(vo, ct.c_int64), hp._ptr(co, ct.c_int64), T.shape[0], hp._ptr(lits, ct.c_int32))
    v = np.zeros(10, np.uint8)
    nu = np.zeros(10)
    out = np.zeros(10, np.uint8)
    assert lib.hp_unit_propagate(ct.byref(cnf), 1, 1, v.ctypes.data, nu.ctypes.data, out.ctypes.data, 0) == hp.HP_EINVAL
    assert lib.hp_unit_propagate(ct.byref(cnf), 0, 1, None, nu.ctypes.data, out.ctypes.data, 0) == hp.HP_EINVAL
    assert lib.hp_unit_propagate(ct.byref(cnf), 0, 1, v.ctypes.data, nu.ctypes.data, out.ctypes.data, -1) == hp.HP_EINVAL
    bad = T.copy()
    bad[0, 0] = 11                             # literal beyond the variable count
    with pytest.raises(hp.HpError):
        hp.unit_propagate([bad], [10], 0, np.zeros((1, 10), np.uint8), np.zeros((1, 10)))
