"""Host-side input generation: synthetic formulas, DIMACS I/O, chain init."""
import numpy as np
import pytest

from paper_2311_02101_amd import workload as wl


def test_random_formula_shape_lengths_and_distinct_vars():
    T = wl.random_formula(4096, 1)
    K, C = T.shape
    assert (K, C) == (7, 6 * 4096)
    assert np.all(T != 0) and np.all(np.abs(T) <= 4096)
    # clause length = number of distinct literals (padding repeats the first)
    lens = np.array([len(set(T[:, c])) for c in range(0, C, 7)])
    assert set(np.unique(lens)) <= {2, 3, 4, 5, 6, 7}
    frac2 = np.mean(lens == 2)
    assert 0.45 < frac2 < 0.55
    # distinct variables inside each clause, padding repeats the first literal
    for c in range(0, C, 97):
        col = T[:, c]
        L = len(set(col))
        assert len(set(np.abs(col[:L]))) == L
        assert np.all(col[L:] == col[0])
    # polarities are balanced
    assert 0.45 < np.mean(T > 0) < 0.55


def test_generator_is_deterministic_and_seed_dependent():
    assert np.array_equal(wl.random_formula(256, 0), wl.random_formula(256, 0))
    assert not np.array_equal(wl.random_formula(256, 0), wl.random_formula(256, 1))
    assert np.array_equal(wl.initial_state(3, 50, 2), wl.initial_state(3, 50, 2))
    v = wl.initial_state(64, 4096, 1)
    assert v.dtype == np.uint8 and set(np.unique(v)) == {0, 1}
    assert abs(v.mean() - 0.5) < 0.01


def test_uneven_sizes_log_uniform():
    n = wl.uneven_sizes(1024, 3)
    assert n.min() >= 64 and n.max() <= 16384
    med = np.median(n)
    assert 700 < med < 1400          # geometric midpoint 1024


def test_dimacs_round_trip_and_errors():
    T = wl.random_formula(20, 4, ratio=2, k=7)
    n, clauses = wl.read_dimacs(wl.write_dimacs(20, T))
    assert n == 20 and np.array_equal(wl.pad_clauses(clauses, 7), T)
    n, cl = wl.read_dimacs("c hi\np cnf 4 2\n1 2 -3 4 0\n-1\n 2 0\n")
    assert cl == [[1, 2, -3, 4], [-1, 2]]
    with pytest.raises(ValueError):
        wl.read_dimacs("p wcnf 3 1\n1 2 0\n")
    with pytest.raises(ValueError):
        wl.read_dimacs("p cnf 2 1\n1 5 0\n")
    with pytest.raises(ValueError):
        wl.pad_clauses([[1, 2, 3, 4]], 3)


def test_temperature_split():
    assert list(wl.default_temperatures(4, 2)) == [0, 0, 1, 1]
    assert list(wl.default_temperatures(3, 2)) == [0, 0, 1]
    assert list(wl.default_temperatures(1, 1)) == [0]
    assert wl.hidden_units_for(3) == 3 and wl.hidden_units_for(7) == 8


def test_bench_work_model_of_the_clustered_model():
    """bench.py's ALU model for the size-clustered model: clause lengths as the
    oracle reads them, one Philox block and 3 draws for lengths <= 3, two
    blocks and len + 1 draws above, plus the visible groups."""
    import bench
    from oracle import clustered as CL
    n = 300
    T = wl.random_formula(n, 5, lengths=[1, 2, 3, 4, 7], probs=[0.2, 0.3, 0.2, 0.15, 0.15])
    lens = bench.clause_lengths(T)
    assert np.array_equal(lens, CL.clause_lengths(T, n))
    calls, draws, slots = bench.chain_sweep_work_clustered(n, T)
    big = lens > 3
    assert calls == int(np.sum(np.where(big, 2, 1))) + (n + 3) // 4
    assert draws == int(np.sum(np.where(big, lens + 1, 3))) + n
    assert slots == calls * bench.PHILOX_SLOTS + draws * bench.DRAW_SLOTS
    # the padded model: every clause draws L = 8 units from two blocks
    c2, d2, _ = bench.chain_sweep_work(n, T.shape[1], 8)
    assert c2 == 2 * T.shape[1] + (n + 3) // 4 and d2 == 8 * T.shape[1] + n


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and a
    message, before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
