"""Pins of the unit-propagation and merge oracle (Sec. 3.4; the exchange of
the appendix program) against the paper's worked example, hand-derived
cases, an independent fixpoint implementation and plain-Python counting."""
import itertools

import numpy as np
import pytest

from oracle import up as U
from paper_2311_02101_amd import workload as wl
from tests.parity import golden_fields, golden_lines


def _table(clauses, k=3):
    return wl.pad_clauses(clauses, k)


def _eval(clauses, x):
    return sum(any((x[abs(l) - 1] == 1) == (l > 0) for l in c) for c in clauses)


def test_worked_example_sec3_4():
    name = "sec3_4_unit_propagation.txt"
    clauses = [[int(t) for t in part.split()] for part in golden_fields(name)["clauses"].split("|")]
    line = [ln for ln in golden_lines(name) if ln.startswith("up:")][0]
    left, res = line[3:].split("->")
    nu, v = [np.array([float(t) for t in part.split()]) for part in left.split("|")]
    got = U.prioritized_up(_table(clauses), 4, v.astype(np.uint8), nu)
    assert list(got) == [int(t) for t in res.split()]


def test_queue_order_and_clause_order():
    """Hand-derived.  Variables a, x, y, z, d = 1..5; a and d are held (highest
    nu) at False.  Clauses: 0 (not x or z), 1 (not y or not z), 2 (a or x),
    3 (a or y).  The first pass over the clauses makes x (clause 2) and then
    y (clause 3) true; the FIFO queue takes x first, so clause 0 makes z true
    and clause 1 is a conflict.  A LIFO queue would take y first and make z
    false instead."""
    clauses = [[-2, 4], [-3, -4], [1, 2], [1, 3]]
    nu = np.array([0.9, 0.3, 0.2, 0.1, 0.8])
    stats = {}
    got = U.prioritized_up(_table(clauses, 2), 5, np.zeros(5, np.uint8), nu, stats)
    assert list(got) == [0, 1, 1, 1, 0]
    assert stats["conflicts"] == 2          # clause 1, met from y and again from z


def _naive(clauses, n, v, nu):
    """Independent restatement: assign, then re-scan all clauses until no
    clause is unit; no conflict handling beyond skipping."""
    order = sorted(range(n), key=lambda i: (-nu[i], i))
    val = [None] * n

    def closure():
        changed = True
        while changed:
            changed = False
            for c in clauses:
                vals = [None if val[abs(l) - 1] is None else (val[abs(l) - 1] == (1 if l > 0 else 0)) for l in c]
                if any(x is True for x in vals):
                    continue
                free = [l for l, x in zip(c, vals) if x is None]
                if len(set(free)) == 1:
                    l = free[0]
                    val[abs(l) - 1] = 1 if l > 0 else 0
                    changed = True

    for i in order[:n // 2]:
        val[i] = int(v[i])
    closure()
    for i in order[n // 2:]:
        if val[i] is None:
            val[i] = int(v[i])
            closure()
    return np.array(val, dtype=np.uint8)


def test_conflict_free_runs_match_the_fixpoint_definition():
    """Without conflicts the propagation closure does not depend on the order
    of implications, so the FIFO procedure must equal a plain fixpoint."""
    rng = np.random.default_rng(5)
    checked = 0
    for trial in range(1000):
        n = int(rng.integers(4, 14))
        C = int(rng.integers(3, 2 * n))
        clauses = []
        for _ in range(C):
            k = int(rng.integers(1, 4))
            vs = rng.choice(n, size=min(k, n), replace=False) + 1
            clauses.append([int(x) * (1 if rng.random() < 0.5 else -1) for x in vs])
        v = rng.integers(0, 2, n).astype(np.uint8)
        nu = rng.random(n)
        stats = {}
        got = U.prioritized_up(_table(clauses), n, v, nu, stats)
        if stats.get("conflicts", 0) == 0:
            assert np.array_equal(got, _naive(clauses, n, v, nu)), trial
            checked += 1
    assert checked >= 150


def test_properties_on_random_formulas():
    rng = np.random.default_rng(6)
    for trial in range(60):
        n = 40
        T = wl.random_formula(n, 100 + trial, ratio=4)
        clauses = U.clause_literals(T, n)
        v = rng.integers(0, 2, n).astype(np.uint8)
        nu = rng.random(n)
        stats = {}
        got = U.prioritized_up(T, n, v, nu, stats)
        order = U.priority_order(nu)
        # held variables keep their sampled values
        assert all(got[i] == v[i] for i in order[:n // 2])
        # a variable moved away from its sample is the only true literal of some clause
        for i in np.nonzero(got != v)[0]:
            assert any(sum((got[abs(l) - 1] == 1) == (l > 0) for l in c) == 1 and
                       any(abs(l) - 1 == i and (got[i] == 1) == (l > 0) for l in c) for c in clauses)
        # every falsified clause was met as a conflict
        falsified = len(clauses) - _eval(clauses, got)
        assert falsified <= stats.get("conflicts", 0)


def test_all_variables_held_is_identity_for_n1_and_n2():
    # N = 2: one variable held; the other recomputed from a unit clause
    T = _table([[2], [1, 2]], 2)
    got = U.prioritized_up(T, 2, np.array([1, 0], np.uint8), np.array([0.5, 0.1]))
    assert list(got) == [1, 1]
    got = U.prioritized_up(_table([[1]], 1), 1, np.array([0], np.uint8), np.array([0.3]))
    assert list(got) == [1]            # N = 1: nothing held, the unit clause decides


def test_merge_keeps_the_best_rows_and_prefers_returned_states_on_ties():
    clauses = [[1], [2], [3], [-1, -2]]
    T = _table(clauses, 2)
    v = np.array([[1, 0, 1], [1, 1, 1], [0, 1, 1]], np.uint8)        # counts 3, 3, 3
    v_up = np.array([[1, 0, 1], [1, 1, 0], [0, 0, 0]], np.uint8)     # counts 3, 2, 1
    nu = np.array([[0.1] * 3, [0.2] * 3, [0.3] * 3])
    counts = [_eval(clauses, x) for x in np.vstack([v, v_up])]
    assert counts == [3, 3, 3, 3, 2, 1]
    vn, nun = U.merge_topb(T, 3, v, nu, v_up)
    # stable ascending order of the counts: rows 5, 4, 0, 1, 2, 3; the last
    # three keep the returned row 3 over the current row 0 (equal counts)
    assert np.array_equal(vn, np.vstack([v[1], v[2], v_up[0]]))
    assert np.allclose(nun, np.vstack([nu[1], nu[2], nu[0]]))


def test_planted_ascending_priority_is_caught(monkeypatch):
    monkeypatch.setattr(U, "priority_order", lambda nu: sorted(range(len(nu)), key=lambda i: (nu[i], i)))
    with pytest.raises(AssertionError):
        test_worked_example_sec3_4()


def test_planted_lifo_queue_is_caught(monkeypatch):
    import collections

    class Lifo(collections.deque):
        def popleft(self):
            return self.pop()

    monkeypatch.setattr(U, "deque", Lifo)
    with pytest.raises(AssertionError):
        test_queue_order_and_clause_order()
