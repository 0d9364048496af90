"""Oracle for the prioritized unit-propagation heuristic and the top-B merge
(Sec. 3.4; the exchange in the appendix program).  Test infrastructure: only
tests/ and the measurement scripts' CPU legs use it.

Sec. 3.4 states the heuristic in outline (its details are in a cited paper):
variables are ranked by the moving average nu of their conditional variance;
the floor(N/2) variables with the highest nu are held at their sampled values,
the others are unassigned and recomputed by unit propagation, which extends a
partial assignment by the values its clauses imply.  Reading taken here:

  1. priority order: nu descending, ties by variable index ascending;
  2. the first floor(N/2) variables of that order take their sampled values;
  3. every clause is examined once, in clause order: a clause with no true
     literal and exactly one unassigned literal makes that literal true (the
     variable is assigned and queued); a clause with no true and no
     unassigned literal is a conflict and is left unsatisfied;
  4. propagation (FIFO): a variable taken from the queue has every clause
     holding its literal as false examined as in 3, in clause order;
  5. the remaining variables, in priority order: a variable still unassigned
     takes its sampled value, is queued and propagated as in 4.

A clause is the set of its distinct literals (padding copies and repeats
count once).

The merge follows the appendix program: the current states and the returned
ones are stacked (current first), counted, ordered by a stable ascending sort
of the counts, and the last B rows are kept (ties favour the returned
states); nu is stacked as [nu; nu], so a returned state takes the variance
average of the chain it replaces.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from .rbmsat import clause_count, normalize_table, plan


def clause_literals(T, n_vars):
    """Distinct literals (signed, 1-based) of every clause of a padded table."""
    T = normalize_table(np.asarray(T), n_vars)
    out = []
    for c in range(T.shape[1]):
        seen = []
        for lit in T[:, c]:
            lit = int(lit)
            if lit not in seen:
                seen.append(lit)
        out.append(seen)
    return out


def priority_order(nu):
    nu = np.asarray(nu, dtype=np.float64)
    return sorted(range(len(nu)), key=lambda i: (-nu[i], i))


def prioritized_up(T, n_vars, v, nu, stats=None):
    """New assignment of one chain (uint8 [N]) from its sample v and nu."""
    clauses = clause_literals(T, n_vars)
    occ = [[] for _ in range(n_vars)]            # clauses holding variable i
    for c, lits in enumerate(clauses):
        for lit in lits:
            occ[abs(lit) - 1].append(c)
    val = [None] * n_vars
    queue = deque()
    conflicts = 0

    def lit_value(lit):
        x = val[abs(lit) - 1]
        if x is None:
            return None
        return x if lit > 0 else 1 - x

    def assign(i, x):
        val[i] = x
        queue.append(i)

    def examine(c):
        nonlocal conflicts
        lits = clauses[c]
        values = [lit_value(lit) for lit in lits]
        if any(x == 1 for x in values):
            return
        free = [lit for lit, x in zip(lits, values) if x is None]
        if len(free) == 1:
            lit = free[0]
            assign(abs(lit) - 1, 1 if lit > 0 else 0)
        elif not free:
            conflicts += 1

    def propagate():
        while queue:
            i = queue.popleft()
            for c in occ[i]:
                # only clauses in which variable i's literal is now false
                if any(abs(lit) - 1 == i and lit_value(lit) == 0 for lit in clauses[c]):
                    examine(c)

    order = priority_order(nu)
    half = n_vars // 2
    v = np.asarray(v)
    for i in order[:half]:
        val[i] = int(v[i])
    for c in range(len(clauses)):
        examine(c)
    propagate()
    for i in order[half:]:
        if val[i] is None:
            assign(i, int(v[i]))
            propagate()
    if stats is not None:
        stats["conflicts"] = stats.get("conflicts", 0) + conflicts
    return np.array(val, dtype=np.uint8)


def merge_topb(T, n_vars, v, nu, v_up):
    """Stack [v; v_up], count, keep the last B rows of a stable ascending sort
    of the counts; nu rows follow [nu; nu].  Returns (v_new, nu_new)."""
    v = np.asarray(v)
    B = v.shape[0]
    stacked = np.vstack([v, np.asarray(v_up)])
    counts = clause_count(stacked.astype(np.uint8), plan(T, n_vars, np.zeros((T.shape[0], 1)), np.zeros(1)))
    ranks = np.argsort(counts, kind="stable")[-B:]
    nu2 = np.vstack([np.asarray(nu), np.asarray(nu)])
    return stacked[ranks], nu2[ranks]
