"""Oracle for the size-clustered formula-RBM (Sec. 4): clauses grouped by
their length, every group with the canonical OR-gate RBM of its own size,
the groups coupled by summing their contributions to the visible logits.
Test infrastructure: only tests/ use it.

Reading taken here (Sec. 4 states the idea in one sentence; the hidden-unit
count is given for K >= 3 only):
  * the length l of a clause is its column of the padded table without the
    trailing copies of its first literal (1 <= l <= K);
  * lengths 1..3 use the K = 3 RBM (L = 3), their inputs padded to 3 by
    repeating the first literal; a length l >= 4 uses the K = l RBM with
    L = l + 1 hidden units;
  * hidden unit j of clause c draws word j mod 4 of Philox block 2c + j div 4
    (phase 0): the stride of two blocks per clause of the padded model with
    L = 8, so a formula whose clauses all have 7 literals gives the padded
    model's samples exactly;
  * everything else (count, best, visible conditional, EMA, draws) is the
    padded model's (rbmsat.sweep).
"""
from __future__ import annotations

import numpy as np

from . import rbmsat as _rbmsat
from .rbmsat import (HIDDEN, State, contributions, hidden_logits, literal_truth, normalize_table, plan,
                     scatter_add, sigmoid, uniforms, visible_uniforms)


def hidden_units(K):
    return 3 if K == 3 else K + 1


def clause_lengths(T, n_vars):
    T = normalize_table(np.asarray(T), n_vars)
    K, C = T.shape
    out = np.empty(C, np.int64)
    for c in range(C):
        l = K
        while l > 1 and T[l - 1, c] == T[0, c]:
            l -= 1
        out[c] = l
    return out


class ClusteredPlan:
    """full: plan of the padded table (gather, count, scatter indices);
    groups: list of (K, L, clause indices, plan of rows 0..K-1 of those
    clauses with the K-input RBMs)."""

    def __init__(self, T, n_vars, rbms):
        T = normalize_table(np.asarray(T), n_vars)
        self.n_vars = n_vars
        K = T.shape[0]
        self.full = plan(T, n_vars, np.zeros((1, K, 1)), np.zeros((1, 1)))
        lens = clause_lengths(T, n_vars)
        self.groups = []
        for Kg in (3, 4, 5, 6, 7):
            cs = np.nonzero(np.maximum(lens, 3) == Kg)[0]
            if len(cs) == 0:
                continue
            if Kg > K:
                raise ValueError("clause longer than the table width")
            W, b = rbms[Kg]
            sub = np.ascontiguousarray(T[:Kg, cs])
            self.groups.append((Kg, hidden_units(Kg), cs, plan(sub, n_vars, W, b)))


def hidden_probabilities(g, cp: ClusteredPlan, tau):
    """p(h = 1 | v) of every group, [B][L_g][C_g] each, from the gathered
    values g [B][K][C] of the padded table (eqs. 2, 6 with each clause's RBM)."""
    out = []
    for Kg, Lg, cs, sp in cp.groups:
        gs = g[:, :Kg, :][:, :, cs].astype(np.float64)
        out.append(sigmoid(hidden_logits(gs, sp, int(tau))))
    return out


def visible_logits(h_groups, cp: ClusteredPlan, tau):
    """x [B][N]: every group's contributions (l^(c) = W^(c) h^(c)) summed per
    variable in ascending (clause, slot) order (eq. 7, d = 0)."""
    pf = cp.full
    B = h_groups[0].shape[0]
    ell = np.zeros((B, pf.K, pf.C))
    for (Kg, Lg, cs, sp), h in zip(cp.groups, h_groups):
        ell[:, :Kg, cs] = contributions(h.astype(np.float64), sp, int(tau))
    return scatter_add(ell, pf)             # unused slots add 0.0


def sweep(st: State, cp: ClusteredPlan, temps, *, alpha: float, seed: int, formula_id: int = 0,
          chain_ids=None):
    B = st.v.shape[0]
    temps = np.asarray(temps, dtype=np.int64)
    chain_ids = np.arange(B) if chain_ids is None else np.asarray(chain_ids, np.int64)
    t = st.t
    pf = cp.full
    g, lit = literal_truth(st.v, pf)
    s = lit.any(axis=1).sum(axis=1).astype(np.int64)
    better = s > st.s_max
    st.s_max = np.where(better, s, st.s_max)
    st.best[better] = st.v[better]
    u8 = uniforms(seed, formula_id, t, chain_ids, HIDDEN, pf.C, 8)      # [B][C][8], blocks 2c, 2c+1
    x = np.zeros((B, pf.n_vars))
    hid_margin = np.inf
    for tau in np.unique(temps):
        sel = np.nonzero(temps == tau)[0]
        ph = hidden_probabilities(g[sel], cp, tau)
        us = [np.transpose(u8[sel][:, cs, :Lg], (0, 2, 1)) for (Kg, Lg, cs, sp) in cp.groups]
        hs = [(u < p).astype(np.float64) for u, p in zip(us, ph)]
        hid_margin = min([hid_margin] + [float(np.abs(u - p).min()) for u, p in zip(us, ph)])
        x[sel] = visible_logits(hs, cp, tau)
    rho = sigmoid(x)
    st.nu = _rbmsat.variance_ema(st.nu, rho, alpha)
    u_v = visible_uniforms(seed, formula_id, t, chain_ids, pf.n_vars)
    st.v = (u_v < rho).astype(np.uint8)
    st.t = t + 1
    return dict(x=x, rho=rho, u_v=u_v, hid_margin=hid_margin)


def run(st: State, cp: ClusteredPlan, temps, n_sweeps, *, alpha, seed, formula_id=0, chain_ids=None):
    for _ in range(n_sweeps):
        sweep(st, cp, temps, alpha=alpha, seed=seed, formula_id=formula_id, chain_ids=chain_ids)
    return st


def formula_free_energy(v, cp: ClusteredPlan, tau):
    """F(v) = sum over clauses of the free energy (eq. 1) of the clause's own
    RBM after the negation transform, on the raw values: the visible
    marginal of the clustered formula-RBM is p(v) ~ exp(-F(v))."""
    from .rbmsat import free_energy
    v = np.atleast_2d(np.asarray(v, dtype=np.uint8))
    out = np.zeros(v.shape[0])
    for Kg, Lg, cs, sp in cp.groups:
        gv = literal_truth(v, sp)[0].astype(np.float64)                     # [B][K_g][C_g]
        for j in range(len(cs)):
            out += free_energy(gv[:, :, j], sp.W[tau][:, :, j], sp.b[tau][:, j])
    return out
