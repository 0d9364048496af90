"""Oracle for replica exchange (parallel tempering) across the ensemble of
free-energy targets.  Test infrastructure: only tests/ use it.

Chains sample the formula-RBM of their temperature tau, whose marginal over
the visible units is p_tau(v) ~ exp(-F_tau(v)) with F_tau the formula free
energy (eq. 5: the sum of the clause free energies, eq. 1, after the negation
transform of eq. 4).  A swap round proposes, for adjacent temperatures
(tau, tau + 1), to exchange the temperatures of two chains a (at tau) and b
(at tau + 1); the proposal keeps every p_tau invariant when accepted with
probability min(1, exp(D)),

    D = F_tau(v_a) + F_tau+1(v_b) - F_tau(v_b) - F_tau+1(v_a).

Reading taken here (the paper names tempering as an extension only):
  * rounds alternate between the pairs (tau, tau+1) with tau even (parity 0)
    and tau odd (parity 1);
  * inside a formula, the k-th chain (by chain index) at tau is paired with
    the k-th chain at tau + 1;
  * the acceptance draw of pair (a, b) is U = (w >> 8) 2^-24 with w word 0 of
    Philox4x32-10 at counter (t mod 2^32, a, 2^31 - 1, t div 2^32) and the
    sweep generator's key for the formula (a block index no sweep uses);
    the swap happens iff U < exp(min(D, 0)).
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32
from .rbmsat import free_energy, literal_truth, plan

SWAP_BLOCK = (1 << 31) - 1


def clause_free_energies(T, n_vars, W, b, v):
    """F_tau(v) for every chain and temperature: [B][T_count], as the sum over
    clauses (in clause order) of the clause free energy of the literal values."""
    W = np.asarray(W, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    p = plan(T, n_vars, W, b)
    lit = literal_truth(np.asarray(v, dtype=np.uint8), p)[1].astype(np.float64)   # [B][K][C]
    out = np.zeros((lit.shape[0], W.shape[0]))
    for tau in range(W.shape[0]):
        per_clause = free_energy(np.moveaxis(lit, 1, 2), W[tau], b[tau])   # [B][C]
        for c in range(per_clause.shape[1]):                              # clause order
            out[:, tau] += per_clause[:, c]
    return out


def swap_uniform(seed, formula_id, t, a):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    key = (seed & 0xFFFFFFFF, ((seed >> 32) ^ int(formula_id)) & 0xFFFFFFFF)
    w = philox4x32((t & 0xFFFFFFFF, int(a), SWAP_BLOCK, (t >> 32) & 0xFFFFFFFF), key)[0]
    return (int(w) >> 8) * 2.0 ** -24


def swap_round(temps, F, parity, t, seed, formula_id=0, record=None):
    """New temperatures of the chains of one formula.  temps: [B] ints,
    F: [B][T] free energies of the current states."""
    temps = np.array(temps, dtype=np.int64, copy=True)
    n_t = F.shape[1]
    old = temps.copy()
    for tau in range(parity, n_t - 1, 2):
        lo = [c for c in range(len(old)) if old[c] == tau]
        hi = [c for c in range(len(old)) if old[c] == tau + 1]
        for a, bb in zip(lo, hi):
            D = F[a, tau] + F[bb, tau + 1] - F[bb, tau] - F[a, tau + 1]
            u = swap_uniform(seed, formula_id, t, a)
            acc = u < np.exp(min(D, 0.0))
            if record is not None:
                record.append((a, bb, D, u, bool(acc)))
            if acc:
                temps[a], temps[bb] = tau + 1, tau
    return temps
