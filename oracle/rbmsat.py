"""Plain CPU FP64 oracle of the RbmSAT block-Gibbs sweep.

Part of the test oracle (see ``oracle/__init__``): not used by the product
path, shares no code with it.

Everything here follows the paper's equations and the order of operations of
its appendix program (Fig. "A simplified implementation of RbmSAT"), in FP64
NumPy, vectorised over chains and clauses but with every reduction written as
an explicit ascending loop so its rounding order is visible:

  plan       -- polarity = sign T, idx = |T| - 1, negation transform (eq. 4)
                W[k,l,c] = pol_kc W_c[k,l],
                b[l,c]   = b_c[l] + sum_k W_c[k,l] (1 - pol_kc)/2.
  sweep      -- one Gibbs round in the appendix program's order:
                gather, clause count (OR of true literals), best tracking,
                hidden conditional (eqs. 2, 6) and Bernoulli draw,
                per-clause contributions l = W_f^(c) h^(c) (Sec. 3.1 "Gibbs
                sampling in a formula-RBM"), scatter-add (eq. 7, d = 0),
                visible conditional (eq. 3), variance EMA (Sec. 3.4) and
                Bernoulli draw.

Readings where the text is silent or inconsistent:
  * clause count: a literal is true iff (pol > 0) == v; the program's product
    "(polarity > 0) * c" would miss satisfied negated literals, whereas the
    text describes comparing thresholded signs with the values and OR-ing.
  * zero entries of T (Sec. 3.1 padding) are replaced by the clause's first
    non-zero literal (Sec. 3.3 pads by repetition with the same polarity).
  * visible bias d = 0 (Sec. 3.1 states that the formula-RBM needs none).
  * best assignment: replaced only on a strict improvement s > s_max.
  * randomness: U(t, b, phase, j) from Philox4x32-10 (see ``uniforms``);
    a draw is 1 iff U < p (the Bernoulli semantics of the program).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .philox import philox4x32

HIDDEN, VISIBLE = 0, 1
TWO_M24 = 2.0 ** -24


# ---------------------------------------------------------------------------
# Eq. 1: RBM free energy (pins only; the sweep never evaluates it)
# ---------------------------------------------------------------------------

def free_energy(v, W, b, d=None):
    """F(v) = -d^T v - sum_j log(1 + exp(b_j + sum_k W_kj v_k))   (eq. 1).

    v: [..., K] binary, W: [K, L], b: [L], d: [K] or None (= 0)."""
    v = np.asarray(v, dtype=np.float64)
    z = v @ W + b
    f = -np.sum(np.logaddexp(0.0, z), axis=-1)
    if d is not None:
        f = f - v @ d
    return f


def sigmoid(z):
    """Logistic function sigma(z) = 1 / (1 + exp(-z)) (Sec. 2.1)."""
    return 1.0 / (1.0 + np.exp(-z))


# ---------------------------------------------------------------------------
# Plan: padding normalisation, negation transform, formula assembly
# ---------------------------------------------------------------------------

def normalize_table(T, n_vars: int) -> np.ndarray:
    """Return a copy of the signed 1-based [K][C] table with zero entries
    replaced by the clause's first non-zero literal.  Raises ValueError on an
    all-zero clause or a literal outside [-n_vars, n_vars]."""
    T = np.array(T, dtype=np.int64, copy=True)
    if T.ndim != 2:
        raise ValueError("T must be [K][C]")
    if np.any(np.abs(T) > n_vars):
        raise ValueError("literal index exceeds n_vars")
    K, C = T.shape
    for c in range(C):
        col = T[:, c]
        nz = col[col != 0]
        if nz.size == 0:
            raise ValueError(f"clause {c} has no literal")
        col[col == 0] = nz[0]
    return T


@dataclass
class Plan:
    n_vars: int
    pol: np.ndarray     # [K][C] in {-1, +1}
    idx: np.ndarray     # [K][C] 0-based variable index
    W: np.ndarray       # [T][K][L][C] per-clause weights (eq. 4)
    b: np.ndarray       # [T][L][C]    per-clause hidden biases (eq. 4)

    @property
    def K(self):
        return self.pol.shape[0]

    @property
    def C(self):
        return self.pol.shape[1]

    @property
    def L(self):
        return self.W.shape[2]


def plan(T, n_vars: int, W_c, b_c) -> Plan:
    """Formula-RBM assembly (Sec. 3.1) with the negation transform (eq. 4).

    T: [K][C] signed 1-based literals; W_c: [n_temps][K][L]; b_c: [n_temps][L].
    For clause c with Lambda = diag(pol_{.,c}):
        W^(c) = Lambda W_c,   b^(c) = b_c + 1/2 (1 - diag Lambda) W_c
    where the second term sums over the clause inputs k in ascending order."""
    T = normalize_table(T, n_vars)
    W_c = np.asarray(W_c, dtype=np.float64)
    b_c = np.asarray(b_c, dtype=np.float64)
    if W_c.ndim == 2:
        W_c, b_c = W_c[None], b_c[None]
    K, C = T.shape
    if W_c.shape[1] != K:
        raise ValueError("W_c must be [n_temps][K][L]")
    pol = np.sign(T).astype(np.int64)
    idx = np.abs(T) - 1
    n_t, _, L = W_c.shape
    W = np.empty((n_t, K, L, C))
    b = np.empty((n_t, L, C))
    for t in range(n_t):
        W[t] = pol[:, None, :] * W_c[t][:, :, None]
        acc = np.repeat(b_c[t][:, None], C, axis=1)
        for k in range(K):
            acc = acc + W_c[t][k][:, None] * ((1 - pol[k]) / 2.0)[None, :]
        b[t] = acc
    return Plan(n_vars, pol, idx, W, b)


# ---------------------------------------------------------------------------
# Clause count (gather + OR + sum)
# ---------------------------------------------------------------------------

def literal_truth(v, p: Plan):
    """g[b,k,c] = v[b, idx_kc]; literal true iff g == [pol_kc > 0]."""
    g = np.asarray(v)[:, p.idx]                       # [B][K][C]
    return g, (g == (p.pol > 0)[None])


def clause_count(v, p: Plan):
    """Number of satisfied clauses per chain: sum_c OR_k lit[b,k,c]."""
    _, lit = literal_truth(v, p)
    return lit.any(axis=1).sum(axis=1).astype(np.int64)


def brute_force_maxsat(T, n_vars: int) -> int:
    """Maximum number of simultaneously satisfiable clauses, by enumerating
    every assignment (tiny n_vars only)."""
    T = normalize_table(T, n_vars)
    m = np.arange(2 ** n_vars)
    V = ((m[:, None] >> np.arange(n_vars)[None, :]) & 1).astype(np.uint8)
    pol = np.sign(T)
    idx = np.abs(T) - 1
    sat = (V[:, idx] == (pol > 0)[None]).any(axis=1).sum(axis=1)
    return int(sat.max())


# ---------------------------------------------------------------------------
# Counter-based uniforms
# ---------------------------------------------------------------------------

def _key(seed: int, formula_id: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, ((seed >> 32) ^ int(formula_id)) & 0xFFFFFFFF)


def uniforms(seed: int, formula_id: int, t: int, chains, phase: int, n_groups: int,
             per_group: int):
    """U(t, b, phase, j) for j = (group, r), r < per_group.

    Draws of one group (one clause's hidden units, or 4 consecutive visible
    units) come from consecutive Philox blocks: block = group * ceil(per_group/4)
    + r // 4, word r % 4.  Counter = (t mod 2^32, chain, phase*2^31 + block,
    t div 2^32); key = (seed mod 2^32, (seed div 2^32) xor formula_id).
    U = (word >> 8) * 2^-24 in [0, 1 - 2^-24].

    Returns float64 [len(chains)][n_groups][per_group]."""
    chains = np.atleast_1d(np.asarray(chains, dtype=np.int64))
    nb = -(-per_group // 4)
    block = np.arange(n_groups * nb, dtype=np.uint64).reshape(n_groups, nb)   # [G][nb]
    ctr = (np.uint64(t & 0xFFFFFFFF),
           chains[:, None, None].astype(np.uint64),
           (np.uint64(phase) << np.uint64(31)) | block[None],
           np.uint64((t >> 32) & 0xFFFFFFFF))
    words = philox4x32(ctr, _key(seed, formula_id))                          # [B][G][nb][4]
    w = words.reshape(len(chains), n_groups, nb * 4)[:, :, :per_group]       # word r of group
    return (w >> np.uint64(8)).astype(np.float64) * TWO_M24


def hidden_uniforms(seed, formula_id, t, chains, C, L):
    """U_h[b, l, c] for the L hidden units of every clause."""
    u = uniforms(seed, formula_id, t, chains, HIDDEN, C, L)                   # [B][C][L]
    return np.transpose(u, (0, 2, 1))


def visible_uniforms(seed, formula_id, t, chains, N):
    """U_v[b, i] for the N visible units (4 consecutive units per block)."""
    g = -(-N // 4)
    u = uniforms(seed, formula_id, t, chains, VISIBLE, g, 4)                  # [B][G][4]
    return u.reshape(len(np.atleast_1d(chains)), g * 4)[:, :N]


# ---------------------------------------------------------------------------
# One Gibbs sweep
# ---------------------------------------------------------------------------

@dataclass
class State:
    v: np.ndarray       # [B][N] uint8
    nu: np.ndarray      # [B][N] float64
    s_max: np.ndarray   # [B] int64
    best: np.ndarray    # [B][N] uint8
    t: int

    def copy(self):
        return State(self.v.copy(), self.nu.copy(), self.s_max.copy(),
                     self.best.copy(), int(self.t))


def initial(v0) -> State:
    """Initial chain state: v = v0, nu = 0.25, s_max = 0, best = v0, t = 0
    (the appendix program initialises nu to 0.25 and s_max to 0)."""
    v0 = np.asarray(v0, dtype=np.uint8)
    return State(v0.copy(), np.full(v0.shape, 0.25), np.zeros(v0.shape[0], np.int64),
                 v0.copy(), 0)


def hidden_logits(g, p: Plan, tau: int):
    """z[b,l,c] = b[l,c] + sum_{k ascending} g[b,k,c] W[k,l,c]   (eqs. 2, 6)."""
    z = np.broadcast_to(p.b[tau][None], (g.shape[0], p.L, p.C)).copy()
    for k in range(p.K):
        z = z + g[:, k, None, :] * p.W[tau][k][None]
    return z


def contributions(h, p: Plan, tau: int):
    """l[b,k,c] = sum_{l ascending} W[k,l,c] h[b,l,c]  (l^(c) = W_f^(c) h^(c))."""
    ell = np.zeros((h.shape[0], p.K, p.C))
    for l in range(p.L):
        ell = ell + p.W[tau][:, l, :][None] * h[:, l, None, :]
    return ell


def scatter_add(ell, p: Plan):
    """x[b,i] = sum over clause slots (c ascending, then k ascending) with
    idx_kc = i of l[b,k,c]   (eq. 7 with d = 0).

    ``np.add.at`` accumulates unbuffered, one index at a time in the order
    the index arrays are traversed; the slots are laid out c-major so each
    x[b,i] is summed in ascending (c, k) order."""
    B = ell.shape[0]
    x = np.zeros((B, p.n_vars))
    var = np.broadcast_to(p.idx.T.reshape(1, -1), (B, p.K * p.C))
    row = np.broadcast_to(np.arange(B)[:, None], var.shape)
    np.add.at(x, (row, var), np.transpose(ell, (0, 2, 1)).reshape(B, -1))
    return x


def sweep(st: State, p: Plan, temps, *, alpha: float, seed: int, formula_id: int = 0,
          chain_ids=None, record: bool = False):
    """One block-Gibbs round on every chain, in the appendix program's order.
    Mutates ``st`` and returns a record dict (empty unless ``record``)."""
    B = st.v.shape[0]
    temps = np.asarray(temps, dtype=np.int64)
    chain_ids = np.arange(B) if chain_ids is None else np.asarray(chain_ids, np.int64)
    t = st.t
    # gather + clause count + best tracking
    g, lit = literal_truth(st.v, p)
    s = lit.any(axis=1).sum(axis=1).astype(np.int64)
    better = s > st.s_max
    st.s_max = np.where(better, s, st.s_max)
    st.best[better] = st.v[better]
    # hidden conditional and draw, contributions, scatter -- per temperature
    x = np.zeros((B, p.n_vars))
    rec = {}
    if record:
        rec = dict(s=s.copy(), p_h=np.zeros((B, p.L, p.C)), u_h=np.zeros((B, p.L, p.C)),
                   h=np.zeros((B, p.L, p.C), np.uint8))
    u_h = hidden_uniforms(seed, formula_id, t, chain_ids, p.C, p.L)
    for tau in np.unique(temps):
        sel = np.nonzero(temps == tau)[0]
        z = hidden_logits(g[sel].astype(np.float64), p, int(tau))
        ph = sigmoid(z)
        h = (u_h[sel] < ph).astype(np.float64)
        ell = contributions(h, p, int(tau))
        x[sel] = scatter_add(ell, p)
        if record:
            rec["p_h"][sel], rec["u_h"][sel], rec["h"][sel] = ph, u_h[sel], h
    # visible conditional, variance EMA, draw
    rho = sigmoid(x)
    st.nu = variance_ema(st.nu, rho, alpha)
    u_v = visible_uniforms(seed, formula_id, t, chain_ids, p.n_vars)
    st.v = (u_v < rho).astype(np.uint8)
    st.t = t + 1
    if record:
        rec.update(x=x, rho=rho, u_v=u_v)
    return rec


def variance_ema(nu, rho, alpha: float):
    """Moving average of the visible units' conditional variance (Sec. 3.4,
    the priority of prioritized unit propagation): the variance of the
    Bernoulli(rho) draw of a unit is rho (1 - rho), and every sweep moves nu
    a fraction alpha towards it, nu <- (1 - alpha) nu + alpha rho (1 - rho).
    The appendix program starts nu at 0.25 (the variance at rho = 1/2)."""
    return (1 - alpha) * nu + alpha * rho * (1 - rho)


def count_and_track(st: State, p: Plan):
    """The count/best step alone (a zero-sweep run): returns s."""
    s = clause_count(st.v, p)
    better = s > st.s_max
    st.s_max = np.where(better, s, st.s_max)
    st.best[better] = st.v[better]
    return s


def run(st: State, p: Plan, temps, n_sweeps: int, *, alpha: float, seed: int,
        formula_id: int = 0, chain_ids=None) -> State:
    """Advance every chain ``n_sweeps`` rounds (a zero-sweep run only counts
    the current state and updates s_max / best).  Returns ``st`` (mutated)."""
    if n_sweeps == 0:
        count_and_track(st, p)
        return st
    for _ in range(n_sweeps):
        sweep(st, p, temps, alpha=alpha, seed=seed, formula_id=formula_id,
              chain_ids=chain_ids)
    return st


# ---------------------------------------------------------------------------
# Dense formula-RBM (pins only): W_f [N][C*L], b_f [C*L]
# ---------------------------------------------------------------------------

def dense_formula_rbm(p: Plan, tau: int = 0):
    """Instantiate the N x CL formula-RBM weight matrix that the sparse form
    never builds (Sec. 3.1): hidden unit (c, l) sits in column c*L + l, and a
    variable repeated inside a clause accumulates its rows."""
    N, K, L, C = p.n_vars, p.K, p.L, p.C
    Wf = np.zeros((N, C * L))
    for c in range(C):
        for k in range(K):
            Wf[p.idx[k, c], c * L:(c + 1) * L] += p.W[tau][k, :, c]
    bf = p.b[tau].T.reshape(-1)           # [C*L], column c*L + l
    return Wf, bf
