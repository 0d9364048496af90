"""Seeded synthetic inputs for the RbmSAT block-Gibbs path.

This module only *makes inputs*: CNF index tables, initial chain states,
temperature assignments and canonical OR-gate RBM parameter sets.  It holds
none of the method's arithmetic (no free energies, conditionals, sampling or
clause counting), so both the CPU oracle and the HIP path can consume what it
produces without sharing any computation.

Conventions (Sec. 3.3 "Scalable TPU implementation"):

* A formula is a signed, 1-based index table ``T`` of shape ``[K][C]``
  (variable-major, clause-minor); column ``c`` lists the literals of clause
  ``c`` and a negative entry is a negated variable, so the column
  ``(1, 2, -3, 4)`` is ``v1 or v2 or not v3 or v4``.
* Clauses shorter than ``K`` are padded by repeating a literal with the same
  polarity (Sec. 3.3); this module always repeats the clause's first literal.
* Chain states are ``uint8`` arrays of shape ``[B][N]`` holding 0/1.

The synthetic generator stands in for the MaxSAT-Evaluation incomplete
unweighted instances of Sec. 4 (not available here).  It keeps that section's
envelope: clause size <= 7, "few large and many small clauses", and an
over-constrained clause/variable ratio so the optimum leaves clauses
unsatisfied.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

# Clause-length mix of the synthetic formulas: mostly short clauses with a
# thin tail up to the maximum width 7 (Sec. 4 "few large and many small").
LENGTHS = np.array([2, 3, 4, 5, 6, 7], dtype=np.int64)
LENGTH_PROBS = np.array([0.50, 0.30, 0.05, 0.05, 0.05, 0.05])
CLAUSE_RATIO = 6          # C = 6 N
K_DEFAULT = 7             # maximum clause size handled (Sec. 3.1, K <= 7)

# Free-energy targets F* listed for the pretrained OR-gate ensembles
# (appendix "Pretraining"): the 1-accelerator pair and the 16-target list.
FSTAR_PAIR = (0.068, 0.528)
FSTAR_16 = tuple(round(0.068 + 0.030 * i, 3) for i in range(16))

_WEIGHTS_JSON = os.path.join(os.path.dirname(__file__), "or_gate_weights.json")

# stream tags for SeedSequence spawning; each input kind gets its own stream
_S_FORMULA, _S_STATE, _S_WEIGHTS, _S_SIZES = 0, 1, 2, 3


def _rng(seed: int, *tags: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, *tags])))


def pad_clauses(clauses, k: int) -> np.ndarray:
    """Pack a list of clauses (lists of signed 1-based literals) into a
    ``[k][C]`` int32 table, padding short clauses by repeating their first
    literal (Sec. 3.3)."""
    c = len(clauses)
    table = np.zeros((k, c), dtype=np.int32)
    for j, cl in enumerate(clauses):
        if len(cl) == 0 or len(cl) > k:
            raise ValueError(f"clause {j} has {len(cl)} literals (allowed 1..{k})")
        for i in range(k):
            table[i, j] = cl[i] if i < len(cl) else cl[0]
    return table


def random_formula(n_vars: int, seed: int, *, ratio: int = CLAUSE_RATIO,
                   k: int = K_DEFAULT, lengths=LENGTHS, probs=LENGTH_PROBS,
                   tag: int = 0) -> np.ndarray:
    """Random MaxSAT instance with ``C = ratio * n_vars`` clauses.

    Each clause draws its length from ``probs`` over ``lengths``, then that
    many *distinct* variables uniformly, then each literal's polarity as the
    sign of an N(0,1) draw.  Returns the padded ``[k][C]`` signed table."""
    lengths = np.asarray(lengths, dtype=np.int64)
    if n_vars < int(lengths.max()):
        raise ValueError("n_vars must be at least the longest clause length")
    rng = _rng(seed, _S_FORMULA, tag)
    n_cl = ratio * n_vars
    lens = rng.choice(lengths, size=n_cl, p=probs)
    kk = int(lengths.max())
    var = rng.integers(0, n_vars, size=(n_cl, kk))
    # redraw rows whose first len entries are not distinct (rejection)
    col = np.arange(kk)[None, :]
    while True:
        srt = np.sort(np.where(col < lens[:, None], var, -1 - col), axis=1)
        bad = np.any(srt[:, 1:] == srt[:, :-1], axis=1)
        if not bad.any():
            break
        var[bad] = rng.integers(0, n_vars, size=(int(bad.sum()), kk))
    sign = np.where(rng.standard_normal(size=(n_cl, kk)) >= 0.0, 1, -1)
    lit = (var + 1) * sign
    # pad by repeating the first literal
    lit = np.where(col < lens[:, None], lit, lit[:, :1])
    table = np.empty((k, n_cl), dtype=np.int32)
    table[:kk] = lit.T
    table[kk:] = lit[:, :1].T
    return table


def uneven_sizes(n_formulas: int, seed: int, lo: int = 64, hi: int = 16384) -> np.ndarray:
    """Formula sizes log-uniform in [lo, hi] (rounded to integers)."""
    rng = _rng(seed, _S_SIZES)
    u = rng.uniform(math.log(lo), math.log(hi), size=n_formulas)
    return np.clip(np.rint(np.exp(u)).astype(np.int64), lo, hi)


def initial_state(n_chains: int, n_vars: int, seed: int, tag: int = 0) -> np.ndarray:
    """Uniform random assignments: v = [z > 0] with z ~ N(0,1), i.e. a
    Bernoulli(1/2) draw per variable (Sec. 3.2 "initialized from a uniform
    distribution over assignments")."""
    rng = _rng(seed, _S_STATE, tag)
    return (rng.standard_normal(size=(n_chains, n_vars)) > 0.0).astype(np.uint8)


def default_temperatures(n_chains: int, n_temps: int) -> np.ndarray:
    """Chain -> temperature index: the chains are split into ``n_temps``
    contiguous, near-equal groups (with two targets: first half / second
    half), matching one OR-gate RBM per temperature (Sec. 3.2)."""
    b = np.arange(n_chains, dtype=np.int64)
    return ((b * n_temps) // max(n_chains, 1)).astype(np.int32)


def gaussian_rbm(n_temps: int, k: int, l: int, seed: int):
    """Parity-stress OR-gate parameters W_c ~ N(0,1)^[T,K,L], b_c ~ N(0,1)^[T,L]."""
    rng = _rng(seed, _S_WEIGHTS)
    return rng.standard_normal((n_temps, k, l)), rng.standard_normal((n_temps, l))


def hidden_units_for(k: int) -> int:
    """Hidden units per clause-RBM: 3 for clause size 3, K+1 for K in [4,7]
    (appendix "Pretraining")."""
    return 3 if k <= 3 else k + 1


def pretrained_rbm(k: int, targets=FSTAR_PAIR):
    """Canonical OR-gate RBMs fitted by ``or_gate_fit`` (one per F* target).
    Returns (W_c [T,K,L], b_c [T,L], max residuals [T])."""
    with open(_WEIGHTS_JSON) as fh:
        db = json.load(fh)
    ws, bs, res = [], [], []
    for f in targets:
        key = f"K{k}_F{f:.3f}"
        if key not in db["fits"]:
            raise KeyError(f"no pretrained OR-gate RBM for {key}")
        e = db["fits"][key]
        ws.append(np.array(e["W"], dtype=np.float64))
        bs.append(np.array(e["b"], dtype=np.float64))
        res.append(e["max_abs_residual"])
    return np.stack(ws), np.stack(bs), np.array(res)


def pretrained_size_rbms(targets=FSTAR_PAIR, k_max: int = 7):
    """The canonical RBMs of the size-clustered model (Sec. 4): {K: (W [T][K][L_K],
    b [T][L_K])} for K = 3 .. k_max, L_K = 3 for K = 3 and K + 1 otherwise,
    fitted to the same F* targets."""
    out = {}
    for K in range(3, max(k_max, 3) + 1):
        W, b, _ = pretrained_rbm(K, targets)
        out[K] = (W, b)
    return out


# ---------------------------------------------------------------------------
# DIMACS CNF reader (unweighted, "p cnf N C" header, 0-terminated clauses)
# ---------------------------------------------------------------------------

def read_dimacs(text: str):
    """Parse DIMACS CNF text.  Returns (n_vars, list of clauses).

    Weighted formats (``p wcnf``) are rejected: every clause is a unit-weight
    soft clause in this method (Sec. 4 "does not handle weighted clauses")."""
    n_vars = n_cl = None
    clauses, cur = [], []
    for raw in text.splitlines():
        line = raw.strip()
        if not line or line[0] in "c%":
            continue
        if line[0] == "p":
            parts = line.split()
            if len(parts) < 4 or parts[1] != "cnf":
                raise ValueError(f"unsupported problem line: {line!r}")
            n_vars, n_cl = int(parts[2]), int(parts[3])
            continue
        for tok in line.split():
            x = int(tok)
            if x == 0:
                if not cur:
                    raise ValueError("empty clause")
                clauses.append(cur)
                cur = []
            else:
                cur.append(x)
    if cur:
        clauses.append(cur)
    if n_vars is None:
        raise ValueError("missing 'p cnf' line")
    if n_cl is not None and n_cl != len(clauses):
        raise ValueError(f"header says {n_cl} clauses, found {len(clauses)}")
    for cl in clauses:
        for x in cl:
            if abs(x) > n_vars:
                raise ValueError(f"literal {x} exceeds n_vars={n_vars}")
    return n_vars, clauses


def write_dimacs(n_vars: int, table: np.ndarray) -> str:
    """Serialise a padded ``[K][C]`` table as DIMACS (padding kept)."""
    out = [f"p cnf {n_vars} {table.shape[1]}"]
    for c in range(table.shape[1]):
        out.append(" ".join(str(int(x)) for x in table[:, c]) + " 0")
    return "\n".join(out) + "\n"


# ---------------------------------------------------------------------------
# Named workloads (sizes and seeds of the measured configurations)
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n_vars: list            # per formula
    chains: int             # B per formula
    sweeps: int
    seed: int
    precision: str          # "f64" | "f32" | "mixed"
    tables: list = field(default_factory=list)   # per formula [K][C]
    v0: list = field(default_factory=list)       # per formula [B][N]
    W: np.ndarray = None    # [T][K][L]
    b: np.ndarray = None    # [T][L]
    temps: np.ndarray = None  # [B]
    alpha: float = 1e-3
    size_rbms: dict = None    # size-clustered model {K: (W, b)}, None = padded


def make_workload(name: str, n_vars, chains: int, seed: int, *, sweeps: int = 500,
                  precision: str = "f64", weights: str = "pretrained",
                  k: int = K_DEFAULT, ratio: int = CLAUSE_RATIO) -> Workload:
    n_list = [int(n) for n in np.atleast_1d(n_vars)]
    l = hidden_units_for(k)
    if weights == "pretrained":
        W, b, _ = pretrained_rbm(k, FSTAR_PAIR)
    elif weights == "gaussian":
        W, b = gaussian_rbm(len(FSTAR_PAIR), k, l, seed)
    else:
        raise ValueError(weights)
    n_temps = 1 if chains == 1 else W.shape[0]
    W, b = W[:n_temps], b[:n_temps]
    wl = Workload(name, n_list, chains, sweeps, seed, precision, W=W, b=b,
                  temps=default_temperatures(chains, n_temps))
    for f, n in enumerate(n_list):
        wl.tables.append(random_formula(n, seed, ratio=ratio, k=k, tag=f))
        wl.v0.append(initial_state(chains, n, seed, tag=f))
    return wl


# the five measured configurations (sizes, chains, seeds, precision)
CONFIGS = {
    "plain_n256_b1": dict(n_vars=256, chains=1, seed=0, precision="f64"),
    "plain_n4096_b64": dict(n_vars=4096, chains=64, seed=1, precision="f64"),
    "mixed_n8192_b256": dict(n_vars=8192, chains=256, seed=2, precision="mixed"),
    "uneven_1024x64": dict(n_vars=None, chains=64, seed=3, precision="f32"),
    "learned_n2048": dict(n_vars=2048, chains=32, seed=4, precision="f32"),
}


def config_workload(name: str, **over) -> Workload:
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    if cfg["n_vars"] is None:
        cfg["n_vars"] = uneven_sizes(1024, cfg["seed"])
    return make_workload(name, **cfg)
