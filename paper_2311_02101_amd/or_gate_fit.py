"""Fit canonical OR-gate RBMs by free-energy regression (host tool, FP64).

Sec. 3.1 "Learning OR gate RBM parameters": because a clause has at most
K <= 7 inputs, all 2^K inputs are enumerated and the RBM parameters are
fitted by least squares of the free energy (eq. 1, visible bias d = 0)
against the OR-gate targets: 0 for the all-false input and F_s = -F* for every
satisfying input (Sec. 3.1 "OR gate as an RBM"; F_s < 0, so the printed
positive targets F* are magnitudes).  The appendix fixes Adam with learning
rate 1e-3, 3 hidden units for K = 3 and K+1 for K in [4, 7].

The exact fit is unattainable (F(0) = -sum_j softplus(b_j) < 0), so every
fit records its largest absolute residual.  The paper does not publish its
fitted values; this tool regenerates them and stores them as JSON:

    python -m paper_2311_02101_amd.or_gate_fit            # writes or_gate_weights.json
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

from .workload import FSTAR_16, FSTAR_PAIR, hidden_units_for

OUT = os.path.join(os.path.dirname(__file__), "or_gate_weights.json")


def _inputs(k: int) -> np.ndarray:
    m = np.arange(2 ** k)
    return ((m[:, None] >> np.arange(k)[None, :]) & 1).astype(np.float64)   # [2^K, K]


def _softplus(z):
    return np.logaddexp(0.0, z)


def _sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def fit(k: int, f_star: float, *, steps: int = 60000, lr: float = 1e-3,
        seed: int = 0, l: int | None = None):
    """Adam on L(W,b) = F(0)^2 + sum_{v != 0} (F(v) + F*)^2, full batch."""
    l = hidden_units_for(k) if l is None else l
    x = _inputs(k)
    target = np.full(2 ** k, -f_star)
    target[0] = 0.0
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, k, int(f_star * 1000)])))
    W = 0.5 * rng.standard_normal((k, l))
    b = -2.0 + 0.5 * rng.standard_normal(l)
    params = [W, b]
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    b1, b2, eps = 0.9, 0.999, 1e-8
    for it in range(1, steps + 1):
        z = x @ W + b                                   # [2^K, L]
        F = -_softplus(z).sum(axis=1)                   # eq. 1 with d = 0
        r = F - target
        dz = -(2.0 * r)[:, None] * _sigmoid(z)          # dLoss/dz
        grads = [x.T @ dz, dz.sum(axis=0)]
        for p, g, mm, vv in zip(params, grads, m, v):
            mm *= b1
            mm += (1 - b1) * g
            vv *= b2
            vv += (1 - b2) * g * g
            p -= lr * (mm / (1 - b1 ** it)) / (np.sqrt(vv / (1 - b2 ** it)) + eps)
    F = -_softplus(x @ W + b).sum(axis=1)
    res = F - target
    return W, b, float(np.max(np.abs(res))), float(np.sum(res * res))


def main(argv=None):
    targets = sorted(set(FSTAR_16) | set(FSTAR_PAIR))
    ks = [3, 4, 5, 6, 7]
    db = {"note": "canonical OR-gate RBMs fitted by free-energy regression "
                  "(Adam, lr 1e-3, full batch over all 2^K inputs, d = 0)",
          "fits": {}}
    for k in ks:
        for f in targets:
            W, b, mx, sse = fit(k, f)
            db["fits"][f"K{k}_F{f:.3f}"] = {
                "K": k, "L": int(W.shape[1]), "F_star": f,
                "W": W.tolist(), "b": b.tolist(),
                "max_abs_residual": mx, "sse": sse}
            print(f"K={k} F*={f:.3f} L={W.shape[1]} max|res|={mx:.3e}", flush=True)
    with open(OUT, "w") as fh:
        json.dump(db, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
