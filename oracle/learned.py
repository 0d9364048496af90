"""CPU FP64 oracle of the learned initial-assignment model.

Part of the test oracle (see ``oracle/__init__``): not used by the product
path, shares no code with it.

The paper suggests combining RbmSAT with learned components that generate
good initial assignments (Sec. 2, related work on learned SAT policies).  The
model here maps per-variable occurrence statistics of a formula to
q_i = P(v_i = 1) with a two-layer perceptron, trained on labels the sampler
itself produces; chains are then initialised from Bernoulli(q).

Specification mirrored by the HIP kernels:
  features   -- 32 per variable, all exact dyadic values before one rounding
                to bfloat16 (round to nearest even):
                  0..13  count of clauses of real length l = 1..7 holding the
                         variable positively (even index) / negated (odd), / 8
                  14, 15 positive / negated occurrences, / 8
                  16     (positive - negated occurrences) / 8
                  17, 18 sum over positive / negated occurrences of 2^-l
                  19     difference of the two
                  20..31 zero (padding of the 32-wide input)
                The real length of a clause ignores the padding copies of its
                first literal (trailing repeats).
  network    -- pre = x W1 + b1, h = relu(pre), o = h w2 + b2, q = sigmoid(o);
                W1 [32][256] and w2 [256] are used rounded to bfloat16, the
                biases in full precision.
  loss       -- mean binary cross-entropy of q against labels y in [0, 1].
  gradients  -- of the mean loss; the hidden-layer gradient dh is rounded to
                bfloat16 before it multiplies the inputs (dW1 = x^T bf16(dh)).
  Adam       -- Kingma & Ba: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
                p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
  init draw  -- v0_i = [U < q_i] with U from the sweep generator at the
                reserved time t = 2^64 - 1, visible phase, unit i.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32
from .rbmsat import normalize_table

F_IN = 32
HIDDEN = 256


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32)
    # NaN/inf pass through unchanged (not produced by the features here)
    return np.where(np.isfinite(f), out, f).astype(np.float64)


def real_lengths(T):
    """Real length of every clause: K minus the trailing copies of literal 0."""
    K, C = T.shape
    lens = np.full(C, K, dtype=np.int64)
    for c in range(C):
        L = K
        while L > 1 and T[L - 1, c] == T[0, c]:
            L -= 1
        lens[c] = L
    return lens


def features(T, n_vars):
    """Per-variable features [N][32] (float64, before the bfloat16 rounding)."""
    T = normalize_table(T, n_vars)
    lens = real_lengths(T)
    feat = np.zeros((n_vars, F_IN))
    for c in range(T.shape[1]):
        L = int(lens[c])
        for k in range(L):
            lit = int(T[k, c])
            i, neg = abs(lit) - 1, int(lit < 0)
            feat[i, 2 * (L - 1) + neg] += 1.0 / 8.0
            feat[i, 15 if neg else 14] += 1.0 / 8.0
            feat[i, 18 if neg else 17] += 2.0 ** -L
    feat[:, 16] = feat[:, 14] - feat[:, 15]
    feat[:, 19] = feat[:, 17] - feat[:, 18]
    return feat


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(x, W1, b1, w2, b2, quantize=True):
    """q and the intermediates, with the bf16-rounded weights (quantize=False
    uses the weights as given, for derivative checks)."""
    x = np.asarray(x, dtype=np.float64)
    Q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    pre = x @ Q(W1) + b1
    h = np.maximum(pre, 0.0)
    o = h @ Q(w2) + b2
    return sigmoid(o), dict(pre=pre, h=h, o=o)


def loss(x, y, W1, b1, w2, b2, quantize=True):
    q, mid = forward(x, W1, b1, w2, b2, quantize)
    o = mid["o"]
    # -(y log q + (1 - y) log(1 - q)) = softplus(o) - y o
    return float(np.mean(np.logaddexp(0.0, o) - y * o))


def gradients(x, y, W1, b1, w2, b2, quantize=True):
    """Gradients of the mean loss: dict(W1, b1, w2, b2).  quantize=False
    skips every bfloat16 rounding (the exact chain rule)."""
    x = np.asarray(x, dtype=np.float64)
    Q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    R = x.shape[0]
    q, mid = forward(x, W1, b1, w2, b2, quantize)
    g = (q - y) / R                                   # dL/do
    h, pre = mid["h"], mid["pre"]
    dw2 = h.T @ g
    db2 = np.sum(g)
    dh = np.outer(g, Q(w2)) * (pre > 0.0)
    db1 = np.sum(dh, axis=0)
    dW1 = x.T @ Q(dh)
    return dict(W1=dW1, b1=db1, w2=dw2, b2=np.array([db2]))


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    p = p - lr * (m / (1 - beta1 ** step)) / (np.sqrt(v / (1 - beta2 ** step)) + eps)
    return p, m, v


def init_assignment(q, seed, formula_id, chains):
    """v0[b, i] = [U < q_i] with U at the reserved time t = 2^64 - 1."""
    q = np.asarray(q, dtype=np.float64)
    n = q.shape[0]
    chains = np.atleast_1d(np.asarray(chains, dtype=np.int64))
    g = -(-n // 4)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    key = (seed & 0xFFFFFFFF, ((seed >> 32) ^ int(formula_id)) & 0xFFFFFFFF)
    ctr = (np.uint64(0xFFFFFFFF), chains[:, None].astype(np.uint64),
           np.uint64(1 << 31) | np.arange(g, dtype=np.uint64)[None, :], np.uint64(0xFFFFFFFF))
    w = philox4x32(ctr, key).reshape(len(chains), g * 4)[:, :n]
    u = (w >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    return (u < q[None, :]).astype(np.uint8)
