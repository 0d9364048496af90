"""Pins of the learned-initializer oracle (CPU)."""
import numpy as np
import pytest

from oracle import learned as M
from oracle import rbmsat as R
from paper_2311_02101_amd import workload as wl


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10 ** rng.uniform(-6, 6, 20000),
                        # exact ties between two bfloat16 neighbours
                        (np.arange(1, 2000) * 2 + 1) * 2.0 ** -8 * 2.0 ** rng.integers(-5, 5, 1999)])
    ours = M.bf16_round(x)
    theirs = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, theirs)


def test_features_by_hand():
    # clauses: (v1 or not v2), (v2 or v3 or not v1) padded to K = 4 by repeating v2
    T = wl.pad_clauses([[1, -2], [2, 3, -1]], 4)
    f = M.features(T, 3)
    # v1: positive in a length-2 clause, negated in a length-3 clause
    assert f[0, 2] == 1 / 8 and f[0, 5] == 1 / 8 and f[0, 14] == 1 / 8 and f[0, 15] == 1 / 8
    assert f[0, 17] == 2 ** -2 and f[0, 18] == 2 ** -3 and f[0, 19] == 2 ** -2 - 2 ** -3
    # v2: negated in the length-2 clause, positive in the length-3 clause (padding ignored)
    assert f[1, 3] == 1 / 8 and f[1, 4] == 1 / 8 and f[1, 14] == 1 / 8 and f[1, 15] == 1 / 8
    # v3: one positive occurrence, length 3
    assert f[2, 4] == 1 / 8 and f[2, 16] == 1 / 8 and f[2, 17] == 2 ** -3
    assert np.all(f[:, 20:] == 0)
    assert np.array_equal(M.real_lengths(T), [2, 3])


def test_features_are_exact_dyadics():
    T = wl.random_formula(512, 3)
    f = M.features(T, 512)
    assert np.all(f * 2 ** 10 == np.floor(f * 2 ** 10))   # multiples of 2^-10
    # counts add up: every real literal appears once in the length/sign counts
    lens = M.real_lengths(R.normalize_table(T, 512))
    assert np.isclose(f[:, 0:14].sum() * 8, lens.sum())


def _net(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    W1 = M.bf16_round(scale * rng.standard_normal((M.F_IN, M.HIDDEN)))
    b1 = 0.1 * rng.standard_normal(M.HIDDEN)
    w2 = M.bf16_round(scale * rng.standard_normal(M.HIDDEN))
    b2 = np.array(0.05)
    return W1, b1, w2, b2


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    x = M.bf16_round(rng.standard_normal((64, M.F_IN)))
    y = rng.uniform(0, 1, 64)
    W1, b1, w2, b2 = _net(2)
    g = M.gradients(x, y, W1, b1, w2, b2, quantize=False)
    eps = 1e-6
    for name, arr, idx in [("W1", W1, (3, 17)), ("W1", W1, (31, 200)), ("b1", b1, (5,)),
                           ("w2", w2, (9,)), ("w2", w2, (255,))]:
        a = arr.copy()
        a[idx] += eps
        args = dict(W1=W1, b1=b1, w2=w2, b2=b2)
        args[name] = a
        lp = M.loss(x, y, quantize=False, **args)
        a[idx] -= 2 * eps
        lm = M.loss(x, y, quantize=False, **args)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[name][idx]) < 1e-7 * max(1.0, abs(fd))
    lp = M.loss(x, y, W1, b1, w2, b2 + eps, quantize=False)
    lm = M.loss(x, y, W1, b1, w2, b2 - eps, quantize=False)
    assert abs((lp - lm) / (2 * eps) - g["b2"][0]) < 1e-7
    # the specified (bf16-rounded dh) gradient stays within the rounding bound
    gq = M.gradients(x, y, W1, b1, w2, b2)
    q, mid = M.forward(x, W1, b1, w2, b2)
    dh = np.outer((q - y) / 64, w2) * (mid["pre"] > 0)
    bound = np.abs(x).T @ np.abs(dh) * 2.0 ** -8
    assert np.all(np.abs(gq["W1"] - g["W1"]) <= bound + 1e-18)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p, g = rng.standard_normal(100), rng.standard_normal(100)
    p1, m1, v1 = M.adam(p, g, np.zeros(100), np.zeros(100), 1, lr=1e-3)
    assert np.allclose(p - p1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_init_draw_matches_sweep_generator_and_frequencies():
    q = np.linspace(0, 1, 4000)
    v = M.init_assignment(q, 7, 2, np.arange(64))
    u = R.visible_uniforms(7, 2, 2 ** 64 - 1, np.arange(64), 4000)
    assert np.array_equal(v, (u < q[None, :]).astype(np.uint8))
    assert np.all(v[:, 0] == 0) and np.all(v[:, -1] == 1)
    assert abs(v.mean() - 0.5) < 0.01


def test_training_reduces_loss_on_a_learnable_target():
    rng = np.random.default_rng(4)
    x = M.bf16_round(rng.standard_normal((512, M.F_IN)))
    y = (x[:, 0] - x[:, 1] > 0).astype(np.float64)
    W1, b1, w2, b2 = _net(5)
    params = dict(W1=W1, b1=b1, w2=w2, b2=np.array([0.0]))
    mom = {k: (np.zeros_like(v), np.zeros_like(v)) for k, v in params.items()}
    l0 = M.loss(x, y, params["W1"], params["b1"], params["w2"], params["b2"][0])
    for step in range(1, 201):
        g = M.gradients(x, y, params["W1"], params["b1"], params["w2"], params["b2"][0])
        for k in params:
            params[k], m, v = M.adam(params[k], g[k], *mom[k], step, lr=1e-2)
            mom[k] = (m, v)
    l1 = M.loss(x, y, params["W1"], params["b1"], params["w2"], params["b2"][0])
    assert l1 < 0.3 * l0
