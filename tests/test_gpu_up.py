"""The unit-propagation exchange on the GPU: the device top-B merge against
the oracle's, and the whole driver (sampling, snapshot, host propagation
overlapped with sampling, merge) against a step-by-step replay built from the
oracle's propagation and merge."""
import numpy as np
import pytest

from oracle import up as U
from paper_2311_02101_amd import hp, workload as wl
from tests.parity import say

pytestmark = pytest.mark.gpu


def _sync():
    import torch
    torch.cuda.synchronize()


def _batch(seed):
    sizes = [40, 97, 23]
    tables = [wl.random_formula(n, seed, tag=f, ratio=4) for f, n in enumerate(sizes)]
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    return sizes, tables, W, b


def test_merge_matches_oracle(hip):
    import torch
    sizes, tables, W, b = _batch(3)
    B = 6
    plan = hp.Plan(tables, sizes, W, b, chains=B, precision="f64", seed=3)
    st = plan.new_state([wl.initial_state(B, n, 3, tag=f) for f, n in enumerate(sizes)])
    plan.run(st, 7)
    _sync()
    rng = np.random.default_rng(4)
    before = [st.formula(f) for f in range(len(sizes))]
    cand_parts = []
    for f, n in enumerate(sizes):
        c = rng.integers(0, 2, (B, n)).astype(np.uint8)
        c[1] = before[f][0][4]                  # equal counts: the returned row must win
        c[3] = before[f][0][0]
        cand_parts.append(c)
    cand = torch.tensor(np.concatenate([c.ravel() for c in cand_parts]), device="cuda")
    say("[merge] 3 formulas x 6 chains")
    plan.merge_candidates(st, cand)
    _sync()
    for f, n in enumerate(sizes):
        v0, nu0, s0, b0 = before[f]
        want_v, want_nu = U.merge_topb(tables[f], n, v0, nu0, cand_parts[f])
        v1, nu1, s1, b1 = st.formula(f)
        assert np.array_equal(v1, want_v) and np.array_equal(nu1, want_nu)
        assert np.array_equal(s1, s0) and np.array_equal(b1, b0)
    plan.free()


def test_solver_matches_oracle_replay(hip):
    """solve() = sampling segments + snapshot + oracle UP + upw more sweeps +
    oracle merge, replayed by hand on a second plan with the same seed."""
    from paper_2311_02101_amd import solver
    sizes, tables, W, b = _batch(5)
    B, S, upp, upw = 8, 260, 100, 30
    temps = wl.default_temperatures(B, 2)
    v0 = [wl.initial_state(B, n, 5, tag=f) for f, n in enumerate(sizes)]
    say("[solver] driver run")
    p1 = hp.Plan(tables, sizes, W, b, chains=B, temps=temps, precision="f64", seed=5)
    s1 = p1.new_state(v0)
    stats = solver.solve(p1, tables, s1, S, upp, upw, threads=4)
    _sync()
    assert stats["exchanges"] == 2
    say("[solver] replay")
    p2 = hp.Plan(tables, sizes, W, b, chains=B, temps=temps, precision="f64", seed=5)
    s2 = p2.new_state(v0)
    t = 0
    for send in (100, 200):
        p2.run(s2, send - t)
        _sync()
        snap = [s2.formula(f) for f in range(len(sizes))]
        p2.run(s2, upw)
        _sync()
        for f, n in enumerate(sizes):
            up = np.stack([U.prioritized_up(tables[f], n, snap[f][0][c], snap[f][1][c]) for c in range(B)])
            v, nu, _, _ = s2.formula(f)
            vn, nun = U.merge_topb(tables[f], n, v, nu, up)
            s2.set_formula(f, v=vn, nu=nun)
        t = send + upw
    p2.run(s2, S - t)
    _sync()
    for f in range(len(sizes)):
        for a, c in zip(s1.formula(f), s2.formula(f)):
            assert np.array_equal(a, c)
    p1.free()
    p2.free()
