"""Learned initial assignments for the block-Gibbs search.

A 32 -> 256 -> 1 perceptron maps per-variable occurrence statistics of a
formula to q_i = P(v_i = 1).  It is trained on labels the sampler itself
produces -- the fraction of chains whose best assignment sets v_i after a
plain run from uniform starts -- and then seeds half of the chains of a new
formula with v_i ~ Bernoulli(q_i) while the other half keep uniform starts.
The plain method is thereby the fallback, and the exact satisfied-clause
count judges the two halves.

Every step runs in the library's HIP kernels (features, MFMA forward and
backward, Adam, initial draws, label reduction); this module only allocates
buffers and drives the loop.

    python -m paper_2311_02101_amd.learned --instances 100000   # full-size training run
    python -m paper_2311_02101_amd.learned --mlp-bench 4194304  # MLP kernels alone (JSON)
    python -m paper_2311_02101_amd.learned --equal-accuracy 256 # learned form vs plain at equal accuracy
"""
from __future__ import annotations

import argparse
import ctypes as ct
import json
import os
import sys
import time

import numpy as np

from . import hp
from . import workload as wl

F_IN, HIDDEN = 32, 256
N_PARAMS = F_IN * HIDDEN + 2 * HIDDEN + 1
MLP_PARTS = 1024                     # rows of the backward pass's partial-sum workspace
WEIGHTS_JSON = os.path.join(os.path.dirname(os.path.abspath(__file__)), "learned_init_weights.json")


class HpMlp(ct.Structure):
    _fields_ = [("params", ct.c_void_p), ("adam_m", ct.c_void_p), ("adam_v", ct.c_void_p),
                ("grad", ct.c_void_p), ("w_bf16", ct.c_void_p), ("partials", ct.c_void_p)]


def _lib():
    lib = hp.load()
    if not getattr(lib, "_mlp_bound", False):
        lib.hp_features.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
        lib.hp_mlp_sync.argtypes = [ct.POINTER(HpMlp), ct.c_void_p]
        lib.hp_mlp_forward.argtypes = [ct.POINTER(HpMlp), ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p]
        lib.hp_mlp_backward.argtypes = [ct.POINTER(HpMlp), ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p,
                                        ct.c_void_p]
        lib.hp_mlp_adam.argtypes = [ct.POINTER(HpMlp), ct.c_float, ct.c_float, ct.c_float, ct.c_float,
                                    ct.c_int64, ct.c_void_p]
        lib.hp_init_chains.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int32,
                                       ct.POINTER(hp.HpState), ct.c_void_p]
        lib.hp_chain_mean.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
        for n in ("hp_features", "hp_mlp_sync", "hp_mlp_forward", "hp_mlp_backward", "hp_mlp_adam",
                  "hp_init_chains", "hp_chain_mean"):
            getattr(lib, n).restype = ct.c_int
        lib._mlp_bound = True
    return lib


def _stream():
    import torch
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


class MLP:
    """Device parameters (FP32 master, Adam moments, gradient, bf16 copies)."""

    def __init__(self, seed: int = 4, params: np.ndarray | None = None, device="cuda"):
        import torch
        if params is None:
            rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 77])))
            params = np.zeros(N_PARAMS)
            params[:F_IN * HIDDEN] = rng.standard_normal(F_IN * HIDDEN) * np.sqrt(2.0 / F_IN)
            params[F_IN * HIDDEN + HIDDEN:F_IN * HIDDEN + 2 * HIDDEN] = \
                rng.standard_normal(HIDDEN) * np.sqrt(1.0 / HIDDEN)
        f32 = dict(dtype=torch.float32, device=device)
        self.params = torch.tensor(np.asarray(params, dtype=np.float32), **f32)
        self.m = torch.zeros(N_PARAMS, **f32)
        self.v = torch.zeros(N_PARAMS, **f32)
        self.grad = torch.zeros(N_PARAMS, **f32)
        self.w_bf16 = torch.zeros(F_IN * HIDDEN + HIDDEN, dtype=torch.int16, device=device)
        self.partials = torch.empty(MLP_PARTS * (N_PARAMS + 1), **f32)
        self.loss_buf = torch.zeros(1, **f32)
        self.step = 0
        self.sync()

    def c_struct(self):
        return HpMlp(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                     self.grad.data_ptr(), self.w_bf16.data_ptr(), self.partials.data_ptr())

    def sync(self):
        hp._check(_lib().hp_mlp_sync(ct.byref(self.c_struct()), _stream()))

    def forward(self, x, q=None):
        import torch
        rows = x.shape[0]
        if q is None:
            q = torch.empty(rows, dtype=torch.float32, device=x.device)
        hp._check(_lib().hp_mlp_forward(ct.byref(self.c_struct()), ct.c_void_p(x.data_ptr()), rows,
                                        ct.c_void_p(q.data_ptr()), _stream()))
        return q

    def backward(self, x, y):
        """Fill self.grad with the gradient of the mean loss; returns the
        (device) summed loss tensor."""
        hp._check(_lib().hp_mlp_backward(ct.byref(self.c_struct()), ct.c_void_p(x.data_ptr()),
                                         ct.c_void_p(y.data_ptr()), x.shape[0],
                                         ct.c_void_p(self.loss_buf.data_ptr()), _stream()))
        return self.loss_buf

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        hp._check(_lib().hp_mlp_adam(ct.byref(self.c_struct()), lr, beta1, beta2, eps, self.step,
                                     _stream()))

    def host_params(self):
        return self.params.cpu().numpy().astype(np.float64)

    def save(self, path=WEIGHTS_JSON, **meta):
        with open(path, "w") as fh:
            json.dump({"params": self.host_params().tolist(), **meta}, fh)

    @classmethod
    def load(cls, path=WEIGHTS_JSON, device="cuda"):
        with open(path) as fh:
            d = json.load(fh)
        return cls(params=np.array(d["params"]), device=device), d


def features(plan):
    """bf16 feature rows [sum N][32] (torch int16 holding the bit patterns)."""
    import torch
    x = torch.empty((plan.total_vars, F_IN), dtype=torch.int16, device="cuda")
    hp._check(_lib().hp_features(plan._h, ct.c_void_p(x.data_ptr()), _stream()))
    return x


def init_chains(plan, q, state, chain_lo, chain_hi):
    hp._check(_lib().hp_init_chains(plan._h, ct.c_void_p(q.data_ptr()), int(chain_lo), int(chain_hi),
                                    ct.byref(state.c_struct()), _stream()))


def chain_mean(plan, arr):
    import torch
    out = torch.empty(plan.total_vars, dtype=torch.float32, device="cuda")
    hp._check(_lib().hp_chain_mean(plan._h, ct.c_void_p(arr.data_ptr()), ct.c_void_p(out.data_ptr()),
                                   _stream()))
    return out


# ---------------------------------------------------------------------------
# data, training and evaluation
# ---------------------------------------------------------------------------

def _formulas(n_formulas, n_vars, seed, first=0):
    return [wl.random_formula(n_vars, seed, tag=first + f) for f in range(n_formulas)]


def _formula_task(args):
    n_vars, seed, tag = args
    return wl.random_formula(n_vars, seed, tag=tag)


class FormulaPool:
    """Host worker processes that generate formulas (NumPy only, never the
    GPU).  Create it before the process first uses the GPU: the workers are
    forked."""

    def __init__(self, workers):
        import multiprocessing as mp
        self.pool = mp.get_context("fork").Pool(workers) if workers > 1 else None

    def submit(self, n_formulas, n_vars, seed, first):
        tasks = [(n_vars, seed, first + f) for f in range(n_formulas)]
        if self.pool is None:
            res = [_formula_task(t) for t in tasks]
            return lambda: res
        handle = self.pool.map_async(_formula_task, tasks, chunksize=8)
        return lambda: handle.get()

    def close(self):
        if self.pool is not None:
            self.pool.close()
            self.pool.join()


def make_dataset(n_formulas, n_vars=2048, seed=4, chains=32, sweeps=500, batch=256, first=0,
                 log=None, pool=None):
    """Features and labels from the method itself: for each formula, run the
    plain sampler from uniform starts and label every variable with the
    fraction of chains whose best assignment sets it.  Returns device tensors
    x [rows][32] (bf16 bits) and y [rows].  With a FormulaPool the next
    batch of formulas is generated while the GPU labels the current one."""
    import torch
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    temps = wl.default_temperatures(chains, 2)
    xs, ys = [], []
    src = pool if pool is not None else FormulaPool(0)
    t_start = time.time()
    starts = list(range(0, n_formulas, batch))
    pending = src.submit(min(batch, n_formulas), n_vars, seed, first) if starts else None
    for j, lo in enumerate(starts):
        k = min(batch, n_formulas - lo)
        tables = pending()
        if j + 1 < len(starts):
            nlo = starts[j + 1]
            pending = src.submit(min(batch, n_formulas - nlo), n_vars, seed, first + nlo)
        plan = hp.Plan(tables, [n_vars] * k, W, b, chains=chains, temps=temps, precision="f32",
                       seed=seed + 1000 * (first + lo))
        st = plan.new_state([wl.initial_state(chains, n_vars, seed, tag=first + lo + f) for f in range(k)])
        plan.run(st, sweeps)
        xs.append(features(plan))
        ys.append(chain_mean(plan, st.best))
        torch.cuda.synchronize()
        plan.check()              # labels of a void (failed split exchange) run are refused
        plan.free()
        if log:
            log(f"labelled {lo + k}/{n_formulas} formulas ({time.time() - t_start:.1f} s)")
    return torch.cat(xs), torch.cat(ys)


def train(net, x, y, epochs=3, batch_rows=1 << 18, lr=1e-3, log=None):
    import torch
    rows = x.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(1234)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(rows // batch_rows if rows >= batch_rows else 1, generator=gen)
        tot = 0.0
        for bi in perm.tolist():
            lo = bi * batch_rows
            hi = min(rows, lo + batch_rows)
            loss = net.backward(x[lo:hi], y[lo:hi])
            net.adam(lr=lr)
            tot += float(loss.item()) / (hi - lo)
        losses.append(tot / len(perm))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss {losses[-1]:.5f}")
    return losses


def evaluate(net, n_formulas, n_vars=2048, seed=4, chains=64, sweeps=(20, 100, 500), first=10 ** 6):
    """Held-out comparison on formulas never used in training: chains
    [0, B/2) start from Bernoulli(q), chains [B/2, B) from uniform; for each
    sweep budget report the mean best count of each half (the better of the
    two is the answer, so the plain method is the fallback)."""
    import torch
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    tables = _formulas(n_formulas, n_vars, seed, first)
    # both halves use the same temperature split (first half of each half at
    # the low target) so the comparison is paired
    half = chains // 2
    temps = np.concatenate([wl.default_temperatures(half, 2)] * 2).astype(np.int32)
    plan = hp.Plan(tables, [n_vars] * n_formulas, W, b, chains=chains, temps=temps, precision="f32",
                   seed=seed + 7)
    st = plan.new_state([wl.initial_state(chains, n_vars, seed, tag=first + f) for f in range(n_formulas)])
    q = net.forward(features(plan))
    init_chains(plan, q, st, 0, half)
    plan.run(st, 0)
    out = {}
    done = 0
    for s in sweeps:
        plan.run(st, s - done)
        done = s
        plan.run(st, 0)
        torch.cuda.synchronize()
        plan.check()
        smax = st.s_max.cpu().numpy().reshape(n_formulas, chains)
        mlp_best = smax[:, :half].max(axis=1)
        uni_best = smax[:, half:].max(axis=1)
        out[s] = dict(mlp=float(mlp_best.mean()), uniform=float(uni_best.mean()),
                      gain=float((mlp_best - uni_best).mean()),
                      wins=int((mlp_best > uni_best).sum()), losses=int((mlp_best < uni_best).sum()),
                      fallback_used=int((uni_best > mlp_best).sum()),
                      clauses=int(tables[0].shape[1]))
    plan.free()
    return out


def _event_seconds(fn):
    """HIP-event time of fn() on the current stream (synchronised)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def equal_accuracy(net, n_formulas, n_vars=2048, seed=4, chains=64, budget=20, step=5, max_sweeps=1000,
                   first=10 ** 6, precisions=("f64", "f32")):
    """Speed-up of the learned form over the plain method at equal accuracy.

    Accuracy is the mean over the formulas of the best satisfied-clause
    count of all B chains.  Learned form (FP32): chains [0, B/2) start from
    Bernoulli(q), chains [B/2, B) uniform, `budget` sweeps.  Plain method, in
    each of `precisions`: all B chains uniform (the same initial states,
    temperatures and random streams as the learned run's uniform half), run
    `step` sweeps at a time until its accuracy reaches the learned form's.
    Times are HIP-event times of fresh runs: the learned form's includes the
    features, the forward pass and the initial draws; the plain form's is one
    run of the sweeps it needed.  Per formula, the sweeps the plain run needs
    to reach that formula's learned count are reported too (max_sweeps + step
    where it never does)."""
    import torch
    W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_PAIR)
    tables = _formulas(n_formulas, n_vars, seed, first)
    ns = [n_vars] * n_formulas
    half = chains // 2
    temps = np.concatenate([wl.default_temperatures(half, 2)] * 2).astype(np.int32)
    v0 = [wl.initial_state(chains, n_vars, seed, tag=first + f) for f in range(n_formulas)]

    def best_of(plan, st):
        plan.check()
        return st.s_max.cpu().numpy().reshape(n_formulas, chains).max(axis=1)

    lplan = hp.Plan(tables, ns, W, b, chains=chains, temps=temps, precision="f32", seed=seed + 7)

    def learned_run(st):
        q = net.forward(features(lplan))
        init_chains(lplan, q, st, 0, half)
        lplan.run(st, budget)
        lplan.run(st, 0)

    learned_run(lplan.new_state(v0))                       # warm-up (module load, first launches)
    st = lplan.new_state(v0)
    torch.cuda.synchronize()
    t_learned = _event_seconds(lambda: learned_run(st))
    target_f = best_of(lplan, st)
    lplan.free()
    target = float(target_f.mean())
    out = {"formulas": n_formulas, "n_vars": n_vars, "chains": chains, "budget": budget, "step": step,
           "learned": {"precision": "f32", "sweeps": budget, "accuracy": target, "seconds": t_learned}}
    for prec in precisions:
        plan = hp.Plan(tables, ns, W, b, chains=chains, temps=temps, precision=prec, seed=seed + 7)
        st = plan.new_state(v0)
        plan.run(st, 0)
        need_f = np.full(n_formulas, max_sweeps + step)
        need, acc, done = None, [], 0
        while done < max_sweeps:
            plan.run(st, step)
            plan.run(st, 0)
            done += step
            best = best_of(plan, st)
            acc.append((done, float(best.mean())))
            need_f[(need_f > max_sweeps) & (best >= target_f)] = done
            if need is None and best.mean() >= target:
                need = done
            if need is not None and (need_f <= max_sweeps).all():
                break
        res = {"precision": prec, "sweeps_to_equal_accuracy": need, "accuracy_by_sweeps": acc,
               "per_formula_sweeps_median": float(np.median(need_f)),
               "per_formula_reached": int((need_f <= max_sweeps).sum())}
        if need is not None:
            plan.run(plan.new_state(v0), need)             # warm-up of the same launch
            st = plan.new_state(v0)
            torch.cuda.synchronize()
            res["seconds"] = _event_seconds(lambda: (plan.run(st, need), plan.run(st, 0)))
            res["accuracy"] = float(best_of(plan, st).mean())
            res["speedup_of_learned_form"] = res["seconds"] / t_learned
        plan.free()
        out["plain_" + prec] = res
    return out


def mlp_bench(rows, rounds=5, seed=4):
    """Time the MLP kernels alone on `rows` random feature rows: forward, and
    the training step (backward kernel with the forward recomputed, the
    fixed-order reduction of its partial sums, Adam), `rounds` times each after a
    warm-up.  Algorithmic work per row: the forward product 2 * 32 * 256 and
    the output 2 * 256 flops; the backward recomputes the forward and adds
    dh = w2 * relu'(h) (256), dW1 = x^T dh (2 * 32 * 256) and dw2 (2 * 256).
    Bytes per row: 64 of bfloat16 features, 4 of label, 4 of output."""
    import torch
    net = MLP(seed=seed)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    feat = torch.rand(rows, F_IN, generator=gen).to("cuda")
    x = feat.to(torch.bfloat16).view(torch.int16)
    y = torch.rand(rows, generator=gen).to("cuda")
    q = torch.empty(rows, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(rounds):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / rounds

    t_fwd = timed(lambda: net.forward(x, q))
    t_bwd = timed(lambda: (net.backward(x, y), net.adam()))
    fwd_flops = rows * (2 * F_IN * HIDDEN + 2 * HIDDEN)
    bwd_flops = rows * (2 * F_IN * HIDDEN + 2 * HIDDEN + HIDDEN + 2 * F_IN * HIDDEN + 2 * HIDDEN)
    return {"rows": rows, "forward_s": t_fwd, "forward_rows_per_s": rows / t_fwd,
            "forward_tflops": fwd_flops / t_fwd / 1e12, "forward_hbm_gbs": rows * (64 + 4) / t_fwd / 1e9,
            "train_step_s": t_bwd, "train_rows_per_s": rows / t_bwd, "train_tflops": bwd_flops / t_bwd / 1e12,
            "train_hbm_gbs": rows * (64 + 4) / t_bwd / 1e9, "mfma_bf16_peak_tflops": 2500.0}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--mlp-bench", type=int, default=0,
                    help="only time the MLP kernels on this many random feature rows and print JSON")
    ap.add_argument("--instances", type=int, default=100000)
    ap.add_argument("--n-vars", type=int, default=2048)
    ap.add_argument("--label-sweeps", type=int, default=500)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--eval", type=int, default=256)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--out", default=WEIGHTS_JSON)
    ap.add_argument("--workers", type=int, default=16, help="host processes generating formulas")
    ap.add_argument("--equal-accuracy", type=int, default=0,
                    help="only compare the committed network's learned form with the plain method at equal "
                         "accuracy on this many held-out formulas and print JSON")
    ap.add_argument("--budget", type=int, default=20, help="sweeps of the learned form (--equal-accuracy)")
    ap.add_argument("--step", type=int, default=1, help="sweeps between the plain runs' counts (--equal-accuracy)")
    args = ap.parse_args(argv)
    if args.mlp_bench > 0:
        print(json.dumps(mlp_bench(args.mlp_bench)), flush=True)
        return 0
    if args.equal_accuracy > 0:
        net, _ = MLP.load()
        print(json.dumps(equal_accuracy(net, args.equal_accuracy, args.n_vars, args.seed,
                                        budget=args.budget, step=args.step)), flush=True)
        return 0
    pool = FormulaPool(args.workers)      # forked before the GPU is used

    def log(msg):
        print(f"[learned] {msg}", file=sys.stderr, flush=True)

    t0 = time.time()
    x, y = make_dataset(args.instances, args.n_vars, args.seed, sweeps=args.label_sweeps, log=log, pool=pool)
    pool.close()
    t1 = time.time()
    net = MLP(seed=args.seed)
    losses = train(net, x, y, epochs=args.epochs, log=log)
    t2 = time.time()
    ev = evaluate(net, args.eval, args.n_vars, args.seed)
    net.save(args.out, instances=args.instances, n_vars=args.n_vars, epochs=args.epochs,
             losses=losses, evaluation={str(k): v for k, v in ev.items()})
    print(json.dumps({"instances": args.instances, "label_s": t1 - t0, "train_s": t2 - t1,
                      "losses": losses, "evaluation": ev}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
