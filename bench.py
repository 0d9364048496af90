"""Benchmark of the block-Gibbs hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--precision f64|f32] [--workload NAME]
                    [--model padded|clustered]

Default workload: the formula N = 4096, C = 24576 (K = 7, L = 8) with its 64
chains.  One step advances every formula of the workload 500 sweeps on all
its chains (one dispatch of 500 Gibbs rounds, the appendix "Batching
operations"); an instance is one formula so advanced.  Inputs are resident in
HBM before timing.  Prints ONE JSON line with throughput (instances/s), the
ALU roofline of the sweep kernels and the CPU oracle baseline timed on a
bounded sample.  --workload uneven_1024x64 runs the batch of 1024 formulas of
log-uniform size 64..16384 (64 chains each) through size-class launches in
one hipGraph, autotuned first.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# ---------------------------------------------------------------------------
# ALU cost model of one chain-sweep (K = 7, L = 8, C = 6N):
#   Philox4x32-10 calls: C * ceil(L/4) hidden + ceil(N/4) visible
#   one call = 10 rounds x (2 v_mad_u64_u32 + 2 three-input XORs, gfx950's
#            v_bitop3_b32) = 40 VALU instructions, each one issue slot per
#            lane (a Philox-only loop with 2-input XORs measures 55 lane-slots
#            per call for its ~58 instructions at the rated clock), less the
#            3 of the first two rounds that depend only on the counter words
#            shared by a whole chain-sweep (computed once per chain-sweep):
#            37 per call
#   each Bernoulli draw adds a shift and an unsigned compare (2 slots)
# Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32 T lane-slots/s.
# ---------------------------------------------------------------------------
PHILOX_SLOTS = 37
DRAW_SLOTS = 2
PEAK_SLOTS = 256 * 64 * 2.4e9
MFMA_BF16_PEAK = 2.5e15          # dense BF16 MFMA, MI355X


def chain_sweep_work(n_vars, n_clauses, L):
    calls = n_clauses * -(-L // 4) + -(-n_vars // 4)
    draws = n_clauses * L + n_vars
    return calls, draws, calls * PHILOX_SLOTS + draws * DRAW_SLOTS


def clause_lengths(table):
    """Length of every clause of a padded [K][C] table: K minus the trailing
    copies of its first literal."""
    t = np.asarray(table)
    same = t == t[:1]
    k = t.shape[0]
    lens = np.full(t.shape[1], k)
    for j in range(k - 1, 0, -1):
        run = np.all(same[j:], axis=0)
        lens = np.where(run, j, lens)
    return lens


def chain_sweep_work_clustered(n_vars, table):
    """The same model for the size-clustered formula-RBM: a clause of length
    len draws L = 3 hidden units (one Philox call) when len <= 3, else len + 1
    units (two calls)."""
    lens = clause_lengths(table)
    big = lens > 3
    calls = int(np.sum(np.where(big, 2, 1))) + -(-n_vars // 4)
    draws = int(np.sum(np.where(big, lens + 1, 3))) + n_vars
    return calls, draws, calls * PHILOX_SLOTS + draws * DRAW_SLOTS


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "mixed"])
    ap.add_argument("--workload", default="plain_n4096_b64")
    ap.add_argument("--sweeps", type=int, default=500)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--kernel", default="auto", choices=["auto", "push", "pull"])
    ap.add_argument("--split", type=int, default=0, help="workgroups per chain (0 = automatic)")
    ap.add_argument("--cpu-sweeps", type=int, default=25,
                    help="sweeps of the oracle sample (all chains; about 13 s of CPU work on the "
                         "default workload); 0 skips the CPU leg")
    ap.add_argument("--graph", type=int, default=-1, help="hipGraph replay (default: on for batches)")
    ap.add_argument("--tune", type=int, default=-1, help="autotune first (default: on for batches)")
    ap.add_argument("--model", default="padded", choices=["padded", "clustered"],
                    help="padded formula-RBM (K = 7, L = 8 for every clause) or the size-clustered one")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run y = -x over this many MiB (a plain streaming kernel whose "
                         "FETCH_SIZE / WRITE_SIZE calibrate the HBM counters), then exit")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(chains and formulas would shard across GPUs with no per-sweep exchange)",
              file=sys.stderr, flush=True)
        return 2

    import torch
    from paper_2311_02101_amd import hp, workload as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                          "launches": 3}), flush=True)
        return 0

    progress(f"workload {args.workload}: generating inputs")
    w = wl.config_workload(args.workload, precision=args.precision)
    B = w.chains
    L = w.W.shape[2]
    batch = len(w.n_vars) > 1
    use_graph = (args.graph if args.graph >= 0 else int(batch)) == 1
    clustered = args.model == "clustered"
    w.size_rbms = wl.pretrained_size_rbms() if clustered else None
    plan = hp.Plan(w.tables, w.n_vars, w.W, w.b, chains=B, temps=w.temps,
                   precision=args.precision, alpha=w.alpha, seed=w.seed, threads=args.threads,
                   kernel=args.kernel, split=args.split, graph=use_graph, size_rbms=w.size_rbms)
    progress(f"planned: {plan.info()['n_buckets']} launch(es)")
    if (args.tune if args.tune >= 0 else int(batch)) == 1:
        plan.tune(n_sweeps=3)
        progress(f"tuned: workgroup sizes {plan.info()['bucket_threads']}")
    st = plan.new_state(w.v0, device=dev)
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        plan.run(st, args.sweeps, stream)
        torch.cuda.synchronize()
        progress(f"warmup step {i + 1}/{args.warmup} done")

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        plan.run(st, args.sweeps, stream)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.check()
    progress(f"timed {args.steps} steps in {wall:.3f} s")
    launch_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    avg_launch_s = float(np.mean(launch_ms)) * 1e-3

    instances = args.steps * len(w.n_vars)
    value = instances / wall
    calls = draws = slots = 0
    for n, t in zip(w.n_vars, w.tables):
        c1, d1, s1 = chain_sweep_work_clustered(n, t) if clustered else chain_sweep_work(n, t.shape[1], L)
        calls, draws, slots = calls + c1, draws + d1, slots + s1
    per_launch_slots = slots * B * args.sweeps
    achieved = per_launch_slots / avg_launch_s
    kernel_name = ("sweep_pull_kernel" if args.kernel == "pull" else
                   "sweep_split_kernel" if plan.split > 1 else "sweep_push_kernel")
    info = plan.info()
    traffic = measured_traffic(kernel_name, args.workload, args.precision, plan.split,
                               info["bucket_threads"][0])
    N = w.n_vars[0] if not batch else int(sum(w.n_vars))
    C = w.tables[0].shape[1] if not batch else int(sum(t.shape[1] for t in w.tables))
    out = {
        "metric": "instances/sec at oracle-matched tolerance; fraction of HBM/MFMA roofline",
        "value": value, "unit": "instances/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": args.workload, "formulas": len(w.n_vars), "model": args.model,
                   "n_vars": N, "clauses": C, "K": 7, "L": L if not clustered else "3 or len + 1",
                   "chains": B, "sweeps_per_step": args.sweeps, "temperatures": list(wl.FSTAR_PAIR),
                   "graph": use_graph,
                   "threads": plan_threads(args.threads), "kernel": args.kernel,
                   "launch": info,
                   "parallelism": "single GPU"},
        "chain_sweeps_per_s": B * args.sweeps * instances / wall,
        "draws_per_s": draws * B * args.sweeps * args.steps / wall,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "T VALU lane-slots/s", "frac": achieved / PEAK_SLOTS,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "kernel": kernel_name,
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "philox_calls_per_chain_sweep": calls, "draws_per_chain_sweep": draws},
    }
    if args.precision == "mixed":
        # two v_mfma_f32_32x32x16_bf16 per 32 clauses per chain-sweep (hidden
        # logits and contributions, four BF16 limb pairs each)
        tiles = sum(-(-t.shape[1] // 32) for t in w.tables)
        mfma_flops = tiles * 2 * (32 * 32 * 16 * 2) * B * args.sweeps
        out["mfma"] = {"flops_per_launch": mfma_flops, "achieved_tflops": mfma_flops / avg_launch_s / 1e12,
                       "peak_tflops": MFMA_BF16_PEAK / 1e12, "frac": mfma_flops / avg_launch_s / MFMA_BF16_PEAK}
    if args.cpu_sweeps > 0:
        out["cpu_baseline"] = cpu_baseline(w, plan, args.cpu_sweeps, args.precision, dev)
    print(json.dumps(out), flush=True)
    plan.free()
    return 0


def measured_traffic(kernel, workload, precision, split, threads):
    """HBM bytes per launch from the committed counter runs (profiles/traffic.json),
    or None when no run matches this launch or the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec["entries"].get(f"{kernel}|{workload}|{precision}|G{split}|T{threads}")
    if ent is None:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != ent["sources_sha256"]:
        return None
    return (ent["fetch_kib"] * ent["fetch_factor"] + ent["write_kib"] * ent["write_factor"]) * 1024.0


def plan_threads(t):
    return t if t else 1024


def cpu_baseline(w, plan, sweeps, precision, dev):
    """Time the oracle (as it stands) on a bounded sample of the workload and
    compare the GPU's result for the same sample (parity of the timed
    configuration).  Single formula: all chains for ``sweeps`` sweeps.
    Batches: 8 formulas spread over the sizes, 4 chains each, 2 sweeps.
    The rate is scaled to instances/s of the whole workload by its total
    chain-sweep work, weighted by formula size."""
    import torch
    from oracle import clustered as CL
    from oracle import rbmsat as R

    batch = len(w.n_vars) > 1
    if batch:
        order = np.argsort(w.n_vars)
        pick = [int(order[i]) for i in np.linspace(0, len(order) - 1, 8).astype(int)]
        chains, sw = np.arange(4), 2
    else:
        pick, chains, sw = [0], np.arange(w.chains), sweeps
    el = 0.0
    work_done = 0.0
    parity = {"v_mismatches": 0, "s_max_equal": True, "best_equal": True, "nu_max_rel_err": 0.0}
    st = plan.new_state(w.v0, device=dev)
    plan.run(st, sw)
    torch.cuda.synchronize()
    for f in pick:
        ost = R.initial(w.v0[f][chains])
        t0 = time.perf_counter()
        if w.size_rbms is not None:
            cp = CL.ClusteredPlan(w.tables[f], w.n_vars[f], w.size_rbms)
            CL.run(ost, cp, w.temps[chains], sw, alpha=w.alpha, seed=w.seed, formula_id=f, chain_ids=chains)
        else:
            op = R.plan(w.tables[f], w.n_vars[f], w.W, w.b)
            R.run(ost, op, w.temps[chains], sw, alpha=w.alpha, seed=w.seed, formula_id=f,
                  chain_ids=chains)
        el += time.perf_counter() - t0
        work_done += len(chains) * sw * w.n_vars[f]
        v, nu, s_max, best = st.formula(f)
        v, nu, s_max, best = v[chains], nu[chains], s_max[chains], best[chains]
        parity["v_mismatches"] += int(np.sum(v != ost.v))
        parity["s_max_equal"] &= bool(np.array_equal(s_max, ost.s_max))
        parity["best_equal"] &= bool(np.array_equal(best, ost.best))
        parity["nu_max_rel_err"] = max(parity["nu_max_rel_err"],
                                       float(np.max(np.abs(nu - ost.nu) / ost.nu)))
    # seconds per (chain-sweep x variable), then per step of the workload
    rate = el / work_done
    step_work = w.chains * 500 * float(sum(w.n_vars))
    per_step = rate * step_work
    sample = (f"{len(pick)} formulas (N = {sorted(w.n_vars[f] for f in pick)}) x {len(chains)} chains "
              f"x {sw} sweeps" if batch else f"{w.chains} chains x {sw} sweeps") + \
        f" of the same workload ({el:.1f} s single-threaded NumPy FP64), scaled to 500 sweeps"
    return {"value": len(w.n_vars) / per_step, "unit": "instances/s", "cores": 1, "kind": "oracle",
            "sample": sample, "chain_sweeps_per_s": w.chains * 500 * len(w.n_vars) / per_step,
            "parity": parity}


if __name__ == "__main__":
    sys.exit(main())
