"""Benchmark of the block-Gibbs hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision f64|f32|mixed]
                    [--model padded|clustered]

Default workload: the uneven batch of 1024 formulas with N log-uniform in
[64, 16384] (C = 6N, K = 7, L = 8, seed 3), 64 chains each, FP32: size-class
launches of the sweep kernel forked over side streams and captured in one
hipGraph, their workgroup shapes autotuned before timing.  One step advances
every formula 500 sweeps on all its chains (one dispatch of 500 Gibbs rounds,
the appendix "Batching operations"); an instance is one formula so advanced.
``--workload plain_n4096_b64`` runs the single 4096-variable formula with its
64 chains (FP64 by default).  Inputs are resident in HBM before timing.

Prints ONE JSON line with throughput (instances/s), the ALU roofline of the
sweep kernels and the CPU oracle baseline.  The oracle legs run before the
GPU is touched: on one core, and on all cores (one process per chain slice);
a third process records teacher-forcing snapshots of a few chains, which the
GPU then replays sweep by sweep in the timed launch configuration to check
parity (the FP32 class: visible draws may differ only within the tie bound).
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
METRIC = "instances/sec at oracle-matched tolerance; fraction of HBM/MFMA roofline"
TIE = {"f32": 2e-6}              # FP32 class: |U - rho_oracle| of a draw allowed to differ
NU_RTOL = {"f32": 1e-5, "f64": 1e-12, "mixed": 1e-12}


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


# ---------------------------------------------------------------------------
# CPU oracle legs (child processes started before the GPU is initialised)
# ---------------------------------------------------------------------------

def _oracle_worker(job, barrier, out_q):
    """One oracle process: build the oracle plans of its formulas, wait at the
    barrier (so every process of a leg starts sweeping together), run its
    chains for the given sweeps and report wall-clock start/end of the sweep
    loop.  With record=True it also returns per-sweep teacher-forcing
    snapshots: the state before every sweep and |U - rho| of every visible
    draw, plus the smallest hidden-draw margin."""
    from oracle import clustered as CL
    from oracle import rbmsat as R
    plans = {}
    for f, t in job["formulas"].items():
        if job["size_rbms"] is not None:
            plans[f] = CL.ClusteredPlan(t["table"], t["n"], job["size_rbms"])
        else:
            plans[f] = R.plan(t["table"], t["n"], job["W"], job["b"])
    barrier.wait()
    t0 = time.time()
    snaps = {}
    for f, t in job["formulas"].items():
        ch = np.asarray(job["chains"], dtype=np.int64)
        st = R.initial(t["v0"][ch])
        temps = job["temps"][ch]
        seq = []
        for _ in range(job["sweeps"]):
            if job["record"]:
                seq.append(dict(v=st.v.copy(), nu=st.nu.copy(), s_max=st.s_max.copy(), best=st.best.copy(),
                                t=st.t))
            if job["size_rbms"] is not None:
                rec = CL.sweep(st, plans[f], temps, alpha=job["alpha"], seed=job["seed"], formula_id=f,
                               chain_ids=ch)
                hid = rec["hid_margin"]
            else:
                rec = R.sweep(st, plans[f], temps, alpha=job["alpha"], seed=job["seed"], formula_id=f,
                              chain_ids=ch, record=job["record"])
                hid = float(np.abs(rec["u_h"] - rec["p_h"]).min()) if job["record"] else None
            if job["record"]:
                seq[-1]["vis_margin"] = np.abs(rec["u_v"] - rec["rho"]).astype(np.float32)
                seq[-1]["hid_margin"] = hid
        if job["record"]:
            seq.append(dict(v=st.v.copy(), nu=st.nu.copy(), s_max=st.s_max.copy(), best=st.best.copy(), t=st.t))
            snaps[f] = seq
    out_q.put({"t0": t0, "t1": time.time(), "snaps": snaps})


def _run_leg(jobs):
    """Run one process per job (spawned interpreters: no torch, no GPU),
    released together by a barrier; returns (wall seconds of the sweep
    loops, results)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(len(jobs))
    q = ctx.Queue()
    env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in env_keys}
    for k in env_keys:                      # each oracle process computes on one core
        os.environ[k] = "1"
    try:
        procs = [ctx.Process(target=_oracle_worker, args=(j, barrier, q)) for j in jobs]
        for p in procs:
            p.start()
        res = [q.get() for _ in procs]
        for p in procs:
            p.join()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    if any(p.exitcode != 0 for p in procs):
        raise RuntimeError("an oracle process failed")
    return max(r["t1"] for r in res) - min(r["t0"] for r in res), res


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    logical = len(os.sched_getaffinity(0))
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return model, logical, min(logical, cap) if cap > 0 else logical


def oracle_legs(w, cpu_sweeps, progress):
    """Time the oracle on a bounded sample of the workload, single-core and
    on all cores, and record teacher-forcing snapshots for the GPU parity
    check.  Single formula: all chains x cpu_sweeps sweeps; batches: 16
    formulas spread over the sizes x all chains x 5 sweeps (about 25 s on
    one core for the 1024-formula batch).  Returns the timing summary and the
    snapshots."""
    batch = len(w.n_vars) > 1
    if batch:
        order = np.argsort(w.n_vars, kind="stable")
        pick = sorted({int(order[i]) for i in np.linspace(0, len(order) - 1, 16).astype(int)})
        chains = np.arange(w.chains)
        sweeps = 5
        par_chains = np.array(sorted({0, w.chains // 2 - 1, w.chains // 2, w.chains - 1}))
    else:
        pick, chains, sweeps = [0], np.arange(w.chains), cpu_sweeps
        par_chains = np.unique(np.linspace(0, w.chains - 1, min(8, w.chains)).astype(int))
    model, logical, cores = host_cpu()
    forms = {f: {"table": w.tables[f], "n": w.n_vars[f], "v0": w.v0[f]} for f in pick}
    base = dict(formulas=forms, W=w.W, b=w.b, temps=np.asarray(w.temps), alpha=w.alpha, seed=w.seed,
                size_rbms=w.size_rbms, sweeps=sweeps, record=False)
    work = float(len(chains) * sweeps * sum(w.n_vars[f] for f in pick))     # chain-sweep x variables
    step_work = w.chains * 500 * float(sum(w.n_vars))
    progress(f"oracle, 1 core: {len(pick)} formulas x {len(chains)} chains x {sweeps} sweeps")
    t1, _ = _run_leg([dict(base, chains=chains)])
    slices = [chains[k::cores] for k in range(cores) if len(chains[k::cores])]
    progress(f"oracle, {len(slices)} cores: one process per chain slice")
    tn, _ = _run_leg([dict(base, chains=s) for s in slices])
    progress(f"oracle snapshots for parity: {len(par_chains)} chains x {sweeps} sweeps")
    _, res = _run_leg([dict(base, chains=par_chains, record=True)])
    sample = (f"{len(pick)} formulas (N = {sorted(w.n_vars[f] for f in pick)}) x {len(chains)} chains x "
              f"{sweeps} sweeps" if batch else f"{len(chains)} chains x {sweeps} sweeps") + \
        " of the same workload (NumPy FP64), scaled to 500 sweeps of every formula and chain by the " \
        "chain-sweep x variable count"
    out = {"value": len(w.n_vars) / (tn / work * step_work), "unit": "instances/s", "cores": len(slices),
           "kind": "oracle", "sample": sample, "cpu_model": model, "host_logical_cpus": logical,
           "sample_seconds_all_cores": tn,
           "single_core": {"value": len(w.n_vars) / (t1 / work * step_work), "cores": 1,
                           "sample_seconds": t1},
           "chain_sweeps_per_s": w.chains * 500 * len(w.n_vars) / (tn / work * step_work)}
    return out, {"pick": pick, "chains": par_chains, "sweeps": sweeps, "snaps": res[0]["snaps"]}


def gpu_parity(plan, w, snap, precision, tie):
    """Teacher-forced replay of the oracle snapshots in the benchmark's own
    plan: before every sweep the sampled chains of the sampled formulas get
    the oracle's state, the plan runs one sweep (every formula), and the new
    state is compared with the oracle's: s_max and best exactly, nu within the
    class's relative bound, and every differing visible draw must be a tie
    (|U - rho_oracle| <= tie)."""
    import torch
    st = plan.new_state(w.v0)
    ch = snap["chains"]
    out = {"formulas": len(snap["pick"]), "chains": len(ch), "sweeps": snap["sweeps"], "teacher_forced": True,
           "v_mismatches": 0, "non_tie_mismatches": 0, "s_max_equal": True, "best_equal": True,
           "nu_max_rel_err": 0.0, "tie_bound": tie, "hidden_undecidable": 0}
    for s in range(snap["sweeps"]):
        for f in snap["pick"]:
            a = snap["snaps"][f][s]
            st.set_formula(f, v=a["v"], nu=a["nu"], s_max=a["s_max"], best=a["best"], chains=ch)
        st.set_t(snap["snaps"][snap["pick"][0]][s]["t"])
        plan.run(st, 1)
        torch.cuda.synchronize()
        for f in snap["pick"]:
            a, z = snap["snaps"][f][s], snap["snaps"][f][s + 1]
            v, nu, s_max, best = st.formula(f, chains=ch)
            diff = v != z["v"]
            out["v_mismatches"] += int(diff.sum())
            out["non_tie_mismatches"] += int(np.sum(a["vis_margin"][diff] > tie))
            out["s_max_equal"] &= bool(np.array_equal(s_max, z["s_max"]))
            out["best_equal"] &= bool(np.array_equal(best, z["best"]))
            out["nu_max_rel_err"] = max(out["nu_max_rel_err"], float(np.max(np.abs(nu - z["nu"]) / z["nu"])))
            if a["hid_margin"] is not None and a["hid_margin"] <= 3e-11:
                out["hidden_undecidable"] += 1
    out["ok"] = bool(out["non_tie_mismatches"] == 0 and out["s_max_equal"] and out["best_equal"]
                     and out["nu_max_rel_err"] <= NU_RTOL[precision])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uneven_1024x64")
    ap.add_argument("--precision", default=None, choices=["f64", "f32", "mixed"],
                    help="default: the workload's own (FP32 for the uneven batch, FP64 for plain_n4096_b64)")
    ap.add_argument("--sweeps", type=int, default=500)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--kernel", default="auto", choices=["auto", "push", "pull"])
    ap.add_argument("--split", type=int, default=0, help="workgroups per chain (0 = automatic)")
    ap.add_argument("--cpu-sweeps", type=int, default=25,
                    help="oracle sample sweeps on a single formula (all chains; about 13 s of CPU work on "
                         "plain_n4096_b64); batches use 5 sweeps of all chains of 16 formulas; 0 skips the "
                         "CPU legs and the parity check")
    ap.add_argument("--graph", type=int, default=-1, help="hipGraph replay (default: on for batches)")
    ap.add_argument("--tune", type=int, default=-1, help="autotune first (default: on for batches)")
    ap.add_argument("--model", default="padded", choices=["padded", "clustered"],
                    help="padded formula-RBM (K = 7, L = 8 for every clause) or the size-clustered one")
    ap.add_argument("--philox-probe", type=int, default=0,
                    help="only time the sweep generator alone (hp_philox_xor) on this many M Philox blocks "
                         "and report VALU lane-slots per block at the rated clock, then exit")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run y = -x over this many MiB (a plain streaming kernel whose "
                         "FETCH_SIZE / WRITE_SIZE calibrate the HBM counters), then exit")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(chains and formulas would shard across GPUs with no per-sweep exchange)",
              file=sys.stderr, flush=True)
        return 2

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.philox_probe > 0:
        # every SIMD lane of the chip busy: 256 CUs x 4 SIMDs x 64 lanes x 8 waves
        import torch
        from paper_2311_02101_amd import hp
        n_out = 256 * 4 * 64 * 8
        blocks = max(1, args.philox_probe * (1 << 20) // n_out)
        out = torch.empty(n_out, dtype=torch.int32, device="cuda")
        hp.philox_xor(1, 0, 0, 0, 0, blocks, n_out, out)         # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for rep in range(3):
            hp.philox_xor(1, 0, rep, 0, 0, blocks, n_out, out)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / 3
        calls = n_out * blocks
        print(json.dumps({"philox_blocks": calls, "seconds": sec, "blocks_per_s": calls / sec,
                          "lane_slots_per_block": PEAK_SLOTS * sec / calls,
                          "model_slots_per_block": PHILOX_SLOTS,
                          "note": "two interleaved blocks per step, first two rounds from per-sweep constants, "
                                  "plus about 3 XORs per block to reduce the words"}), flush=True)
        return 0

    if args.copy_probe_mib > 0:
        import torch
        dev = torch.device("cuda:0")
        n = args.copy_probe_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                          "launches": 3}), flush=True)
        return 0

    from paper_2311_02101_amd import workload as wl
    progress(f"workload {args.workload}: generating inputs")
    w = wl.config_workload(args.workload, **({"precision": args.precision} if args.precision else {}))
    precision = w.precision
    clustered = args.model == "clustered"
    w.size_rbms = wl.pretrained_size_rbms() if clustered else None

    cpu = snap = None
    if args.cpu_sweeps > 0:
        cpu, snap = oracle_legs(w, args.cpu_sweeps, progress)

    import torch
    from paper_2311_02101_amd import hp
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    B = w.chains
    L = w.W.shape[2]
    batch = len(w.n_vars) > 1
    use_graph = (args.graph if args.graph >= 0 else int(batch)) == 1
    plan = hp.Plan(w.tables, w.n_vars, w.W, w.b, chains=B, temps=w.temps,
                   precision=precision, alpha=w.alpha, seed=w.seed, threads=args.threads,
                   kernel=args.kernel, split=args.split, graph=use_graph, size_rbms=w.size_rbms)
    progress(f"planned: {plan.info()['n_buckets']} launch(es)")
    if (args.tune if args.tune >= 0 else int(batch)) == 1:
        plan.tune(n_sweeps=10)
        progress(f"tuned: workgroup sizes {plan.info()['bucket_threads']}, table layouts "
                 f"{plan.info()['bucket_kind']}")
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
    # the tuner's shapes vary a little from run to run (timing noise), so a
    # tuned batch's counters are keyed by "tuned"
    tuned = (args.tune if args.tune >= 0 else int(batch)) == 1
    tkey = "tuned" if tuned else ",".join(str(t) for t in info["bucket_threads"]) if batch else \
        str(info["bucket_threads"][0])
    traffic = measured_traffic(kernel_name, args.workload, precision, plan.split, tkey)
    N = w.n_vars[0] if not batch else int(sum(w.n_vars))
    C = w.tables[0].shape[1] if not batch else int(sum(t.shape[1] for t in w.tables))
    out = {
        "metric": METRIC,
        "value": value, "unit": "instances/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": precision, "data": "synthetic",
        "config": {"workload": args.workload, "formulas": len(w.n_vars), "model": args.model,
                   "n_vars": N, "clauses": C, "K": 7, "L": L if not clustered else "3 or len + 1",
                   "chains": B, "sweeps_per_step": args.sweeps, "temperatures": list(wl.FSTAR_PAIR),
                   "graph": use_graph, "tuned": tuned,
                   "threads": args.threads or "automatic", "kernel": args.kernel,
                   "launch": info, "parallelism": "single GPU"},
        "chain_sweeps_per_s": B * args.sweeps * instances / wall,
        "draws_per_s": draws * B * args.sweeps * args.steps / wall,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "T VALU lane-slots/s", "frac": achieved / PEAK_SLOTS,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "kernel": kernel_name + (" (size-class launches of one graph replay)" if batch else ""),
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "philox_calls_per_chain_sweep": calls, "draws_per_chain_sweep": draws},
    }
    if precision == "mixed":
        # two v_mfma_f32_32x32x16_bf16 per 32 clauses per chain-sweep (hidden
        # logits and contributions, four BF16 limb pairs each)
        tiles = sum(-(-t.shape[1] // 32) for t in w.tables)
        mfma_flops = tiles * 2 * (32 * 32 * 16 * 2) * B * args.sweeps
        out["mfma"] = {"flops_per_launch": mfma_flops, "achieved_tflops": mfma_flops / avg_launch_s / 1e12,
                       "peak_tflops": MFMA_BF16_PEAK / 1e12, "frac": mfma_flops / avg_launch_s / MFMA_BF16_PEAK}
    if cpu is not None:
        if precision == "f32":
            tie = TIE["f32"]
        else:
            # FP64 classes: contributions rounded to the fixed-point grid 2^-S
            slots = max(int(np.bincount(np.abs(t).ravel()).max()) for t in w.tables)
            tie = 0.25 * slots * 2.0 ** -(info["fx_shift"] + 1) + 1e-15
        progress("parity: teacher-forced replay of the oracle snapshots")
        cpu["parity"] = gpu_parity(plan, w, snap, precision, tie)
        out["cpu_baseline"] = cpu
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


if __name__ == "__main__":
    sys.exit(main())
