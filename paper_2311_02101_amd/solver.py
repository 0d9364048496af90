"""Sampling with the periodic unit-propagation exchange (Sec. 3.4; the
appendix program's exchange).

Every ``upp`` sweeps the chains' (v, nu) are copied to pinned host memory;
host threads run the prioritized unit propagation (``hp_unit_propagate``) on
every formula while the GPU samples ``upw`` more sweeps; then the returned
assignments are merged on the device (``hp_merge_candidates``: stack under the
current states, count, keep the best B per formula).  The GPU never waits for
the host except at the merge, which needs the host's result.

    python -m paper_2311_02101_amd.solver [--workload NAME] [--sweeps S] [--upp P] [--upw W]

runs the same workload plain, with the exchange, with replica exchange
between the temperatures (``--temper`` sweeps apart) and with both (same
seeds), plus the plain method given the slowest variant's wall time, and
prints the best satisfied-clause counts and the timings as one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import threading
import time

import numpy as np

from . import hp
from . import workload as wl


def _host_views(plan, host_v, host_nu):
    """Per-formula [B][N_f] numpy views of flat host buffers (state layout)."""
    out = []
    for f in range(plan.F):
        lo, hi = int(plan.var_offset[f]) * plan.B, int(plan.var_offset[f + 1]) * plan.B
        n = plan.n_vars[f]
        out.append((host_v[lo:hi].reshape(plan.B, n), host_nu[lo:hi].reshape(plan.B, n)))
    return out


class _Sampler:
    """Runs sweeps, inserting a replica-exchange round (``hp_temper``, parity
    alternating) after every ``every`` sweeps counted over the whole solve."""

    def __init__(self, plan, state, every, stream):
        self.plan, self.state, self.every, self.stream = plan, state, every, stream
        self.since = 0
        self.rounds = 0

    def advance(self, n):
        if self.every <= 0:
            self.plan.run(self.state, n, self.stream)
            return
        while n > 0:
            step = min(n, self.every - self.since)
            self.plan.run(self.state, step, self.stream)
            n -= step
            self.since += step
            if self.since == self.every:
                self.plan.temper(self.state, self.rounds % 2, self.stream)
                self.rounds += 1
                self.since = 0


def solve(plan, tables, state, sweeps, upp=0, upw=0, threads=0, stream=None, temper_every=0):
    """Advance ``state`` by ``sweeps`` sweeps with an exchange every ``upp``
    sweeps whose result is merged ``upw`` sweeps later (0 < upw < upp; upp = 0:
    no exchange) and, with temper_every > 0, a replica-exchange round after
    every temper_every sweeps.  Returns statistics."""
    import torch
    stream = torch.cuda.current_stream() if stream is None else stream
    sampler = _Sampler(plan, state, temper_every, stream)
    if upp <= 0:
        sampler.advance(sweeps)
        return {"temper_rounds": sampler.rounds}
    if not (0 < upw < upp):
        raise ValueError("need 0 < upw < upp")
    host_v = torch.empty(state.v.shape, dtype=torch.uint8, pin_memory=True)
    host_nu = torch.empty(state.nu.shape, dtype=state.nu.dtype, pin_memory=True)
    cand_host = torch.empty(state.v.shape, dtype=torch.uint8, pin_memory=True)
    cand = torch.empty_like(state.v)
    views = _host_views(plan, host_v.numpy(), host_nu.numpy())
    cand_views = _host_views(plan, cand_host.numpy(), host_nu.numpy())
    stats = {"exchanges": 0, "host_s": 0.0, "wait_s": 0.0}
    t = 0
    next_send = upp
    while t < sweeps:
        run_to = min(next_send, sweeps)
        sampler.advance(run_to - t)
        t = run_to
        if t < next_send:
            break
        next_send += upp
        if t + upw > sweeps:
            continue
        # send: snapshot (v, nu) into pinned memory, propagate on host threads
        with torch.cuda.stream(stream):
            host_v.copy_(state.v, non_blocking=True)
            host_nu.copy_(state.nu, non_blocking=True)
        ready = torch.cuda.Event()
        ready.record(stream)
        err = []

        def work():
            try:
                t0 = time.perf_counter()
                ready.synchronize()
                for f, (v, nu) in enumerate(views):
                    cand_views[f][0][...] = hp.unit_propagate(tables, plan.n_vars, f, v,
                                                              nu.astype(np.float64), threads)
                stats["host_s"] += time.perf_counter() - t0
            except Exception as e:          # re-raised on the caller's thread
                err.append(e)

        th = threading.Thread(target=work)
        th.start()
        sampler.advance(upw)                # the GPU keeps sampling meanwhile
        t += upw
        t0 = time.perf_counter()
        th.join()
        stats["wait_s"] += time.perf_counter() - t0
        if err:
            raise err[0]
        with torch.cuda.stream(stream):
            cand.copy_(cand_host, non_blocking=True)
        plan.merge_candidates(state, cand, stream)
        stats["exchanges"] += 1
    stats["temper_rounds"] = sampler.rounds
    return stats


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="plain_n4096_b64")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "mixed"])
    ap.add_argument("--sweeps", type=int, default=5000)
    ap.add_argument("--upp", type=int, default=500)
    ap.add_argument("--upw", type=int, default=100)
    ap.add_argument("--threads", type=int, default=16)
    ap.add_argument("--temper", type=int, default=10, help="sweeps between replica-exchange rounds")
    ap.add_argument("--targets", type=int, default=2, choices=[2, 16],
                    help="free-energy targets: the pair of the 1-accelerator runs or the 16-target list")
    ap.add_argument("--formulas", type=int, default=0, help="limit a batch workload to its first formulas")
    ap.add_argument("--model", default="padded", choices=["padded", "clustered"],
                    help="padded formula-RBM or the size-clustered one (an RBM per clause length)")
    args = ap.parse_args(argv)
    w = wl.config_workload(args.workload, precision=args.precision)
    tables, n_vars, v0 = w.tables, w.n_vars, w.v0
    W, b, temps = w.W, w.b, w.temps
    targets = wl.FSTAR_PAIR
    if args.targets == 16:
        targets = wl.FSTAR_16
        W, b, _ = wl.pretrained_rbm(7, wl.FSTAR_16)
        temps = wl.default_temperatures(w.chains, 16)
    size_rbms = wl.pretrained_size_rbms(targets) if args.model == "clustered" else None
    if args.formulas:
        tables, n_vars, v0 = tables[:args.formulas], n_vars[:args.formulas], v0[:args.formulas]
    out = {"workload": args.workload, "sweeps": args.sweeps, "upp": args.upp, "upw": args.upw,
           "temper_every": args.temper, "targets": args.targets, "chains": w.chains, "formulas": len(tables),
           "host_threads": args.threads, "model": args.model}

    def run(sweeps, upp=0, temper=0):
        plan = hp.Plan(tables, n_vars, W, b, chains=w.chains, temps=temps, precision=args.precision,
                       alpha=w.alpha, seed=w.seed, size_rbms=size_rbms)
        st = plan.new_state(v0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = solve(plan, tables, st, sweeps, upp, args.upw, args.threads, temper_every=temper)
        plan.run(st, 0)                     # count the final states too
        torch.cuda.synchronize()
        plan.check()                        # a failed split exchange voids the run
        wall = time.perf_counter() - t0
        best = [int(st.formula(f)[2].max()) for f in range(len(tables))]
        if temper:
            # chains that ended at another temperature than they started at
            stats["moved_chains"] = float(np.mean(plan.current_temps() != np.asarray(temps)[None, :]))
        plan.free()
        return {"sweeps": sweeps, "best_mean": float(np.mean(best)), "best": best[:8], "seconds": wall, **stats}

    out["plain"] = run(args.sweeps)
    out["with_up"] = run(args.sweeps, upp=args.upp)
    out["with_tempering"] = run(args.sweeps, temper=args.temper)
    out["with_both"] = run(args.sweeps, upp=args.upp, temper=args.temper)
    # the plain method given the wall time of the slowest variant
    slowest = max(out[k]["seconds"] for k in ("with_up", "with_tempering", "with_both"))
    eq = int(round(args.sweeps * slowest / out["plain"]["seconds"]))
    out["plain_equal_time"] = run(max(eq, args.sweeps))
    for k in ("with_up", "with_tempering", "with_both"):
        out["gain_" + k] = out[k]["best_mean"] - out["plain_equal_time"]["best_mean"]
    for k in ("plain", "with_up", "with_tempering", "with_both", "plain_equal_time"):
        print(f"[solver] {k}: {out[k]['sweeps']} sweeps, mean best {out[k]['best_mean']:.2f} "
              f"in {out[k]['seconds']:.3f} s", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
