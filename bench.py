#!/usr/bin/env python3
"""Throughput of the explicit energy-conserving PIC step on one MI355X.

One "step" is one full ESEC2 step (predictor gather, push, both deposits, field updates,
Gamma correction with fallback count, energy record) over every particle.  The default
workload is the 1D-1V two-stream instability with 10,000,000 particles, 512 cells,
quadratic shapes and dt = 0.05.  Inputs are generated on the host, copied to HBM, and the
timed region (HIP events on the library's stream) covers only the steps.

Prints one JSON line: particle-steps/s, the roofline of the dominant kernel (pass B,
measured with HIP events around its launches), and the oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (FP64, 10M particles) at ≤1e-11 energy error; % HBM roofline"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per particle and launch of each particle pass (structure of
# arrays, FP64): pass A reads x and v; pass B reads x, v and writes x, v.
def alg_bytes(nv):
    state = 8 * (1 + nv)
    return {"pass_a": state, "pass_b": 2 * state}


def workload_for(name):
    import workloads
    return workloads.by_name(name)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="two_stream_1d1v_512c_10M")
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--deposit-mode", default="auto")
    ap.add_argument("--rebin-every", type=int, default=0)
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=8,
                    help="oracle steps of the same workload for the CPU baseline (0: skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the 1D grid would be all-reduced across GPUs; not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2411_09605_amd import Pic

    wl = workload_for(args.workload)
    print(f"[bench] workload {args.workload}: {wl.n_particles} particles, {wl.n_cells} cells, "
          f"order {wl.order}, dt {wl.dt}", file=sys.stderr, flush=True)
    knobs = dict(block_threads=args.block_threads, grid_blocks=args.grid_blocks,
                 deposit_mode=args.deposit_mode, rebin_every=args.rebin_every,
                 record_capacity=max(4096, args.steps + args.warmup + args.profile_steps + 8))
    gpu = Pic.from_workload(wl, device="cuda:0", **knobs)
    gpu.step(args.warmup)
    gpu.diagnostics()
    torch.cuda.synchronize()

    stream = gpu.stream
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    gpu.step(args.steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    recs = gpu.diagnostics()
    print(f"[bench] timed {args.steps} steps in {ms:.2f} ms", file=sys.stderr, flush=True)

    # per-kernel durations from HIP events around each launch (separate segment)
    prof = None
    if args.profile_steps > 0:
        gpu.profile(True)
        gpu.step(args.profile_steps)
        prof = gpu.profile_read()
        gpu.profile(False)
        gpu.diagnostics()

    n = wl.n_particles
    value = n * args.steps / (ms * 1e-3)
    kernels = {}
    roofline = None
    if prof:
        ab = alg_bytes(wl.nv)
        for k, (tms, cnt) in prof.items():
            if cnt:
                avg_us = tms / cnt * 1e3
                entry = {"avg_us": round(avg_us, 3), "launches": cnt}
                if k in ab:
                    gbs = ab[k] * n / (avg_us * 1e-6) / 1e9
                    entry["alg_GBps"] = round(gbs, 1)
                kernels[k] = entry
        b = kernels["pass_b"]
        roofline = {"bound": "hbm", "achieved": b["alg_GBps"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(b["alg_GBps"] / HBM_PEAK_GBS, 4),
                    "traffic": None, "kernel": "k_pass_b",
                    "alg_bytes_per_particle": alg_bytes(wl.nv)["pass_b"]}

    cpu = None
    if args.cpu_steps > 0:
        import oracle
        ost = oracle.State(wl)
        ost.run(0)                       # initial Gauss solve outside the timing
        c0 = time.perf_counter()
        ost.run(args.cpu_steps)
        cs = time.perf_counter() - c0
        cpu = {"value": n * args.cpu_steps / cs, "unit": "particle-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{args.cpu_steps} steps of the full {n}-particle workload, "
                         f"single-threaded C oracle, {cs:.1f} s"}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_particles": n, "n_cells": wl.n_cells,
                   "shape_order": wl.order, "scheme": wl.scheme, "dt": wl.dt,
                   "nv": wl.nv, "block_threads": args.block_threads,
                   "grid_blocks": args.grid_blocks, "deposit_mode": args.deposit_mode,
                   "rebin_every": args.rebin_every},
        "max_rel_energy_err": float(np.max(recs["rel_energy_err"])) if len(recs) else None,
        "fallbacks": int(np.sum(recs["fallbacks"])) if len(recs) else None,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    gpu.destroy()


if __name__ == "__main__":
    main()
