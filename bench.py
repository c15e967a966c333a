#!/usr/bin/env python3
"""Throughput of the explicit energy-conserving PIC step on one MI355X.

One "step" is one full ESEC2 step (predictor gather, push, both deposits, field updates,
Gamma correction with fallback count, energy record) over every particle.  The default
workload is the 1D-1V two-stream instability with 10,000,000 particles, 512 cells,
quadratic shapes and dt = 0.05.  Inputs are generated on the host, copied to HBM, and the
timed region (HIP events on the library's stream) covers only the steps.

Prints one JSON line: particle-steps/s, the roofline of the dominant kernel (pass B,
measured with HIP events around its launches), and the oracle timed on the host cores.

``--form adjoint`` times the adjoint form on the two-stream gradient workload (1e6
particles, 256 cells, 500 steps, 8 density modes): the loss forward with checkpoints
every 50 steps plus the reverse sweep, against the plain forward step on the same run.

``--form batched`` instead times the batched ensemble (512 Landau runs of 10^4 .. 10^6
particles, about 1.1e8 in all) advanced together from a replayed hipGraph, with the launch
shape picked by the autotuner, against the plain step run sequentially over the same
runs; it prints one JSON line of its own.
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
# arrays, FP64): pass A reads x and v; pass B reads x, v and writes x, v.  ESEC1 runs one
# pass per step (reported as pass B), which reads and writes the state once.
def alg_bytes(nv, scheme="esec2"):
    state = 8 * (1 + nv)
    if scheme in ("esec1", "standard"):
        # one particle pass per step (the standard scheme's field launch, timed as
        # pass A, moves no particle data)
        return {"pass_b": 2 * state}
    return {"pass_a": state, "pass_b": 2 * state}


PROFILE_DIR = os.path.join(ROOT, "profiles")


def source_digest():
    """Digest of the GPU sources; a stored counter profile applies only to the same one."""
    import hashlib
    h = hashlib.sha256()
    for rel in ("paper_2411_09605_amd/csrc/pic_device.hpp", "paper_2411_09605_amd/csrc/pic_adjoint.hpp",
                "paper_2411_09605_amd/csrc/pic_lib.hip", "paper_2411_09605_amd/csrc/pic_types.hpp",
                "paper_2411_09605_amd/csrc/pic_host.cpp", "include/pic.h"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload, config):
    """HBM bytes per launch of pass B from the stored counter profile of this workload and
    launch shape, or None when there is none or the kernels changed since."""
    path = os.path.join(PROFILE_DIR, f"{workload}_pass_b_traffic.json")
    try:
        with open(path) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        return None
    if doc.get("source_digest") != source_digest():
        return None
    for k in ("block_threads", "grid_blocks", "rebin_every", "deposit_mode", "scheme"):
        if doc.get("config", {}).get(k) != config.get(k):
            return None
    return doc.get("traffic_bytes_per_launch")


def copy_calibration():
    """Plain copies of 160 MB (1e7 x 2 doubles): the bytes each counter should report."""
    import torch
    a = torch.ones(20_000_000, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read_per_launch": a.numel() * 8,
                      "bytes_written_per_launch": a.numel() * 8, "launches": 10}), flush=True)


def energy_report(recs):
    """Energy error over the run: the largest |TE - TE0| / TE0, the largest before the
    first Gamma fallback (the method conserves energy exactly until then), the last step
    at which the error is still within 1e-11, and the largest of the paper's measure
    delta^n = (TE^n - min_k TE^k) / TE^0 over the records (section 5.1)."""
    import numpy as np
    err = recs["rel_energy_err"]
    clean = recs["fallbacks_total"] == 0
    bad = np.nonzero(err > 1e-11)[0]
    tot = recs["total"]
    return {"max_rel_err": float(err.max()),
            "max_delta_n": float(((tot - tot.min()) / tot[0]).max()),
            "max_rel_err_before_first_fallback": float(err[clean].max()) if clean.any() else None,
            "first_fallback_step": int(recs["step"][~clean][0]) if (~clean).any() else None,
            "within_1e-11_through_step": int(recs["step"][bad[0] - 1]) if len(bad)
            else int(recs["step"][-1]),
            "fallbacks": int(recs["fallbacks_total"][-1]),
            "steps_recorded": int(len(recs))}


def bench_batched(args):
    """Batched ensemble: aggregate particle-steps/s, against plain steps run by run."""
    import numpy as np
    import torch
    import workloads
    from paper_2411_09605_amd import Pic, PicBatch, pack_runs
    from paper_2411_09605_amd import autotune

    runs = workloads.batched_landau()
    ntot = sum(r.n_particles for r in runs)
    print(f"[bench] batched: {len(runs)} runs, {ntot} particles", file=sys.stderr, flush=True)
    packed = pack_runs(runs, "cuda:0")
    tuned = autotune.tune(runs, packed=packed, use_cache=False)
    print(f"[bench] tuned {tuned['block_threads']} threads, chunk {tuned['chunk']}",
          file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    G = args.graph_steps
    steps = max(G, args.steps // G * G) if G > 0 else args.steps
    with torch.cuda.stream(stream):
        b = PicBatch(packed=packed, block_threads=tuned["block_threads"], chunk=tuned["chunk"],
                     graph_steps=G, stream=stream,
                     record_capacity=steps + args.warmup + 8)
        b.step(args.warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    value = ntot * steps / (ms * 1e-3)
    per_run = [energy_report(b.diagnostics(k)) for k in range(len(runs))]
    clean = [e["max_rel_err"] for e in per_run if e["fallbacks"] == 0]
    b.destroy()
    del b, packed
    torch.cuda.empty_cache()
    print(f"[bench] batched {steps} steps in {ms:.2f} ms", file=sys.stderr, flush=True)

    # the plain step, run after run, on the same runs
    ctxs = [Pic.from_workload(r, device="cuda:0") for r in runs]
    for c in ctxs:
        c.step(1)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    cur = torch.cuda.current_stream()
    s0.record(cur)
    for c in ctxs:
        c.step(args.seq_steps)
    s1.record(cur)
    torch.cuda.synchronize()
    seq_ms = s0.elapsed_time(s1)
    seq_value = ntot * args.seq_steps / (seq_ms * 1e-3)
    for c in ctxs:
        c.destroy()
    alg = alg_bytes(1)
    step_bytes = (alg["pass_a"] + alg["pass_b"]) * ntot
    achieved = step_bytes / (ms / steps * 1e-3) / 1e9
    out = {
        "metric": "aggregate particle-steps/s, batched ensemble of 512 Landau runs (FP64)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batched_landau_512runs", "n_runs": len(runs),
                   "n_particles_total": ntot, "shape_order": runs[0].order,
                   "scheme": runs[0].scheme, "dt": runs[0].dt, "graph_steps": G,
                   "block_threads": tuned["block_threads"], "chunk": tuned["chunk"]},
        "sequential_plain": {"value": seq_value, "steps": args.seq_steps,
                             "ms_per_step": seq_ms / args.seq_steps},
        "speedup_vs_sequential": value / seq_value,
        "energy": {"runs_without_fallback": len(clean),
                   "max_rel_err_runs_without_fallback": max(clean) if clean else None,
                   "runs_with_fallbacks": len(runs) - len(clean),
                   "fallbacks": int(sum(e["fallbacks"] for e in per_run))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole step (k_batch_pass_a + k_batch_pass_b)",
                     "alg_bytes_per_particle_step": alg["pass_a"] + alg["pass_b"]},
        "autotune": tuned["trials"],
    }
    print(json.dumps(out), flush=True)


def bench_dt_sweep(args):
    """Section 5.1 (Fig. maxerrs_vs_dt): maximum energy error and Gamma fallbacks against
    dt for ESEC2, ESEC1 and the standard scheme on the Landau workload (1e5 particles, 64
    cells, tent, alpha 0.01) over t = 20, in 1D-1V and with the paper's two velocity
    components (v_y thermal, run as 1D-3V).  One JSON line; the headline value is ESEC2's
    largest energy error with two velocity components up to dt = 1."""
    import numpy as np
    import torch
    import workloads
    from paper_2411_09605_amd import Pic

    T = 20.0
    rows = []
    for variant, builder in (("1v", workloads.landau), ("2v", workloads.landau_2v)):
        for dt in (0.05, 0.1, 0.2, 0.4, 0.7, 1.0):
            steps = int(round(T / dt))
            for scheme in ("esec2", "esec1", "standard"):
                wl = builder(n_particles=100_000, n_cells=64, dt=dt, steps=steps)
                g = Pic.from_workload(wl, scheme=scheme, device="cuda:0",
                                      record_capacity=steps + 8)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(g.stream)
                g.step(steps)
                e1.record(g.stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                recs = g.diagnostics()
                g.destroy()
                en = energy_report(recs)
                ab = sum(alg_bytes(wl.nv, scheme).values()) * wl.n_particles
                gbs = ab / (ms / steps * 1e-3) / 1e9
                rows.append({"velocity_space": variant, "dt": dt, "scheme": scheme,
                             "steps": steps, "max_rel_err": en["max_rel_err"],
                             "max_delta_n": en["max_delta_n"], "fallbacks": en["fallbacks"],
                             "max_fallbacks_per_step": int(recs["fallbacks"].max()),
                             "ms_per_step": ms / steps, "step_GBps": round(gbs, 1),
                             "step_frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4)})
                print(f"[bench] dt sweep {variant} dt {dt} {scheme}: err {en['max_rel_err']:.2e}"
                      f" fallbacks {en['fallbacks']}", file=sys.stderr, flush=True)
    head = max(r["max_rel_err"] for r in rows if r["velocity_space"] == "2v"
               and r["scheme"] == "esec2")
    total_steps = sum(r["steps"] for r in rows)
    total_ms = sum(r["ms_per_step"] * r["steps"] for r in rows)
    out = {"metric": "max fractional energy error vs dt, Landau 1e5 x 64 (FP64); ESEC2 with "
                     "two velocity components, dt <= 1",
           "value": head, "unit": "fractional energy error", "n_gpus": 1,
           "steps": total_steps, "warmup": 0, "ms_per_step": total_ms / total_steps,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "landau_1d1v_64c_100k and landau_2v_64c_100k", "t_end": T,
                      "schemes": ["esec2", "esec1", "standard"]},
           "rows": rows}
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Adjoint form: (forward + backward) time against the forward-only plain step."""
    import numpy as np
    import torch
    import workloads
    from paper_2411_09605_amd import Pic, PicAdjoint

    wl = workloads.by_name("adjoint_two_stream_256c_1M")
    m = wl.meta
    n, N = wl.n_particles, wl.steps
    every = 50
    adj = PicAdjoint.from_workload(wl, checkpoint_every=every)
    theta = (m["alphas"], m["v_beam"], m["v_spread"])
    for _ in range(2):                                   # warm-up
        adj.forward(*theta)
        adj.backward(1.0)
    torch.cuda.synchronize()
    reps = 3
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    f_ms, b_ms = [], []
    for _ in range(reps):
        ev[0].record(adj.stream)
        adj.forward(*theta, sync=False)
        ev[1].record(adj.stream)
        adj.backward(1.0, sync=False)
        ev[2].record(adj.stream)
        torch.cuda.synchronize()
        f_ms.append(ev[0].elapsed_time(ev[1]))
        b_ms.append(ev[1].elapsed_time(ev[2]))
    J = float(adj.loss.cpu()[0])
    grad = adj.grad.cpu().numpy().tolist()
    recs = adj.records()
    adj.destroy()
    # the plain step on the same run (same sampled particles as the generator's)
    gpu = Pic.from_workload(wl, device="cuda:0", record_capacity=N + 8)
    gpu.step(20)
    gpu.diagnostics()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(gpu.stream)
    gpu.step(N)
    e1.record(gpu.stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    gpu.destroy()
    fb = float(np.median(f_ms))
    bb = float(np.median(b_ms))
    total = fb + bb
    out = {
        "metric": "adjoint (forward + backward) time vs forward-only plain step, two-stream "
                  "gradient workload (FP64)",
        "value": n * N / (total * 1e-3), "unit": "particle-steps/s (forward + backward)",
        "n_gpus": 1, "steps": N, "warmup": 2, "ms_per_step": total / N,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "adjoint_two_stream_256c_1M", "n_particles": n,
                   "n_cells": wl.n_cells, "shape_order": wl.order, "dt": wl.dt,
                   "n_modes": len(m["alphas"]), "checkpoint_every": every},
        "forward_ms": fb, "backward_ms": bb, "plain_forward_ms": plain_ms,
        "ratio_to_plain_forward": total / plain_ms,
        "loss": J, "grad": grad,
        "energy": energy_report(recs),
    }
    print(json.dumps(out), flush=True)


def host_info():
    """The benchmark host's CPU: logical CPUs this process may use and the model name."""
    info = {"nproc": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else os.cpu_count(), "cpu_count": os.cpu_count(), "cpu_model": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return info


def workload_for(name):
    import workloads
    return workloads.by_name(name)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="two_stream_1d1v_512c_10M")
    ap.add_argument("--scheme", default=None,
                    choices=("esec2", "esec1", "emec_li", "emec_psatd", "emec_lf", "standard"),
                    help="scheme to run the workload with (default: the workload's own)")
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--deposit-mode", default="auto")
    ap.add_argument("--rebin-every", type=int, default=0)
    ap.add_argument("--deterministic", action="store_true",
                    help="PIC_F_DETERMINISTIC (bit-reproducible current sums)")
    ap.add_argument("--dt", type=float, default=None,
                    help="time step instead of the workload's (e.g. EMEC(LF) needs c dt <= h)")
    ap.add_argument("--charge-conserving", action="store_true",
                    help="PIC_F_CHARGE_CONSERVING (exact charge conservation; ESEC2 with "
                         "tent shapes: the workload is run with shape order 1)")
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle steps of the same workload for the CPU baseline (0: skip)")
    ap.add_argument("--late-start", type=int, default=1000,
                    help="also time --late-steps steps from this step on, after the "
                         "instability has saturated (0: skip)")
    ap.add_argument("--late-steps", type=int, default=20)
    ap.add_argument("--form", choices=("plain", "batched", "adjoint", "dt_sweep"), default="plain")
    ap.add_argument("--graph-steps", type=int, default=50,
                    help="batched form: steps per captured hipGraph")
    ap.add_argument("--seq-steps", type=int, default=20,
                    help="batched form: steps of the sequential plain-step comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of known size (for scaling the HBM "
                         "counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the 1D grid would be all-reduced across GPUs; not built)", file=sys.stderr)
        sys.exit(2)

    if args.form == "batched":
        return bench_batched(args)
    if args.form == "adjoint":
        return bench_adjoint(args)
    if args.form == "dt_sweep":
        return bench_dt_sweep(args)

    import numpy as np
    import torch
    from paper_2411_09605_amd import Pic

    wl = workload_for(args.workload)
    if args.scheme:
        wl.scheme = args.scheme
    if args.charge_conserving:
        wl.order = 1
    if args.dt is not None:
        wl.dt = args.dt
    print(f"[bench] workload {args.workload}: {wl.n_particles} particles, {wl.n_cells} cells, "
          f"order {wl.order}, dt {wl.dt}", file=sys.stderr, flush=True)
    knobs = dict(block_threads=args.block_threads, grid_blocks=args.grid_blocks,
                 deposit_mode=args.deposit_mode, rebin_every=args.rebin_every,
                 deterministic=args.deterministic, charge_conserving=args.charge_conserving,
                 record_capacity=max(4096, args.steps + args.warmup + args.profile_steps
                                     + args.late_start + args.late_steps + 8))
    gpu = Pic.from_workload(wl, device="cuda:0", **knobs)
    gpu.step(args.warmup)
    warm_recs = gpu.diagnostics()
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
    energy = energy_report(np.concatenate([warm_recs, recs]))

    # per-kernel durations from HIP events around each launch (separate segment)
    prof = None
    prof_recs = []
    if args.profile_steps > 0:
        gpu.profile(True)
        gpu.step(args.profile_steps)
        prof = gpu.profile_read()
        gpu.profile(False)
        prof_recs = [gpu.diagnostics()]

    # a window after the instability has saturated (particles no longer move as two
    # beams; the fallback Gamma := 1 appears), reached by running the steps in between
    late = None
    done = args.warmup + args.steps + (args.profile_steps if args.profile_steps > 0 else 0)
    if args.late_start > done:
        gpu.step(args.late_start - done)
        skip_recs = gpu.diagnostics()
        torch.cuda.synchronize()
        l0 = torch.cuda.Event(enable_timing=True)
        l1 = torch.cuda.Event(enable_timing=True)
        l0.record(stream)
        gpu.step(args.late_steps)
        l1.record(stream)
        torch.cuda.synchronize()
        lms = l0.elapsed_time(l1)
        all_recs = np.concatenate([warm_recs, recs] + prof_recs + [skip_recs, gpu.diagnostics()])
        late = {"start_step": args.late_start, "steps": args.late_steps,
                "ms_per_step": lms / args.late_steps,
                "value": wl.n_particles * args.late_steps / (lms * 1e-3),
                "energy_through_window": energy_report(all_recs)}

    n = wl.n_particles
    value = n * args.steps / (ms * 1e-3)
    kernels = {}
    roofline = None
    if prof:
        ab = alg_bytes(wl.nv, wl.scheme)
        for k, (tms, cnt) in prof.items():
            if cnt:
                avg_us = tms / cnt * 1e3
                entry = {"avg_us": round(avg_us, 3), "launches": cnt}
                if k in ab:
                    gbs = ab[k] * n / (avg_us * 1e-6) / 1e9
                    entry["alg_GBps"] = round(gbs, 1)
                kernels[k] = entry
        b = kernels["pass_b"]
        shape = {"block_threads": gpu.block_threads, "grid_blocks": gpu.grid_blocks,
                 "rebin_every": args.rebin_every, "deposit_mode": args.deposit_mode,
                 "scheme": wl.scheme}
        roofline = {"bound": "hbm", "achieved": b["alg_GBps"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(b["alg_GBps"] / HBM_PEAK_GBS, 4),
                    "traffic": stored_traffic(args.workload, shape),
                    "kernel": {"esec1": "k_esec1", "standard": "k_std_pass"}.get(wl.scheme, "k_pass_b"),
                    "alg_bytes_per_particle": ab["pass_b"],
                    "alg_bytes_per_launch": ab["pass_b"] * n}

    cpu = None
    if args.cpu_steps > 0:
        import oracle
        ost = oracle.State(wl, charge_conserving=args.charge_conserving)
        ost.run(0)                       # initial Gauss solve outside the timing
        c0 = time.perf_counter()
        ost.run(args.cpu_steps)
        cs = time.perf_counter() - c0
        # the oracle is plain single-threaded C: it uses one of the host's cores
        cpu = {"value": n * args.cpu_steps / cs, "unit": "particle-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{args.cpu_steps} steps of the full {n}-particle workload, "
                         f"single-threaded C oracle, {cs:.1f} s",
               "host": host_info()}

    # the whole step against the same roofline: algorithmic bytes of both passes per step
    ab_all = alg_bytes(wl.nv, wl.scheme)
    step_bytes = sum(ab_all.values()) * n
    step_gbs = step_bytes / (ms / args.steps * 1e-3) / 1e9
    state_bytes = n * 8 * (1 + wl.nv)
    step_roof = {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                 "alg_bytes_per_particle_step": sum(ab_all.values()),
                 "state_bytes": state_bytes,
                 # MI355X's Infinity Cache (MALL) holds 256 MB: a smaller state can stay in
                 # it between the two passes, so part of the traffic never reaches HBM
                 "state_fits_infinity_cache": state_bytes <= 256e6}

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
                   "nv": wl.nv, "block_threads": gpu.block_threads,
                   "grid_blocks": gpu.grid_blocks, "deposit_mode": args.deposit_mode,
                   "rebin_every": args.rebin_every, "deterministic": args.deterministic,
                   "charge_conserving": args.charge_conserving},
        "energy": energy,
        "roofline": roofline,
        "step_roofline": step_roof,
        "kernels": kernels,
        "late_window": late,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    gpu.destroy()


if __name__ == "__main__":
    main()
