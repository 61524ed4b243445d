#!/usr/bin/env python3
"""Throughput of the WFP march on one MI355X: scatterer-steps per second.

Workload: the periodic multiband problem (M = 1e4 springs, beta log-uniform in
[0.1, 100], 8 Gaussian wave packets with angular carriers 50..500, dt = 1e-3,
K = 3141, W = 35, p = 8), FP64.  A step is one time level of the march (spread,
FFT, mode update, inverse FFT, local sum + interpolation, solve).  Plan
creation (sorting, tables, local weights) happens before timing, as in the
paper's timings; the timed region starts with every input resident in HBM.

Printed: one JSON line on stdout (diagnostics on stderr).
  value       M * steps / seconds over the timed steps
  parity      max |sigma_gpu - sigma_oracle| / max |sigma_oracle| against the
              stored oracle values (tests/golden/multiband_sigma.npz)
  roofline    the dominant kernel, timed with HIP events on the plan's stream in
              a second pass over the same steps; algorithmic bytes per launch
              as stated in the design notes
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scatterer-steps/s (M*N_t/s) at 1e-10 rel err; batched & adjoint vs plain"
HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden", "multiband_sigma.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_bytes(info, stage):
    """Algorithmic bytes one launch of a stage must move (minimum traffic)."""
    M, K, nf, W, mm = info["M"], info["K"], info["n_fine"], info["W"], info["m_max"]
    nnz = info["n_weights_nonzero"]
    if stage == "local":
        # nonzero local weights (lag >= 1), the density stack, per-row data
        # (x, beta, rhs out, start/count, offset), the type-2 grid
        return 8 * nnz + 8 * (mm - 1) * M + 40 * M + 8 * nf
    if stage == "modes":
        # FFT output rows k and N/2-k, dk1, dk2, p/q tables, spectra ring, alpha,
        # alpha', write ring slot, alpha, alpha', y
        return (K + 1) * (32 + 16 + 16 * W + 16 * W + 48 + 16 + 32 + 16)
    if stage == "spread":
        return 16 * M + 8 * 2 * nf + 8 * nf
    if stage in ("fft_fwd", "fft_inv"):
        return 16 * nf
    if stage == "solve":
        return 8 * M * 4
    return 0


def check_golden(sig_rows, save_every, steps):
    if not os.path.exists(GOLDEN):
        return None
    g = np.load(GOLDEN)
    smax = float(g["sigma_max"])
    worst = 0.0
    n_cmp = 0
    for L, row in zip(g["full_levels"], g["full"]):
        if L < steps and L % save_every == 0:
            worst = max(worst, float(np.max(np.abs(sig_rows[L // save_every] - row))))
            n_cmp += row.size
    every = int(g["strided_every"])
    sample = g["sample"]
    for i, row in enumerate(g["strided"]):
        L = i * every
        if L < steps and L % save_every == 0:
            worst = max(worst, float(np.max(np.abs(sig_rows[L // save_every][sample] - row))))
            n_cmp += row.size
    return dict(rel_err=worst / smax, compared=n_cmp, tol=1e-10)


def cpu_baseline(p, n_steps):
    from oracle.march import Oracle, incident_driving
    from oracle.params import Params
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    t0 = time.perf_counter()
    o = Oracle(p["x"], p["beta"], Params(dt=p["dt"]), incident_driving(p["x"], p["beta"], p["packets"], True))
    pre = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(n_steps):
        o.step()
    el = time.perf_counter() - t0
    M = p["x"].size
    return {"value": M * n_steps / el, "unit": "scatterer-steps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"same workload, levels 0..{n_steps - 1} of the CPU oracle (direct sums, sparse LU), "
                      f"timed after its {pre:.0f} s set-up"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the march has no multi-GPU "
              "path in this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2507_07823_amd import wfp, workloads

    torch.cuda.set_device(0)
    p = workloads.multiband_periodic()
    M = p["x"].size
    t0 = time.perf_counter()
    plan = wfp.Plan(p, p["dt"])
    info = plan.info
    log(f"plan: {time.perf_counter() - t0:.2f} s, info {info}")
    if args.warmup:
        plan.march(args.warmup)
    plan.reset()
    save_every = 50
    rows = (args.steps + save_every - 1) // save_every
    sig = torch.empty((rows, M), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(args.steps, sig, save_every)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = M * args.steps / elapsed
    log(f"timed {args.steps} steps in {elapsed:.4f} s -> {value:.4e} scatterer-steps/s")
    parity = check_golden(sig.cpu().numpy(), save_every, args.steps)
    log(f"parity vs oracle: {parity}")

    roofline, stages = None, None
    if not args.no_profile:
        plan.reset()
        plan.set_profiling(True)
        plan.run(args.steps)
        prof = plan.profile()
        plan.set_profiling(False)
        stages = {}
        for s, (ms, n) in prof.items():
            if n:
                avg = ms / n
                b = stage_bytes(info, s)
                stages[s] = {"avg_us": 1e3 * avg, "launches": n, "bytes": b,
                             "GBps": (b / (avg * 1e-3) / 1e9) if b else None}
        log("stages:", json.dumps(stages))
        dom = max(stages, key=lambda s: stages[s]["avg_us"] * stages[s]["launches"])
        st = stages[dom]
        achieved = st["GBps"]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
                    "avg_launch_us": st["avg_us"], "bytes_per_launch": st["bytes"]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, args.cpu_steps)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": METRIC, "value": value, "unit": "scatterer-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "periodic multiband springs", "M": M, "dt": p["dt"], "K": info["K"],
                   "W": info["W"], "p": info["p"], "n_fine": info["n_fine"], "pairs": info["n_pairs"],
                   "levels_timed": args.steps, "parallelism": "single GPU"},
        "parity": parity, "roofline": roofline, "stages": stages, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
