#!/usr/bin/env python3
"""Throughput of the WFP march on one MI355X: scatterer-steps per second.

Headline workload: the clumped free-space problem at full size (M = 1e6 springs
uniform in the box with 10 % in 100 Gaussian clumps of width 1e-3, a
Gaussian-modulated plane wave of angular frequency 1000, dt = 5e-4, K = 6250,
W = 35, p = 8, local weights evaluated on the fly), FP64.  A step is one time
level of the march (spread, FFT, mode update, boundary projection when due,
inverse FFT, local sum, solve).  Plan creation (sorting, tables, solve
factors) happens before timing, as in the paper's timings; the timed region
starts with every input resident in HBM.

Printed: one JSON line on stdout (diagnostics on stderr).
  value       M * steps / seconds over the timed steps
  parity      one level of the same plan from a seeded synthetic state against
              stored oracle values (tests/golden/clumped_level.npz): the new
              spectrum and alpha, alpha' at every mode, the explicit local sum
              at 96 sampled springs and the residual of the per-step system there
  roofline    the on-the-fly local sum (the dominant kernel), timed with HIP
              events on the plan's stream in a second pass (while timing, the
              library runs every stage on that stream, so the kernel is timed
              alone); algorithmic flops per launch = ordered neighbour pairs x
              1.6 kflop
  cpu_baseline  the FP64 CPU oracle on the same distribution at M = 1e4, run in
              a child process beside the GPU legs
Secondary legs (each in its own key): the periodic multiband workload (M = 1e4)
with its stored-oracle parity, the gradient pass, the batched form, the
scaling study, the convergence test, the filters and the disordered runs.
"""
import argparse
import csv
import hashlib
import json
import math
import os
import re
import subprocess
import sys
import time
from collections import defaultdict

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scatterer-steps/s (M*N_t/s) at 1e-10 rel err; batched & adjoint vs plain"
HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden", "multiband_sigma.npz")
CLUMPED_GOLDEN = os.path.join(ROOT, "tests", "golden", "clumped_level.npz")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2507_07823_amd", "csrc", "wfp_kernels.hip")
COPY_BYTES = 1 << 28          # the calibration copy moves 256 MiB

# Per kernel: its own source text (from the first marker up to the second)
# and the committed counter summary of its HBM traffic.
KERNELS = {
    "wfp::k_local_rhs": dict(
        region=("// Local sum of lags m0 <= m < m1", "// The lag-1 part of the right-hand side local sum"),
        traffic=os.path.join(ROOT, "profiles", "k_local_rhs.periodic-multiband-M1e4.traffic.txt")),
    "wfp::k_local_otf_sym": dict(
        region=("// Local sum of lags m >= 1 with the weights evaluated on the fly, each",
                "#define WFP_OTFS_INST"),
        traffic=os.path.join(ROOT, "profiles", "k_local_otf_sym.clumped-free-space-M1e6.traffic.txt")),
}


def kernel_source_hash(kernel):
    """SHA-256 of a kernel's source region: its counter summary holds only
    while that text is unchanged."""
    a_mark, b_mark = KERNELS[kernel]["region"]
    with open(KERNEL_SOURCE, encoding="utf-8") as f:
        src = f.read()
    a = src.index(a_mark)
    b = src.index(b_mark, a)
    return hashlib.sha256(src[a:b].encode("utf-8")).hexdigest()


def read_traffic(kernel):
    """HBM bytes per launch of a kernel from its committed counter summary, or
    None when it is missing or the kernel source has changed since the
    counters were taken."""
    fn = KERNELS[kernel]["traffic"]
    if not os.path.exists(fn):
        return None
    kv = {}
    with open(fn) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash(kernel):
        return None
    return float(kv["traffic_bytes_per_dispatch"])


def _kname(name):
    """Kernel name without return type, template arguments and parameters."""
    n = name.split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    return re.sub(r"<.*>", "", n)


def _counter_means(d, counter):
    """Mean per dispatch of one counter, per kernel, from a rocprofv3 --pmc run."""
    acc = defaultdict(list)
    for fn in os.listdir(d):
        if fn.endswith("counter_collection.csv"):
            with open(os.path.join(d, fn)) as f:
                for r in csv.DictReader(f):
                    if r["Counter_Name"] == counter:
                        acc[_kname(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def pmc_summary(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, kernel="wfp::k_local_otf_sym"):
    """Text summary: FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of ``kernel``,
    each scaled by what the counter reads for a 256 MiB device copy."""
    cf = _counter_means(cal_fetch_dir, "FETCH_SIZE")["__amd_rocclr_copyBuffer"][0]
    cw = _counter_means(cal_write_dir, "WRITE_SIZE")["__amd_rocclr_copyBuffer"][0]
    ff = COPY_BYTES / 1024.0 / cf
    fw = COPY_BYTES / 1024.0 / cw
    fe, n = _counter_means(fetch_dir, "FETCH_SIZE")[kernel]
    wr, _ = _counter_means(write_dir, "WRITE_SIZE")[kernel]
    traffic = 1024.0 * (fe * ff + wr * fw)
    return "\n".join([
        f"kernel: {kernel}",
        f"kernel_source_sha256: {kernel_source_hash(kernel)}",
        f"dispatches: {n}",
        f"FETCH_SIZE_KiB_per_dispatch: {fe:.3f}",
        f"WRITE_SIZE_KiB_per_dispatch: {wr:.3f}",
        f"copy_256MiB_FETCH_SIZE_KiB: {cf:.3f}",
        f"copy_256MiB_WRITE_SIZE_KiB: {cw:.3f}",
        f"fetch_scale: {ff:.4f}",
        f"write_scale: {fw:.4f}",
        f"traffic_bytes_per_dispatch: {traffic:.0f}",
    ])


def counters_summary(dirs, kernel, avg_ms, pairs, nodes=35):
    """Per-dispatch means of every counter of ``kernel`` in the given
    rocprofv3 --pmc runs, and the derived VALU/LDS/FP64 figures of the
    pair-once local sum (256 compute units in 8 XCDs, GRBM_GUI_ACTIVE summed
    over the XCDs; one (unordered pair, node) step per lane)."""
    vals, n = {}, 0
    for d in dirs:
        for fn in os.listdir(d):
            if fn.endswith("counter_collection.csv"):
                names = set()
                with open(os.path.join(d, fn)) as f:
                    for r in csv.DictReader(f):
                        names.add(r["Counter_Name"])
                for c in sorted(names):
                    m, n = _counter_means(d, c)[kernel]
                    vals[c] = m
    steps = pairs / 2 * nodes / 64
    busy = vals["SQ_ACTIVE_INST_VALU"] / 256 / (vals["GRBM_GUI_ACTIVE"] / 8)
    flops = 64 * vals["SQ_INSTS_VALU_FLOPS_FP64"]
    f64 = vals["SQ_INSTS_VALU_FMA_F64"] + vals["SQ_INSTS_VALU_ADD_F64"] + vals["SQ_INSTS_VALU_MUL_F64"]
    lines = [f"kernel: {kernel}", f"kernel_source_sha256: {kernel_source_hash(kernel)}", f"dispatches: {n}", ""]
    lines += [f"{c}: {v:.6g}" for c, v in sorted(vals.items())]
    if "SQ_LDS_IDX_ACTIVE" in vals:
        lines.append(f"LDS_busy (SQ_LDS_IDX_ACTIVE per CU-cycle): "
                     f"{vals['SQ_LDS_IDX_ACTIVE'] / 256 / (vals['GRBM_GUI_ACTIVE'] / 8):.3f}")
    lines += [
        f"VALU_busy: {busy:.3f}",
        f"VALU_lanes_active: {vals['SQ_THREAD_CYCLES_VALU'] / (64 * vals['SQ_ACTIVE_INST_VALU']):.4f}",
        f"LDS_active_fraction: {vals['SQ_ACTIVE_INST_LDS'] / 256 / (vals['GRBM_GUI_ACTIVE'] / 8):.3f}",
        f"FP64_flops_executed: {flops:.4g}",
        f"FP64_executed_TFLOPs_at_{avg_ms:g}ms: {flops / (avg_ms * 1e-3) / 1e12:.2f}",
        f"FP64_executed_fraction_of_78.6_peak: {flops / (avg_ms * 1e-3) / 78.6e12:.3f}",
        f"FP64_share_of_VALU_instructions: {f64 / vals['SQ_INSTS_VALU']:.3f}",
        f"VALU_instructions_per_node_wavefront: {vals['SQ_INSTS_VALU'] / steps:.1f}",
        f"LDS_instructions_per_node_wavefront: {vals['SQ_INSTS_LDS'] / steps:.2f}",
        f"LDS_bank_conflicts_per_LDS_instruction: {vals['SQ_LDS_BANK_CONFLICT'] / vals['SQ_INSTS_LDS']:.2e}",
    ]
    return "\n".join(lines)


def trace_tail_mean(d, kernel, n):
    """Mean duration (us) of the last n dispatches of `kernel` in a rocprofv3
    kernel trace (kernel_trace.csv), e.g. bench.py's timed-alone pass."""
    durs = []
    for fn in os.listdir(d):
        if fn.endswith("kernel_trace.csv"):
            with open(os.path.join(d, fn)) as f:
                for r in csv.DictReader(f):
                    if _kname(r["Kernel_Name"]) == kernel:
                        durs.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    durs.sort()
    tail = [x for _, x in durs[-n:]]
    return sum(tail) / len(tail) / 1e3 if tail else None


def stats_summary(d, top=20):
    """Text table of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    rows = []
    for fn in os.listdir(d):
        if fn.endswith("kernel_stats.csv"):
            with open(os.path.join(d, fn)) as f:
                rows += list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"{'kernel':<32} {'calls':>7} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}"]
    for r in rows[:top]:
        out.append(f"{_kname(r['Name'])[:32]:<32} {int(r['Calls']):>7} {float(r['AverageNs']) / 1e3:>10.3f} "
                   f"{float(r['MinNs']) / 1e3:>10.3f} {float(r['MaxNs']) / 1e3:>10.3f} "
                   f"{float(r['Percentage']):>6.2f}")
    return "\n".join(out)


def copy_calibration():
    """A plain 256 MiB device-to-device copy, three times (counter calibration)."""
    import torch
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log("copied 3 x 256 MiB")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_bytes(info, stage):
    """Algorithmic bytes one launch of a stage must move (minimum traffic)."""
    M, K, nf, W, mm = info["M"], info["K"], info["n_fine"], info["W"], info["m_max"]
    nnz = info["n_weights_nonzero"]
    if stage == "local":
        # the lags >= 2 kernel: nonzero weights of lags 2 .. m_max - 1, those
        # density levels, the per-row lag table (8 bytes per lag), neighbour
        # start and packed offset per row, one double out per row
        nl = mm - 2
        return 8 * (nnz - info["n_weights_lag1"]) + 8 * nl * M + 8 * nl * M + 20 * M
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


def check_golden(plan, M):
    """The multiband plan from level 0 through the stored oracle levels (an
    untimed march): the full density rows and the sampled springs every 100th
    level up to the last full level, compared with the oracle's.  Reports the
    levels compared and whether any compared row carries the scattered field
    (max |sigma| above 1e-3 of the run's maximum), so that a check made
    before the pulse arrives cannot pass as parity."""
    import torch
    if not os.path.exists(GOLDEN):
        return None
    g = np.load(GOLDEN)
    smax = float(g["sigma_max"])
    last = int(max(L for L in g["full_levels"] if L <= 1000))
    plan.reset()
    sig = torch.empty((last + 1, M), dtype=torch.float64, device="cuda")
    plan.run(last + 1, sig, 1)
    torch.cuda.synchronize()
    s = sig.cpu().numpy()
    worst, n_cmp, live, levels = 0.0, 0, 0.0, []
    for L, row in zip(g["full_levels"], g["full"]):
        if L <= last:
            worst = max(worst, float(np.max(np.abs(s[L] - row))))
            n_cmp += row.size
            live = max(live, float(np.max(np.abs(row))))
            levels.append(int(L))
    every = int(g["strided_every"])
    sample = g["sample"]
    n_strided = 0
    for i, row in enumerate(g["strided"]):
        L = i * every
        if L <= last:
            worst = max(worst, float(np.max(np.abs(s[L][sample] - row))))
            n_cmp += row.size
            n_strided += 1
    return dict(rel_err=worst / smax, compared=n_cmp, full_levels=levels,
                sampled_levels=f"0..{last} every {every} ({n_strided} levels, {sample.size} springs)",
                field_present=bool(live > 1e-3 * smax), tol=1e-10)


def clumped_parity(plan, p):
    """One level of the headline plan from the seeded synthetic state of
    workloads.clumped_level_state (a level where the boundary projection is
    due), against the stored oracle values: the new spectrum and alpha, alpha'
    at every mode, the explicit local sum at 96 sampled springs, and there the
    residual sigma_j + sum_l S_jl sigma_l - b_j of the per-step system."""
    import torch
    from paper_2507_07823_amd import workloads
    if not os.path.exists(CLUMPED_GOLDEN):
        return None
    g = np.load(CLUMPED_GOLDEN)
    info = plan.info
    M, K, W, mm = info["M"], info["K"], info["W"], info["m_max"]
    st, _ = workloads.clumped_level_state(M, K, W, mm)

    def dev(z):
        return torch.from_numpy(np.ascontiguousarray(np.stack([z.real, z.imag], -1))).cuda()

    plan.set_state(int(g["L"]), torch.from_numpy(st["hist"]).cuda(), dev(st["ring"]), dev(st["alpha"]),
                   dev(st["dalpha"]))
    loc = plan.local_part()
    sig, _ = plan.march(1, receivers=False)
    e = plan.get_state()
    torch.cuda.synchronize()
    loc = loc.cpu().numpy()
    sig = sig.cpu().numpy()[0]
    ring = e["ring"].cpu().numpy()
    a = e["alpha"].cpu().numpy()
    da = e["dalpha"].cpu().numpy()

    def rho(x, y):
        return float(np.max(np.abs(x - y)) / np.max(np.abs(y)))

    rows = g["rows"]
    ptr, idx, val = g["nb_ptr"], g["nb_idx"], g["nb_val"]
    res = np.array([sig[j] + val[ptr[i]:ptr[i + 1]] @ sig[idx[ptr[i]:ptr[i + 1]]] - g["rhs"][i]
                    for i, j in enumerate(rows)])
    out = {"level": int(g["L"]),
           "spectrum": rho(ring[0, :, 0] + 1j * ring[0, :, 1], g["spectrum"]),
           "alpha": rho(a[:, 0] + 1j * a[:, 1], g["alpha"]),
           "dalpha": rho(da[:, 0] + 1j * da[:, 1], g["dalpha"]),
           "local_sum_sampled": rho(loc[rows], g["local"]),
           "residual_sampled": float(np.max(np.abs(res)) / np.max(np.abs(g["rhs"]))),
           "modes": int(K + 1), "sampled_springs": int(rows.size), "tol": 1e-10}
    out["rel_err"] = max(out[k] for k in ("spectrum", "alpha", "dalpha", "local_sum_sampled", "residual_sampled"))
    return out


def cpu_baseline(levels):
    """The FP64 CPU oracle (direct sums, per-pair weights, sparse LU) on the
    clumped free-space distribution at M = 1e4 (beta ~ U[1, 10]), timed over
    `levels` levels after its set-up."""
    from oracle.march import Oracle, incident_driving
    from oracle.params import Params
    from paper_2507_07823_amd import workloads
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    p = workloads.clumped_free_space(M=10_000, clump_beta=(1.0, 10.0))
    t0 = time.perf_counter()
    o = Oracle(p["x"], p["beta"], Params(dt=p["dt"], boundary=1),
               incident_driving(p["x"], p["beta"], p["packets"], False))
    pre = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(levels):
        o.step()
    el = time.perf_counter() - t0
    M = p["x"].size
    return {"value": M * levels / el, "unit": "scatterer-steps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"the clumped free-space distribution at M = {M} (K = 6250, dt = 5e-4), levels "
                      f"0..{levels - 1} of the CPU oracle, timed after its {pre:.0f} s set-up"}


def _adjoint_run(p, levels, every, positions=True, local_mode=0):
    """Forward march then gradient pass over `levels` levels of the adjoint
    workload on a plan with checkpoint_every = `every` (> 0: checkpoints, the
    gradient pass replays each segment; < 0: every level recorded in blocks of
    -every levels, no replay).  A first gradient call over one block or
    segment (derivative-weight set-up) is not timed."""
    import torch
    from paper_2507_07823_amd import wfp
    M, R = p["x"].size, p["x_recv"].size
    t0 = time.perf_counter()
    plan = wfp.Plan(p, p["dt"], checkpoint_every=every, local_mode=local_mode)
    setup = time.perf_counter() - t0
    u = torch.empty((levels, R), dtype=torch.float64, device="cuda")
    first = min(levels, abs(every))
    plan.run(first, None, 1, u[:first])
    plan.gradient(p["dt"] * u[:first], positions=positions)   # warm-up and one-time set-up
    plan.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(levels, None, 1, u)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    log(f"adjoint workload, checkpoint_every {every}, local_mode {local_mode}: forward {levels} levels {t_fwd:.2f} s")
    e = p["dt"] * u                                  # dJ/du of J = dt/2 sum u^2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gb, gx = plan.gradient(e, positions=positions)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    log(f"  gradient pass ({'beta, x' if positions else 'beta'}) {t_bwd:.2f} s")
    ok = bool(torch.isfinite(gb).all() and (gx is None or torch.isfinite(gx).all()))
    info = plan.query_info()
    plan.close()
    return {"levels": levels, "checkpoint_every": every, "local_mode": info["local_mode"],
            "gradients": "beta, x" if positions else "beta", "plan_setup_s": setup, "forward_s": t_fwd,
            "gradient_s": t_bwd, "forward_scatterer_steps_per_s": M * levels / t_fwd,
            "forward_plus_gradient_scatterer_steps_per_s": M * levels / (t_fwd + t_bwd),
            "gradient_over_forward_time": t_bwd / t_fwd, "device_bytes": info["device_bytes"], "finite": ok}


def adjoint_leg(levels, every):
    """Forward + gradient pass on the adjoint workload (M = 1e5 springs, 64
    receivers, dt = 1e-3): with the weights stored per ordered pair over
    `levels` levels with every level recorded (blocks of `every`) and over at
    most 1000 levels with checkpoints every `every` levels (the replayed
    form), over `levels` levels recorded with the weights stored once per
    unordered pair (the library's choice for this workload), and over at most
    1000 levels recorded with the weights evaluated on the fly, against a plain
    forward march (weights per ordered pair, no checkpoints, no recording) of
    the same levels."""
    import torch
    from paper_2507_07823_amd import wfp, workloads
    p = workloads.adjoint_periodic()
    M, R = p["x"].size, p["x_recv"].size
    plain = wfp.Plan(p, p["dt"], local_mode=1)
    u = torch.empty((levels, R), dtype=torch.float64, device="cuda")
    plain.run(10, None, 1, u[:10])
    plain.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain.run(levels, None, 1, u)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log(f"adjoint workload: plain forward {levels} levels {t_plain:.2f} s")
    plain.close()
    del u
    rec = _adjoint_run(p, levels, -every, local_mode=1)
    ck = _adjoint_run(p, min(levels, 1000), every, local_mode=1)
    # the weights (and derivative weights) stored once per unordered pair
    po = _adjoint_run(p, levels, -every, local_mode=3)
    # nothing stored: weights and derivative weights evaluated on the fly
    of = _adjoint_run(p, min(levels, 1000), -every, local_mode=2)
    return {"workload": "periodic adjoint", "M": M, "R": R, "levels": levels,
            "beta": [round(float(p["beta"].min()), 4), round(float(p["beta"].max()), 4)],
            "plain_forward_s": t_plain, "plain_scatterer_steps_per_s": M * levels / t_plain,
            "recorded": rec, "checkpointed": ck, "pair_once_recorded": po, "on_the_fly_recorded": of,
            "forward_plus_gradient_over_plain_time": (rec["forward_s"] + rec["gradient_s"]) / t_plain}


def batch_leg(n_inst, levels, m_max, trial_levels=3, uneven=True):
    """The batched form on uneven periodic instances (M log-uniform in
    [100, m_max], dt in {1e-3, 2e-3, 5e-3}, beta ~ U[1, 10] scaled per
    instance to keep the dense-medium number <= 0.1, one random pulse each),
    autotuned, against the same instances marched one plain plan at a
    time.  With `uneven`, instance i marches its own level count
    levels - (i mod 4) levels / 8 (wfp_batch_set_levels), the plain plans the
    same counts; the rate counts each instance's own levels."""
    import torch
    from paper_2507_07823_amd import wfp, workloads
    insts = workloads.batch_instances(n=n_inst, n_steps=levels, m_range=(100, m_max))
    ends = [levels - (i % 4) * levels // 8 if uneven else levels for i in range(len(insts))]
    work = int(sum(p["x"].size * e for p, e in zip(insts, ends)))
    total_m = int(sum(p["x"].size for p in insts))
    t0 = time.perf_counter()
    b = wfp.Batch(insts, [p["dt"] for p in insts])
    setup = time.perf_counter() - t0
    n_otf = sum(1 for i in range(b.n) if b.plan(i).info["local_mode"] == 2)
    shape = b.autotune(trial_levels)
    b.set_levels(ends)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(levels)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.set_levels(None)
    b.reset()
    plans = [b.plan(i) for i in range(b.n)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, e in zip(plans, ends):
        pl.run(e)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    b.reset()
    b.close()
    return {"workload": "batched periodic instances", "instances": n_inst, "M_range": [100, m_max],
            "total_M": total_m, "levels": levels, "level_counts": "own" if uneven else "equal",
            "scatterer_steps": work, "plan_setup_s": setup, "instances_on_the_fly": n_otf,
            "autotuned": {"rows_per_block": shape[0], "xcd_remap": shape[1], "spread_pass": shape[2]},
            "batched_scatterer_steps_per_s": work / t_batch,
            "plain_one_by_one_scatterer_steps_per_s": work / t_plain,
            "batched_over_plain": t_plain / t_batch}


# Algorithmic FP64 operations of the on-the-fly local sum per ordered
# neighbour pair: N_L = 35 quadrature nodes, each a node lag, a window weight
# and a degree-7 interpolant of the source's history (about 46 flops), 1.6
# kflop in all (the method's per-pair estimate).
OTF_FLOPS_PER_PAIR = 1600.0
FP64_VECTOR_PEAK_TFLOPS = 78.6


def balanced_leg(levels, sizes, autotune_levels):
    """The free-space scaling study of Section 6.2 (springs uniform in [-2, 2],
    beta in [0.1, 3], p = 6, dt chosen for about 100 neighbours; weights stored
    per ordered pair, whose HBM-bound local sum the per-stage rates describe)
    at each M of `sizes`: set-up time, the schedule wfp_plan_autotune picks,
    the rate over `levels` levels from rest (the
    per-level work does not depend on the densities) and the per-stage times
    of a second, profiled pass.  The paper's CPU rate for this study is
    quoted as context (other hardware, M up to 1e6)."""
    import torch
    from paper_2507_07823_amd import wfp, workloads
    rows = []
    for M in sizes:
        lv = levels if M < 500_000 else max(levels // 5, 50)
        p = workloads.paper_balanced_free_space(M)
        t0 = time.perf_counter()
        plan = wfp.Plan(p, p["dt"], p=p["p"], local_mode=1)
        setup = time.perf_counter() - t0
        plan.autotune(autotune_levels if M < 500_000 else max(autotune_levels // 5, 3))
        info = plan.info
        plan.run(min(lv, 100))
        torch.cuda.synchronize()
        plan.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run(lv)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        plan.reset()
        plan.set_profiling(True)
        plan.run(lv)
        prof = plan.profile()
        plan.set_profiling(False)
        plan.close()
        stages = {k: 1e3 * v[0] / v[1] for k, v in prof.items() if v[1]}
        row = {"M": M, "dt": p["dt"], "K": info["K"], "p": info["p"], "n_fine": info["n_fine"],
               "mean_neighbours": info["n_pairs"] / M, "local_mode": info["local_mode"],
               "solve_mode": info["solve_mode"], "overlap_cus": info["overlap_cus"], "plan_setup_s": setup,
               "levels": lv,
               "ms_per_level": 1e3 * el / lv, "scatterer_steps_per_s": M * lv / el, "stages_us": stages}
        if info["local_mode"] == 1 and "local" in stages:     # stored weights: HBM-bound local sum
            row["local_GBps"] = stage_bytes(info, "local") / (stages["local"] * 1e-6) / 1e9
        rows.append(row)
        log(f"balanced M={M}: {rows[-1]}")
    return {"workload": "free-space scaling study (Section 6.2), p = 6, about 100 neighbours", "sizes": rows,
            "paper_context": {"scatterer_steps_per_s": 1.5e5, "hardware": "2 x Xeon Platinum 8362 (64 cores)",
                              "note": "the paper's asymptotic CPU rate for this study, M up to 1e6"}}


def convergence_leg(sizes=(10, 100), orders=(2, 4, 6, 8), dts=(0.0125, 0.00625, 0.003125)):
    """The convergence test of Section 6.1 on the GPU: prescribed Gaussian
    densities at M springs in [-1, 1] (free space), the march driven by the
    data they imply (wfp_run_driven), the field at 10 receivers in [-1, 1]
    compared with the exact field at 10 times covering 0 < t < 6 pi.  Reports
    the maximum grid error per (M, p, dt) and the observed orders."""
    import torch
    from paper_2507_07823_amd import wfp, workloads
    T = 6.0 * math.pi
    xg = np.linspace(-1.0, 1.0, 10)
    out = []
    for M in sizes:
        prob = workloads.manufactured_springs(M)
        for dt in dts:
            n = int(math.floor(T / dt)) + 1
            lv = np.minimum(np.round(np.arange(1, 11) * (T / 10) / dt).astype(int), n - 1)
            ex = np.array([workloads.manufactured_potential(xg, L * dt, prob["x"], prob["mu"], prob["t0"])
                           for L in lv])
            g = torch.from_numpy(np.ascontiguousarray(workloads.manufactured_data(prob, dt, n))).cuda()
            for p in orders:
                plan = wfp.Plan(dict(prob, x_recv=xg), dt, p=p)
                t0 = time.perf_counter()
                _, u = plan.march_driven(g, save_every=n)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                plan.close()
                err = float(np.max(np.abs(u.cpu().numpy()[lv] - ex)))
                out.append({"M": M, "p": p, "dt": dt, "levels": n, "max_grid_error": err, "march_s": el})
    for r in out:
        prev = [q for q in out if q["M"] == r["M"] and q["p"] == r["p"] and q["dt"] == 2 * r["dt"]]
        r["observed_order"] = math.log2(prev[0]["max_grid_error"] / r["max_grid_error"]) if prev else None
    return {"workload": "manufactured solution (Section 6.1), free space, 10 x 10 space-time grid, T = 6 pi",
            "runs": out}


def filters_leg():
    """The filter demonstrations of Section 6.4 (free space, dt = 0.01): the
    two-spring cavity (9426 levels) and arrays of 10 and 200 springs (25134
    levels), the march time of each and, for the cavity, the frequencies the
    downstream total field passes (peaks of the Hann-windowed transform of the
    total field over that of the incident wave).  The paper's run times (a laptop, other hardware) are
    quoted as context."""
    import torch
    from paper_2507_07823_amd import wfp, workloads
    paper_s = {2: 16.0, 10: 91.0, 200: 114.0}
    rows = []
    for prob in [workloads.fabry_perot()] + workloads.spring_arrays():
        M, n = prob["x"].size, prob["n_steps"]
        t0 = time.perf_counter()
        plan = wfp.Plan(prob, prob["dt"], p=prob["p"])
        setup = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, u = plan.march(n, save_every=n)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        plan.close()
        t = np.arange(n) * prob["dt"]
        inc = np.exp(-prob["mu"] * (prob["x_recv"][0] - t - prob["t0"]) ** 2)
        tot = u.cpu().numpy()[:, 0] + inc
        row = {"M": M, "beta": float(prob["beta"][0]), "p": prob["p"], "levels": n, "plan_setup_s": setup,
               "march_s": el, "paper_s": paper_s[M], "max_transmitted": float(np.max(np.abs(tot)))}
        if M == 2:
            # Hann-windowed transfer ratio over the run, w in [1, 11]
            win = 0.5 - 0.5 * np.cos(2 * np.pi * t / t[-1])
            w = np.linspace(1.0, 11.0, 4001)
            ph = np.exp(1j * np.outer(w, t))
            T = np.abs(ph @ (tot * win)) / np.abs(ph @ inc)
            row["transmission_peaks"] = [float(w[i]) for i in range(1, w.size - 1)
                                         if T[i] > T[i - 1] and T[i] > T[i + 1] and T[i] > 0.2 * T.max()]
        rows.append(row)
        log(f"filter M={M}: {row}")
    return {"workload": "spring filters (Section 6.4), free space, dt = 0.01", "runs": rows}


def disordered_leg(large_levels):
    """The long disordered runs of Section 6.3 (random springs on [-2, 2], a
    pulse of width sqrt(8) times the mean spacing, p = 8): M = 1e3 marched
    in full (72044 levels) and at dt / 2 (144088 levels), the estimated error
    of the first from the second at 50 receivers; M = 1e4 timed over its
    first `large_levels` levels (of 720440).  The paper's times (a laptop,
    other hardware) are quoted as context."""
    import torch
    from paper_2507_07823_amd import wfp, workloads
    out = {"workload": "disordered springs (Section 6.3), free space, p = 8"}
    us = []
    for rf in (1, 2):
        prob = workloads.disordered_long(1000, refine=rf)
        n = prob["n_steps"]
        plan = wfp.Plan(prob, prob["dt"], p=prob["p"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, u = plan.march(n, save_every=n)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"M1000_dt{'' if rf == 1 else '_half'}"] = {"dt": prob["dt"], "K": plan.info["K"], "levels": n,
                                                         "march_s": el, "ms_per_level": 1e3 * el / n}
        plan.close()
        us.append(u.cpu().numpy())
    ref = us[1][::2][: us[0].shape[0]]
    out["M1000_estimated_rel_error"] = float(np.max(np.abs(us[0] - ref)) / np.max(np.abs(ref)))
    out["M1000_paper"] = {"s_per_level": 0.02, "total_min": 24}
    if large_levels > 0:
        prob = workloads.disordered_long(10_000)
        plan = wfp.Plan(prob, prob["dt"], p=prob["p"])
        plan.run(50)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run(large_levels)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ms = 1e3 * el / large_levels
        out["M10000"] = {"dt": prob["dt"], "K": plan.info["K"], "levels_timed": large_levels, "ms_per_level": ms,
                         "projected_full_run_min": ms * prob["n_steps"] / 6e4,
                         "paper": {"s_per_level": 0.15, "total_h": 29.5}}
        plan.close()
    log(f"disordered leg: {out}")
    return out


def disordered_full(M=10_000, chunk=50_000, refines=(1, 2)):
    """The long disordered run at M in full, at dt and at dt / 2 (for M = 1e4:
    720440 and 1440880 levels), marched in chunks with a progress line per
    chunk; returns the times and the estimated error of the dt run at its 50
    receivers."""
    import torch
    from paper_2507_07823_amd import wfp, workloads
    out = {"workload": f"disordered springs (Section 6.3), M = {M}, full run", "M": M}
    us = []
    for rf in refines:
        prob = workloads.disordered_long(M, refine=rf)
        n, R = prob["n_steps"], prob["x_recv"].size
        t0 = time.perf_counter()
        plan = wfp.Plan(prob, prob["dt"], p=prob["p"])
        setup = time.perf_counter() - t0
        u = torch.empty((n, R), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            plan.run(b - a, None, 1, u[a:b])
            torch.cuda.synchronize()
            log(f"disordered M={M} refine={rf}: level {b} of {n}, {time.perf_counter() - t0:.1f} s")
        el = time.perf_counter() - t0
        out[f"refine{rf}"] = {"dt": prob["dt"], "K": plan.info["K"], "n_fine": plan.info["n_fine"], "levels": n,
                              "plan_setup_s": setup, "march_s": el, "ms_per_level": 1e3 * el / n}
        plan.close()
        us.append(u.cpu().numpy())
        del u
    if len(us) == 2:
        ref = us[1][::2][: us[0].shape[0]]
        out["estimated_rel_error"] = float(np.max(np.abs(us[0] - ref)) / np.max(np.abs(ref)))
        out["field_max"] = float(np.max(np.abs(ref)))
    return out


def lds_ceiling():
    """LDS read rates of this GPU from the committed probe program (built
    beside the library): a dict with the ceiling (16-byte reads) and the rate
    of the 8-byte pair reads the local sum issues, or None if it is missing or
    fails."""
    probe = os.path.join(ROOT, "paper_2507_07823_amd", "lds_probe")
    if not os.path.exists(probe):
        return None
    try:
        r = subprocess.run([probe], capture_output=True, text=True, timeout=60)
        d = json.loads(r.stdout.strip().splitlines()[-1])
        return {"ceiling": float(d["lds_read_bytes_per_s"]), "b64x2": float(d["ds_read2st64_b64_bytes_per_s"])}
    except (subprocess.SubprocessError, ValueError, IndexError, KeyError, OSError):
        return None


def headline(steps, warmup, profile_levels):
    """The clumped free-space workload at full size (M = 1e6): set-up, `warmup`
    untimed levels, `steps` timed levels, then a profiled pass of
    `profile_levels` levels for the per-stage times and the roofline of the
    on-the-fly local sum, then the one-level parity check."""
    import torch
    from paper_2507_07823_amd import wfp, workloads
    p = workloads.clumped_free_space()
    M = p["x"].size
    t0 = time.perf_counter()
    plan = wfp.Plan(p, p["dt"])
    setup = time.perf_counter() - t0
    info = plan.info
    log(f"clumped plan: {setup:.2f} s, info {info}")
    if warmup:
        plan.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {steps} levels in {elapsed:.3f} s -> {M * steps / elapsed:.4e} scatterer-steps/s")
    roofline, stages = None, None
    if profile_levels:
        plan.set_profiling(True)
        plan.run(profile_levels)
        prof = plan.profile()
        plan.set_profiling(False)
        stages = {k: {"avg_ms": v[0] / v[1], "launches": v[1]} for k, v in prof.items() if v[1]}
        ms, n = prof["local"]
        avg = ms / n
        flops = info["n_pairs"] * OTF_FLOPS_PER_PAIR
        achieved = flops / (avg * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": "wfp::k_local_otf_sym (+ k_local_otf_reduce)", "achieved": achieved,
                    "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                    "traffic": read_traffic("wfp::k_local_otf_sym"), "avg_launch_ms": avg,
                    "flops_per_launch": flops, "flop_count": "ordered neighbour pairs x 1.6 kflop",
                    "timed_with": "HIP events on the plan's stream"}
        # the operands each lane reads from LDS per (unordered pair, node): the
        # source and row stencils (p values each) and the window piece,
        # against this GPU's LDS read throughput measured by the probe (its
        # ceiling, 16-byte reads; and the rate of the 8-byte pair reads that
        # carry the stencils)
        lds = info["n_pairs"] / 2 * info["n_gl_local"] * (2 * info["p"] + 6) * 8.0
        roofline["lds_operand_bytes_per_launch"] = lds
        roofline["lds_operand_GBps"] = lds / (avg * 1e-3) / 1e9
        ceiling = lds_ceiling()
        if ceiling:
            roofline["lds_ceiling_GBps"] = ceiling["ceiling"] / 1e9
            roofline["lds_frac"] = roofline["lds_operand_GBps"] / roofline["lds_ceiling_GBps"]
            roofline["lds_read2_b64_GBps"] = ceiling["b64x2"] / 1e9
        log(f"stages: {json.dumps(stages)}")
    parity = clumped_parity(plan, p)
    log(f"parity vs oracle: {parity}")
    plan.close()
    cfg = {"workload": "clumped free space (10 % of springs in 100 Gaussian clumps of width 1e-3)",
           "M": M, "dt": p["dt"], "K": info["K"], "W": info["W"], "p": info["p"], "n_fine": info["n_fine"],
           "pairs": info["n_pairs"], "local_mode": "on the fly", "solve_mode": info["solve_mode"],
           "beta_uniform": [round(float(p["beta"][:M - M // 10].min()), 4),
                            round(float(p["beta"][:M - M // 10].max()), 4)],
           "beta_clumped": list(workloads.CLUMP_BETA),
           "levels_timed": steps, "parallelism": "single GPU", "plan_setup_s": setup}
    return dict(value=M * steps / elapsed, elapsed=elapsed, config=cfg, parity=parity, roofline=roofline,
                stages=stages)


def multiband_leg(steps, warmup, overlap_cus, autotune_levels):
    """The periodic multiband workload (M = 1e4, weights stored per ordered
    pair): rate over `steps` levels, the roofline of its local sum
    (HBM-bound) and parity with the stored oracle march; then the rate with
    the weights stored once per pair (the library's choice for this
    workload) on the same schedule."""
    import torch
    from paper_2507_07823_amd import wfp, workloads
    p = workloads.multiband_periodic()
    M = p["x"].size
    t0 = time.perf_counter()
    plan = wfp.Plan(p, p["dt"], overlap_cus=overlap_cus, local_mode=1)
    setup = time.perf_counter() - t0
    if overlap_cus == 0:
        pick = plan.autotune(autotune_levels)
        log(f"multiband autotune: overlap_cus {pick}")
    info = plan.info
    if warmup:
        plan.march(warmup)
    plan.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.reset()
    plan.set_profiling(True)
    plan.run(steps)
    prof = plan.profile()
    plan.set_profiling(False)
    stages = {}
    for s_, (ms, n) in prof.items():
        if n:
            avg = ms / n
            b = stage_bytes(info, s_)
            stages[s_] = {"avg_us": 1e3 * avg, "launches": n, "bytes": b,
                          "GBps": (b / (avg * 1e-3) / 1e9) if b else None}
    st = stages["local"]
    roofline = {"bound": "hbm", "kernel": "wfp::k_local_rhs", "achieved": st["GBps"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": st["GBps"] / HBM_PEAK_GBS, "traffic": read_traffic("wfp::k_local_rhs"),
                "avg_launch_us": st["avg_us"], "bytes_per_launch": st["bytes"]}
    parity = check_golden(plan, M)
    plan.close()
    po = wfp.Plan(p, p["dt"], overlap_cus=info["overlap_cus"], local_mode=3)
    po.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    po.run(steps)
    torch.cuda.synchronize()
    t_po = time.perf_counter() - t0
    po.close()
    pair_once = {"local_mode": 3, "ms_per_level": 1e3 * t_po / steps, "scatterer_steps_per_s": M * steps / t_po}
    out = {"workload": "periodic multiband springs (beta log-uniform in [0.1, 10])", "M": M, "dt": p["dt"],
           "K": info["K"], "p": info["p"], "pairs": info["n_pairs"], "overlap_cus": info["overlap_cus"],
           "plan_setup_s": setup, "levels": steps, "ms_per_level": 1e3 * elapsed / steps,
           "scatterer_steps_per_s": M * steps / elapsed, "roofline": roofline, "stages": stages, "parity": parity,
           "pair_once": pair_once}
    log(f"multiband leg: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed levels of the headline workload")
    ap.add_argument("--warmup", type=int, default=3, help="untimed levels before them")
    ap.add_argument("--profile-levels", type=int, default=5,
                    help="levels of the headline's profiled pass (roofline, stage times; 0 skips it)")
    ap.add_argument("--cpu-levels", type=int, default=40, help="levels of the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only run the CPU oracle baseline and print its JSON (the child process of a bench run)")
    ap.add_argument("--multiband-levels", type=int, default=2000,
                    help="levels of the periodic multiband leg (0 skips it)")
    ap.add_argument("--adjoint-levels", type=int, default=5000,
                    help="levels of the adjoint leg (0 skips it)")
    ap.add_argument("--batch-levels", type=int, default=200, help="levels of the batched leg (0 skips it)")
    ap.add_argument("--batch-instances", type=int, default=512)
    ap.add_argument("--batch-max-m", type=int, default=10_000,
                    help="largest M of the batched leg (1e5 is the full recipe; its large instances then "
                         "evaluate their local weights on the fly and a level takes about a second)")
    ap.add_argument("--batch-full-levels", type=int, default=50,
                    help="levels of a second batched leg over the full M range [100, 1e5] (0 skips it)")
    ap.add_argument("--no-convergence", action="store_true", help="skip the manufactured-solution leg")
    ap.add_argument("--no-filters", action="store_true", help="skip the spring-filter leg")
    ap.add_argument("--disordered-full", action="store_true",
                    help="only run the M = 1e4 disordered run in full at dt and dt/2 (about 15 GPU-minutes) "
                         "and print its result")
    ap.add_argument("--disordered-refines", type=str, default="1,2",
                    help="with --disordered-full: the runs to make (1 = dt, 2 = dt/2; both give the error estimate)")
    ap.add_argument("--disordered-levels", type=int, default=20000,
                    help="levels timed at M = 1e4 in the disordered leg (negative skips the leg)")
    ap.add_argument("--balanced-levels", type=int, default=500,
                    help="levels per size of the free-space scaling-study leg (0 skips it)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the adjoint leg (--adjoint-levels levels) and print its result")
    ap.add_argument("--balanced-only", action="store_true",
                    help="only run the scaling-study leg (for counter runs of its kernels) and print its result")
    ap.add_argument("--balanced-sizes", type=str, default="1000,10000,100000,1000000",
                    help="comma-separated M of the scaling-study leg")
    ap.add_argument("--headline-only", action="store_true",
                    help="only run the headline workload (for profiler runs) and print its JSON line")
    ap.add_argument("--overlap-cus", type=int, default=0,
                    help="multiband plan parameter overlap_cus (0: chosen by wfp_plan_autotune, -1: one stream)")
    ap.add_argument("--autotune-levels", type=int, default=30,
                    help="trial levels per candidate schedule of wfp_plan_autotune")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 256 MiB copy used to calibrate the HBM counters")
    ap.add_argument("--pmc-summary", nargs=5, metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR",
                                                       "KERNEL"),
                    help="print the traffic summary of rocprofv3 --pmc runs and exit")
    ap.add_argument("--stats-summary", metavar="DIR", help="print a rocprofv3 --stats table and exit")
    ap.add_argument("--counters-summary", nargs="+", metavar="ARG",
                    help="DIR [DIR ...] KERNEL AVG_MS PAIRS: print the counters of KERNEL from rocprofv3 --pmc "
                         "runs, with the VALU/LDS/FP64 figures derived at a launch time of AVG_MS over PAIRS "
                         "ordered neighbour pairs, and exit")
    ap.add_argument("--trace-tail", nargs=3, metavar=("DIR", "KERNEL", "N"),
                    help="print the mean duration of the last N dispatches of KERNEL in a kernel trace and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        print(pmc_summary(*args.pmc_summary[:4], kernel=args.pmc_summary[4]))
        return
    if args.stats_summary:
        print(stats_summary(args.stats_summary))
        return
    if args.counters_summary:
        *dirs, k, ms, pairs = args.counters_summary
        print(counters_summary(dirs, k, float(ms), float(pairs)))
        return
    if args.trace_tail:
        d, k, n = args.trace_tail
        print(f"{k}: mean of the last {n} dispatches {trace_tail_mean(d, k, int(n)):.3f} us")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library runs the march "
              "on one GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.cpu_levels)), flush=True)
        return
    # the CPU oracle baseline runs in a child process beside the GPU legs
    child = None
    if not (args.no_cpu_baseline or args.headline_only or args.balanced_only or args.disordered_full
            or args.copy_calibration or args.adjoint_only):
        child = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                                  "--cpu-levels", str(args.cpu_levels)], stdout=subprocess.PIPE, text=True)
    try:
        out = run_gpu_legs(args)
    finally:
        cpu = None
        if child is not None:
            so, _ = child.communicate()
            try:
                cpu = json.loads(so.strip().splitlines()[-1])
            except (ValueError, IndexError):
                cpu = None
            log(f"cpu baseline: {cpu}")
    if out is None:
        return
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def run_gpu_legs(args):
    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return None
    if args.balanced_only:
        print(json.dumps(balanced_leg(args.balanced_levels, [int(v) for v in args.balanced_sizes.split(",")],
                                      args.autotune_levels)), flush=True)
        return None
    if args.disordered_full:
        print(json.dumps(disordered_full(refines=[int(v) for v in args.disordered_refines.split(",")])),
              flush=True)
        return None
    if args.adjoint_only:
        print(json.dumps(adjoint_leg(args.adjoint_levels, 250)), flush=True)
        return None
    h = headline(args.steps, args.warmup, args.profile_levels)
    out = {
        "metric": METRIC, "value": h["value"], "unit": "scatterer-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * h["elapsed"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": h["config"], "parity": h["parity"], "roofline": h["roofline"], "stages": h["stages"],
    }
    if args.headline_only:
        return out
    if args.multiband_levels > 0:
        out["multiband"] = multiband_leg(args.multiband_levels, 200, args.overlap_cus, args.autotune_levels)
    if args.adjoint_levels > 0:
        out["adjoint"] = adjoint_leg(args.adjoint_levels, 250)
        log(f"adjoint leg: {out['adjoint']}")
    if args.batch_levels > 0:
        out["batch"] = batch_leg(args.batch_instances, args.batch_levels, args.batch_max_m)
        log(f"batch leg: {out['batch']}")
    if args.batch_full_levels > 0:
        out["batch_full_range"] = batch_leg(args.batch_instances, args.batch_full_levels, 100_000, trial_levels=1)
        log(f"full-range batch leg: {out['batch_full_range']}")
    if args.balanced_levels > 0:
        out["balanced"] = balanced_leg(args.balanced_levels, [int(v) for v in args.balanced_sizes.split(",")],
                                       args.autotune_levels)
    if not args.no_convergence:
        out["convergence"] = convergence_leg()
        log("convergence leg:", json.dumps(out["convergence"]))
    if not args.no_filters:
        out["filters"] = filters_leg()
    if args.disordered_levels >= 0:
        out["disordered"] = disordered_leg(args.disordered_levels)
    return out


if __name__ == "__main__":
    main()
