"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Metric: rho(a, b) = max |a - b| / max |b| over every compared entry; the bar
is 1e-10 (both sides run the same discrete scheme in FP64; the HIP path
replaces exponential sums by NUFFTs of ~1e-15 relative accuracy and the LU
solve by converged Jacobi sweeps).
"""
import math
import sys

import numpy as np
import pytest

from oracle.march import Oracle, incident_driving
from oracle.params import FREE_SPACE, PERIODIC, Params
from paper_2507_07823_amd import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-10


def rho(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def wfp():
    import torch
    assert torch.cuda.is_available()
    from paper_2507_07823_amd import wfp as w
    w.load_library()
    return w


def oracle_for(prob, **kw):
    prm = Params(dt=prob["dt"], boundary=prob["boundary"], **kw)
    periodic = prob["boundary"] == PERIODIC
    drv = incident_driving(prob["x"], prob["beta"], prob["packets"], periodic)
    return Oracle(prob["x"], prob["beta"], prm, drv, x_recv=prob.get("x_recv"))


def gpu_march(w, prob, n, save_every=1, **kw):
    plan = w.Plan(prob, prob["dt"], **kw)
    sig, u = plan.march(n, save_every)
    import torch
    torch.cuda.synchronize()
    out = sig.cpu().numpy(), (None if u is None else u.cpu().numpy()), plan.info
    plan.close()
    return out


def test_small_periodic_full_march(wfp):
    p = workloads.small_periodic()
    n = p["n_steps"] + 1
    say(f"case small_periodic M={p['x'].size} levels={n}")
    g, _, info = gpu_march(wfp, p, n)
    o, _ = oracle_for(p).run(n)
    assert info["K"] == 314 and info["W"] == 35 and info["m_max"] == 39
    r = rho(g, o)
    say(f"rho={r:.3e} iters={info['solve_iters']}")
    assert r < TOL


def _state_to_gpu(st):
    import torch
    c = lambda z: torch.from_numpy(np.ascontiguousarray(np.stack([z.real, z.imag], -1))).cuda()
    return dict(hist=torch.from_numpy(np.ascontiguousarray(st["hist"])).cuda(), ring=c(st["ring"]),
                alpha=c(st["alpha"]), dalpha=c(st["dalpha"]))


def _state_from_gpu(st):
    c = lambda t: t.cpu().numpy()[..., 0] + 1j * t.cpu().numpy()[..., 1]
    return dict(L=st["L"], hist=st["hist"].cpu().numpy(), ring=c(st["ring"]), alpha=c(st["alpha"]),
                dalpha=c(st["dalpha"]))


@pytest.mark.parametrize("boundary", [PERIODIC, FREE_SPACE])
def test_steps_from_synthetic_state(wfp, boundary):
    """Both sides start from the same seeded mid-run state and advance a few
    levels; every state component is compared (spectrum ring -> type-1 NUFFT
    + FFT; alpha -> FIR + propagator (+ RBC); sigma -> type-2, local sum,
    driving data and solve).  Several solve tiles and a ragged last tile."""
    import torch
    rng = np.random.default_rng(11)
    M = 1100
    if boundary == PERIODIC:
        dt = 2e-3
        x = rng.uniform(-math.pi, math.pi, M)
    else:
        dt = 5e-3
        x = rng.uniform(-2.0, 2.0, M)
    beta = rng.uniform(1, 10, M)
    pk = np.array([[1.0, -1.0, 0.1, 20.0, 0.3], [0.5, 0.5, 0.2, 0.0, 0.0]])
    p = dict(x=x, beta=beta, packets=pk, boundary=boundary, dt=dt, x_recv=np.zeros(0))
    o = oracle_for(p)
    prm = o.prm
    st = workloads.random_state(5, M, prm.K, prm.W, prm.m_max)
    # start at a level where the RBC fires after the first step (free space)
    L0 = 3 * prm.rbc_period - 1 if boundary == FREE_SPACE else 1234
    plan = wfp.Plan(p, dt)
    say(f"case synthetic_state boundary={boundary} M={M} K={prm.K} L0={L0}")
    gst = _state_to_gpu(st)
    plan.set_state(L0, gst["hist"], gst["ring"], gst["alpha"], gst["dalpha"])
    o.set_state(dict(L=L0, **st))
    for step in range(3):
        plan.run(1)
        o.step()
        torch.cuda.synchronize()
        g = _state_from_gpu(plan.get_state())
        e = o.get_state()
        assert g["L"] == e["L"]
        rs = rho(g["ring"][0], e["ring"][0])
        ra = rho(g["alpha"], e["alpha"])
        rd = rho(g["dalpha"], e["dalpha"])
        rh = rho(g["hist"][0], e["hist"][0])
        say(f"step {step}: ring {rs:.2e} alpha {ra:.2e} dalpha {rd:.2e} sigma {rh:.2e}")
        assert rs < 1e-12 and ra < 1e-12 and rd < 1e-12 and rh < 1e-12
        assert rho(g["hist"][:step + 1], e["hist"][:step + 1]) < 1e-12
        assert np.array_equal(g["hist"][step + 1:], e["hist"][step + 1:])   # inputs, moved untouched
    plan.close()


def test_receivers_small(wfp):
    p = workloads.periodic_single_pulse(21, 24, 0.01, 500, n_recv=9)
    p["x_recv"] = np.concatenate([p["x_recv"], [p["x"][3], p["x"][5] + 0.004, -3.1]])
    n = 501
    say(f"case receivers M=24 R={p['x_recv'].size}")
    g, gu, _ = gpu_march(wfp, p, n)
    o, ou = oracle_for(p).run(n)
    say(f"rho sigma {rho(g, o):.2e} u {rho(gu, ou):.2e}")
    assert rho(g, o) < TOL and rho(gu, ou) < TOL


def test_free_space_with_rbc(wfp):
    rng = np.random.default_rng(5)
    M = 40
    x = rng.uniform(-0.5, 1.5, M)
    beta = rng.uniform(1, 10, M)
    xr = np.array([-1.8, -0.2, 1.7])
    p = dict(x=x, beta=beta, packets=np.array([[1.0, -2.5, 0.2, 0.0, 0.0]]), boundary=FREE_SPACE, dt=0.01,
             x_recv=xr)
    n = 1100
    say(f"case free_space M={M} levels={n}")
    g, gu, info = gpu_march(wfp, p, n)
    o, ou = oracle_for(p).run(n)
    assert info["K"] == 256 and info["rbc_period"] == 43
    say(f"rho sigma {rho(g, o):.2e} u {rho(gu, ou):.2e}")
    assert rho(g, o) < TOL and rho(gu, ou) < TOL


def test_checkpoint_resume_is_bitwise(wfp):
    import torch
    p = workloads.small_periodic()
    plan = wfp.Plan(p, p["dt"])
    a1, _ = plan.march(150)
    st = plan.get_state()
    st = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in st.items()}
    a2, _ = plan.march(200)
    plan.reset()
    b0, _ = plan.march(10)
    plan.set_state(st["L"], st["hist"], st["ring"], st["alpha"], st["dalpha"])
    b2, _ = plan.march(200)
    torch.cuda.synchronize()
    assert torch.equal(a2, b2)
    plan.close()


def test_save_every_ragged_and_order(wfp):
    p = workloads.small_periodic()
    g1, _, _ = gpu_march(wfp, p, 101, save_every=1)
    g7, _, _ = gpu_march(wfp, p, 101, save_every=7)
    assert g7.shape == (15, 16)
    assert np.array_equal(g7, g1[::7])


def test_edge_single_spring_and_close_pair(wfp):
    """M = 1 (closed-form case) and two springs closer than dt (coupled solve)."""
    for x, beta in [(np.array([1.0]), np.array([5.0])), (np.array([0.5, 0.5037, 1.2]), np.array([9.0, 7.0, 2.0]))]:
        p = dict(x=x, beta=beta, packets=np.array([[1.0, -2.0, 0.3, 0.0, 0.0]]), boundary=PERIODIC, dt=0.01,
                 x_recv=np.zeros(0))
        g, _, info = gpu_march(wfp, p, 401)
        o, _ = oracle_for(p).run(401)
        say(f"edge M={x.size} rho={rho(g, o):.2e} iters={info['solve_iters']}")
        assert rho(g, o) < TOL


def test_interpolation_order_4(wfp):
    p = workloads.periodic_single_pulse(8, 30, 0.01, 300)
    g, _, _ = gpu_march(wfp, p, 301, p=4)
    o, _ = oracle_for(p, p=4).run(301)
    assert rho(g, o) < TOL


def test_multiband_full_size_against_stored_oracle(wfp):
    """The throughput workload at full size (M = 1e4, dt = 1e-3, levels
    0..10000, in the launch configuration bench.py times) against the stored
    oracle values of tests/golden/multiband_sigma.npz (written by
    tests/golden/make_golden.py from the oracle alone): every density at
    levels 250, 1000, 4000 and 10000 and 200 sampled springs every 100 levels."""
    import os
    import torch
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "multiband_sigma.npz"))
    p = workloads.multiband_periodic()
    n = int(g["n_levels"])
    say(f"multiband full size: M={p['x'].size} levels={n}")
    plan = wfp.Plan(p, p["dt"])
    every = 50
    sig = torch.empty(((n + every - 1) // every, p["x"].size), dtype=torch.float64, device="cuda")
    plan.run(n, sig, every)
    torch.cuda.synchronize()
    s = sig.cpu().numpy()
    plan.close()
    smax = float(g["sigma_max"])
    worst = 0.0
    for L, row in zip(g["full_levels"], g["full"]):
        worst = max(worst, float(np.max(np.abs(s[L // every] - row))))
    for i, row in enumerate(g["strided"]):
        L = i * int(g["strided_every"])
        worst = max(worst, float(np.max(np.abs(s[L // every][g["sample"]] - row))))
    say(f"  rho = {worst / smax:.2e}")
    assert worst / smax < TOL


def test_dense_cluster_global_solve(wfp):
    """400 springs inside an interval of length 0.01 at dt = 1e-3: about 80
    nearby sources per row along one run, more than an LDS tile holds, so the
    solve takes the global-sweep path (solve_mode 1)."""
    rng = np.random.default_rng(21)
    M = 400
    x = rng.uniform(0.5, 0.51, M)
    beta = rng.uniform(0.1, 1.0, M)
    prob = dict(x=x, beta=beta, packets=np.array([[1.0, 0.2, 0.03, 0.0, 0.0]]), boundary=PERIODIC,
                x_recv=np.array([0.49, 0.505, 0.53]), dt=1e-3)
    n = 300
    say(f"dense cluster: M={M} dt=1e-3 levels={n}")
    sig, u, info = gpu_march(wfp, prob, n)
    assert info["solve_mode"] == 1
    o = oracle_for(prob)
    ref, uref = o.run(n)
    assert np.max(np.abs(ref)) > 1e-3
    e1, e2 = rho(sig, ref), rho(u, uref)
    say(f"  rho(sigma) = {e1:.2e}  rho(u) = {e2:.2e}")
    assert e1 < TOL and e2 < TOL


def test_concurrent_chain_is_bitwise_identical(wfp):
    """The history chain on its own compute units (overlap_cus > 0) computes
    exactly what the single-stream level computes, receivers included."""
    import torch
    p = workloads.multiband_periodic()
    p = dict(p, x_recv=np.linspace(-1.0, 2.0, 8))
    n = 300
    out = []
    for cus in (-1, 32):
        plan = wfp.Plan(p, p["dt"], overlap_cus=cus)
        assert plan.info["overlap_cus"] == cus
        sig, u = plan.march(n, 7)
        torch.cuda.synchronize()
        out.append((sig.cpu().numpy(), u.cpu().numpy()))
        plan.close()
    say(f"concurrent chain: M={p['x'].size} levels={n}")
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    plan = wfp.Plan(p, p["dt"])
    say(f"  library choice: overlap_cus = {plan.info['overlap_cus']}")
    plan.close()


def test_autotune_keeps_results_and_level(wfp):
    """wfp_plan_autotune picks one of its candidate splits, leaves the plan at
    level 0 with zero history, and the march that follows equals the
    one-stream march bit for bit."""
    import torch
    p = workloads.paper_balanced_free_space(10_000)
    n = 200
    ref = wfp.Plan(p, p["dt"], p=6, overlap_cus=-1)
    sref, _ = ref.march(n, 9)
    torch.cuda.synchronize()
    ref.close()
    plan = wfp.Plan(p, p["dt"], p=6)
    with pytest.raises(wfp.WFPError):
        plan.autotune(0)
    pick = plan.autotune(3)
    say(f"autotune: overlap_cus = {pick}")
    assert pick in (-1, 32, 64, 96, 128) and plan.info["overlap_cus"] == pick and plan.info["level"] == 0
    sig, _ = plan.march(n, 9)
    torch.cuda.synchronize()
    assert np.array_equal(sig.cpu().numpy(), sref.cpu().numpy())
    with pytest.raises(wfp.WFPError):
        plan.autotune(3)                      # not at level 0
    plan.close()


def test_pipelined_runs_of_any_length(wfp):
    """The pipelined schedule (next level's local sum started while the
    current level is finished) split into runs of 1, 2, 3 and 257 levels, with
    a state restored in between and the driving data crossing a block of
    levels: bit for bit the one-stream march."""
    import torch
    p = workloads.multiband_periodic()
    runs = [1, 2, 3, 257, 1]
    out = []
    for cus in (-1, 32):
        plan = wfp.Plan(p, p["dt"], overlap_cus=cus)
        i = plan.info
        gst = _state_to_gpu(workloads.random_state(6, i["M"], i["K"], i["W"], i["m_max"]))
        plan.set_state(5000, gst["hist"], gst["ring"], gst["alpha"], gst["dalpha"])
        rows = []
        for k in runs:
            sig, _ = plan.march(k)
            rows.append(sig)
        st = plan.get_state()
        st = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in st.items()}
        more, _ = plan.march(40)
        plan.set_state(st["L"], st["hist"], st["ring"], st["alpha"], st["dalpha"])
        again, _ = plan.march(40)
        torch.cuda.synchronize()
        assert torch.equal(more, again)
        out.append(torch.cat(rows + [more]).cpu().numpy())
        plan.close()
    say(f"pipelined runs {runs} + 40 (restored): levels {out[0].shape[0]}")
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("case", ["free_space_stored", "periodic_on_the_fly"])
def test_overlap_forced_matches_one_stream(wfp, case):
    """Concurrent schedules the library does not pick by itself, forced with
    overlap_cus = 32: free space with stored weights (the RBC projection on the
    chain's queue, receivers on) and on-the-fly weights (the local sum on its
    own queue): bit for bit the one-stream march."""
    import torch
    rng = np.random.default_rng(21)
    if case == "free_space_stored":
        prm = Params(dt=5e-3, boundary=FREE_SPACE)
        lo, hi = prm.omega
        x = rng.uniform(lo + 0.1, hi - 0.1, 3000)
        p = dict(x=x, beta=rng.uniform(1, 10, x.size), packets=np.array([[1.0, lo - 0.2, 0.1, 20.0, 0.0]]),
                 boundary=FREE_SPACE, dt=prm.dt, x_recv=np.array([lo + 0.05, 0.0, hi - 0.05]))
        kw = dict(local_mode=1)
    else:
        p = workloads.small_periodic()
        kw = dict(local_mode=2)
    n = 160
    out = []
    for cus in (-1, 32):
        plan = wfp.Plan(p, p["dt"], overlap_cus=cus, **kw)
        assert plan.info["overlap_cus"] == cus
        sig, u = plan.march(n)
        torch.cuda.synchronize()
        out.append((sig.cpu().numpy(), None if u is None else u.cpu().numpy()))
        plan.close()
    say(f"forced overlap, {case}: levels={n} max |sigma| = {np.max(np.abs(out[0][0])):.3e}")
    assert np.max(np.abs(out[0][0])) > 0
    assert np.array_equal(out[0][0], out[1][0])
    if out[0][1] is not None:
        assert np.array_equal(out[0][1], out[1][1])


def test_check_finite(wfp):
    """check_finite: a healthy march returns OK with the same densities bit for
    bit; a NaN planted in the density history (from the host, through
    wfp_set_state) reaches the new level and wfp_run returns WFP_ENONFINITE."""
    import torch
    p = workloads.small_periodic()
    plain = wfp.Plan(p, p["dt"])
    a, _ = plain.march(120)
    plain.close()
    plan = wfp.Plan(p, p["dt"], check_finite=1)
    b, _ = plan.march(120)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    st = plan.get_state()
    hist = st["hist"].clone()
    hist[3, 5] = float("nan")
    plan.set_state(st["L"], hist, st["ring"], st["alpha"], st["dalpha"])
    say("check_finite: NaN planted in the density history at lag 4")
    with pytest.raises(wfp.WFPError) as ei:
        plan.run(1)
    assert ei.value.status == wfp.WFP_ENONFINITE
    assert plan.level == st["L"] + 1
    plan.close()


def test_solve_wrapper_matches_plan(wfp):
    """wfp.solve (plan, march, release in one call; tensors in or out)
    returns what a plan marched by hand returns."""
    import torch
    p = workloads.periodic_single_pulse(21, 24, 0.01, 300, n_recv=5)
    plan = wfp.Plan(p, p["dt"])
    s1, u1 = plan.march(300, 3)
    torch.cuda.synchronize()
    plan.close()
    u2, s2 = wfp.solve(torch.from_numpy(p["x"]), p["beta"], p["packets"], p["dt"], 300, boundary=0,
                       x_recv=p["x_recv"], save_every=3)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2) and torch.equal(u1, u2)
