"""Parity of the HIP path with the FP64 CPU oracle on the free-space scaling
study of Section 6.2 (springs uniform in [-2, 2], beta in [0.1, 3], Gaussian
pulse exp(-30 (s + 3)^2), p = 6, dt such that the mean neighbour count is
about 100).

* M = 1e3 (K = 512): a full march from rest through the pulse's passage,
  every density of every level against the oracle.
* M = 2e4 (K = 10240), and 400 springs at the time steps of the study's
  M = 1e5 (K = 51200 = 200 x 256) and M = 1e6 (K = 524288, a fine grid of
  2.5e6 points whose rows take the 1024-thread passes): three levels from a seeded mid-run state across a
  boundary correction (computed over workgroups at these K), against the
  oracle's values stored by tests/golden/make_golden.py.
"""
import os
import sys

import numpy as np
import pytest

from oracle.march import Oracle, incident_driving
from oracle.params import FREE_SPACE, Params
from paper_2507_07823_amd import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-10
GOLDEN_DIR = os.path.join(os.path.dirname(__file__), "golden")


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


def test_balanced_small_full_march(wfp):
    import torch
    p = workloads.paper_balanced_free_space(1000)
    n = 700                                   # t = 4: the pulse has crossed [-2, 2]
    say(f"case balanced M=1000 p=6 levels={n}")
    plan = wfp.Plan(p, p["dt"], p=p["p"])
    info = plan.info
    sig, _ = plan.march(n)
    torch.cuda.synchronize()
    g = sig.cpu().numpy()
    plan.close()
    prm = Params(dt=p["dt"], boundary=FREE_SPACE, p=p["p"])
    o = Oracle(p["x"], p["beta"], prm, incident_driving(p["x"], p["beta"], p["packets"], False))
    e, _ = o.run(n)
    assert info["K"] == prm.K == 512 and info["p"] == 6 and info["m_max"] == 38
    assert 90 < info["n_pairs"] / 1000 < 110          # mean neighbours ~ 100 (self included)
    assert np.max(np.abs(e)) > 1e-3                   # the pulse has driven the springs
    r = rho(g, e)
    say(f"rho={r:.3e} rbc_period={info['rbc_period']} solve_mode={info['solve_mode']}")
    assert r < TOL


@pytest.mark.parametrize("case", ["balanced", "midgrid", "longgrid", "disordered"])
def test_long_grids_from_state(wfp, case):
    """Three levels from a seeded mid-run state (the boundary projection due
    after the first) against stored oracle levels: the scaling study at
    M = 2e4, its longest grids (K = 51200, 524288) at 400 springs, and the
    long disordered run of Section 6.3 at M = 1e3 (K = 20480, p = 8)."""
    import torch
    g = np.load(os.path.join(GOLDEN_DIR, f"{case}_state_steps.npz"))
    M = int(g["M"])
    if case == "balanced":
        p = workloads.paper_balanced_free_space(M)
    elif case == "disordered":
        p = workloads.disordered_long(M)
    elif case == "midgrid":
        p = workloads.long_grid_free_space(M, spread=0.2, study_M=100_000)
    else:
        p = workloads.long_grid_free_space(M)
    prm = Params(dt=p["dt"], boundary=FREE_SPACE, p=p["p"])
    assert prm.K == int(g["K"])
    st = workloads.random_state(int(g["state_seed"]), M, prm.K, prm.W, prm.m_max)
    L0 = int(g["L0"])
    say(f"case {case}-state M={M} K={prm.K} L0={L0}")
    plan = wfp.Plan(p, p["dt"], p=p["p"])
    assert plan.info["K"] == prm.K and plan.info["rbc_period"] == prm.rbc_period
    c = lambda z: torch.from_numpy(np.ascontiguousarray(np.stack([z.real, z.imag], -1))).cuda()
    plan.set_state(L0, torch.from_numpy(np.ascontiguousarray(st["hist"])).cuda(), c(st["ring"]),
                   c(st["alpha"]), c(st["dalpha"]))
    for step in range(g["sigma"].shape[0]):
        plan.run(1)
        torch.cuda.synchronize()
        s = plan.get_state()
        r = rho(s["hist"][0].cpu().numpy(), g["sigma"][step])
        say(f"step {step}: sigma {r:.2e}")
        assert r < TOL
    cz = lambda t: t.cpu().numpy()[..., 0] + 1j * t.cpu().numpy()[..., 1]
    k = int(g["mode_stride"])
    ra = rho(cz(s["alpha"])[::k], g["alpha"])
    rd = rho(cz(s["dalpha"])[::k], g["dalpha"])
    rs = rho(cz(s["ring"])[0][::k], g["spectrum"])
    say(f"alpha {ra:.2e} dalpha {rd:.2e} spectrum {rs:.2e}")
    assert ra < TOL and rd < TOL and rs < TOL
    plan.close()
