"""Stored local weights once per unordered pair (local_mode 3): Q_m depends on
the distance alone (Section 4.1), so each pair's weights are stored once, per
row and lag over the row's upper source range, and applied to both rows (the
on-the-fly layout's column sums and per-row reduce).  Checked against the
weights stored per ordered pair (local_mode 1) and against the oracle,
including upper ranges that wrap past pi in the periodic box and a dense
cluster of nearby springs."""
import sys

import numpy as np
import pytest

from oracle.march import Oracle, incident_driving
from oracle.params import FREE_SPACE, PERIODIC, Params
from paper_2507_07823_amd import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-10


def rho(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


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


def _march(w, prob, n, **kw):
    import torch
    plan = w.Plan(prob, prob["dt"], **kw)
    sig, u = plan.march(n)
    torch.cuda.synchronize()
    out = sig.cpu().numpy(), (None if u is None else u.cpu().numpy()), plan.info
    plan.close()
    return out


def _oracle(p, n, boundary=PERIODIC):
    o = Oracle(p["x"], p["beta"], Params(dt=p["dt"], boundary=boundary),
               incident_driving(p["x"], p["beta"], p["packets"], boundary == PERIODIC),
               x_recv=p["x_recv"] if p["x_recv"].size else None)
    return o.run(n)


def test_pair_once_matches_stored_multiband(wfp):
    p = workloads.multiband_periodic()
    n = 300
    s1, _, i1 = _march(wfp, p, n, local_mode=1)
    s3, _, i3 = _march(wfp, p, n, local_mode=3)
    assert i1["local_mode"] == 1 and i3["local_mode"] == 3
    e = rho(s3, s1)
    say(f"pair-once vs per-pair stored weights, multiband M=1e4, {n} levels: rho = {e:.2e}; "
        f"weights stored {i3['n_weights_stored']} vs {i1['n_weights_stored']}")
    assert e < 1e-12
    assert i3["n_weights_stored"] < 0.6 * i1["n_weights_stored"]


def test_pair_once_small_periodic_against_oracle(wfp):
    p = workloads.small_periodic()
    n = 600
    sig, _, info = _march(wfp, p, n, local_mode=3)
    assert info["local_mode"] == 3
    ref, _ = _oracle(dict(p, x_recv=np.zeros(0)), n)
    e = rho(sig, ref)
    say(f"pair-once small periodic vs oracle: rho = {e:.2e}")
    assert e < TOL


def test_pair_once_free_space_with_receivers_against_oracle(wfp):
    rng = np.random.default_rng(17)
    M, dt = 40, 0.0125
    prm = Params(dt=dt, boundary=FREE_SPACE)
    lo, hi = prm.omega
    x = rng.uniform(lo + 0.6, hi - 0.3, M)
    beta = rng.uniform(1.0, 10.0, M)
    p = dict(x=x, beta=beta, packets=np.array([[1.0, lo - 0.1, 0.08, 20.0, 0.0]]), boundary=FREE_SPACE,
             x_recv=np.array([lo + 0.3, 0.0, hi - 0.1]), dt=dt)
    n = 500
    sig, u, info = _march(wfp, p, n, local_mode=3)
    ref, uref = _oracle(p, n, FREE_SPACE)
    e1, e2 = rho(sig, ref), rho(u, uref)
    say(f"pair-once free space vs oracle: rho(sigma) = {e1:.2e} rho(u) = {e2:.2e}")
    assert e1 < TOL and e2 < TOL


def test_pair_once_wrapping_upper_ranges_against_oracle(wfp):
    """60 springs within 0.3 of the periodic seam (x near +pi and -pi), dt =
    0.01 (delta = 0.35): most upper ranges continue past the last sorted
    spring to the first ones."""
    rng = np.random.default_rng(23)
    x = np.concatenate([rng.uniform(np.pi - 0.3, np.pi, 30), rng.uniform(-np.pi, -np.pi + 0.3, 30)])
    beta = rng.uniform(1.0, 10.0, 60)
    p = dict(x=x, beta=beta, packets=np.array([[1.0, 0.0, 0.1, 0.0, 0.0]]), boundary=PERIODIC,
             x_recv=np.zeros(0), dt=0.01)
    n = 450
    sig, _, info = _march(wfp, p, n, local_mode=3)
    assert info["local_mode"] == 3
    ref, _ = _oracle(p, n)
    e = rho(sig, ref)
    say(f"pair-once across the periodic seam vs oracle: rho = {e:.2e} (max |sigma| {np.max(np.abs(ref)):.2e})")
    assert e < TOL and np.max(np.abs(ref)) > 1e-2


def test_pair_once_dense_cluster_against_oracle(wfp):
    """400 springs within 0.01 at dt = 1e-3: every pair nearby or
    intermediate, the global-sweep solve."""
    rng = np.random.default_rng(21)
    x = rng.uniform(0.5, 0.51, 400)
    beta = rng.uniform(0.1, 1.0, 400)
    p = dict(x=x, beta=beta, packets=np.array([[1.0, 0.2, 0.03, 0.0, 0.0]]), boundary=PERIODIC,
             x_recv=np.zeros(0), dt=1e-3)
    n = 400
    sig, _, info = _march(wfp, p, n, local_mode=3)
    assert info["local_mode"] == 3 and info["solve_mode"] == 1
    ref, _ = _oracle(p, n)
    e = rho(sig, ref)
    say(f"pair-once dense cluster vs oracle: rho = {e:.2e}")
    assert e < TOL


def test_pair_once_dense_cluster_across_the_seam_against_oracle(wfp):
    """300 springs within 0.005 of the periodic seam at dt = 1e-3: upper
    ranges of about 150 sources (two sources per lane in the pair-once
    kernels), which run past the last sorted spring to the first, so density
    pairs straddle source M - 1 and source 0."""
    rng = np.random.default_rng(31)
    x = np.mod(np.pi + rng.uniform(-0.005, 0.005, 300) + np.pi, 2 * np.pi) - np.pi
    beta = rng.uniform(0.05, 0.5, 300)
    p = dict(x=x, beta=beta, packets=np.array([[1.0, np.pi - 0.2, 0.03, 0.0, 0.0]]), boundary=PERIODIC,
             x_recv=np.zeros(0), dt=1e-3)
    xs = np.sort(x)
    gap = np.diff(np.concatenate([xs, xs[:1] + 2 * np.pi]))
    assert np.max(gap) > np.pi                      # one cluster across the seam
    n = 350
    sig, _, info = _march(wfp, p, n, local_mode=3)
    assert info["local_mode"] == 3
    assert info["n_pairs"] / 2 / x.size > 96         # long upper ranges: two sources per lane
    ref, _ = _oracle(p, n)
    e = rho(sig, ref)
    say(f"pair-once dense cluster across the seam vs oracle: rho = {e:.2e} (max |sigma| {np.max(np.abs(ref)):.2e})")
    assert e < TOL and np.max(np.abs(ref)) > 1e-2


def test_pair_once_gradient(wfp):
    """With weights stored once per unordered pair the gradient pass gives
    both gradients (checked against the oracle in tests/test_gpu_adjoint.py)."""
    import torch
    p = workloads.small_periodic()
    p = dict(p, x_recv=np.array([0.5, 1.5]))
    plan = wfp.Plan(p, p["dt"], local_mode=3, checkpoint_every=20)
    u = torch.empty((40, 2), dtype=torch.float64, device="cuda")
    plan.run(40, None, 1, u)
    gb, gx = plan.gradient(u)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(gb).all() and torch.isfinite(gx).all()) and float(gb.abs().max()) > 0
    plan.close()


@pytest.mark.parametrize("p", [2, 4, 6, 10, 12])
def test_every_interpolation_order_matches_stored(wfp, p):
    """The on-the-fly kernel (local_mode 2, one template per p) and the
    pair-once stored weights (local_mode 3) against the weights stored per
    ordered pair (local_mode 1) at every even p other than 8: 120 random
    springs in the periodic box, 250 levels."""
    rng = np.random.default_rng(40 + p)
    x = rng.uniform(-np.pi + 1.2, np.pi, 120)
    beta = rng.uniform(1.0, 10.0, 120)
    prob = dict(x=x, beta=beta, packets=np.array([[1.0, -np.pi + 0.6, 0.05, 0.0, 0.0]]), boundary=PERIODIC,
                x_recv=np.zeros(0), dt=5e-3)
    n = 250
    s1, _, i1 = _march(wfp, prob, n, local_mode=1, p=p)
    s2, _, i2 = _march(wfp, prob, n, local_mode=2, p=p)
    s3, _, i3 = _march(wfp, prob, n, local_mode=3, p=p)
    assert (i1["p"], i2["p"], i3["p"]) == (p, p, p)
    e2, e3 = rho(s2, s1), rho(s3, s1)
    say(f"p = {p}: on the fly {e2:.2e}, pair-once stored {e3:.2e} against per-pair stored (max |sigma| "
        f"{np.max(np.abs(s1)):.2e})")
    assert e2 < 1e-12 and e3 < 1e-12 and np.max(np.abs(s1)) > 1e-2
