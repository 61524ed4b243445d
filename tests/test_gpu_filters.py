"""The filter demonstrations of Section 6.4 through the HIP path, against
the exact solution for point springs (oracle.exact.spring_array_field: the
frequency-domain solve per frequency and its inverse transform, pinned in
test_oracle_exact.py) and, for the two-spring cavity, against the oracle
march.  The total field downstream is the incident wave plus the receiver's
scattered field; errors are measured against the incident wave's unit
amplitude (the arrays transmit as little as 3e-5 of it).  Stiffness 100 at
dt = 0.01 runs at p = 6: the p = 8 local rule is unstable there."""
import math
import sys

import numpy as np
import pytest

from oracle.exact import spring_array_field, spring_array_transmission
from oracle.march import Oracle, incident_driving
from oracle.params import FREE_SPACE, Params
from paper_2507_07823_amd import workloads

pytestmark = pytest.mark.gpu


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


def total_field(prob, u):
    t = np.arange(u.shape[0]) * prob["dt"]
    return u[:, 0] + np.exp(-prob["mu"] * (prob["x_recv"][0] - t - prob["t0"]) ** 2)


def gpu_march(w, prob):
    import torch
    plan = w.Plan(prob, prob["dt"], p=prob["p"])
    sig, u = plan.march(prob["n_steps"], save_every=1)
    torch.cuda.synchronize()
    out = sig.cpu().numpy(), u.cpu().numpy()
    plan.close()
    return out


def check_exact(prob, tot, n_samples=150, dw=5e-5, transmission=None):
    lv = np.linspace(0, prob["n_steps"] - 1, n_samples).astype(int)
    ex = spring_array_field(prob["x_recv"][0], lv * prob["dt"], prob["x"], prob["beta"], prob["mu"], prob["t0"],
                            dw=dw, transmission=transmission)
    return float(np.max(np.abs(tot[lv] - ex))), float(np.max(np.abs(ex)))


def test_fabry_perot_exact_and_oracle(wfp):
    prob = workloads.fabry_perot()
    say(f"case fabry-perot levels={prob['n_steps']}")
    sig, u = gpu_march(wfp, prob)
    tot = total_field(prob, u)
    err, peak = check_exact(prob, tot)
    say(f"against the exact field: {err:.2e} (transmitted peak {peak:.2e})")
    assert err < 1e-9 and peak > 1e-3
    prm = Params(dt=prob["dt"], boundary=FREE_SPACE, p=prob["p"])
    o = Oracle(prob["x"], prob["beta"], prm, incident_driving(prob["x"], prob["beta"], prob["packets"], False),
               x_recv=prob["x_recv"])
    es, eu = o.run(prob["n_steps"])
    rs = float(np.max(np.abs(sig - es)) / np.max(np.abs(es)))
    ru = float(np.max(np.abs(u - eu)) / np.max(np.abs(eu)))
    say(f"against the oracle: sigma {rs:.2e} u {ru:.2e}")
    assert rs < 1e-10 and ru < 1e-10
    # the cavity passes frequencies near multiples of pi / L (L = 1): the
    # peaks of the Hann-windowed transfer ratio over the run sit at the exact
    # resonances (maxima of |T(w)|)
    n = tot.size
    t = np.arange(n) * prob["dt"]
    win = 0.5 - 0.5 * np.cos(2 * np.pi * t / t[-1])
    inc = np.exp(-prob["mu"] * (prob["x_recv"][0] - t - prob["t0"]) ** 2)
    w = np.linspace(1.0, 11.0, 4001)
    ph = np.exp(1j * np.outer(w, t))
    R = np.abs(ph @ (tot * win)) / np.abs(ph @ inc)
    peaks = [w[i] for i in range(1, w.size - 1) if R[i] > R[i - 1] and R[i] > R[i + 1] and R[i] > 0.2 * R.max()]
    we = np.linspace(1.0, 11.0, 200001)
    Te = np.abs(spring_array_transmission(we, prob["x"], prob["beta"]))
    exact = [we[i] for i in range(1, we.size - 1) if Te[i] > Te[i - 1] and Te[i] > Te[i + 1]]
    say(f"transmission peaks {np.round(peaks, 3)}, exact resonances {np.round(exact, 4)}")
    assert len(peaks) == len(exact) == 3
    assert max(abs(a - b) for a, b in zip(peaks, exact)) < 0.01
    assert all(abs(e / math.pi - k) < 0.07 for k, e in zip((1, 2, 3), exact))


@pytest.mark.parametrize("which", [0, 1])
def test_spring_array_exact(wfp, which):
    """The ten springs of stiffness 100 (p = 6) and the 200 springs of
    stiffness 1 (p = 8), 25134 levels, against the exact field (the 200-spring
    one by transfer matrices, spring_chain_transmission)."""
    from oracle.exact import spring_chain_transmission
    prob = workloads.spring_arrays()[which]
    say(f"case array M={prob['x'].size} beta={prob['beta'][0]:g} p={prob['p']} levels={prob['n_steps']}")
    _, u = gpu_march(wfp, prob)
    if which == 0:
        err, peak = check_exact(prob, total_field(prob, u))
    else:
        err, peak = check_exact(prob, total_field(prob, u), dw=4e-4, transmission=spring_chain_transmission)
    say(f"against the exact field: {err:.2e} (peak of the total field {peak:.2e})")
    assert err < 1e-9
