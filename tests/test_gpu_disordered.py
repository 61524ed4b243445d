"""The long disordered run of Section 6.3 at M = 1e3 through the HIP path:
1000 random springs, a pulse of width sqrt(8) times the mean spacing, p = 8,
72044 levels of dt = 1.308e-4 (about 3 pi), the field at 50 receivers; its
accuracy estimated, as the paper does, against the same run at dt / 2
(144088 levels) at the common times."""
import sys

import numpy as np
import pytest

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


def run(w, prob):
    import torch
    plan = w.Plan(prob, prob["dt"], p=prob["p"])
    info = plan.info
    n = prob["n_steps"]
    _, u = plan.march(n, save_every=n)
    torch.cuda.synchronize()
    out = u.cpu().numpy()
    plan.close()
    return out, info


def test_disordered_self_convergence(wfp):
    a = workloads.disordered_long(1000)
    b = workloads.disordered_long(1000, refine=2)
    say(f"case disordered M=1000 levels {a['n_steps']} and {b['n_steps']}")
    ua, ia = run(wfp, a)
    ub, ib = run(wfp, b)
    assert ia["K"] == 20480 and ib["K"] == 40960 and ia["p"] == 8
    assert np.all(np.isfinite(ua)) and np.all(np.isfinite(ub))
    ref = ub[::2][: ua.shape[0]]
    scale = np.max(np.abs(ref))
    est = float(np.max(np.abs(ua - ref)) / scale)
    say(f"field max {scale:.3e}, estimated relative error at dt {est:.2e}")
    assert scale > 1e-2 and est < 1e-6
