"""wfp_run_noalloc (no device allocation: the driving-data block in the
library's static per-GPU scratch) against wfp_run through the C ABI: two
calls in a row on one GPU, the second with a smaller problem (the scratch
still holds the first call's data), each compared with wfp_run on an
identical plan."""
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


def _pair(wfp, p, n, save_every, **kw):
    """The same march by wfp_run and by wfp_run_noalloc on two identical plans."""
    import torch
    out = []
    for noalloc in (False, True):
        plan = wfp.Plan(p, p["dt"], **kw)
        M, R = plan.info["M"], plan.info["R"]
        sig = torch.full((-(-n // save_every), M), float("nan"), dtype=torch.float64, device="cuda")
        u = torch.full((n, max(R, 1)), float("nan"), dtype=torch.float64, device="cuda") if R else None
        (plan.run_noalloc if noalloc else plan.run)(n, sig, save_every, u)
        torch.cuda.synchronize()
        out.append((sig.cpu().numpy(), None if u is None else u.cpu().numpy(), plan.level))
        plan.close()
    return out


def _rho(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_noalloc_matches_run_twice_second_smaller(wfp):
    # first call: 5000 periodic springs (the block holds 209 levels), finite check on
    big = workloads.multiband_periodic(M=5000)
    (s1, _, l1), (s2, _, l2) = _pair(wfp, big, 420, 7, check_finite=1)
    say(f"M=5000 periodic: levels {l1}/{l2}, rho = {_rho(s2, s1):.2e}, bitwise {np.array_equal(s1, s2)}")
    assert l1 == l2 == 420
    assert np.isfinite(s2).all() and np.max(np.abs(s1)) > 0
    assert _rho(s2, s1) < 1e-12
    # second call: 300 free-space springs with receivers
    small = workloads.periodic_single_pulse(33, 300, 0.0125, 500, x_range=(-1.0, 1.0), n_recv=5)
    small["boundary"] = 1
    (s1, u1, l1), (s2, u2, l2) = _pair(wfp, small, 500, 1)
    say(f"M=300 free space: rho(sigma) = {_rho(s2, s1):.2e}, rho(u) = {_rho(u2, u1):.2e}, "
        f"bitwise {np.array_equal(s1, s2) and np.array_equal(u1, u2)}")
    assert l1 == l2 == 500
    assert np.isfinite(s2).all() and np.isfinite(u2).all() and np.max(np.abs(u1)) > 0
    assert _rho(s2, s1) < 1e-12 and _rho(u2, u1) < 1e-12


def test_noalloc_refuses_checkpointing_plans(wfp):
    p = workloads.small_periodic()
    plan = wfp.Plan(p, p["dt"], checkpoint_every=50)
    with pytest.raises(wfp.WFPError) as e:
        plan.run_noalloc(10)
    assert e.value.status == wfp.WFP_EINVAL
    plan.close()
