"""The batched form (wfp_batch_*): every instance of a batch computes what its
own plan computes (same kernel bodies and reduction order; inlined into the
batched kernels the compiler contracts some multiply-adds differently, so the
two agree to rounding -- ~5e-14 after 137 levels -- not bitwise; the bar here is
rho <= 1e-12), one small instance is also checked against the oracle, and
the autotuned launch shape does not change any result (bitwise: the same
batched kernels run, only their block shape changes)."""
import sys

import numpy as np
import pytest

from oracle.march import Oracle, incident_driving
from oracle.params import Params
from paper_2507_07823_amd import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-12


def rho(a, b):
    a, b = np.asarray(a), np.asarray(b)
    m = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / m) if m > 0 else float(np.max(np.abs(a)))


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


def _instances():
    """Uneven instances: the small parity case, random springs at three time
    steps (different K and fine grids), and a dense cluster that takes the
    global-sweep solve."""
    out = [workloads.small_periodic()]
    rng = np.random.default_rng(31)
    for i, (M, dt) in enumerate([(300, 5e-3), (1200, 2e-3), (57, 1e-2), (2500, 1e-3)]):
        x = rng.uniform(-np.pi + 1.2, np.pi, M)
        beta = rng.uniform(1.0, 10.0, M)
        out.append(dict(x=x, beta=beta, packets=np.array([[1.0, -np.pi + 0.6, 0.05 + 0.01 * i, 0.0, 0.0]]),
                        boundary=0, dt=dt))
    x = rng.uniform(0.5, 0.51, 400)
    out.append(dict(x=x, beta=rng.uniform(0.1, 1.0, 400), packets=np.array([[1.0, 0.2, 0.03, 0.0, 0.0]]),
                    boundary=0, dt=1e-3))
    for p in out:
        p["x_recv"] = np.zeros(0)
    return out


def _plain(w, p, n):
    import torch
    plan = w.Plan(p, p["dt"])
    sig = torch.empty((n, p["x"].size), dtype=torch.float64, device="cuda")
    plan.run(n, sig, 1)
    st = plan.get_state()
    torch.cuda.synchronize()
    out = sig[-1].cpu().numpy(), {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in st.items()}, plan.info
    plan.close()
    return out


def _batch_run(b, insts, n):
    import torch
    fin = [torch.empty(p["x"].size, dtype=torch.float64, device="cuda") for p in insts]
    b.run(n, fin)
    torch.cuda.synchronize()
    return [f.cpu().numpy() for f in fin]


def test_batch_matches_plain_plans(wfp):
    import torch
    insts = _instances()
    n = 137
    say(f"batch: {len(insts)} instances, M = {[p['x'].size for p in insts]}, levels {n}")
    b = wfp.Batch(insts, [p["dt"] for p in insts])
    fin = _batch_run(b, insts, n)
    assert b.level == n
    modes = []
    worst = 0.0
    for i, p in enumerate(insts):
        last, st, info = _plain(wfp, p, n)
        modes.append(info["solve_mode"])
        bst = b.plan(i).get_state()
        torch.cuda.synchronize()
        errs = {"sigma": rho(fin[i], last)}
        for k in ("hist", "ring", "alpha", "dalpha"):
            errs[k] = rho(bst[k].cpu().numpy(), st[k])
        say(f"  instance {i} (M={p['x'].size}, dt={p['dt']:g}, solve_mode={info['solve_mode']}): "
            + " ".join(f"{k} {v:.1e}" for k, v in errs.items()))
        worst = max(worst, max(errs.values()))
        assert bst["L"] == st["L"] == n
    assert worst <= TOL
    assert 1 in modes and 0 in modes          # both solve paths are exercised
    b.close()


def test_batch_instance_against_oracle(wfp):
    insts = _instances()
    n = 200
    b = wfp.Batch(insts, [p["dt"] for p in insts])
    fin = _batch_run(b, insts, n)
    b.close()
    p = insts[0]
    o = Oracle(p["x"], p["beta"], Params(dt=p["dt"]), incident_driving(p["x"], p["beta"], p["packets"], True))
    ref, _ = o.run(n)
    err = float(np.max(np.abs(fin[0] - ref[-1])) / np.max(np.abs(ref)))
    say(f"batch instance 0 vs oracle at level {n - 1}: rho = {err:.2e}")
    assert err < 1e-10


def test_autotune_and_reset_keep_results(wfp):
    insts = _instances()
    n = 60
    b = wfp.Batch(insts, [p["dt"] for p in insts])
    first = _batch_run(b, insts, n)
    b.reset()
    assert b.level == 0
    shape = b.autotune(3)
    say(f"autotuned launch shape: rows per block {shape[0]}, xcd remap {shape[1]}, spread pass {shape[2]}")
    assert shape[0] in (4, 8) and shape[1] in (0, 1) and shape[2] in (0, 1)
    assert b.level == 0
    again = _batch_run(b, insts, n)
    for a, c in zip(first, again):
        assert np.array_equal(a, c)
    # every launch shape, the spread tile included, computes the same bits
    for rows in (4, 8):
        for xcd in (0, 1):
            for sp in (0, 1):
                b.reset()
                b.set_shape(rows, xcd, sp)
                out = _batch_run(b, insts, n)
                say(f"  shape ({rows}, {xcd}, {sp})")
                for a, c in zip(first, out):
                    assert np.array_equal(a, c)
    with pytest.raises(wfp.WFPError):
        b.set_shape(6, 0, 0)
    b.close()


@pytest.mark.parametrize("modes", [[2, 1, 2, 1, 2, 1], [3, 1, 3, 2, 3, 1]])
def test_batch_with_mixed_local_modes(wfp, modes):
    """Instances whose local weights are evaluated on the fly (local_mode 2)
    or stored once per unordered pair (local_mode 3) next to ones stored per
    ordered pair: each matches its own plan with the same mode."""
    import torch
    insts = _instances()
    n = 90
    b = wfp.Batch(insts, [p["dt"] for p in insts], per_instance=[{"local_mode": m} for m in modes])
    fin = _batch_run(b, insts, n)
    worst = 0.0
    for i, p in enumerate(insts):
        assert b.plan(i).info["local_mode"] == modes[i]
        last, _, _ = _plain(wfp, dict(p), n) if modes[i] == 1 else _plain_mode(wfp, p, n, modes[i])
        e = rho(fin[i], last)
        say(f"  instance {i} local_mode {modes[i]}: rho {e:.1e}")
        worst = max(worst, e)
    b.close()
    assert worst <= TOL


def _plain_mode(w, p, n, mode):
    import torch
    plan = w.Plan(p, p["dt"], local_mode=mode)
    sig = torch.empty((n, p["x"].size), dtype=torch.float64, device="cuda")
    plan.run(n, sig, 1)
    torch.cuda.synchronize()
    out = sig[-1].cpu().numpy(), None, plan.info
    plan.close()
    return out


def test_batch_receivers_match_plain_plans(wfp):
    """Receivers in the batched form: each instance's field at its receivers,
    level by level over two runs (the second starting where the first ended),
    equals its own plan's to 1e-12 of the unit incident amplitude (before the
    scattered field arrives the values are ~1e-19 rounding noise, so the bar
    is absolute); instances without receivers and runs without receiver
    outputs write nothing."""
    import torch
    insts = _instances()[:4]
    rng = np.random.default_rng(7)
    for i, p in enumerate(insts):
        p["x_recv"] = rng.uniform(-np.pi + 1.2, np.pi, [5, 0, 9, 3][i])
    n1, n2 = 150, 110
    say(f"batch receivers: R = {[p['x_recv'].size for p in insts]}, levels {n1} + {n2}")
    b = wfp.Batch(insts, [p["dt"] for p in insts])
    out = []
    for n in (n1, n2):
        u = [torch.full((n, max(p["x_recv"].size, 1)), -7.0, dtype=torch.float64, device="cuda") if p["x_recv"].size
             else None for p in insts]
        b.run(n, None, u)
        torch.cuda.synchronize()
        out.append([None if t is None else t.cpu().numpy() for t in u])
    b.run(5)                                       # no receiver outputs: the earlier buffers are left alone
    torch.cuda.synchronize()
    worst, seen = 0.0, 0.0
    for i, p in enumerate(insts):
        R = p["x_recv"].size
        if R == 0:
            continue
        plan = wfp.Plan(p, p["dt"])
        _, uref = plan.march(n1 + n2)
        torch.cuda.synchronize()
        ref = uref.cpu().numpy()
        plan.close()
        got = np.concatenate([out[0][i], out[1][i]])
        err = float(np.max(np.abs(got - ref)))
        worst = max(worst, err)
        seen = max(seen, float(np.max(np.abs(ref))))
        say(f"  instance {i}: R = {R}, max |u| = {np.max(np.abs(ref)):.2e}, max |batch - plan| = {err:.2e}")
    assert worst < 1e-12 and seen > 1e-3
    b.close()


GOLDEN_DIR = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _load_golden_module():
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN_DIR, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_batch_recipe_instances_against_oracle(wfp):
    """The batched workload's instances with M <= 1e4 among its first 24,
    marched together, each for its own level count N_i (1125..2000,
    wfp_batch_set_levels): sampled springs at levels 499, 999, 1499 and every
    spring at each instance's last level against the oracle's own marches
    (tests/golden/batch_recipe.npz)."""
    import os
    import torch
    g = np.load(os.path.join(GOLDEN_DIR, "batch_recipe.npz"))
    cases = _load_golden_module().batch_recipe_cases()
    assert [c[0] for c in cases] == list(g["index"])
    insts = [c[1] for c in cases]
    ends = [c[2] for c in cases]
    say(f"batch recipe: {len(insts)} instances, M = {[p['x'].size for p in insts]}, levels {ends}")
    b = wfp.Batch(insts, [p["dt"] for p in insts])
    b.set_levels(ends)
    worst = 0.0
    for L1 in (500, 1000, 1500, 2000):
        fin = [torch.full((p["x"].size,), float("nan"), dtype=torch.float64, device="cuda") for p in insts]
        b.run(L1 - b.level, fin)
        torch.cuda.synchronize()
        for k, (i, p, n) in enumerate(cases):
            got = fin[k].cpu().numpy()
            smax = float(g["sigma_max"][k])
            if L1 - 1 < n:                       # still marching: level L1 - 1
                key = f"at{L1 - 1}_{i}"
                if key in g:
                    e = float(np.max(np.abs(got[g[f"sample_{i}"]] - g[key]))) / smax
                    worst = max(worst, e)
            elif L1 == 2000 or L1 - 500 < n:     # its last level
                assert b.plan(k).level == n
                e = float(np.max(np.abs(got - g[f"last_{i}"]))) / smax
                worst = max(worst, e)
    say(f"  worst rho over the compared levels: {worst:.2e}")
    assert worst < 1e-10
    assert b.level == 2000
    b.close()


def test_batch_paths_against_oracle(wfp):
    """Five instances that between them take every batched kernel path (tiled
    Jacobi solve, global sweeps with a wavefront per row, local weights on the
    fly, receivers, direct small-run solve), each with its own level count:
    their last levels and receivers at every level against the oracle
    (tests/golden/batch_paths.npz); receiver rows at and beyond an instance's
    end are left untouched."""
    import os
    import torch
    g = np.load(os.path.join(GOLDEN_DIR, "batch_paths.npz"))
    cases = _load_golden_module().batch_paths_cases()
    insts = [c[0] for c in cases]
    ends = [c[1] for c in cases]
    modes = [c[2] for c in cases]
    n = max(ends)
    b = wfp.Batch(insts, [p["dt"] for p in insts], per_instance=[{"local_mode": m} for m in modes])
    infos = [b.plan(i).info for i in range(b.n)]
    say("batch paths: " + "; ".join(f"M={q['M']} solve_mode={q['solve_mode']} tiles={q['n_solve_tiles']} "
                                    f"direct={q['n_direct_tiles']} wave={q['sweep_wave']} local_mode={q['local_mode']} "
                                    f"R={q['R']}" for q in infos))
    assert infos[0]["solve_mode"] == 0 and infos[0]["n_solve_tiles"] > 0
    assert infos[1]["solve_mode"] == 1 and infos[1]["sweep_wave"] == 1
    assert infos[2]["local_mode"] == 2 and infos[2]["R"] == 3
    assert infos[4]["n_direct_tiles"] > 0
    b.set_levels(ends)
    fin = [torch.empty(p["x"].size, dtype=torch.float64, device="cuda") for p in insts]
    rec = [torch.full((n, p["x_recv"].size), float("nan"), dtype=torch.float64, device="cuda")
           if p["x_recv"].size else None for p in insts]
    b.run(n, fin, rec)
    torch.cuda.synchronize()
    for i, p in enumerate(insts):
        smax = float(g[f"smax_{i}"])
        e = float(np.max(np.abs(fin[i].cpu().numpy() - g[f"last_{i}"]))) / smax
        msg = f"  instance {i}: levels {ends[i]} rho(last sigma) = {e:.2e}"
        assert b.plan(i).level == ends[i]
        assert e < 1e-10
        if rec[i] is not None:
            u = rec[i].cpu().numpy()
            ref = g[f"recv_{i}"]
            eu = rho(u[:ends[i]], ref)
            msg += f" rho(receivers) = {eu:.2e}"
            assert eu < 1e-10 and np.max(np.abs(ref)) > 1e-3       # the scattered field reaches them
            assert np.isnan(u[ends[i]:]).all()
        say(msg)
    b.close()
