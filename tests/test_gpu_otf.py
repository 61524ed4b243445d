"""Local weights evaluated on the fly (local_mode 2): the same discrete scheme
as the stored weights, regrouped by quadrature node.  Checked against the
stored path and the oracle at small sizes, and at the clumped free-space
workload's full size (M = 1e6, where stored weights would need ~1.1 TB)
against the oracle's local sum on sampled springs from a synthetic state."""
import sys

import numpy as np
import pytest

from oracle.local import local_weights
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


def _march(w, p, n, **kw):
    import torch
    plan = w.Plan(p, p["dt"], **kw)
    sig, u = plan.march(n)
    torch.cuda.synchronize()
    out = sig.cpu().numpy(), (None if u is None else u.cpu().numpy()), plan.info
    plan.close()
    return out


def test_otf_matches_stored_weights_multiband(wfp):
    p = workloads.multiband_periodic()
    n = 300
    s1, _, i1 = _march(wfp, p, n, local_mode=1)
    s2, _, i2 = _march(wfp, p, n, local_mode=2)
    assert i1["local_mode"] == 1 and i2["local_mode"] == 2
    e = rho(s2, s1)
    say(f"on-the-fly vs stored weights, multiband M=1e4, {n} levels: rho = {e:.2e}")
    assert e < 1e-12


def test_otf_small_periodic_against_oracle(wfp):
    p = workloads.small_periodic()
    n = 600
    sig, _, info = _march(wfp, p, n, local_mode=2)
    assert info["local_mode"] == 2
    o = Oracle(p["x"], p["beta"], Params(dt=p["dt"]), incident_driving(p["x"], p["beta"], p["packets"], True))
    ref, _ = o.run(n)
    e = rho(sig, ref)
    say(f"on-the-fly small periodic vs oracle: rho = {e:.2e}")
    assert e < TOL


def test_otf_free_space_with_receivers_against_oracle(wfp):
    rng = np.random.default_rng(17)
    M, dt = 40, 0.0125
    prm = Params(dt=dt, boundary=FREE_SPACE)
    lo, hi = prm.omega
    x = rng.uniform(lo + 0.6, hi - 0.3, M)
    beta = rng.uniform(1.0, 10.0, M)
    p = dict(x=x, beta=beta, packets=np.array([[1.0, lo - 0.1, 0.08, 20.0, 0.0]]), boundary=FREE_SPACE,
             x_recv=np.array([lo + 0.3, 0.0, hi - 0.1]), dt=dt)
    n = 500
    sig, u, info = _march(wfp, p, n, local_mode=2)
    o = Oracle(x, beta, prm, incident_driving(x, beta, p["packets"], False), x_recv=p["x_recv"])
    ref, uref = o.run(n)
    e1, e2 = rho(sig, ref), rho(u, uref)
    say(f"on-the-fly free space vs oracle: rho(sigma) = {e1:.2e} rho(u) = {e2:.2e}  K={info['K']}")
    assert e1 < TOL and e2 < TOL


@pytest.fixture(scope="module")
def clumped(wfp):
    """The clumped free-space workload at full size (M = 1e6) and its plan,
    shared by the tests below (creating it takes most of their time)."""
    p = workloads.clumped_free_space()
    say(f"clumped free space full size: M={p['x'].size} dt={p['dt']}")
    plan = wfp.Plan(p, p["dt"])
    info = plan.info
    say(f"  plan: local_mode={info['local_mode']} pairs={info['n_pairs']} solve_mode={info['solve_mode']} "
        f"K={info['K']} rbc_period={info['rbc_period']}")
    yield p, plan, info
    plan.close()


def _sample_rows(M, seed):
    """48 springs of the uniform part and 48 in clumps (the workload puts the
    clumped 10 % last)."""
    rng = np.random.default_rng(seed)
    n_un = int(round(0.9 * M))
    return np.concatenate([rng.choice(n_un, 48, replace=False), n_un + rng.choice(M - n_un, 48, replace=False)])


def _near(x, j, prm):
    d = np.abs(x - x[j])
    nb = np.nonzero(d < prm.delta)[0]
    return nb, local_weights(d[nb], prm.dt, prm.W, prm.p, prm.delta, prm.b, prm.n_gl_local)


def test_local_part_clumped_full_size_sampled(clumped):
    """M = 1e6 clumped free-space springs: the plan chooses on-the-fly weights;
    from a synthetic density history the local part at 96 sampled springs
    (half of them in clumps) is compared with the oracle's sum over the
    springs within delta of each, with the oracle's weights."""
    import torch
    p, plan, info = clumped
    M = p["x"].size
    assert info["local_mode"] == 2
    mm, K, W = info["m_max"], info["K"], info["W"]
    g = torch.Generator().manual_seed(123)
    hist = torch.randn((mm, M), generator=g, dtype=torch.float64)
    ring = torch.zeros((W, K + 1, 2), dtype=torch.float64)
    a = torch.zeros((K + 1, 2), dtype=torch.float64)
    plan.set_state(5000, hist.cuda(), ring.cuda(), a.cuda(), a.clone().cuda())
    loc = plan.local_part().cpu().numpy()
    prm = Params(dt=p["dt"], boundary=FREE_SPACE)
    x = p["x"]
    h = hist.numpy()
    worst, scale = 0.0, 0.0
    for j in _sample_rows(M, 7):
        nb, Q = _near(x, j, prm)
        ref = 0.5 * sum(float(Q[:, m] @ h[m - 1, nb]) for m in range(1, prm.m_max))
        worst = max(worst, abs(loc[j] - ref))
        scale = max(scale, abs(ref))
    say(f"  sampled local part: max |gpu - oracle| = {worst:.2e}, max |oracle| = {scale:.2e}, "
        f"rho = {worst / scale:.2e}")
    assert worst / scale < 1e-12


def test_one_level_clumped_full_size(clumped):
    """One whole level at M = 1e6 (free space, K = 6250, a level on which the
    radiation-boundary projection is due) from a synthetic state: random
    density history, random spectra ring and mode state; the newest density
    level is nonzero at 2000 springs so that the oracle's direct spectrum
    stays cheap.  Checked against the oracle's pieces of a level:
    * the new ring slot (type-1 transform of the newest level) and the
      advanced alpha, alpha' (FIR, propagator, projection), every mode;
    * at 96 sampled springs, the residual of the per-step system,
      sigma_j + sum_l S_jl sigma_l - b_j, with b_j = -(g_j + local sum +
      beta_j u_H(x_j)) formed by the oracle (u_H from its own alpha) and
      sigma from the GPU: a property that holds at any size."""
    import torch
    from oracle.history import mode_step, pq_tables, rotation
    from oracle.rbc import rbc_project
    p, plan, info = clumped
    x, beta = p["x"], p["beta"]
    M = x.size
    prm = Params(dt=p["dt"], boundary=FREE_SPACE)
    mm, K, W = info["m_max"], info["K"], info["W"]
    assert (mm, K, W) == (prm.m_max, prm.K, prm.W)
    L = prm.rbc_period * (5000 // prm.rbc_period + 1)
    rng = np.random.default_rng(321)
    hist = rng.standard_normal((mm, M))
    hist[0] = 0.0
    hot = _sample_rows(M, 11)
    hot = np.unique(np.concatenate([hot, rng.choice(M, 1904, replace=False)]))
    hist[0, hot] = rng.standard_normal(hot.size)
    ring = rng.standard_normal((W, K + 1)) + 1j * rng.standard_normal((W, K + 1))
    alpha = rng.standard_normal(K + 1) + 1j * rng.standard_normal(K + 1)
    dalpha = rng.standard_normal(K + 1) + 1j * rng.standard_normal(K + 1)
    # the field and the densities are real: the k = 0 terms of a reachable state are real
    ring[:, 0] = ring[:, 0].real
    alpha[0], dalpha[0] = alpha[0].real, dalpha[0].real

    def dev(z):
        return torch.from_numpy(np.ascontiguousarray(np.stack([z.real, z.imag], -1))).cuda()

    plan.set_state(L, torch.from_numpy(hist).cuda(), dev(ring), dev(alpha), dev(dalpha))
    sig, _ = plan.march(1, receivers=False)
    st = plan.get_state()
    torch.cuda.synchronize()
    sig = sig.cpu().numpy()[0]
    ring_g = st["ring"].cpu().numpy()
    a_g = st["alpha"].cpu().numpy()
    da_g = st["dalpha"].cpu().numpy()
    a_g, da_g = a_g[:, 0] + 1j * a_g[:, 1], da_g[:, 0] + 1j * da_g[:, 1]
    s_new_g = ring_g[0, :, 0] + 1j * ring_g[0, :, 1]
    assert st["L"] == L + 1

    # oracle: spectrum, ring push, mode step, projection (the level is a multiple of its period)
    k = np.arange(K + 1)
    s_new = (np.exp(1j * np.outer(k, x[hot])) @ hist[0, hot]) / (2 * np.pi)
    ring_o = np.concatenate([s_new[None], ring[:-1]])
    P, Q = pq_tables(K, prm.dt, W, prm.delta, prm.b, prm.n_gl_pq)
    a_o, da_o = mode_step(alpha, dalpha, ring_o, P, Q, rotation(K, prm.dt), prm.dt)
    assert L % prm.rbc_period == 0
    a_o, da_o = rbc_project(a_o, da_o, prm)
    e_s, e_a, e_d = rho(s_new_g, s_new), rho(a_g, a_o), rho(da_g, da_o)
    say(f"  level {L}: rho(new spectrum) = {e_s:.2e}  rho(alpha) = {e_a:.2e}  rho(alpha') = {e_d:.2e}")
    if max(e_a, e_d) >= TOL:
        ka, kd = int(np.argmax(np.abs(a_g - a_o))), int(np.argmax(np.abs(da_g - da_o)))
        a_n, da_n = mode_step(alpha, dalpha, ring_o, P, Q, rotation(K, prm.dt), prm.dt)
        say(f"  worst modes: alpha k={ka} gpu {a_g[ka]} oracle {a_o[ka]}; alpha' k={kd} gpu {da_g[kd]} "
            f"oracle {da_o[kd]}; without projection rho = {rho(a_g, a_n):.2e} {rho(da_g, da_n):.2e}")
    assert e_s < TOL and e_a < TOL and e_d < TOL

    # sampled residuals of (I + S) sigma = b
    rows = _sample_rows(M, 7)
    wk = np.where(k == 0, 1.0, 2.0) * a_o
    t = L * prm.dt
    g = incident_driving(x[rows], beta[rows], p["packets"], False)(t)
    res, bmax = 0.0, 0.0
    for i, j in enumerate(rows):
        nb, Qw = _near(x, j, prm)
        hb = 0.5 * beta[j]
        local = hb * sum(float(Qw[:, m] @ hist[m - 1, nb]) for m in range(1, prm.m_max + 1))
        uH = float(np.cos(k * x[j]) @ wk.real + np.sin(k * x[j]) @ wk.imag)
        b = -(g[i] + local + beta[j] * uH)
        r = sig[j] + hb * float(Qw[:, 0] @ sig[nb]) - b
        res, bmax = max(res, abs(r)), max(bmax, abs(b))
    say(f"  sampled residual of the per-step system: max |r| = {res:.2e}, max |b| = {bmax:.2e}, "
        f"rho = {res / bmax:.2e}")
    assert res / bmax < TOL
