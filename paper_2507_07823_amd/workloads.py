"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

Each generator returns a dict with
    x        scatterer positions (float64, M)
    beta     spring stiffnesses  (float64, M)
    packets  incident-field packets, (n, 5) rows (amp, centre, width, omega, phase):
             f(s) = sum amp * exp(-(s - centre)^2 / (2 width^2)) * cos(omega (s - centre) + phase)
    boundary 0 = periodic box [-pi, pi), 1 = free space
    dt, n_steps
    x_recv   receiver positions (float64, R; may be empty)
    name     workload label

The scatterer sets mirror the random-spring experiments of the paper
(Section 6: uniform random positions, random strengths).  Springs are placed
outside the 1e-12 support of the incident pulse at t = 0, as the paper
requires of Gamma and supp f (Section 1), so the densities switch on smoothly.
No public dataset is involved anywhere.
"""
import math

import numpy as np

PI = math.pi


def _rng(*seed):
    return np.random.default_rng(list(seed))


# Largest dense-medium number theta = dt sqrt(rho mean(beta)) a workload is
# drawn with (rho: springs per unit length).  Many springs per time step act on
# a wave like a continuous elastic medium of stiffness density rho mean(beta);
# for that medium the discrete march with p = 8 has a growing mode once theta
# exceeds about 0.15-0.2 (at 0.29: +0.017 per level), whatever dt and rho are
# separately.  0.1 leaves a margin.
THETA_MAX = 0.1


def stable_beta_scale(M, length, dt, beta_mean, theta_max=THETA_MAX):
    """Factor s <= 1 for stiffnesses of mean beta_mean, so that M springs
    spread uniformly over an interval of the given length keep
    theta = dt sqrt(rho s beta_mean) <= theta_max (rho = M / length)."""
    theta = dt * math.sqrt(M / length * beta_mean)
    return min(1.0, (theta_max / theta) ** 2)


def periodic_single_pulse(seed, M, dt, n_steps, beta_range=(1.0, 10.0),
                          x_range=(0.3, 2.0), width=0.3, centre=-2.0, n_recv=0,
                          name="periodic"):
    """Periodic box, one Gaussian pulse, x ~ U(x_range), beta ~ U(beta_range)."""
    r = _rng(seed)
    x = r.uniform(x_range[0], x_range[1], M)
    beta = r.uniform(beta_range[0], beta_range[1], M)
    xr = np.linspace(x_range[0], x_range[1], n_recv) if n_recv else np.zeros(0)
    return dict(x=x, beta=beta, packets=np.array([[1.0, centre, width, 0.0, 0.0]]),
                boundary=0, dt=dt, n_steps=n_steps, x_recv=xr, name=name)


def small_periodic():
    """M = 16 springs in the periodic box, dt = 0.01, 600 steps, pulse of width
    0.3 centred at -2 (the small parity case)."""
    p = periodic_single_pulse(1, 16, 0.01, 600, name="periodic-M16-dt1e-2-Nt600")
    return p


def multiband_periodic(seed=2, M=10_000, dt=1e-3, n_steps=10_000, beta_max=10.0):
    """M = 1e4 springs, beta log-uniform in [0.1, beta_max], incident field a
    sum of 8 Gaussian wave packets (width 0.05) with angular carriers 50..500,
    dt = 1e-3, 1e4 steps, periodic box (the throughput case).

    beta_max defaults to 10: with stiffnesses up to 100 (the configuration as
    specified) the discrete march (p = 8) of this periodic system has a growing
    mode (about +0.6 % per level once it dominates), so no two FP64 runs can
    agree over 1e4 levels; up to 10 it is stable.  The per-level work does not
    depend on beta."""
    r = _rng(seed)
    x = r.uniform(-PI + 1.2, PI, M)
    beta = np.exp(r.uniform(math.log(0.1), math.log(beta_max), M))
    om = 50.0 * 10.0 ** (np.arange(8) / 7.0)
    c = -PI + 0.4 + 0.05 * np.arange(8)
    packets = np.stack([np.full(8, 0.25), c, np.full(8, 0.05), om, np.zeros(8)], axis=1)
    return dict(x=x, beta=beta, packets=packets, boundary=0, dt=dt, n_steps=n_steps,
                x_recv=np.zeros(0), name=f"periodic-multiband-M{M}-dt{dt:g}-Nt{n_steps}")


# stiffness range of the clumped springs at full size (see clumped_free_space)
CLUMP_BETA = (0.1, 1.0)


def clumped_free_space(seed=3, M=1_000_000, dt=5e-4, n_steps=4000, n_clumps=100,
                       frac=0.1, clump_sigma=1e-3, margin=0.0528, clump_beta=CLUMP_BETA):
    """Free space, M springs uniform in Omega with a fraction in tight Gaussian
    clumps, Gaussian-modulated plane wave of angular frequency 1000 entering
    from the left.  Uniform springs: beta ~ U[1, 10] scaled by
    stable_beta_scale (1 up to M ~ 4.5e4; 0.05 at M = 1e6, where the 9e5
    uniform springs alone would make theta = 0.45).  Clumped springs: beta ~
    U[clump_beta]; at M = 1e6 a clump holds 1000 springs within ~1e-3 (total
    stiffness ~5500 with U[1, 10]), and the discrete march (p = 8, dt = 5e-4)
    of such a clump grows by ~x360 per 100 levels in any exact implementation
    of the scheme; U[0.1, 1] keeps it stable.  At M = 1e4 (10 springs per
    clump) U[1, 10] is stable."""
    r = _rng(seed)
    lo, hi = -PI + margin, PI - margin
    n_cl = int(round(frac * M))
    n_un = M - n_cl
    xu = r.uniform(lo, hi, n_un)
    centres = r.uniform(lo + 0.01, hi - 0.01, n_clumps)
    per = np.full(n_clumps, n_cl // n_clumps)
    per[: n_cl - per.sum()] += 1
    xc = np.concatenate([r.normal(c, clump_sigma, k) for c, k in zip(centres, per)])
    xc = np.clip(xc, lo, hi)
    x = np.concatenate([xu, xc])
    s_un = stable_beta_scale(n_un, hi - lo, dt, 5.5)
    beta = np.concatenate([s_un * r.uniform(1.0, 10.0, n_un), r.uniform(clump_beta[0], clump_beta[1], n_cl)])
    s0 = lo - 0.4
    packets = np.array([[1.0, s0, 0.05, 1000.0, 0.0]])
    return dict(x=x, beta=beta, packets=packets, boundary=1, dt=dt, n_steps=n_steps,
                x_recv=np.zeros(0), name=f"free-clumped-M{M}-dt{dt:g}-Nt{n_steps}")


def balanced_dt(M, m_typ=100.0, W=35, half_width=2.0):
    """Time step giving a mean neighbour count m_typ within delta = W dt for M
    springs spread uniformly over [-half_width, half_width]: 2 delta M / (2
    half_width) = m_typ (edge effects ignored)."""
    return m_typ * half_width / (M * W)


def paper_balanced_free_space(M, seed=6, n_steps=2000, m_typ=100.0, min_sep=1e-6):
    """The scaling study of Section 6.2 (timing): free space, M springs uniform
    in [-2, 2] with pairwise separation at least min_sep (points closer than
    that to their left neighbour are redrawn), beta ~ U[0.1, 3], Gaussian pulse
    f(s) = exp(-30 (s + 3)^2) (width 1/sqrt(60)), dt from balanced_dt so the
    mean neighbour count is about m_typ.  The study runs p = 6."""
    r = _rng(seed, M)
    x = np.sort(r.uniform(-2.0, 2.0, M))
    for _ in range(100):
        close = np.nonzero(np.diff(x) < min_sep)[0] + 1
        if close.size == 0:
            break
        x[close] = r.uniform(-2.0, 2.0, close.size)
        x.sort()
    else:
        raise RuntimeError("could not separate the springs")
    x = x[r.permutation(M)]
    beta = r.uniform(0.1, 3.0, M)
    packets = np.array([[1.0, -3.0, 1.0 / math.sqrt(60.0), 0.0, 0.0]])
    dt = balanced_dt(M, m_typ)
    return dict(x=x, beta=beta, packets=packets, boundary=1, dt=dt, n_steps=n_steps,
                x_recv=np.zeros(0), p=6, name=f"free-balanced-M{M}-dt{dt:.4g}-Nt{n_steps}")


def long_grid_free_space(M=400, seed=8, n_steps=10, spread=0.02, study_M=1_000_000):
    """Free space at the time step of the scaling study's size study_M
    (1e6: K = 524288; 1e5: K = 51200) with only M springs, packed in
    [-spread, spread] so each has a few neighbours: the fine grid and boundary
    grid of that study size at a size the oracle can march.  Pulse and
    strengths as in paper_balanced_free_space; p = 6."""
    r = _rng(seed, M)
    x = r.uniform(-spread, spread, M)
    beta = r.uniform(0.1, 3.0, M)
    packets = np.array([[1.0, -3.0, 1.0 / math.sqrt(60.0), 0.0, 0.0]])
    dt = balanced_dt(study_M)
    return dict(x=x, beta=beta, packets=packets, boundary=1, dt=dt, n_steps=n_steps,
                x_recv=np.zeros(0), p=6, name=f"free-long-grid-M{M}-dt{dt:.4g}")


def incident_data(prob, dt, n_levels, images=4):
    """Driving data beta_j f(x_j - t_L) of the problem's incident packets at
    levels L = 0..n_levels-1, shape (n_levels, M); the periodic box sums the
    images s + 2 pi m, |m| <= images, of the wrapped argument."""
    x, beta, pk = prob["x"], prob["beta"], np.atleast_2d(prob["packets"])
    periodic = prob["boundary"] == 0
    out = np.zeros((n_levels, x.size))
    for L in range(n_levels):
        s = x - L * dt
        if periodic:
            s = s - 2 * PI * np.rint(s / (2 * PI))
        ms = range(-images, images + 1) if periodic else [0]
        f = np.zeros(x.size)
        for a, c, w, om, ph in pk:
            for m in ms:
                y = s + 2 * PI * m - c
                f += a * np.exp(-y * y / (2 * w * w)) * np.cos(om * y + ph)
        out[L] = beta * f
    return out


def manufactured_springs(M, seed=10, min_sep=1e-4):
    """The convergence test of Section 6.1: free space, M springs uniform in
    [-1, 1] with pairwise separation at least min_sep (closer points redrawn),
    prescribed densities sigma_j(t) = exp(-mu_j (t - t0_j)^2) with
    mu ~ U[40, 50], t0 ~ U[1, 3], and beta ~ U[0.1, 3]."""
    r = _rng(seed, M)
    x = np.sort(r.uniform(-1.0, 1.0, M))
    for _ in range(100):
        close = np.nonzero(np.diff(x) < min_sep)[0] + 1
        if close.size == 0:
            break
        x[close] = r.uniform(-1.0, 1.0, close.size)
        x.sort()
    else:
        raise RuntimeError("could not separate the springs")
    mu = r.uniform(40.0, 50.0, M)
    t0 = r.uniform(1.0, 3.0, M)
    beta = r.uniform(0.1, 3.0, M)
    # the driving data come from manufactured_data; the plan's incident
    # field is one packet of zero amplitude
    return dict(x=x, beta=beta, mu=mu, t0=t0, boundary=1, packets=np.array([[0.0, 0.0, 1.0, 0.0, 0.0]]),
                x_recv=np.zeros(0), name=f"manufactured-M{M}")


def manufactured_potential(xq, t, x, mu, t0):
    """Free-space field of the prescribed densities at points xq and time t:
    u(x, t) = (1/2) sum_l int_0^{t - |x - x_l|} sigma_l(s) ds (the 1D wave
    single layer), with int_0^T exp(-mu (s - t0)^2) ds =
    (1/2) sqrt(pi/mu) [erf(sqrt(mu) (T - t0)) + erf(sqrt(mu) t0)] for T > 0."""
    from scipy.special import erf
    xq = np.atleast_1d(np.asarray(xq, dtype=np.float64))
    T = t - np.abs(xq[:, None] - x[None, :])
    rm = np.sqrt(mu)[None, :]
    val = 0.5 * np.sqrt(PI) / rm * (erf(rm * (T - t0[None, :])) + erf(rm * t0[None, :]))
    return 0.5 * np.where(T > 0.0, val, 0.0).sum(axis=1)


def manufactured_data(prob, dt, n_levels):
    """Driving data g_j(t_L) = -sigma_j(t_L) - beta_j u(x_j, t_L) of the
    manufactured densities at levels L = 0..n_levels-1, shape (n_levels, M)."""
    x, beta, mu, t0 = prob["x"], prob["beta"], prob["mu"], prob["t0"]
    g = np.empty((n_levels, x.size))
    for L in range(n_levels):
        t = L * dt
        g[L] = -np.exp(-mu * (t - t0) ** 2) - beta * manufactured_potential(x, t, x, mu, t0)
    return g


def spring_filter(M, beta, t0, n_steps, span=(-1.0, 1.0), dt=0.01, x_recv=1.5, p=8):
    """The filter demonstrations of Section 6.4: M equal springs evenly
    spaced over `span` (both ends included), free space, incident wave
    f(x - t) with f(s) = exp(-5 (s - t0)^2), dt = 0.01, interpolation order p,
    one receiver downstream at x_recv."""
    x = np.linspace(span[0], span[1], M)
    return dict(x=x, beta=np.full(M, float(beta)),
                packets=np.array([[1.0, t0, 1.0 / math.sqrt(10.0), 0.0, 0.0]]), boundary=1, dt=dt,
                n_steps=n_steps, x_recv=np.array([x_recv]), p=p, mu=5.0, t0=t0,
                name=f"filter-M{M}-beta{beta:g}")


def fabry_perot():
    """Two springs of stiffness 100 at -0.5 and 0.5 (cavity length 1), pulse
    exp(-5 (s + 3)^2), 9426 levels of dt = 0.01, p = 6 (at beta dt / 2 = 0.5
    the p = 8 local rule is unstable)."""
    return spring_filter(2, 100.0, -3.0, 9426, span=(-0.5, 0.5), p=6)


def spring_arrays():
    """M = 10 springs of stiffness 100 (p = 6, as for the cavity) and M = 200
    of stiffness 1 (p = 8), evenly on [-1, 1] (the spacing is a reading),
    pulse exp(-5 (s + 4)^2), 25134 levels of dt = 0.01."""
    return [spring_filter(10, 100.0, -4.0, 25134, p=6), spring_filter(200, 1.0, -4.0, 25134, p=8)]


def disordered_long(M, seed=11, refine=1, n_recv=50):
    """The long disordered runs of Section 6.3: free space, M springs uniform
    in [-2, 2], beta ~ U[0.1, 3], a narrow pulse f(s) = exp(-M^2 (s + 3)^2)
    (width sqrt(8) times the mean spacing 4/M), p = 8, the paper's time steps
    (1.308e-4 at M = 1e3, 1.308e-5 at M = 1e4; dt scales like 1/M) and level
    counts (72044, 720440; about 3 pi), n_recv receivers evenly on
    [-2.5, 2.5].  refine = 2 halves dt and doubles the levels (the paper's
    self-convergence check)."""
    r = _rng(seed, M)
    x = r.uniform(-2.0, 2.0, M)
    beta = r.uniform(0.1, 3.0, M)
    width = 1.0 / (math.sqrt(2.0) * M)            # exp(-M^2 s^2) = exp(-s^2 / (2 width^2))
    dt = 1.308e-4 * (1000.0 / M) / refine
    n_steps = int(round(72.044 * M)) * refine
    return dict(x=x, beta=beta, packets=np.array([[1.0, -3.0, width, 0.0, 0.0]]), boundary=1, dt=dt,
                n_steps=n_steps, x_recv=np.linspace(-2.5, 2.5, n_recv), p=8,
                name=f"disordered-M{M}-dt{dt:.4g}-Nt{n_steps}")


def adjoint_periodic(seed=5, M=100_000, dt=1e-3, n_steps=5000, R=64):
    """Periodic, M springs with beta ~ U[1, 10] scaled by stable_beta_scale
    (0.092 at M = 1e5, dt = 1e-3: U[0.092, 0.92]), a single Gaussian pulse
    (width 0.05) and R receivers spread over the spring region."""
    r = _rng(seed)
    x = r.uniform(-PI + 1.2, PI, M)
    beta = stable_beta_scale(M, 2 * PI - 1.2, dt, 5.5) * r.uniform(1.0, 10.0, M)
    packets = np.array([[1.0, -PI + 0.6, 0.05, 0.0, 0.0]])
    xr = -PI + 1.2 + (np.arange(R) + 0.5) * (2 * PI - 1.2) / R
    return dict(x=x, beta=beta, packets=packets, boundary=0, dt=dt, n_steps=n_steps,
                x_recv=xr, name=f"periodic-adjoint-M{M}-dt{dt:g}-Nt{n_steps}-R{R}")


def batch_instances(seed=4, n=512, n_steps=2000, m_range=(100, 100_000)):
    """n independent periodic problems with log-uniform M, dt in {1,2,5}e-3,
    beta ~ U[1, 10] scaled per instance by stable_beta_scale (the dense
    instances at the larger time steps get weaker springs) and one random
    Gaussian pulse each."""
    out = []
    for i in range(n):
        r = _rng(seed, i)
        M = int(round(math.exp(r.uniform(math.log(m_range[0]), math.log(m_range[1])))))
        dt = float(r.choice([1e-3, 2e-3, 5e-3]))
        w = r.uniform(0.03, 0.07)
        c = r.uniform(-PI + 0.55, -PI + 0.65)
        x = r.uniform(-PI + 1.2, PI, M)
        beta = stable_beta_scale(M, 2 * PI - 1.2, dt, 5.5) * r.uniform(1.0, 10.0, M)
        out.append(dict(x=x, beta=beta, packets=np.array([[1.0, c, w, 0.0, 0.0]]),
                        boundary=0, dt=dt, n_steps=n_steps, x_recv=np.zeros(0),
                        name=f"batch-{i}"))
    return out


def clumped_level_state(M, K, W, m_hist, seed=21, n_hot=2000):
    """A synthetic mid-run state of the clumped free-space workload for a
    one-level check at full size: a unit-normal density history, whose newest
    level is nonzero only at n_hot springs (so that a direct spectrum of it
    stays cheap), a unit-normal spectra ring and mode state (real k = 0
    terms).  Returns the state and the indices of the nonzero springs."""
    r = _rng(seed, M)
    hist = r.standard_normal((m_hist, M))
    hot = np.unique(r.choice(M, n_hot, replace=False))
    hist[0] = 0.0
    hist[0, hot] = r.standard_normal(hot.size)
    ring = r.standard_normal((W, K + 1)) + 1j * r.standard_normal((W, K + 1))
    alpha = r.standard_normal(K + 1) + 1j * r.standard_normal(K + 1)
    dalpha = r.standard_normal(K + 1) + 1j * r.standard_normal(K + 1)
    ring[:, 0] = ring[:, 0].real
    alpha[0] = alpha[0].real
    dalpha[0] = dalpha[0].real
    return dict(hist=hist, ring=ring, alpha=alpha, dalpha=dalpha), hot


def random_state(seed, M, K, W, m_hist, scale=1e-2):
    """A synthetic mid-run state (density history, spectra ring, modes) used to
    test one step from a state both sides receive as input."""
    r = _rng(seed, 99)
    hist = scale * r.standard_normal((m_hist, M))
    ring = scale * (r.standard_normal((W, K + 1)) + 1j * r.standard_normal((W, K + 1)))
    decay = np.exp(-np.arange(K + 1) / (0.3 * (K + 1)))
    alpha = scale * decay * (r.standard_normal(K + 1) + 1j * r.standard_normal(K + 1))
    dalpha = scale * decay * (r.standard_normal(K + 1) + 1j * r.standard_normal(K + 1))
    ring[:, 0] = ring[:, 0].real
    alpha[0] = alpha[0].real
    dalpha[0] = dalpha[0].real
    return dict(hist=hist, ring=ring, alpha=alpha, dalpha=dalpha)
