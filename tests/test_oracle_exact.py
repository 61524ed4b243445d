"""Pins of the whole oracle march against results fixed independently of it:
closed forms (M = 1, manufactured densities) and a brute-force solve of the
Volterra system written as delay-differential equations."""
import math

import numpy as np
import pytest

from oracle.exact import (manufactured_driving, manufactured_field, gaussian_density,
                          single_spring)
from oracle.march import Oracle, incident_driving
from oracle.params import FREE_SPACE, PERIODIC, Params
from oracle.volterra import solve_delay_system

PULSE = np.array([[1.0, -2.0, 0.3, 0.0, 0.0]])


@pytest.mark.parametrize("beta", [1.0, 5.0, 10.0])
def test_single_spring_closed_form(beta):
    """M = 1: -sigma - (beta/2) int_0^t sigma = g (Section 5.1), closed form in erfc.
    Fixes the sign conventions, the history factor beta_j u_H and the solve."""
    x = np.array([1.0])
    b = np.array([beta])
    prm = Params(dt=0.01)
    o = Oracle(x, b, prm, incident_driving(x, b, PULSE, True))
    sig, _ = o.run(601)
    t = np.arange(601) * prm.dt
    ref, _ = single_spring(t, 1.0, beta, 1.0, -2.0, 0.3)
    assert np.max(np.abs(sig[:, 0] - ref)) < 1e-10 * np.max(np.abs(ref))


def test_field_at_receiver_single_spring():
    """u(x, t) = 1/2 I(t - |x - x_1|) for one spring (eq. (singleLayerSol))."""
    x = np.array([1.0])
    b = np.array([4.0])
    xr = np.array([1.0, 1.2, 0.9])
    prm = Params(dt=0.01)
    o = Oracle(x, b, prm, incident_driving(x, b, PULSE, True), x_recv=xr)
    _, u = o.run(501)
    for n in range(0, 501, 25):
        t = n * prm.dt
        ref = np.array([0.5 * single_spring(np.array([t - abs(r - 1.0)]), 1.0, 4.0, 1.0, -2.0, 0.3)[1][0]
                        if t > abs(r - 1.0) else 0.0 for r in xr])
        assert np.max(np.abs(u[n] - ref)) < 1e-10


@pytest.mark.parametrize("periodic", [True, False])
def test_split_invariant_prescribed_densities(periodic):
    """u_L + u_H equals the potential of prescribed Gaussian densities (eqs.
    (localSol), (historySol) sum to (SLPp)/(singleLayerSol)); pins the local
    weights, the history modes, the image sum and (free space) the RBC."""
    rng = np.random.default_rng(7)
    M = 6
    xs = rng.uniform(-0.8, 0.8, M)
    mu = rng.uniform(40, 50, M)
    t0 = rng.uniform(1.0, 2.0, M)
    xr = np.array([-0.5, 0.0, 0.3, xs[0], xs[1] + 0.004])
    prm = Params(dt=0.01, boundary=PERIODIC if periodic else FREE_SPACE)
    o = Oracle(xs, np.ones(M), prm, lambda t: np.zeros(M), x_recv=xr)
    worst = 0.0
    n_levels = 800
    for L in range(n_levels):
        t = L * prm.dt
        u = o.step_prescribed(gaussian_density(t, mu, t0))
        if L % 20 == 0:
            worst = max(worst, np.max(np.abs(u - manufactured_field(xr, t, xs, mu, t0, periodic))))
    assert worst < 1e-10


def test_manufactured_march_converges_at_order_p_plus_1():
    """Manufactured solution (Section 6.1): data g_j = -sigma_j - beta_j u_ex
    from prescribed densities; the march recovers them with error O(dt^{p+1})."""
    rng = np.random.default_rng(3)
    M = 5
    xs = rng.uniform(-1, 1, M)
    mu = rng.uniform(40, 50, M)
    t0 = rng.uniform(1, 3, M)
    beta = rng.uniform(0.1, 3, M)
    errs = []
    for dt in (0.04, 0.02):
        prm = Params(dt=dt, p=4)
        o = Oracle(xs, beta, prm, manufactured_driving(xs, beta, mu, t0, True))
        n = int(round(4.0 / dt)) + 1
        sig, _ = o.run(n)
        t = np.arange(n) * dt
        ex = np.array([gaussian_density(tt, mu, t0) for tt in t])
        errs.append(np.max(np.abs(sig - ex)))
    assert errs[0] / errs[1] > 2 ** 4, errs


def test_manufactured_march_p8_accuracy():
    rng = np.random.default_rng(4)
    M = 5
    xs = rng.uniform(-1, 1, M)
    mu = rng.uniform(40, 50, M)
    t0 = rng.uniform(1, 3, M)
    beta = rng.uniform(0.1, 3, M)
    prm = Params(dt=0.01)
    o = Oracle(xs, beta, prm, manufactured_driving(xs, beta, mu, t0, True))
    sig, _ = o.run(401)
    ex = np.array([gaussian_density(L * prm.dt, mu, t0) for L in range(401)])
    # the error floor is ~M eps (Section 6.1), eps = 1e-12
    assert np.max(np.abs(sig - ex)) < 5e-10


def test_delay_differential_brute_force_periodic():
    """Nearby (d < dt), intermediate and history-only pairs, periodic images:
    the discrete march equals the DDE solution to the scheme's accuracy."""
    x = np.array([0.5, 0.5063, 0.62, 1.9])
    beta = np.array([3.0, 7.0, 5.0, 9.0])
    o = Oracle(x, beta, Params(dt=0.01), incident_driving(x, beta, PULSE, True))
    sig, _ = o.run(401)
    _, ref = solve_delay_system(x, beta, PULSE, True, 4.0, 40)
    assert np.max(np.abs(sig[::10] - ref)) < 1e-9 * np.max(np.abs(ref))


def test_delay_differential_brute_force_free_space_with_rbc():
    """Free space: waves leave the box through the RBC projection; without it
    they would wrap around and hit the springs again after t ~ 8.8."""
    x = np.array([0.5, 0.6, 1.0])
    beta = np.array([3.0, 7.0, 5.0])
    prm = Params(dt=0.01, boundary=FREE_SPACE)
    o = Oracle(x, beta, prm, incident_driving(x, beta, PULSE, False))
    sig, _ = o.run(1101)
    _, ref = solve_delay_system(x, beta, PULSE, False, 11.0, 110)
    assert np.max(np.abs(sig[::10] - ref)) < 1e-9 * np.max(np.abs(ref))


def test_frequency_domain_field_of_springs():
    """The frequency-domain solution for point springs (spring_array_field):
    M = 1 against the closed form in erfc (Section 5.1), M = 3 against the
    oracle march's total field at a receiver right of the springs (free
    space, waves leaving through the RBC)."""
    from oracle.exact import spring_array_field, spring_array_transmission
    # one spring: |T|^2 = 4 w^2 / (4 w^2 + beta^2), the textbook point scatterer
    w = np.array([0.5, 2.0, 7.0])
    T = spring_array_transmission(w, [0.3], [4.0])
    assert np.max(np.abs(np.abs(T) ** 2 - 4 * w * w / (4 * w * w + 16.0))) < 1e-15
    mu, t0 = 5.0, -3.0
    # M = 1
    x1, b1, xr = 0.3, 4.0, 1.0
    t = np.linspace(0.0, 12.0, 25)
    u = spring_array_field(xr, t, [x1], [b1], mu, t0, dw=2e-3)
    tau = t - (xr - x1)
    _, I = single_spring(np.maximum(tau, 0.0), x1, b1, 1.0, t0, 1.0 / math.sqrt(2.0 * mu))
    ref = np.exp(-mu * (xr - t - t0) ** 2) + 0.5 * np.where(tau > 0.0, I, 0.0)
    assert np.max(np.abs(u - ref)) < 1e-13
    # M = 3, the march (p = 8, dt = 0.01) to 11 time units
    x = np.array([0.5, 0.6, 1.0])
    beta = np.array([3.0, 7.0, 5.0])
    xr = 1.4
    pulse = np.array([[1.0, t0, 1.0 / math.sqrt(2.0 * mu), 0.0, 0.0]])
    prm = Params(dt=0.01, boundary=FREE_SPACE)
    o = Oracle(x, beta, prm, incident_driving(x, beta, pulse, False), x_recv=np.array([xr]))
    _, ur = o.run(1101)
    lv = np.arange(0, 1101, 20)
    tt = lv * prm.dt
    tot = ur[lv, 0] + np.exp(-mu * (xr - tt - t0) ** 2)
    ex = spring_array_field(xr, tt, x, beta, mu, t0, dw=1e-3)
    assert np.max(np.abs(tot - ex)) < 1e-9 * np.max(np.abs(ex))


def test_chain_transmission_matches_the_dense_solve():
    """Transfer matrices (spring_chain_transmission) against the dense
    frequency-domain solve (spring_array_transmission) for the ten-spring
    array of stiffness 100 and unsorted random springs, and the one-spring
    closed form T = 2iw / (2iw - beta)."""
    from oracle.exact import spring_array_transmission, spring_chain_transmission
    w = np.linspace(0.05, 25.0, 997)
    T1 = spring_chain_transmission(w, [0.7], [3.0])
    assert np.max(np.abs(T1 - 2j * w / (2j * w - 3.0))) < 1e-14
    cases = [(np.linspace(-1.0, 1.0, 10), np.full(10, 100.0))]
    rng = np.random.default_rng(3)
    for M in (2, 7, 15):
        cases.append((rng.uniform(-1.0, 1.0, M), rng.uniform(0.1, 20.0, M)))
    for x, beta in cases:
        Td = spring_array_transmission(w, x, beta)
        Tc = spring_chain_transmission(w, x, beta)
        assert np.max(np.abs(Tc - Td)) < 1e-11 * max(1.0, np.max(np.abs(Td))), x.size
