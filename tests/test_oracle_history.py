"""Pins of the oracle's history part (Section 3: eqs. (alphak), (pkqkcomp),
(hkcompdisc), Lemma (alphakEvolutionFormulas))."""
import math

import numpy as np
from scipy.integrate import quad

from oracle.history import influence_kernel, mode_step, pq_tables, rotation
from oracle.params import Params
from oracle.window import phi

PRM = Params(dt=0.01)


def test_pq_vanish_at_support_ends():
    # p_k(t - s), q_k(t - s) vanish at t - s = -dt and t - s = delta (Section 3)
    K, W, dt = 40, PRM.W, PRM.dt
    z, w = np.polynomial.legendre.leggauss(32)
    mu = 0.5 * dt * (z + 1)
    for r in (-dt, PRM.delta):
        for k in (0, 3, 40):
            psi = influence_kernel(k, r + mu, PRM.delta, PRM.b)
            assert np.max(np.abs(psi)) < 1e-9 * np.abs(influence_kernel(k, np.array([PRM.delta / 2]), PRM.delta, PRM.b)).max()


def test_pq_node_count_converged():
    P1, Q1 = pq_tables(60, PRM.dt, PRM.W, PRM.delta, PRM.b, 32)
    P2, Q2 = pq_tables(60, PRM.dt, PRM.W, PRM.delta, PRM.b, 64)
    assert np.max(np.abs(P1 - P2)) < 1e-15 * np.max(np.abs(P2)) * 10
    assert np.max(np.abs(Q1 - Q2)) < 1e-15 * np.max(np.abs(Q2)) * 10


def test_pq_against_direct_quadrature():
    P, Q = pq_tables(20, PRM.dt, PRM.W, PRM.delta, PRM.b, 32)
    dt = PRM.dt
    for k, m in [(0, 0), (0, 17), (7, 3), (20, 30)]:
        sk = (lambda u: (math.sin(k * u) / k) if k else u)
        p = quad(lambda mu: sk(dt - mu) * influence_kernel(k, np.array([m * dt + mu]), PRM.delta, PRM.b)[0], 0, dt, epsabs=1e-18)[0]
        q = quad(lambda mu: math.cos(k * (dt - mu)) * influence_kernel(k, np.array([m * dt + mu]), PRM.delta, PRM.b)[0], 0, dt, epsabs=1e-18)[0]
        assert abs(P[m, k] - p) < 1e-14 * max(abs(p), 1e-3)
        assert abs(Q[m, k] - q) < 1e-14 * max(abs(q), 1e-1)


def test_march_reproduces_windowed_coefficients():
    """alpha_k from the FIR + exact propagator equals eq. (alphak) evaluated by
    adaptive quadrature, for a smooth-start density spectrum S_k(tau)."""
    K, W, dt = PRM.K, PRM.W, PRM.dt
    P, Q = pq_tables(K, dt, W, PRM.delta, PRM.b, 32)
    rot = rotation(K, dt)
    x1 = 1.0
    sig = lambda t: math.exp(-30 * (t - 2.0) ** 2)
    k = np.arange(K + 1)
    ring = np.zeros((W, K + 1), complex)
    a = np.zeros(K + 1, complex)
    da = np.zeros(K + 1, complex)
    n_steps = 230
    for L in range(1, n_steps + 1):
        S = sig((L - 1) * dt) * np.exp(1j * k * x1) / (2 * math.pi)
        ring = np.roll(ring, 1, 0)
        ring[0] = S
        a, da = mode_step(a, da, ring, P, Q, rot, dt)
    t = n_steps * dt
    scale = 0.5 / math.sqrt(30 / math.pi)   # size of the accumulated integral
    for kk in [0, 1, 5, 20, 100]:
        f = lambda tau: ((math.sin(kk * (t - tau)) / kk) if kk else (t - tau)) * phi(np.array([t - tau]), PRM.delta, PRM.b)[0] * sig(tau)
        re = quad(lambda tau: f(tau) * math.cos(kk * x1), 0, t, limit=400, epsabs=1e-16)[0] / (2 * math.pi)
        im = quad(lambda tau: f(tau) * math.sin(kk * x1), 0, t, limit=400, epsabs=1e-16)[0] / (2 * math.pi)
        assert abs(a[kk] - complex(re, im)) < 1e-10 * scale, (kk, a[kk], re, im)


def test_rotation_is_exact_free_propagation():
    # no sources: the propagator moves a periodised right-going pulse exactly
    from oracle.exact import free_wave_field, free_wave_modes
    K, dt = 200, 0.01
    a, da = free_wave_modes(K, -1.0, 0.2)
    c, s, r = rotation(K, dt)
    for _ in range(150):
        a, da = c * a + s * da, r * a + c * da
    x = np.linspace(-math.pi, math.pi, 64, endpoint=False)
    k = np.arange(K + 1)
    wk = np.where(k == 0, 1.0, 2.0)
    u = np.real(np.exp(-1j * np.outer(x, k)) @ (wk * a))
    assert np.max(np.abs(u - free_wave_field(x, 150 * dt, -1.0, 0.2))) < 1e-13


def test_rbc_fft_form_equals_direct_sums():
    # the boundary projection's two sums taken by an FFT of length 2K agree
    # with the same sums evaluated term by term (Section 4.4)
    from oracle.params import FREE_SPACE
    from oracle.rbc import rbc_project, rbc_project_fft
    rng = np.random.default_rng(3)
    for dt in (0.01, 3e-3):
        prm = Params(dt=dt, boundary=FREE_SPACE)
        K = prm.K
        a = rng.standard_normal(K + 1) + 1j * rng.standard_normal(K + 1)
        d = rng.standard_normal(K + 1) + 1j * rng.standard_normal(K + 1)
        a[0] = a[0].real
        d[0] = d[0].real
        u1, v1 = rbc_project(a, d, prm)
        u2, v2 = rbc_project_fft(a, d, prm)
        assert u1[K] == 0 and u2[K] == 0 and v2[K] == 0
        # the direct sums round their phases k x_i (up to K pi) to ~K pi eps
        tol = 8 * K * math.pi * np.finfo(float).eps
        assert np.max(np.abs(u1 - u2)) < tol * np.max(np.abs(u1))
        assert np.max(np.abs(v1 - v2)) < tol * np.max(np.abs(v1))


def test_free_space_pulse_leaves_the_box():
    """Section 4.4: a free pulse represented by its modes travels through the
    box unchanged (exact propagator), and the outgoing-windowing projection
    applied every P levels lets it leave: once it has crossed |x| = pi the
    whole box holds a residual at the window tolerance eps = 1e-12, not the
    periodic image that would re-enter from the other side.  Both directions
    (the left end is the mirror of the right-end formula)."""
    from oracle.params import FREE_SPACE
    from oracle.rbc import rbc_project
    prm = Params(dt=0.01, boundary=FREE_SPACE)
    K = prm.K
    k = np.arange(K + 1)
    x = np.linspace(-math.pi, math.pi, 1501)
    E = np.exp(-1j * np.outer(x, k))
    wk = np.where(k == 0, 1.0, 2.0)
    zero_ring = np.zeros((prm.W, K + 1), np.complex128)
    zero_tab = np.zeros((prm.W, K + 1))
    rot = rotation(K, prm.dt)
    w = 0.08
    inner = np.abs(x) < math.pi - 2 * prm.delta_s
    for direction, c in ((1.0, 1.5), (-1.0, -1.5)):
        # u(x, t) = G(x - direction t), G a Gaussian of width w centred at c:
        # alpha_k = (1/2pi) int G e^{ikx}, alpha'_k = direction i k alpha_k
        a = w / math.sqrt(2 * math.pi) * np.exp(-k * k * w * w / 2) * np.exp(1j * k * c)
        da = direction * 1j * k * a
        gone = None
        for L in range(1, 400):
            a, da = mode_step(a, da, zero_ring, zero_tab, zero_tab, rot, prm.dt)
            if L % prm.rbc_period == 0:
                a, da = rbc_project(a, da, prm)
            t = L * prm.dt
            u = (E @ (wk * a)).real
            exact = np.exp(-(x - c - direction * t) ** 2 / (2 * w * w))
            assert np.max(np.abs(u - exact)[inner]) < 1e-12, (direction, L)
            if abs(c) + t > math.pi + 12 * w and gone is None:
                gone = L
            if gone is not None and L >= gone + prm.rbc_period:
                assert np.max(np.abs(u)) < prm.eps, (direction, L, np.max(np.abs(u)))
        assert gone is not None
