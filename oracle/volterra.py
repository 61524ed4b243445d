"""Brute-force reference: the Volterra system as a delay-differential system.

Differentiating eq. (IEfree) (free space) or eq. (periodicIE) (periodic box)
in t gives, for t > 0,

    sigma_j'(t) = -g_j'(t) - (beta_j/2) sum_l sum_images sigma_l(t - d_jlm),

with d_jlm = |x_j - x_l - 2 pi m| (m = 0 only in free space), sigma_l = 0 for
negative arguments, and sigma_j(0) = -g_j(0) (the equation at t = 0, where
u = 0).  This uses neither the window, nor Fourier modes, nor the local
quadrature, so it pins the whole discrete march independently (up to the
scheme's O(dt^{p+1}) + O(eps) error).

Solved by the method of steps: time is cut into segments no longer than the
smallest positive delay, so every delayed argument falls in an earlier
segment whose dense output (DOP853, 7th order) is kept.  Only small M is
practical.
"""
import math

import numpy as np
from scipy.integrate import solve_ivp


def incident_profile_and_slope(s, packets, periodic):
    """f(s) and f'(s) for the packet sum used by the incident field."""
    s = np.asarray(s, dtype=np.float64)
    if periodic:
        s = s - 2.0 * math.pi * np.round(s / (2.0 * math.pi))
        shifts = [2.0 * math.pi * m for m in range(-4, 5)]
    else:
        shifts = [0.0]
    f = np.zeros_like(s)
    df = np.zeros_like(s)
    for a, c, w, om, ph in np.atleast_2d(packets):
        for sh in shifts:
            y = s + sh - c
            env = a * np.exp(-y * y / (2.0 * w * w))
            f += env * np.cos(om * y + ph)
            df += env * (-(y / (w * w)) * np.cos(om * y + ph) - om * np.sin(om * y + ph))
    return f, df


def solve_delay_system(x, beta, packets, periodic, T, n_out, rtol=1e-13, atol=1e-15):
    """Densities sigma_j(t) at t = 0, T/n_out, ..., T for the incident pulse.

    g_j(t) = beta_j f(x_j - t), so g_j'(t) = -beta_j f'(x_j - t).
    """
    x = np.asarray(x, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    M = x.size
    # delays (j, l, d) with d < T
    delays = []
    for j in range(M):
        for l in range(M):
            ms = range(-3, 4) if periodic else [0]
            for m in ms:
                d = abs(x[j] - x[l] - 2.0 * math.pi * m)
                if d < T:
                    delays.append((j, l, d))
    pos = [d for (_, _, d) in delays if d > 0.0]
    seg = min(pos) if pos else T
    seg = min(seg, T)
    self_terms = [(j, l) for (j, l, d) in delays if d == 0.0]
    lag_terms = [(j, l, d) for (j, l, d) in delays if d > 0.0]
    pieces = []                        # (t0, t1, dense_output)

    def past(l, tau):
        if tau <= 0.0:
            return 0.0
        for (a, b, sol) in pieces:
            if a <= tau <= b:
                return float(sol(tau)[l])
        if pieces and tau <= pieces[-1][1] + 1e-12:      # rounding at a segment end
            return float(pieces[-1][2](pieces[-1][1])[l])
        raise RuntimeError("delayed argument outside the computed history")

    def rhs(t, y):
        _, df = incident_profile_and_slope(x - t, packets, periodic)
        dy = beta * df                 # -g' = beta f'(x - t)
        for (j, l) in self_terms:
            dy[j] -= 0.5 * beta[j] * y[l]
        for (j, l, d) in lag_terms:
            dy[j] -= 0.5 * beta[j] * past(l, t - d)
        return dy

    f0, _ = incident_profile_and_slope(x, packets, periodic)
    y = -beta * f0                     # sigma(0) = -g(0)
    t = 0.0
    while t < T - 1e-15:
        t1 = min(t + seg, T)
        sol = solve_ivp(rhs, (t, t1), y, method="DOP853", rtol=rtol, atol=atol,
                        dense_output=True)
        if not sol.success:
            raise RuntimeError(sol.message)
        pieces.append((t, t1, sol.sol))
        y = sol.y[:, -1]
        t = t1
    ts = np.linspace(0.0, T, n_out + 1)
    out = np.array([[past(l, tt) for l in range(M)] for tt in ts])
    out[0] = -beta * f0
    return ts, out
