"""Closed-form solutions used to pin the oracle (Tier B).

* single_spring: M = 1.  The Volterra equation (IEfree) with one spring is
  -sigma - (beta/2) int_0^t sigma = g (Section 5.1), i.e. the ODE
  I' = -(beta/2) I - g with I = int_0^t sigma, I(0) = 0.  For a Gaussian
  incident pulse f(s) = A exp(-(s-c)^2/(2w^2)) the driving g(t) = beta f(x_1 - t)
  is a Gaussian in t and I has a closed form in erfc (below).  The periodic
  box gives the same solution while t < 2 pi (no image has arrived).
* manufactured: prescribed densities sigma_j(t) = exp(-mu_j (t - t0_j)^2)
  (Section 6.1) generate u_ex through eq. (singleLayerSol) (free space) or
  eq. (SLPp) (periodic, summing the images), and the data
  g_j = -sigma_j - beta_j u_ex(x_j, t).
* free_wave: a periodised right-going Gaussian and its Fourier coefficients,
  u(x, t) = G(x - t) (the homogeneous propagator of Section 3).
"""
import math

import numpy as np
from scipy.special import erfc, erfcx

SQRT_PI = math.sqrt(math.pi)


def single_spring(t, x1, beta, amp, centre, width):
    """sigma(t) and I(t) = int_0^t sigma for one spring (closed form).

    g(t) = beta*amp*exp(-(t - tau0)^2/(2 w^2)) with tau0 = x1 - centre.
    I(t) = -beta*amp * int_0^t e^{-a(t-s)} e^{-(s-tau0)^2/(2w^2)} ds,  a = beta/2,
         = -beta*amp * w sqrt(pi/2) * e^{E} [erfc(-A) - erfc(-B)],
    E = -a (t - tau0) + a^2 w^2 / 2,  A = (t - tau0 - a w^2)/(sqrt2 w),
    B = (-tau0 - a w^2)/(sqrt2 w); written with erfcx to avoid overflow.
    """
    t = np.asarray(t, dtype=np.float64)
    a = 0.5 * beta
    tau0 = x1 - centre
    w = width
    E = -a * (t - tau0) + 0.5 * a * a * w * w
    A = (t - tau0 - a * w * w) / (math.sqrt(2.0) * w)
    B = (-tau0 - a * w * w) / (math.sqrt(2.0) * w)
    bracket = erfcx(-A) * np.exp(E - A * A) - erfcx(-B) * np.exp(E - B * B)
    I = -beta * amp * w * math.sqrt(math.pi / 2.0) * bracket
    g = beta * amp * np.exp(-(t - tau0) ** 2 / (2.0 * w * w))
    sigma = -g - a * I
    return sigma, I


def gaussian_density(t, mu, t0):
    return np.exp(-mu * (t - t0) ** 2)


def gaussian_density_integral(T, mu, t0):
    """int_0^T exp(-mu (tau - t0)^2) dtau for T > 0, else 0 (written with erfc)."""
    T = np.asarray(T, dtype=np.float64)
    rm = np.sqrt(mu)
    val = SQRT_PI / (2.0 * rm) * (erfc(rm * (t0 - T)) - erfc(rm * t0))
    return np.where(T > 0.0, val, 0.0)


def manufactured_field(x, t, xs, mu, t0, periodic, n_images=3):
    """u_ex(x, t) = 1/2 sum_j sum_images int_0^{t - |x - x_j - 2 pi m|} sigma_j.

    x: (P,) targets; xs, mu, t0: (M,) source data.  Free space uses m = 0 only.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    ms = range(-n_images, n_images + 1) if periodic else [0]
    out = np.zeros(x.shape)
    for m in ms:
        d = np.abs(x[:, None] - xs[None, :] - 2.0 * math.pi * m)
        out += 0.5 * gaussian_density_integral(t - d, mu[None, :], t0[None, :]).sum(axis=1)
    return out


def manufactured_driving(xs, beta, mu, t0, periodic):
    """g_j(t) = -sigma_j(t) - beta_j u_ex(x_j, t) for the prescribed densities."""
    def g(t):
        return -gaussian_density(t, mu, t0) - beta * manufactured_field(xs, t, xs, mu, t0, periodic)
    return g


def free_wave_modes(K, centre, width):
    """Fourier data of the periodised u0(x) = exp(-(x-c)^2/(2w^2)) with v0 = -u0'.

    alpha_k = (1/2pi) int_R u0(x) e^{ikx} dx = w/sqrt(2pi) e^{ikc} e^{-k^2 w^2/2};
    alpha'_k = i k alpha_k (a right-going wave has u_t = -u_x).
    """
    k = np.arange(K + 1, dtype=np.float64)
    a = width / math.sqrt(2.0 * math.pi) * np.exp(1j * k * centre - 0.5 * (k * width) ** 2)
    return a, 1j * k * a


def free_wave_field(x, t, centre, width, n_images=4):
    """u(x, t) = sum_m u0(x - t - 2 pi m) (periodised right-going pulse)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape)
    for m in range(-n_images, n_images + 1):
        y = x - t - centre - 2.0 * math.pi * m
        out += np.exp(-y * y / (2.0 * width * width))
    return out
