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


def spring_array_transmission(w, xs, beta):
    """Transmission coefficient T(w) of free-space springs xs, beta at
    frequencies w > 0: the total field right of every spring is
    T(w) F(w) e^{iwx} for an incident wave F(w) e^{iwx}.  With the Green's
    function (1/2) H(t - |x|) -> (i/(2w)) e^{iw|x|} and the spring condition
    -sigma_j = beta_j u_tot(x_j),
        (I + A) v = e^{iw x},   A_jl = (i beta_l/(2w)) e^{iw|x_j - x_l|},
        T = 1 - sum_l (i beta_l/(2w)) e^{-iw x_l} v_l."""
    xs = np.asarray(xs, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    M = xs.size
    d = np.abs(xs[:, None] - xs[None, :])
    out = np.empty(w.size, np.complex128)
    chunk = 4096
    for a in range(0, w.size, chunk):
        ww = w[a:a + chunk]
        A = (1j * beta[None, None, :] / (2.0 * ww[:, None, None])) * np.exp(1j * ww[:, None, None] * d[None, :, :])
        A = A + np.eye(M)[None, :, :]
        v = np.linalg.solve(A, np.exp(1j * ww[:, None] * xs[None, :])[..., None])[..., 0]
        out[a:a + chunk] = 1.0 - ((1j * beta[None, :] / (2.0 * ww[:, None])) * np.exp(-1j * ww[:, None] * xs[None, :])
                                  * v).sum(axis=1)
    return out


def spring_chain_transmission(w, xs, beta):
    """T(w) as spring_array_transmission, by transfer matrices instead of
    the dense solve: in the frequency domain u'' + w^2 u = sum_j beta_j u(x_j)
    delta(x - x_j) (the Green's function's jump -1 in u'), so crossing spring
    j from right to left keeps u and lowers u' by beta_j u(x_j), and between
    springs (u, u') propagates freely.  Starting from u = e^{iwx} right of the
    last spring, the state left of the first one is a e^{iwx} + b e^{-iwx};
    T = 1/a.  O(M) per frequency; xs need not be sorted."""
    order = np.argsort(np.asarray(xs, dtype=np.float64))
    xs = np.asarray(xs, dtype=np.float64)[order]
    beta = np.asarray(beta, dtype=np.float64)[order]
    w = np.asarray(w, dtype=np.float64)
    u = np.exp(1j * w * xs[-1])
    du = 1j * w * u
    for j in range(xs.size - 1, -1, -1):
        du = du - beta[j] * u                       # across spring j, right to left
        if j > 0:
            h = xs[j] - xs[j - 1]                   # back to spring j - 1
            c, sn = np.cos(w * h), np.sin(w * h)
            u, du = c * u - sn / w * du, w * sn * u + c * du
    a = 0.5 * (u + du / (1j * w)) * np.exp(-1j * w * xs[0])
    return 1.0 / a


def spring_array_field(xr, t, xs, beta, mu, t0, w_max=None, dw=None, transmission=None):
    """Total field u_inc + u at a point xr to the right of every spring, for
    the free-space springs xs, beta and the incident wave f(x - t) with
    f(s) = exp(-mu (s - t0)^2), at times t: the inverse transform of
    T(w) F(w) e^{iw xr} (spring_array_transmission), with u(t) =
    (1/2pi) int u^(w) e^{-iwt} dw and F(w) = sqrt(pi/mu) e^{-iw t0}
    e^{-w^2/(4 mu)}, by the trapezoid rule on a midpoint grid of |w| <= w_max
    (the spectrum falls like e^{-w^2/(4 mu)}); it converges geometrically while
    dw is well below the width of the sharpest resonance (the resonances are
    poles a distance ~ that width off the real axis).  `transmission` is
    spring_array_transmission (default) or spring_chain_transmission."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    if w_max is None:
        w_max = math.sqrt(4.0 * mu * 40.0)              # e^{-40} of the peak
    if dw is None:
        dw = 1e-4
    n = int(math.ceil(w_max / dw))
    w = (np.arange(n) + 0.5) * dw                       # w > 0; w < 0 by conjugate symmetry
    F = math.sqrt(math.pi / mu) * np.exp(-1j * w * t0 - w * w / (4.0 * mu))
    U = (transmission or spring_array_transmission)(w, xs, beta) * F * np.exp(1j * w * xr)
    # u(t) = (1/2pi) int U e^{-iwt} dw = (1/pi) Re int_0^inf U e^{-iwt} dw
    out = np.empty(t.size)
    for i, tt in enumerate(t):
        out[i] = (dw / math.pi) * np.real(np.sum(U * np.exp(-1j * w * tt)))
    return out
