"""Free-space radiation-boundary projection P (Section 4.4, eq. (vtilde)).

Acting on the half spectra alpha_k, alpha'_k (k = 0..K):
1. drop k = +-K and evaluate u(x_i) = sum_{|k|<K} alpha_k e^{-ikx_i} and v
   likewise from alpha', on the grid x_i = i h, i = -K..K-1, h = pi/K
   (direct DFT);
2. on the outer grid points, |i| >= K - 2W, roll off with the spatial window
   phi_s of timescale delta_s = W h:
       u~ = phi_s(pi - delta_s - |x|) u,
       v~ = phi_s'(pi - delta_s - |x|) u + phi_s(pi - delta_s - |x|) v
   (the right-end formula of eq. (vtilde); the left end is its mirror image,
   which gives the same expression in |x|);
3. transform back, alpha_k = (1/2K) sum_i u~_i e^{ikx_i} for k = 0..K-1, and
   alpha_K = 0.
The window argument is formed from integers, (K - |i| - W) h, so the end
points of the window support are hit exactly.

rbc_project evaluates both sums as written (dense (2K, K) cosine and sine
tables, so only for K up to a few thousand); rbc_project_fft takes the same
two sums with numpy's FFT of length 2K as the summation step (on x_i =
(i - K) h the phase e^{-ikx_i} is (-1)^k e^{-2 pi i i k / 2K}), for grids too
long for the tables.  The two agree to rounding (pinned in the tests).
"""
import numpy as np

from .window import dphi, phi


def rbc_project(alpha, dalpha, prm):
    K, W, h = prm.K, prm.W, prm.h
    i = np.arange(-K, K)
    x = i * h
    k = np.arange(K)                                  # k = 0..K-1 (k = K dropped)
    wk = np.where(k == 0, 1.0, 2.0)
    ph = np.outer(x, k)                               # (2K, K)
    c, s = np.cos(ph), np.sin(ph)

    def to_grid(a):
        a = wk * a[:K]
        return c @ a.real + s @ a.imag

    u = to_grid(alpha)
    v = to_grid(dalpha)
    outer = np.abs(i) >= K - 2 * W
    arg = (K - np.abs(i[outer]) - W) * h
    rho = phi(arg, prm.delta_s, prm.b)
    drho = dphi(arg, prm.delta_s, prm.b)
    uo, vo = u[outer], v[outer]
    u[outer] = rho * uo
    v[outer] = drho * uo + rho * vo

    def to_modes(g):
        out = np.zeros(K + 1, np.complex128)
        out[:K] = (g @ c + 1j * (g @ s)) / (2 * K)
        return out

    return to_modes(u), to_modes(v)


def _roll_off(u, v, prm):
    K, W, h = prm.K, prm.W, prm.h
    i = np.arange(-K, K)
    outer = np.abs(i) >= K - 2 * W
    arg = (K - np.abs(i[outer]) - W) * h
    rho = phi(arg, prm.delta_s, prm.b)
    drho = dphi(arg, prm.delta_s, prm.b)
    uo, vo = u[outer], v[outer]
    u[outer] = rho * uo
    v[outer] = drho * uo + rho * vo


def rbc_project_fft(alpha, dalpha, prm):
    K = prm.K
    k = np.arange(K)
    sign = np.where(k % 2 == 0, 1.0, -1.0)
    wk = np.where(k == 0, 1.0, 2.0)

    def to_grid(a):
        c = np.zeros(2 * K, np.complex128)
        c[:K] = wk * sign * a[:K]
        return np.fft.fft(c).real          # sum_k wk Re(a_k e^{-ikx_i})

    u = to_grid(alpha)
    v = to_grid(dalpha)
    _roll_off(u, v, prm)

    def to_modes(g):
        out = np.zeros(K + 1, np.complex128)
        out[:K] = sign * np.fft.ifft(g)[:K]     # (1/2K) sum_i g_i e^{ikx_i}
        return out

    return to_modes(u), to_modes(v)
