"""Pieces of one level of the discrete march (eq. (periodicIE_disc)) at a few
selected springs, for sizes where the oracle's whole level (every row of the
local sum, a sparse LU of the full nearby system) is out of reach.  Test
infrastructure like the rest of this package.

All sums are the plain definitions, evaluated directly:
* spectrum_direct: S_k = (1/2pi) sum_j sigma_j e^{ikx_j}, k = 0..K (eq. (densco));
* history_field: u_H(x) = sum_{|k|<=K} alpha_k e^{-ikx} with alpha_{-k} =
  conj(alpha_k) (eq. (historySol1));
* row_pieces: for a target spring j, the explicit local sum
  sum_{m>=1} sum_{l: d_jl < delta} (1/2) Q_m(d_jl) sigma_l^{L-m} (the weights of
  Section 4.1, brute-force neighbour search), and the row of the implicit
  matrix S_jl = (beta_j/2) Q_0(d_jl) over the nearby springs (d_jl < dt).
"""
import math

import numpy as np

from .local import free_distance, local_weights, periodic_distance

TWO_PI = 2.0 * math.pi


def spectrum_direct(x, sigma, K, chunk=512, workers=1, modes=None):
    """S_k for k = 0..K (or the given modes) of densities sigma at positions x
    (eq. (densco)).
    The springs are taken in chunks (in `workers` threads for large M) whose
    partial sums are added in chunk order."""
    x = np.asarray(x, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    k = np.arange(K + 1, dtype=np.float64) if modes is None else np.asarray(modes, dtype=np.float64)
    starts = list(range(0, x.size, chunk))

    def part(a):
        ph = np.outer(k, x[a:a + chunk])
        sg = sigma[a:a + chunk]
        return np.cos(ph) @ sg + 1j * (np.sin(ph) @ sg)

    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            parts = list(ex.map(part, starts))
    else:
        parts = map(part, starts)
    out = np.zeros(k.size, np.complex128)
    for v in parts:
        out += v
    return out / TWO_PI


def history_field(xq, alpha):
    """u_H at the points xq from the half spectrum alpha_0..alpha_K."""
    xq = np.atleast_1d(np.asarray(xq, dtype=np.float64))
    alpha = np.asarray(alpha, dtype=np.complex128)
    k = np.arange(alpha.size, dtype=np.float64)
    w = np.where(k == 0, 1.0, 2.0) * alpha
    ph = np.outer(xq, k)
    return np.cos(ph) @ w.real + np.sin(ph) @ w.imag


def row_pieces(x, beta, hist, j, prm, periodic):
    """(local, nb, S_row) for spring j: the explicit local sum over lags
    m = 1..m_max of hist[m-1] = sigma^{L-m}, the indices of the nearby springs
    and their entries (beta_j/2) Q_0 of the implicit matrix."""
    dist = periodic_distance if periodic else free_distance
    d = dist(x, x[j])
    nb = np.nonzero(d < prm.delta)[0]
    Q = local_weights(d[nb], prm.dt, prm.W, prm.p, prm.delta, prm.b, prm.n_gl_local)
    local = 0.5 * sum(float(Q[:, m] @ hist[m - 1, nb]) for m in range(1, prm.m_max + 1))
    near = Q[:, 0] != 0.0
    return local, nb[near], 0.5 * beta[j] * Q[near, 0]
