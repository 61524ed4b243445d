"""Pins of the oracle's row-sampled pieces of a level (oracle/rows.py)."""
import math

import numpy as np

from oracle.march import Oracle
from oracle.params import FREE_SPACE, PERIODIC, Params
from oracle.rows import history_field, row_pieces, spectrum_direct


def test_spectrum_on_a_uniform_grid_is_the_fft():
    """Springs on the grid x_j = -pi + 2 pi j / N: S_k = (1/2pi) sum_j sigma_j
    e^{ikx_j} = ((-1)^k / 2pi) * N * ifft(sigma)_k (a library transform)."""
    N, K = 64, 20
    x = -math.pi + 2 * math.pi * np.arange(N) / N
    sig = np.random.default_rng(1).standard_normal(N)
    ref = (-1.0) ** np.arange(K + 1) * N * np.fft.ifft(sig)[:K + 1] / (2 * math.pi)
    assert np.max(np.abs(spectrum_direct(x, sig, K) - ref)) < 1e-14


def test_history_field_of_single_modes():
    """alpha = unit at k0 > 0 gives u_H(x) = 2 cos(k0 x); alpha_0 = c gives c;
    alpha_k0 = i gives 2 sin(k0 x) (alpha_{-k} = conj alpha_k)."""
    x = np.linspace(-3, 3, 17)
    a = np.zeros(9, np.complex128)
    a[5] = 1.0
    assert np.max(np.abs(history_field(x, a) - 2 * np.cos(5 * x))) < 1e-14
    a[5] = 1j
    assert np.max(np.abs(history_field(x, a) - 2 * np.sin(5 * x))) < 1e-14
    a[:] = 0
    a[0] = 0.7
    assert np.max(np.abs(history_field(x, a) - 0.7)) < 1e-15


def test_row_pieces_equal_the_assembled_march_rows():
    """The per-row local sum and matrix row (own brute-force neighbour search)
    equal the rows of the march's assembled C and S."""
    rng = np.random.default_rng(5)
    for periodic in (True, False):
        prm = Params(dt=0.01, boundary=PERIODIC if periodic else FREE_SPACE)
        lo, hi = (-math.pi, math.pi) if periodic else prm.omega
        M = 60
        x = rng.uniform(lo, hi, M)
        x[:10] = np.clip(x[0] + rng.uniform(-0.012, 0.012, 10), lo, hi)    # a dense run: nearby pairs
        if periodic:
            x[10:14] = rng.uniform(math.pi - 0.01, math.pi, 4)   # wrapping neighbours
            x[14:18] = rng.uniform(-math.pi, -math.pi + 0.01, 4)
        x = np.where(x >= math.pi, x - 2 * math.pi, x)
        beta = rng.uniform(1, 10, M)
        o = Oracle(x, beta, prm, lambda t: np.zeros(M))
        hist = rng.standard_normal((prm.m_max, M))
        C = o.C @ hist.ravel()
        S = o.S.toarray()
        for j in range(M):
            loc, nb, srow = row_pieces(x, beta, hist, j, prm, periodic)
            assert abs(beta[j] * loc - C[j]) < 1e-13 * (1 + abs(C[j]))
            ref = np.zeros(M)
            ref[nb] = srow
            assert np.max(np.abs(ref - S[j])) < 1e-15
