"""History part: influence kernel, one-step kernels and the mode propagator
(Section 3: eqs. (Fk), (psidef), Lemma (alphakEvolutionFormulas),
(hkgkcomp), (pkqkcomp), (hkcompdisc)).

For mode k (k = 0 meaning the limit k -> 0, Remark r:kzero):
    Psi_k(tau) = 2 cos(k tau) phi'(tau) + (sin(k tau)/k) phi''(tau),
    p_k(r) = int_0^dt sin(k(dt-mu))/k * Psi_k(r+mu) dmu,
    q_k(r) = int_0^dt cos(k(dt-mu))   * Psi_k(r+mu) dmu,
tabulated at r = m dt, m = 0..W-1, by an N_g-point Gauss-Legendre rule.
One step of the exact propagator with the trapezoid driving terms
    h_k = dt sum_{m=0}^{W-1} p_k(m dt) S_k^{n-m},  g_k likewise with q_k,
    alpha_k  <- cos(k dt) alpha_k + sin(k dt)/k alpha'_k + h_k,
    alpha'_k <- -k sin(k dt) alpha_k + cos(k dt) alpha'_k + g_k.
Only k = 0..K is stored: for real densities alpha_{-k} = conj(alpha_k).

Pins: tests/test_oracle_history.py (the march reproduces eq. (alphak) computed
by adaptive quadrature for a smooth-start S_k; p_k, q_k vanish at both ends of
their support; N_g doubling leaves them unchanged).
"""
import numpy as np

from .window import dphi, ddphi


def sin_over_k(k, x):
    """sin(k x)/k with the k -> 0 limit x (Remark r:kzero)."""
    k = np.asarray(k, dtype=np.float64)
    safe = np.where(k == 0, 1.0, k)
    return np.where(k == 0, x, np.sin(k * x) / safe)


def influence_kernel(k, tau, delta, b):
    """Psi_k(tau) of eq. (psidef); support [0, delta]."""
    return 2.0 * np.cos(k * tau) * dphi(tau, delta, b) + sin_over_k(k, tau) * ddphi(tau, delta, b)


def pq_tables(K, dt, W, delta, b, n_gl=32):
    """p_k(m dt), q_k(m dt) for k = 0..K, m = 0..W-1 (eq. (pkqkcomp)).

    Returns two arrays of shape (W, K+1).
    """
    z, w = np.polynomial.legendre.leggauss(n_gl)
    mu = 0.5 * dt * (z + 1.0)             # nodes on [0, dt]
    wmu = 0.5 * dt * w
    k = np.arange(K + 1, dtype=np.float64)[:, None]          # (K+1, 1)
    P = np.empty((W, K + 1))
    Q = np.empty((W, K + 1))
    for m in range(W):
        tau = m * dt + mu                                     # (n_gl,)
        psi = influence_kernel(k, tau[None, :], delta, b)     # (K+1, n_gl)
        ps = sin_over_k(k, (dt - mu)[None, :])
        qc = np.cos(k * (dt - mu)[None, :])
        P[m] = (ps * psi) @ wmu
        Q[m] = (qc * psi) @ wmu
    return P, Q


def rotation(K, dt):
    """Entries of the homogeneous propagator over dt (Section 3):
    c_k = cos(k dt), s_k = sin(k dt)/k, r_k = -k sin(k dt), k = 0..K."""
    k = np.arange(K + 1, dtype=np.float64)
    return np.cos(k * dt), sin_over_k(k, dt), -k * np.sin(k * dt)


def fir(table, ring):
    """dt-free trapezoid sum  sum_{m=0}^{W-1} table[m] * S^{n-m}  (eq. (hkcompdisc)).

    ``ring`` holds the W most recent spectra by age: ``ring[m]`` is S^{n-m}.
    """
    W = table.shape[0]
    acc = np.zeros(ring.shape[1], dtype=np.complex128)
    for m in range(W):
        acc = acc + table[m] * ring[m]
    return acc


def mode_step(alpha, dalpha, ring, P, Q, rot, dt):
    """One application of the Lemma's evolution formulae with eq. (hkcompdisc);
    ``ring[m]`` = S^{n-m}."""
    c, s, r = rot
    hk = dt * fir(P, ring)
    gk = dt * fir(Q, ring)
    return c * alpha + s * dalpha + hk, r * alpha + c * dalpha + gk
