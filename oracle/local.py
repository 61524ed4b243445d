"""Local part: distances, neighbour classes and local quadrature weights
(Definition lambdadef, eqs. (localSol1), (localSol2), (interp) and the
weights Q_m of Section 4.1).

For a target x and a source x_l at distance d = dist(x, x_l) < delta the
integral  int_{t_{n+1}-delta}^{t_{n+1}-d} [1 - phi(t_{n+1}-tau)] sigma_l(tau) dtau
is approximated by one N_L-node Gauss-Legendre rule on its interval, with
sigma_l at each node replaced by the degree-(p-1) polynomial through the p
nearest available grid values sigma_l^{n+1-m}, m_min <= m <= m_max.
Measured in steps before t_{n+1}, node i sits at
    s_i = W - (W - d/dt)(1 + z_i)/2,   z_i in [-1, 1] the Gauss-Legendre nodes,
its weight is ((delta - d)/2) w_i (1 - phi(s_i dt)), and its stencil is the p
consecutive lags starting at max(m_min, floor(s_i) - p/2 + 1); m_min = 0 for a
nearby source (d < dt) and 1 for an intermediate one (dt <= d < delta).
Interpolation weights use the barycentric formula with the equispaced-node
weights (-1)^i C(p-1, i).  Q_m(d) = sum over nodes of node weight times the
node's interpolation weight at lag m; all Q_m vanish for d >= delta.

Pins: tests/test_oracle_local.py (the local quadrature of a prescribed smooth
density reproduces the exact windowed integral; with sigma = 1 the weights sum
to the exact integral of 1 - phi), and the split invariant of
tests/test_oracle_exact.py.
"""
import math

import numpy as np

from .window import phi_sorted

TWO_PI = 2.0 * math.pi


def periodic_distance(a, b):
    """dist(a, b) = min_m |a - b - 2 pi m| for a, b in [-pi, pi)  (Definition lambdadef)."""
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
    return np.where(d > math.pi, TWO_PI - d, d)


def free_distance(a, b):
    return np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))


def barycentric_weights(s, nodes):
    """Lagrange interpolation weights at points s (P,) on integer nodes (P, p).

    Barycentric second form with weights (-1)^i C(p-1, i); exact node hits get
    the unit vector.
    """
    p = nodes.shape[1]
    lam = np.array([(-1) ** i * math.comb(p - 1, i) for i in range(p)], dtype=np.float64)
    diff = s[:, None] - nodes
    hit = diff == 0.0
    safe = np.where(hit, 1.0, diff)
    terms = lam[None, :] / safe
    v = terms / terms.sum(axis=1, keepdims=True)
    anyhit = hit.any(axis=1)
    if anyhit.any():
        v[anyhit] = hit[anyhit].astype(np.float64)
    return v


def local_weights(d, dt, W, p, delta, b, n_gl):
    """Q_m(d) for m = 0..W+p/2 (Section 4.1); d is an array of distances.

    Returns an array of shape (len(d), W + p/2 + 1).
    """
    d = np.atleast_1d(np.asarray(d, dtype=np.float64))
    m_max = W + p // 2
    ncol = m_max + 1
    out = np.zeros((d.size, ncol))
    act = np.nonzero(d < delta)[0]
    if act.size == 0:
        return out
    da = d[act]
    z, wq = np.polynomial.legendre.leggauss(n_gl)
    z, wq = z[::-1], wq[::-1]              # node lags s ascending
    D = da / dt
    m_min = np.where(da < dt, 0, 1)
    half = 0.5 * (delta - da)
    S = W - (W - D)[:, None] * (1.0 + z[None, :]) / 2.0          # (P, n_gl) lags of the nodes
    one_minus_phi = 1.0 - phi_sorted(S * dt, delta, b)
    offs = np.arange(p)
    acc = np.zeros(act.size * ncol)
    base = (np.arange(act.size) * ncol)[:, None]
    for i in range(n_gl):
        s = S[:, i]
        node_w = half * wq[i] * one_minus_phi[:, i]
        m0 = np.maximum(m_min, np.floor(s).astype(np.int64) - p // 2 + 1)
        nodes = m0[:, None] + offs[None, :]
        v = barycentric_weights(s, nodes.astype(np.float64))
        contrib = node_w[:, None] * v
        acc += np.bincount((base + nodes).ravel(), weights=contrib.ravel(),
                           minlength=acc.size)
    out[act] = acc.reshape(act.size, ncol)
    return out


def barycentric_derivative(s, nodes):
    """d/ds of the Lagrange weights of ``barycentric_weights`` (same stencil).

    Off the nodes: v_r' = v_r (-1/(s - n_r) + sum_q A_q/(s - n_q) / sum_q A_q)
    with A_q = lam_q/(s - n_q); at a node n_j the derivative of the Lagrange
    basis is (lam_r/lam_j)/(n_j - n_r) for r != j and minus their sum at j.
    """
    p = nodes.shape[1]
    lam = np.array([(-1) ** i * math.comb(p - 1, i) for i in range(p)], dtype=np.float64)
    diff = s[:, None] - nodes
    hit = diff == 0.0
    safe = np.where(hit, 1.0, diff)
    A = lam[None, :] / safe
    T = A.sum(axis=1, keepdims=True)
    v = A / T
    dv = v * (-1.0 / safe + (A / safe).sum(axis=1, keepdims=True) / T)
    for row in np.nonzero(hit.any(axis=1))[0]:
        j = int(np.nonzero(hit[row])[0][0])
        nj = nodes[row, j]
        d = np.zeros(p)
        for r in range(p):
            if r != j:
                d[r] = (lam[r] / lam[j]) / (nj - nodes[row, r])
        d[j] = -d.sum()
        dv[row] = d
    return dv


def local_weights_dd(d, dt, W, p, delta, b, n_gl):
    """dQ_m/dd for m = 0..W+p/2, the derivative of ``local_weights`` in the
    distance d (for gradients with respect to positions).

    Differentiates each term of Q_m(d) = sum_i node_w_i(d) v_{i,m}(s_i(d)):
        ds_i/dd = (1 + z_i)/(2 dt),
        node_w_i' = -(1/2) w_i (1 - phi(s_i dt)) - ((delta - d)/2) w_i phi'(s_i dt) dt ds_i/dd,
    with the stencil held fixed (it is piecewise constant in d; Q is
    continuous where it changes).  The class switch at d = dt is a jump of
    Q; there the one-sided derivative of the class of d is returned.
    """
    from .window import dphi
    d = np.atleast_1d(np.asarray(d, dtype=np.float64))
    m_max = W + p // 2
    ncol = m_max + 1
    out = np.zeros((d.size, ncol))
    act = np.nonzero(d < delta)[0]
    if act.size == 0:
        return out
    da = d[act]
    z, wq = np.polynomial.legendre.leggauss(n_gl)
    z, wq = z[::-1], wq[::-1]
    D = da / dt
    m_min = np.where(da < dt, 0, 1)
    half = 0.5 * (delta - da)
    S = W - (W - D)[:, None] * (1.0 + z[None, :]) / 2.0
    one_minus_phi = 1.0 - phi_sorted(S * dt, delta, b)
    offs = np.arange(p)
    acc = np.zeros(act.size * ncol)
    base = (np.arange(act.size) * ncol)[:, None]
    for i in range(n_gl):
        s = S[:, i]
        ds = (1.0 + z[i]) / (2.0 * dt)
        node_w = half * wq[i] * one_minus_phi[:, i]
        node_dw = -0.5 * wq[i] * one_minus_phi[:, i] - half * wq[i] * dphi(s * dt, delta, b) * dt * ds
        m0 = np.maximum(m_min, np.floor(s).astype(np.int64) - p // 2 + 1)
        nodes = (m0[:, None] + offs[None, :]).astype(np.float64)
        v = barycentric_weights(s, nodes)
        dv = barycentric_derivative(s, nodes)
        contrib = node_dw[:, None] * v + node_w[:, None] * dv * ds
        acc += np.bincount((base + nodes.astype(np.int64)).ravel(), weights=contrib.ravel(),
                           minlength=acc.size)
    out[act] = acc.reshape(act.size, ncol)
    return out
