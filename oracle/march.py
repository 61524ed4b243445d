"""The fully discrete WFP march (Tier A), plain and slow.

Discrete equation (periodicIE_disc) at t_L = L dt, with the history term read
as beta_j u_H(x_j) (u_H = sum_k alpha_k e^{-ikx}, eq. (historySol1); the
printed factor beta_j/2 contradicts eqs. (historySol), (fcoef) and the jump
condition, see the design notes):

    -(I + S) sigma^L = g^L + sum_{m>=1} C^(m) sigma^{L-m} + diag(beta) u_H(x),

with S_jl = (beta_j/2) Q_0(d_jl) (nearby pairs), C^(m)_jl = (beta_j/2) Q_m(d_jl).
Each level L = 0, 1, 2, ... is computed from the history of levels < L,
which is zero before L = 0 (so sigma^0 solves (I+S) sigma^0 = -g^0):

1. S^{L-1}_k = (1/2pi) sum_j sigma_j^{L-1} e^{ikx_j}, k = 0..K   (eq. (densco), direct sum)
2. push into the ring of the last W spectra, apply the FIR of eq. (hkcompdisc)
   and the Lemma's propagator -> alpha^L, alpha'^L
3. free space only: every P levels apply the RBC projection (Section 4.4)
4. u_H(x) = alpha_0 + 2 Re sum_{k=1}^K alpha_k e^{-ikx}   (direct sum)
5. right-hand side and sparse LU solve for sigma^L
6. receivers: u(x_r, t_L) = 1/2 sum_l sum_{m>=0} Q_m(d_rl) sigma_l^{L-m} + u_H(x_r)

Driving data g_j(t) = beta_j f(x_j - t) (eq. (gj) for a smooth incident field),
f periodised in the periodic box (Section 2).
"""
import math

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from .history import mode_step, pq_tables, rotation
from .local import free_distance, local_weights, periodic_distance
from .params import FREE_SPACE, PERIODIC, Params
from .rbc import rbc_project, rbc_project_fft

# the boundary projection evaluates its sums directly up to this K (dense tables)
RBC_DIRECT_MAX_K = 16384

TWO_PI = 2.0 * math.pi


def incident_profile(s, packets, periodic):
    """f(s) = sum_i a_i exp(-(s-c_i)^2/(2 w_i^2)) cos(omega_i (s-c_i) + ph_i).

    ``packets`` is an (n, 5) array of (a, c, w, omega, ph).  In the periodic
    box f is replaced by its 2 pi-periodisation sum_m f(s + 2 pi m).
    """
    s = np.asarray(s, dtype=np.float64)
    packets = np.atleast_2d(np.asarray(packets, dtype=np.float64))
    if periodic:
        s = s - TWO_PI * np.round(s / TWO_PI)
        shifts = [TWO_PI * m for m in range(-4, 5)]
    else:
        shifts = [0.0]
    out = np.zeros_like(s)
    for a, c, w, om, ph in packets:
        for sh in shifts:
            y = s + sh - c
            out = out + a * np.exp(-y * y / (2.0 * w * w)) * np.cos(om * y + ph)
    return out


def incident_driving(x, beta, packets, periodic):
    """Returns g(L, t) -> beta_j f(x_j - t) for all scatterers (eq. (gj))."""
    x = np.asarray(x, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)

    def g(t):
        return beta * incident_profile(x - t, packets, periodic)
    return g


def neighbour_pairs(targets, sources, delta, periodic, chunk=2048):
    """All (target, source) index pairs with distance < delta, by brute force."""
    dist = periodic_distance if periodic else free_distance
    ti, si, dd = [], [], []
    for a in range(0, len(targets), chunk):
        d = dist(targets[a:a + chunk, None], sources[None, :])
        i, j = np.nonzero(d < delta)
        ti.append(i + a)
        si.append(j)
        dd.append(d[i, j])
    return np.concatenate(ti), np.concatenate(si), np.concatenate(dd)


class Oracle:
    """Step-by-step FP64 march of the discrete WFP scheme.

    x, beta    scatterer positions in [-pi, pi) and stiffnesses (length M)
    params     oracle.params.Params
    driving    callable t -> g(t) (length M)
    x_recv     optional receiver positions
    """

    def __init__(self, x, beta, params: Params, driving, x_recv=None):
        self.x = np.asarray(x, dtype=np.float64)
        self.beta = np.asarray(beta, dtype=np.float64)
        self.M = self.x.size
        self.prm = prm = params
        self.periodic = prm.boundary == PERIODIC
        self.driving = driving
        self.xr = np.zeros(0) if x_recv is None else np.asarray(x_recv, dtype=np.float64)
        K, W = prm.K, prm.W
        if not self.periodic:
            lo, hi = prm.omega
            pts = np.concatenate([self.x, self.xr])
            if np.any(pts < lo) or np.any(pts > hi):
                raise ValueError("free space: scatterers and receivers must lie in Omega")
        # history part tables
        self.P, self.Q = pq_tables(K, prm.dt, W, prm.delta, prm.b, prm.n_gl_pq)
        self.rot = rotation(K, prm.dt)
        k = np.arange(K + 1, dtype=np.float64)
        self.k = k
        self.Ec = np.cos(np.outer(self.x, k))          # (M, K+1)
        self.Es = np.sin(np.outer(self.x, k))
        self.Erc = np.cos(np.outer(self.xr, k))
        self.Ers = np.sin(np.outer(self.xr, k))
        self.wk = np.where(k == 0, 1.0, 2.0)
        # local part: S (implicit, m = 0) and the stacked C^(m), m = 1..m_max
        nm = prm.m_max
        ti, si, d = neighbour_pairs(self.x, self.x, prm.delta, self.periodic)
        Qw = local_weights(d, prm.dt, W, prm.p, prm.delta, prm.b, prm.n_gl_local)
        self.n_pairs = ti.size
        half_beta = 0.5 * self.beta[ti]
        M = self.M
        self.S = sps.csr_matrix((half_beta * Qw[:, 0], (ti, si)), shape=(M, M))
        rows = np.repeat(ti, nm)
        cols = (np.arange(nm)[None, :] * M + si[:, None]).ravel()
        vals = (half_beta[:, None] * Qw[:, 1:nm + 1]).ravel()
        keep = vals != 0.0
        self.C = sps.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(M, nm * M))
        self.lu = spla.splu(sps.csc_matrix(sps.identity(M) + self.S))
        # receivers
        R = self.xr.size
        if R:
            ri, rs, rd = neighbour_pairs(self.xr, self.x, prm.delta, self.periodic)
            Qr = local_weights(rd, prm.dt, W, prm.p, prm.delta, prm.b, prm.n_gl_local)
            self.R0 = sps.csr_matrix((0.5 * Qr[:, 0], (ri, rs)), shape=(R, M))
            rows = np.repeat(ri, nm)
            cols = (np.arange(nm)[None, :] * M + rs[:, None]).ravel()
            vals = (0.5 * Qr[:, 1:nm + 1]).ravel()
            self.Rc = sps.csr_matrix((vals, (rows, cols)), shape=(R, nm * M))
        self.reset()

    # ---- state ---------------------------------------------------------
    def reset(self):
        prm = self.prm
        self.L = 0
        self.hist = np.zeros((prm.m_max, self.M))              # hist[m-1] = sigma^{L-m}
        self.ring = np.zeros((prm.W, prm.K + 1), np.complex128)  # ring[m] = S^{L-2-m}
        self.alpha = np.zeros(prm.K + 1, np.complex128)
        self.dalpha = np.zeros(prm.K + 1, np.complex128)

    def get_state(self):
        return dict(L=self.L, hist=self.hist.copy(), ring=self.ring.copy(),
                    alpha=self.alpha.copy(), dalpha=self.dalpha.copy())

    def set_state(self, st):
        self.L = int(st["L"])
        self.hist = np.array(st["hist"], dtype=np.float64)
        self.ring = np.array(st["ring"], dtype=np.complex128)
        self.alpha = np.array(st["alpha"], dtype=np.complex128)
        self.dalpha = np.array(st["dalpha"], dtype=np.complex128)

    # ---- the pieces of one level ----------------------------------------
    def spectrum(self, sigma):
        """S_k = (1/2pi) sum_j sigma_j e^{ikx_j}, k = 0..K (eq. (densco))."""
        return (sigma @ self.Ec + 1j * (sigma @ self.Es)) / TWO_PI

    def history_field(self, alpha, Ec, Es):
        """u_H(x) = sum_{|k|<=K} alpha_k e^{-ikx} = Re sum_{k>=0} w_k alpha_k e^{-ikx}."""
        a = self.wk * alpha
        return Ec @ a.real + Es @ a.imag

    def advance_modes(self):
        """Steps 1-3: new spectrum, FIR and propagator, RBC when due."""
        prm = self.prm
        S_new = self.spectrum(self.hist[0])
        self.ring = np.roll(self.ring, 1, axis=0)
        self.ring[0] = S_new                                    # ring[m] = S^{L-1-m}
        self.alpha, self.dalpha = mode_step(self.alpha, self.dalpha, self.ring,
                                            self.P, self.Q, self.rot, prm.dt)
        if not self.periodic and self.L > 0 and self.L % prm.rbc_period == 0:
            project = rbc_project if prm.K <= RBC_DIRECT_MAX_K else rbc_project_fft
            self.alpha, self.dalpha = project(self.alpha, self.dalpha, prm)

    def step(self):
        """Compute sigma^L (and receiver values at t_L); advance L."""
        prm = self.prm
        t = self.L * prm.dt
        self.advance_modes()
        uH = self.history_field(self.alpha, self.Ec, self.Es)
        rhs = -(self.driving(t) + self.C @ self.hist.ravel() + self.beta * uH)
        sigma = self.lu.solve(rhs)
        urec = None
        if self.xr.size:
            uHr = self.history_field(self.alpha, self.Erc, self.Ers)
            urec = self.R0 @ sigma + self.Rc @ self.hist.ravel() + uHr
        self.hist = np.roll(self.hist, 1, axis=0)
        self.hist[0] = sigma
        self.L += 1
        return sigma, urec

    def step_prescribed(self, sigma):
        """Advance one level with sigma^L given instead of solved for; returns
        the field at the receivers, u_L + u_H of eqs. (localSol1), (historySol1)."""
        self.advance_modes()
        uHr = self.history_field(self.alpha, self.Erc, self.Ers)
        urec = self.R0 @ sigma + self.Rc @ self.hist.ravel() + uHr
        self.hist = np.roll(self.hist, 1, axis=0)
        self.hist[0] = sigma
        self.L += 1
        return urec

    def run(self, n_levels, save_every=1):
        """March n_levels levels; returns (sigma rows saved every save_every
        levels starting with the first one, receiver values at every level)."""
        sig, rec = [], []
        for i in range(n_levels):
            s, u = self.step()
            if i % save_every == 0:
                sig.append(s)
            if u is not None:
                rec.append(u)
        return np.array(sig), (np.array(rec) if rec else None)
