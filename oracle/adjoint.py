"""Gradient of a receiver misfit through the discrete march (test
infrastructure, like the rest of this package).

The paper has no adjoint; this is the plain reverse-mode transpose of every
step of ``oracle.march.Oracle.step`` (periodic box), taken in reverse order of
the levels, so that for any loss J(u) of the receiver values u_r^L,
L = 0..N-1, it returns dJ/dbeta_j and dJ/dx_j of the fully discrete scheme.

Forward level L (Section 4.2, eq. (periodicIE_disc) with the history term
read as beta_j u_H(x_j)):
    S^{L-1}_k   = (1/2pi) sum_j sigma_j^{L-1} e^{ikx_j}                  (eq. (densco))
    alpha^L     = c alpha^{L-1} + s alpha'^{L-1} + dt sum_m P_m S^{L-1-m} (eq. (hkcompdisc), Lemma)
    alpha'^L    = r alpha^{L-1} + c alpha'^{L-1} + dt sum_m Q_m S^{L-1-m}
    u_H(x)      = sum_k w_k Re(alpha_k^L e^{-ikx}),  w_0 = 1, w_k = 2    (eq. (historySol1))
    v_i         = f(x_i - t_L) + sum_{m>=0} sum_l (1/2) Q_m(d_il) sigma_l^{L-m} + u_H(x_i)
    sigma_i^L   = -beta_i v_i     (solved as (I + S) sigma^L = rhs)
    u_r^L       = sum_{m>=0} sum_l (1/2) Q_m(d_rl) sigma_l^{L-m} + u_H(x_r)

Adjoint variables carry dJ/d(.) of each forward quantity; for a complex
quantity z the adjoint is dJ/dRe z + i dJ/dIm z, so dJ = Re(conj(zbar) dz).
Positions enter through d_il = |wrap(x_i - x_l)| (derivative
sign(wrap(x_i - x_l)), zero for i = l), the phases e^{+-ikx}, and
f(x_i - t).  dQ_m/dd is ``oracle.local.local_weights_dd``.

Pins: tests/test_oracle_adjoint.py (central finite differences of the
oracle's own loss along random directions and single coordinates; the
weight derivative against finite differences of the weights).
"""
import math

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from .local import local_weights, local_weights_dd
from .march import Oracle, incident_driving, neighbour_pairs
from .params import PERIODIC, Params
from .volterra import incident_profile_and_slope

TWO_PI = 2.0 * math.pi


def _wrap(y):
    return y - TWO_PI * np.round(y / TWO_PI)


def _lag_matrices(ti, si, w, shape, nlag):
    """One sparse matrix per lag m: entries w[:, m] at (ti, si)."""
    return [sps.csr_matrix((w[:, m], (ti, si)), shape=shape) for m in range(nlag)]


class AdjointOracle:
    """Forward march with recording, and the reverse sweep, periodic box.

    x, beta, packets   problem data as for ``Oracle``
    params             oracle.params.Params (periodic)
    x_recv             receiver positions (R >= 1)
    """

    def __init__(self, x, beta, packets, params: Params, x_recv):
        if params.boundary != PERIODIC:
            raise ValueError("the adjoint oracle covers the periodic box")
        self.x = np.asarray(x, dtype=np.float64)
        self.beta = np.asarray(beta, dtype=np.float64)
        self.packets = np.atleast_2d(np.asarray(packets, dtype=np.float64))
        self.xr = np.asarray(x_recv, dtype=np.float64)
        self.prm = prm = params
        self.M, self.R = self.x.size, self.xr.size
        self.fwd = Oracle(self.x, self.beta, prm, incident_driving(self.x, self.beta, self.packets, True), self.xr)
        nl = prm.m_max                       # lags 0..m_max-1 are used
        wargs = (prm.dt, prm.W, prm.p, prm.delta, prm.b, prm.n_gl_local)
        ti, si, d = neighbour_pairs(self.x, self.x, prm.delta, True)
        sg = np.sign(_wrap(self.x[ti] - self.x[si]))
        self.Qh = _lag_matrices(ti, si, 0.5 * local_weights(d, *wargs), (self.M, self.M), nl)
        self.DQ = _lag_matrices(ti, si, 0.5 * local_weights_dd(d, *wargs) * sg[:, None], (self.M, self.M), nl)
        ri, rs, rd = neighbour_pairs(self.xr, self.x, prm.delta, True)
        rsg = np.sign(_wrap(self.xr[ri] - self.x[rs]))
        self.RQ = _lag_matrices(ri, rs, 0.5 * local_weights(rd, *wargs), (self.R, self.M), nl)
        self.DR = _lag_matrices(ri, rs, 0.5 * local_weights_dd(rd, *wargs) * rsg[:, None], (self.R, self.M), nl)
        k = np.arange(prm.K + 1, dtype=np.float64)
        self.k = k
        self.wk = np.where(k == 0, 1.0, 2.0)
        self.E = np.exp(1j * np.outer(self.x, k))       # e^{+ikx_j}, (M, K+1)
        self.Er = np.exp(1j * np.outer(self.xr, k))
        A = sps.identity(self.M) + self.fwd.S
        self.luT = spla.splu(sps.csc_matrix(A.T))

    def forward(self, n_levels):
        """March n_levels levels from rest; record sigma^L, alpha^L and u_r^L."""
        self.fwd.reset()
        sig, alp, rec = [], [], []
        for _ in range(n_levels):
            s, u = self.fwd.step()
            sig.append(s)
            alp.append(self.fwd.alpha.copy())
            rec.append(u)
        self.sig = np.array(sig)
        self.alpha = np.array(alp)
        self.urec = np.array(rec)
        return self.urec

    def _uH(self, a, E):
        """u_H at the points of E: sum_k w_k Re(alpha_k e^{-ikx})."""
        return (np.conj(E) @ (self.wk * a)).real

    def _duH(self, a, E):
        """d/dx u_H: sum_k w_k Re(-ik alpha_k e^{-ikx})."""
        return (np.conj(E) @ (-1j * self.k * self.wk * a)).real

    def gradient(self, dJdu):
        """dJ/dbeta and dJ/dx for the recorded forward run, given dJ/du_r^L
        (shape (N, R))."""
        prm = self.prm
        N, M = self.sig.shape
        nl = prm.m_max
        W, dt = prm.W, prm.dt
        c, s, r = self.fwd.rot
        P, Q = self.fwd.P, self.fwd.Q
        sig = self.sig
        sbar = np.zeros((N, M))
        Sbar = np.zeros((N, prm.K + 1), np.complex128)
        abar = np.zeros(prm.K + 1, np.complex128)
        dabar = np.zeros(prm.K + 1, np.complex128)
        gb = np.zeros(M)
        gx = np.zeros(M)
        for L in range(N - 1, -1, -1):
            e = np.asarray(dJdu[L], dtype=np.float64)
            lags = [m for m in range(nl) if L - m >= 0]
            # receivers at level L: u_r^L
            for m in lags:
                sbar[L - m] += self.RQ[m].T @ e
                gx -= sig[L - m] * (self.DR[m].T @ e)
            abar += self.wk * (self.Er.T @ e)
            # the solve at level L: sigma^L = -beta v
            lam = self.luT.solve(sbar[L])
            mu = self.beta * lam
            f, df = incident_profile_and_slope(self.x - L * dt, self.packets, True)
            v = f + self._uH(self.alpha[L], self.E)
            dv = df + self._duH(self.alpha[L], self.E)
            for m in lags:
                v = v + self.Qh[m] @ sig[L - m]
                dv = dv + self.DQ[m] @ sig[L - m]
                gx += sig[L - m] * (self.DQ[m].T @ mu)
            gb -= lam * v
            gx -= mu * dv
            for m in lags:
                if m >= 1:
                    sbar[L - m] -= self.Qh[m].T @ mu
            abar += self.wk * (self.E.T @ (-mu))
            # the mode step of level L
            for m in range(W):
                if L - 1 - m >= 0:
                    Sbar[L - 1 - m] += dt * (P[m] * abar + Q[m] * dabar)
            abar, dabar = c * abar + r * dabar, s * abar + c * dabar
            # the spectrum of level L-1 has all its uses now
            if L >= 1:
                Sb = Sbar[L - 1]
                sbar[L - 1] += (np.conj(self.E) @ Sb).real / TWO_PI
                gx += sig[L - 1] * (self.E @ (1j * self.k * np.conj(Sb))).real / TWO_PI
        return gb, gx


def misfit_loss(u, u_target, dt):
    """J = (dt/2) sum_L sum_r (u_r^L - u*_r^L)^2 and dJ/du."""
    res = u - u_target
    return 0.5 * dt * float(np.sum(res * res)), dt * res
