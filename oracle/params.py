"""Derived parameters of the WFP scheme (Section 3.1, eqs. (Kdt), (W), (b);
Section 4.1 for m_max and N_L; Section 4.4 for the RBC grid).

Readings of the paper where it is silent or inexact (listed in the design
notes of the repository):
* K = floor(pi/dt) in the periodic box (eq. (Kdt) is not an integer); in free
  space the largest K <= pi/dt with 2K a 5-smooth number, so the RBC grid has
  a fast-transform length;
* W = round(2 b / (pi gamma)) (35 for eps = 1e-12, gamma = 1/2);
* p_k, q_k are tabulated at m = 0..W-1 (the indices eq. (hkcompdisc) uses);
* N_L = W Gauss-Legendre nodes for the local rule, N_g = 32 for p_k, q_k;
* m_max = W + p/2 (the largest lag any stencil touches is W-1+p/2);
* RBC grid spacing h = pi/K, spatial window timescale W h, projection period
  ceil(W h / dt) steps, scatterers confined to
  [-pi + 3 max(delta, W h), pi - 3 max(delta, W h)].
"""
import math
from dataclasses import dataclass

from .window import shape_parameter

PERIODIC = 0
FREE_SPACE = 1


def _is_25smooth(n):
    """True if n = 2^a 5^b."""
    for f in (2, 5):
        while n % f == 0 and n > 1:
            n //= f
    return n == 1


@dataclass
class Params:
    dt: float
    boundary: int = PERIODIC
    eps: float = 1e-12
    gamma: float = 0.5
    p: int = 8
    W: int = 0
    K: int = 0
    n_gl_local: int = 0
    n_gl_pq: int = 32
    rbc_period: int = 0

    def __post_init__(self):
        if self.dt <= 0:
            raise ValueError("dt must be positive")
        if self.p < 2 or self.p % 2:
            raise ValueError("p must be even and >= 2")
        self.b = shape_parameter(self.eps)
        if self.W == 0:
            self.W = int(round(2.0 * self.b / (math.pi * self.gamma)))
        self.delta = self.W * self.dt
        if self.K == 0:
            kmax = int(math.floor(math.pi / self.dt))
            if self.boundary == FREE_SPACE:
                k = kmax
                while k > 1 and not _is_25smooth(2 * k):
                    k -= 1
                self.K = k
            else:
                self.K = kmax
        if self.n_gl_local == 0:
            self.n_gl_local = self.W
        self.m_max = self.W + self.p // 2
        self.h = math.pi / self.K                 # RBC grid spacing
        self.delta_s = self.W * self.h            # spatial window timescale
        if self.rbc_period == 0:
            self.rbc_period = int(math.ceil(self.W * self.h / self.dt - 1e-12))
        margin = 3.0 * max(self.delta, self.delta_s)
        self.omega = (-math.pi + margin, math.pi - margin)
        if self.delta >= math.pi:
            raise ValueError("window timescale delta = W dt must be < pi")
        if self.K * self.dt > math.pi * (1 + 1e-14):
            raise ValueError("K dt must not exceed pi (Nyquist)")

    @property
    def nf_modes(self):
        return 2 * self.K + 1
