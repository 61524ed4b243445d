"""Kaiser-Bessel blending window (Section 2, eqs. (KB), (phi), (b)).

phi'(t) = b / (delta sinh b) * I0(b sqrt(1 - (2t/delta - 1)^2)) on [0, delta],
zero outside;  phi(t) = int_0^t phi';  b = ln(1/eps).

phi'' is not printed in the paper; it follows by differentiating (phi):
with s = 2t/delta - 1 and r = sqrt(1 - s^2),
    phi''(t) = -(2 b^2 s / (delta^2 sinh b)) * I1(b r) / r,
and I1(b r)/r -> b/2 as r -> 0.

I0 and I1 are the library routines scipy.special.i0 / i1.

Parity pins: tests/test_oracle_window.py (normalisation phi(delta) = 1 from
eq. (KB) at omega = 0, symmetry phi(t) + phi(delta - t) = 1, the Fourier
transform of phi' against eq. (KB), phi' and phi'' against finite
differences of phi and phi').
"""
import numpy as np
from scipy.special import i0 as _i0, i1 as _i1


def shape_parameter(eps):
    """b = ln(1/eps)  (eq. (b))."""
    return float(np.log(1.0 / eps))


def _bump(u, b):
    """I0(b sqrt(1 - u^2)) for u in [-1, 1]."""
    return _i0(b * np.sqrt(np.clip(1.0 - u * u, 0.0, None)))


def dphi(t, delta, b):
    """phi'(t): the scaled Kaiser-Bessel bump of eq. (phi); zero outside [0, delta]."""
    t = np.asarray(t, dtype=np.float64)
    s = 2.0 * t / delta - 1.0
    inside = (t >= 0.0) & (t <= delta)
    return np.where(inside, b / (delta * np.sinh(b)) * _bump(np.clip(s, -1, 1), b), 0.0)


def ddphi(t, delta, b):
    """phi''(t) = -(2 b^2 s / (delta^2 sinh b)) I1(b r)/r, s = 2t/delta-1, r = sqrt(1-s^2).

    Obtained by differentiating eq. (phi) with d/dz I0(z) = I1(z); zero
    outside [0, delta].
    """
    t = np.asarray(t, dtype=np.float64)
    s = 2.0 * t / delta - 1.0
    inside = (t >= 0.0) & (t <= delta)
    r = np.sqrt(np.clip(1.0 - s * s, 0.0, None))
    x = b * r
    small = x < 1e-6
    xs = np.where(small, 1.0, x)
    i1_over_r = np.where(small, 0.5 * b * (1.0 + x * x / 8.0), b * _i1(xs) / xs)
    val = -(2.0 * b * b * s / (delta * delta * np.sinh(b))) * i1_over_r
    return np.where(inside, val, 0.0)


# Gauss-Legendre rules for the integral of phi'.  The integrand
# I0(b sqrt(1-u^2)) = sum_k (b^2 (1-u^2)/4)^k / (k!)^2 is a polynomial-like
# entire function of u with significant terms up to degree ~2b..4b; 120 nodes
# reach rounding level on [-1, 1] (checked against the closed form of eq. (KB)
# at omega = 0) and 16 nodes on sub-intervals of length <= 0.25.
_ZL, _WL = np.polynomial.legendre.leggauss(120)
_ZS, _WS = np.polynomial.legendre.leggauss(16)


def _integral(u0, u1, b, z, w):
    """int_{u0}^{u1} I0(b sqrt(1-u^2)) du, elementwise, by Gauss-Legendre."""
    mid = 0.5 * (u0 + u1)
    half = 0.5 * (u1 - u0)
    u = mid[..., None] + half[..., None] * z
    return half * (_bump(u, b) @ w)


def phi(t, delta, b):
    """phi(t) = int_0^t phi'(tau) dtau  (eq. (phi)); 0 for t <= 0, 1 for t >= delta.

    In the rescaled variable u = 2 tau/delta - 1:
        phi(t) = (b / (2 sinh b)) int_{-1}^{s} I0(b sqrt(1 - u^2)) du.
    """
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    s = np.clip(2.0 * t / delta - 1.0, -1.0, 1.0)
    out = b / (2.0 * np.sinh(b)) * _integral(np.full_like(s, -1.0), s, b, _ZL, _WL)
    out[t <= 0.0] = 0.0
    out[t >= delta] = 1.0
    return out


def phi_sorted(t, delta, b):
    """phi at points t[..., 0] <= t[..., 1] <= ... (sorted along the last axis).

    Same definition as ``phi``; the integral of phi' is accumulated over the
    consecutive sub-intervals between the points (each by a short rule),
    which is cheaper when many points per row are needed.
    """
    t = np.asarray(t, dtype=np.float64)
    s = np.clip(2.0 * t / delta - 1.0, -1.0, 1.0)
    c = b / (2.0 * np.sinh(b))
    out = np.empty_like(s)
    acc = c * _integral(np.full(s.shape[:-1], -1.0), s[..., 0], b, _ZL, _WL)
    out[..., 0] = acc
    for i in range(1, s.shape[-1]):
        gap = s[..., i] - s[..., i - 1]
        if np.any(gap > 0.25):
            piece = c * _integral(s[..., i - 1], s[..., i], b, _ZL, _WL)
        else:
            piece = c * _integral(s[..., i - 1], s[..., i], b, _ZS, _WS)
        acc = acc + piece
        out[..., i] = acc
    out[t <= 0.0] = 0.0
    out[t >= delta] = 1.0
    return out
