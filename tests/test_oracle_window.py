"""Pins of the oracle's blending window (Section 2, eqs. (KB), (phi), (b))."""
import math

import numpy as np
from scipy.integrate import quad

from oracle.window import dphi, ddphi, phi, phi_sorted, shape_parameter

B = shape_parameter(1e-12)
DELTA = 0.35


def test_shape_parameter():
    # eq. (b): b = ln(1/eps)
    assert abs(B - 12 * math.log(10)) < 1e-14


def test_normalisation_and_symmetry():
    # eq. (KB) at omega = 0 gives int I0(b sqrt(1-t^2)) = 2 sinh(b)/b, so phi(delta) = 1;
    # the bump is even about delta/2, so phi(t) + phi(delta - t) = 1.
    t = np.linspace(0.0, DELTA, 41)
    s = phi(t, DELTA, B) + phi(DELTA - t, DELTA, B)
    assert np.max(np.abs(s - 1.0)) < 2e-15
    total = quad(lambda u: dphi(u, DELTA, B), 0.0, DELTA, epsabs=1e-16, limit=200)[0]
    assert abs(total - 1.0) < 1e-13
    assert phi(np.array([-1.0, 0.0]), DELTA, B).tolist() == [0.0, 0.0]
    assert phi(np.array([DELTA, 2 * DELTA]), DELTA, B).tolist() == [1.0, 1.0]


def test_fourier_transform_matches_kb():
    # Rescaling eq. (KB): int_0^delta phi'(t) e^{iwt} dt
    #   = (b / sinh b) e^{i w delta/2} sinc(sqrt((w delta/2)^2 - b^2)).
    for w in [0.0, 50.0, 150.0, 157.0, 300.0, 900.0]:
        re = quad(lambda t: dphi(t, DELTA, B) * math.cos(w * t), 0, DELTA, limit=400, epsabs=1e-16)[0]
        im = quad(lambda t: dphi(t, DELTA, B) * math.sin(w * t), 0, DELTA, limit=400, epsabs=1e-16)[0]
        z = (w * DELTA / 2) ** 2 - B * B
        sinc = math.sinh(math.sqrt(-z)) / math.sqrt(-z) if z < 0 else (
            math.sin(math.sqrt(z)) / math.sqrt(z) if z > 0 else 1.0)
        ref = B / math.sinh(B) * sinc * complex(math.cos(w * DELTA / 2), math.sin(w * DELTA / 2))
        assert abs(complex(re, im) - ref) < 1e-13 * max(1.0, abs(ref))


def test_bandlimit():
    # the window's eps-bandlimit is 2b/delta: beyond it |FT phi'| is O(eps)
    w = 2 * B / DELTA * 1.05
    re = quad(lambda t: dphi(t, DELTA, B) * math.cos(w * t), 0, DELTA, limit=400, epsabs=1e-17)[0]
    im = quad(lambda t: dphi(t, DELTA, B) * math.sin(w * t), 0, DELTA, limit=400, epsabs=1e-17)[0]
    assert abs(complex(re, im)) < 10 * 2 * B / math.sinh(B)


def test_derivatives_by_finite_differences():
    t = np.linspace(0.02, DELTA - 0.02, 9)
    h = 1e-6
    fd1 = (phi(t + h, DELTA, B) - phi(t - h, DELTA, B)) / (2 * h)
    assert np.max(np.abs(fd1 - dphi(t, DELTA, B))) < 1e-7
    fd2 = (dphi(t + h, DELTA, B) - dphi(t - h, DELTA, B)) / (2 * h)
    assert np.max(np.abs(fd2 - ddphi(t, DELTA, B))) < 1e-6 * np.max(np.abs(fd2))


def test_end_jumps():
    # phi' jumps by b/(delta sinh b) at both ends of its support (I0(0) = 1)
    j = B / (DELTA * math.sinh(B))
    v = dphi(np.array([0.0, DELTA]), DELTA, B)
    assert np.allclose(v, j, rtol=1e-14)


def test_phi_sorted_matches_phi():
    rng = np.random.default_rng(0)
    t = np.sort(rng.uniform(-0.01, DELTA + 0.01, (7, 35)), axis=1)
    a = phi_sorted(t, DELTA, B)
    b = phi(t.ravel(), DELTA, B).reshape(t.shape)
    assert np.max(np.abs(a - b)) < 1e-14
