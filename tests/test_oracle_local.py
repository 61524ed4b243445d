"""Pins of the oracle's local quadrature (Section 4.1: eqs. (localSol2), (interp))."""
import math

import numpy as np
from scipy.integrate import quad

from oracle.local import local_weights, periodic_distance
from oracle.params import Params
from oracle.window import phi

PRM = Params(dt=0.01)


def _exact_window_integral(fn, d, t):
    """int_{t-delta}^{t-d} [1 - phi(t - tau)] fn(tau) dtau."""
    return quad(lambda tau: (1 - phi(np.array([t - tau]), PRM.delta, PRM.b)[0]) * fn(tau),
                t - PRM.delta, t - d, epsabs=1e-17, epsrel=1e-14, limit=400)[0]


def test_weights_integrate_constants_exactly():
    d = np.concatenate([[0.0, 0.5 * PRM.dt, PRM.dt, 0.1234], np.random.default_rng(1).uniform(0, PRM.delta, 6)])
    Q = local_weights(d, PRM.dt, PRM.W, PRM.p, PRM.delta, PRM.b, PRM.n_gl_local)
    for i, di in enumerate(d):
        ref = _exact_window_integral(lambda tau: 1.0, di, 1.0)
        assert abs(Q[i].sum() - ref) < 2e-16 * PRM.delta * 10


def test_weights_vanish_beyond_window_and_respect_classes():
    d = np.array([PRM.delta, PRM.delta * 1.5, 0.02, 0.005])
    Q = local_weights(d, PRM.dt, PRM.W, PRM.p, PRM.delta, PRM.b, PRM.n_gl_local)
    assert np.all(Q[0] == 0) and np.all(Q[1] == 0)
    assert Q[2, 0] == 0.0                 # intermediate source: m_min = 1
    assert Q[3, 0] != 0.0                 # nearby source uses sigma^{n+1}
    assert np.all(Q[:, -1] == 0.0)        # lag W + p/2 is never reached (largest is W-1+p/2)


def test_local_rule_order_of_accuracy():
    """The rule applied to samples of a smooth density converges like dt^(p+1)
    (interpolation error O(dt^p) on an interval of length O(delta))."""
    errs = []
    for dt in (0.02, 0.01):
        prm = Params(dt=dt, p=4)
        f = lambda tau: math.cos(3.0 * tau) + tau * tau
        t = 1.0
        for d in (0.3 * dt, 7.4 * dt):
            Q = local_weights(np.array([d]), dt, prm.W, prm.p, prm.delta, prm.b, prm.n_gl_local)[0]
            samples = np.array([f(t - m * dt) for m in range(Q.size)])
            ref = quad(lambda tau: (1 - phi(np.array([t - tau]), prm.delta, prm.b)[0]) * f(tau),
                       t - prm.delta, t - d, epsabs=1e-17, epsrel=1e-14, limit=400)[0]
            errs.append(abs(Q @ samples - ref))
    # halving dt with p = 4: error ratio ~ 2^5 (allow slack)
    assert errs[0] / errs[2] > 16 and errs[1] / errs[3] > 16


def test_p8_rule_on_smooth_density_is_accurate():
    f = lambda tau: math.exp(-30 * (tau - 0.8) ** 2)
    t = 1.0
    for d in (0.0, 0.004, 0.0123, 0.2):
        Q = local_weights(np.array([d]), PRM.dt, PRM.W, PRM.p, PRM.delta, PRM.b, PRM.n_gl_local)[0]
        samples = np.array([f(t - m * PRM.dt) for m in range(Q.size)])
        assert abs(Q @ samples - _exact_window_integral(f, d, t)) < 1e-11


def test_periodic_distance():
    assert abs(periodic_distance(-3.1, 3.1) - (2 * math.pi - 6.2)) < 1e-15
    assert periodic_distance(0.5, -0.25) == 0.75


def _brute_force_weights(d, prm):
    """Q_m(d) of Section 4.1 written out node by node, independently of the
    oracle's vectorised form: for every Gauss-Legendre node, the p grid lags
    nearest to the node are picked by sorting all allowed lags m_min..m_max
    by their distance to the node (the literal "p nearest available points"),
    and the interpolation weights come from the Lagrange product formula
    (not the barycentric one)."""
    z, w = np.polynomial.legendre.leggauss(prm.n_gl_local)
    m_min = 0 if d < prm.dt else 1
    lags = np.arange(m_min, prm.m_max + 1)
    Q = np.zeros(prm.m_max + 1)
    for zi, wi in zip(z, w):
        tau = (prm.delta - d) / 2 * zi + (prm.delta + d) / 2     # time before t_{n+1}
        s = tau / prm.dt                                          # in steps
        order = np.argsort(np.abs(lags - s), kind="stable")
        stencil = np.sort(lags[order[:prm.p]])
        node_w = (prm.delta - d) / 2 * wi * (1 - phi(np.array([tau]), prm.delta, prm.b)[0])
        for a in stencil:
            ell = 1.0
            for c in stencil:
                if c != a:
                    ell *= (s - c) / (a - c)
            Q[a] += node_w * ell
    return Q


def test_stencil_is_the_p_nearest_available_lags():
    """Each node's stencil is the p lags nearest to it among those allowed
    (eq. (interp)): the oracle's weights equal a brute-force selection by
    sorted distance.  A stencil started one lag newer or older than the
    nearest set fails this at every p."""
    rng = np.random.default_rng(3)
    for p in (2, 4, 6, 8):
        prm = Params(dt=0.01, p=p)
        ds = np.concatenate([[0.0, 0.37 * prm.dt, 0.999 * prm.dt, prm.dt, 1.5 * prm.dt, 12.3 * prm.dt,
                              prm.delta - 0.6 * prm.dt], rng.uniform(0, prm.delta, 4)])
        Q = local_weights(ds, prm.dt, prm.W, p, prm.delta, prm.b, prm.n_gl_local)
        for i, d in enumerate(ds):
            ref = _brute_force_weights(d, prm)
            # the weights are O(dt); rounding of the two forms differs by ~1e-16 dt
            assert np.max(np.abs(Q[i] - ref)) < 1e-14 * prm.dt, (p, d)
