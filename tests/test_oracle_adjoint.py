"""Pins of the oracle's gradient (oracle/adjoint.py): central finite
differences of the oracle's own discrete loss, and of the local weights."""
import math

import numpy as np

from oracle.adjoint import AdjointOracle, misfit_loss
from oracle.local import local_weights, local_weights_dd
from oracle.params import Params

DT = 0.02
N = 150


def _problem(seed=7, M=5, R=3):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0.3, 1.2, M))
    beta = rng.uniform(1.0, 10.0, M)
    packets = np.array([[1.0, -1.0, 0.15, 0.0, 0.0]])
    xr = np.linspace(0.35, 1.15, R)
    return x, beta, packets, xr


def _loss(x, beta, packets, xr, target):
    a = AdjointOracle(x, beta, packets, Params(dt=DT), xr)
    u = a.forward(N)
    return misfit_loss(u, target, DT)[0]


def _setup():
    x, beta, packets, xr = _problem()
    rng = np.random.default_rng(50)
    bstar = beta * (1.0 + 0.05 * rng.standard_normal(beta.size))
    target = AdjointOracle(x, bstar, packets, Params(dt=DT), xr).forward(N)
    a = AdjointOracle(x, beta, packets, Params(dt=DT), xr)
    u = a.forward(N)
    J, dJdu = misfit_loss(u, target, DT)
    gb, gx = a.gradient(dJdu)
    return x, beta, packets, xr, target, J, gb, gx, a


def _no_class_switch(x, h):
    """No pair distance within 2h of dt (where Q jumps)."""
    d = np.abs(x[:, None] - x[None, :])
    return np.all(np.abs(d - DT) > 4 * h)


def test_consistency_of_recorded_forward():
    x, beta, packets, xr, target, J, gb, gx, a = _setup()
    assert J > 0 and np.all(np.isfinite(gb)) and np.all(np.isfinite(gx))
    assert np.abs(a.sig).max() > 1e-3          # the pulse reaches the springs


def test_beta_gradient_matches_finite_differences():
    x, beta, packets, xr, target, J, gb, gx, _ = _setup()
    rng = np.random.default_rng(11)
    for direction in [rng.standard_normal(beta.size), np.eye(beta.size)[2]]:
        h = 1e-5
        jp = _loss(x, beta * (1 + h * direction), packets, xr, target)
        jm = _loss(x, beta * (1 - h * direction), packets, xr, target)
        fd = (jp - jm) / (2 * h)
        an = float(gb @ (beta * direction))
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-300), (fd, an)


def test_position_gradient_matches_finite_differences():
    x, beta, packets, xr, target, J, gb, gx, _ = _setup()
    rng = np.random.default_rng(12)
    h = 1e-6
    assert _no_class_switch(x, h)
    for direction in [rng.standard_normal(x.size), np.eye(x.size)[1], np.eye(x.size)[4]]:
        jp = _loss(x + h * direction, beta, packets, xr, target)
        jm = _loss(x - h * direction, beta, packets, xr, target)
        fd = (jp - jm) / (2 * h)
        an = float(gx @ direction)
        assert abs(fd - an) <= 1e-6 * np.abs(gx).max() * np.abs(direction).sum(), (fd, an)


def test_weight_derivative_matches_finite_differences():
    prm = Params(dt=0.01)
    rng = np.random.default_rng(3)
    d = np.concatenate([rng.uniform(0, prm.dt, 5), rng.uniform(prm.dt, prm.delta, 10)])
    h = 1e-4 * prm.dt
    # keep points whose stencils do not change within [d - 2h, d + 2h]
    z, _ = np.polynomial.legendre.leggauss(prm.n_gl_local)
    lag = lambda dd: prm.W - (prm.W - dd[:, None] / prm.dt) * (1 + z[None, :]) / 2
    keep = np.all(np.floor(lag(d - 2 * h)) == np.floor(lag(d + 2 * h)), axis=1)
    keep &= np.abs(d - prm.dt) > 2 * h
    d = d[keep]
    assert d.size >= 10
    f = lambda dd: local_weights(dd, prm.dt, prm.W, prm.p, prm.delta, prm.b, prm.n_gl_local)
    fd = (-f(d + 2 * h) + 8 * f(d + h) - 8 * f(d - h) + f(d - 2 * h)) / (12 * h)
    an = local_weights_dd(d, prm.dt, prm.W, prm.p, prm.delta, prm.b, prm.n_gl_local)
    rel = np.abs(fd - an).max(axis=1) / np.abs(an).max(axis=1)
    assert rel.max() < 1e-8, rel
    assert math.isfinite(float(an.sum()))


def _clear_of_breaks(x, xr, j, h, prm, z):
    """True if moving spring j by up to +-2h moves no pair distance across a
    point where Q_m(d) is not smooth (d = dt, d = delta, a node's stencil
    shift)."""
    pts = np.concatenate([np.delete(x, j), xr])
    d = np.abs(pts - x[j])
    d = d[d < prm.delta + 3 * h]
    if np.any(np.abs(d - prm.dt) < 3 * h) or np.any(np.abs(d - prm.delta) < 3 * h):
        return False
    base = np.floor(prm.W - (prm.W - d[:, None] / prm.dt) * (1 + z[None, :]) / 2)
    for sg in (-2.0, 2.0):
        D = (d + sg * h) / prm.dt
        if np.any(np.floor(prm.W - (prm.W - D[:, None]) * (1 + z[None, :]) / 2) != base):
            return False
    return True


def test_position_gradient_dense_single_coordinates():
    """A dense slab (100 springs over 0.02 at dt = 4e-3: 20 springs per time
    step, every pair nearby or intermediate, the nearby system fully coupled):
    single-coordinate central differences at springs whose pairs stay clear of
    the points where Q_m(d) is not smooth agree with the gradient.  (Along a
    direction that moves every spring, differences cross such points and do
    not converge to the gradient of the smooth pieces.)"""
    rng = np.random.default_rng(9)
    M, dt, n = 100, 4e-3, 120
    x = rng.uniform(0.5, 0.52, M)
    beta = 0.05 * rng.uniform(1.0, 10.0, M)
    packets = np.array([[1.0, 0.25, 0.03, 0.0, 0.0]])
    xr = np.array([0.49, 0.51, 0.53])
    prm = Params(dt=dt)
    z, _ = np.polynomial.legendre.leggauss(prm.n_gl_local)

    def loss(xx):
        a = AdjointOracle(xx, beta, packets, prm, xr)
        u = a.forward(n)
        return 0.5 * dt * float((u * u).sum()), a, u

    J, a, u = loss(x)
    _, gx = a.gradient(dt * u)
    h = 1e-7
    chosen = [int(j) for j in np.argsort(-np.abs(gx)) if _clear_of_breaks(x, xr, int(j), h, prm, z)][:3]
    assert len(chosen) == 3 and np.abs(gx[chosen]).min() > 0.05 * np.abs(gx).max()
    for j in chosen:
        e = np.zeros(M)
        e[j] = h
        fd = (loss(x + e)[0] - loss(x - e)[0]) / (2 * h)
        assert abs(fd - gx[j]) <= 1e-6 * abs(gx[j]), (j, fd, gx[j])
