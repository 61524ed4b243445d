"""Stability of the discrete march for one spring (a property of the scheme of
Sections 3-4 with p-point interpolation; Section 5 analyses p = 1, 2 only).

Zero driving, a random density history: with p = 8 and dt = 1e-3 the march
decays for beta dt / 2 = 0.2 and grows for beta dt / 2 = 0.4, while p = 4 still
decays at 0.4.  Clusters of nearby stiff springs act like one spring of summed
stiffness, which is why the throughput workload keeps beta <= 10 at M = 1e4,
dt = 1e-3.  At beta dt / 2 = 0.5 (the filter demonstrations of Section 6.4:
beta = 100, dt = 0.01, free space) p = 6 decays and p = 8 grows by ~0.18 per
level, so those run at p = 6."""
import math

import numpy as np
import pytest

from oracle.march import Oracle
from oracle.params import Params


def growth_rate(beta, p, dt=1e-3, n=600):
    prm = Params(dt=dt, p=p)
    o = Oracle(np.array([0.5]), np.array([beta]), prm, lambda t: np.zeros(1))
    o.set_state(dict(L=100, hist=np.random.default_rng(0).standard_normal((prm.m_max, 1)),
                     ring=np.zeros((prm.W, prm.K + 1), complex), alpha=np.zeros(prm.K + 1, complex),
                     dalpha=np.zeros(prm.K + 1, complex)))
    v = [abs(o.step()[0][0]) for _ in range(n)]
    return (math.log(v[-1]) - math.log(v[n // 2])) / (n - n // 2)


@pytest.mark.parametrize("beta,p,stable", [(400.0, 8, True), (800.0, 8, False), (800.0, 4, True)])
def test_single_spring_stability_threshold(beta, p, stable):
    r = growth_rate(beta, p)
    assert (r < 0) == stable, r


@pytest.mark.parametrize("p,stable", [(6, True), (8, False)])
def test_filter_stiffness(p, stable):
    # free space (outgoing waves leave the box), an O(1) random history
    from oracle.params import FREE_SPACE
    prm = Params(dt=0.01, p=p, boundary=FREE_SPACE)
    o = Oracle(np.array([0.5]), np.array([100.0]), prm, lambda t: np.zeros(1))
    o.set_state(dict(L=100, hist=np.random.default_rng(0).standard_normal((prm.m_max, 1)),
                     ring=np.zeros((prm.W, prm.K + 1), complex), alpha=np.zeros(prm.K + 1, complex),
                     dalpha=np.zeros(prm.K + 1, complex)))
    with np.errstate(all="ignore"):
        v = [abs(o.step()[0][0]) for _ in range(3000)]
    if stable:
        assert v[-1] < 1e-3
    else:
        assert not v[-1] < 1e10
