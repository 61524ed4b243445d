"""Writes stored expected values computed by the CPU oracle only.

    python tests/golden/make_golden.py multiband

multiband: the periodic multiband workload (M = 1e4, dt = 1e-3, 1e4 steps)
marched by the oracle for levels 0..n_steps; stores sigma at a few levels for
all scatterers, every 100th level for 200 sampled scatterers, and the max
|sigma| over all levels.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.march import Oracle, incident_driving  # noqa: E402
from oracle.params import Params  # noqa: E402
from paper_2507_07823_amd import workloads  # noqa: E402

FULL_LEVELS = (250, 1000, 4000, 10000)


def multiband():
    p = workloads.multiband_periodic()
    prm = Params(dt=p["dt"])
    t0 = time.time()
    o = Oracle(p["x"], p["beta"], prm, incident_driving(p["x"], p["beta"], p["packets"], True))
    print(f"precompute {time.time() - t0:.1f}s", flush=True)
    n = p["n_steps"] + 1
    sample = np.random.default_rng(12345).choice(p["x"].size, 200, replace=False)
    sample.sort()
    full, strided, smax = {}, [], 0.0
    t0 = time.time()
    for L in range(n):
        s, _ = o.step()
        smax = max(smax, float(np.max(np.abs(s))))
        if L in FULL_LEVELS:
            full[L] = s.copy()
        if L % 100 == 0:
            strided.append(s[sample])
        if L % 500 == 0:
            print(f"level {L} {time.time() - t0:.0f}s", flush=True)
    np.savez_compressed(os.path.join(HERE, "multiband_sigma.npz"),
                        full_levels=np.array(FULL_LEVELS),
                        full=np.array([full[L] for L in FULL_LEVELS]),
                        sample=sample, strided=np.array(strided), strided_every=100,
                        sigma_max=smax, n_levels=n)


if __name__ == "__main__":
    {"multiband": multiband}[sys.argv[1]]()
