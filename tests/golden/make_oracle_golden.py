"""Writes oracle results used as stored expected values by the GPU tests.

Calls only the oracle and the seeded input generators.

* config1_advection16_20steps.npz: the Sec. 4.1 density wave on the
  uniform 16^3 grid of [0,2]^3 (periodic, gamma 1.4, inviscid), 20 two-stage
  steps with dt = 0.5 * (time-step bound of the current state); stores the
  initial state, the dt sequence and the final state.
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1909_01580_amd import workloads as wl  # noqa: E402


def config1():
    n = 16
    Q0 = wl.advection_exact(n)
    prob = oracle.uniform_problem((n, n, n), (0.0, 0.0, 0.0), (2.0, 2.0, 2.0))
    Q = Q0
    dts = []
    for _ in range(20):
        dt = oracle.max_dt(prob, Q, 0.5)
        dts.append(dt)
        Q = oracle.step(prob, Q, dt)
    np.savez_compressed(os.path.join(HERE, "config1_advection16_20steps.npz"), q0=Q0, dt=np.array(dts), q=Q)


if __name__ == "__main__":
    config1()
