"""The Sedov start (Sec. 4) in the oracle: the two-stage step at the printed
CFL of 0.01 loses positivity in the first step, and the step-rejection rule
recovers it.

Pins: the one-stage step and the intermediate state stay physical while the
two-stage result does not, and the failure sits in the six cells two faces
away from the energy cell (the mechanism stated in ``checked_step``); the rule takes
the largest dt / 2^k whose plain step is physical and returns that step
unchanged; the octant's symmetry under exchange of axes and the mass and
energy totals survive the step.
"""

import numpy as np
import pytest

import oracle
from paper_1909_01580_amd import workloads as wl

N, L = 12, 1.2
OCTANT = (("symmetric", "outflow"),) * 3


@pytest.fixture(scope="module")
def start():
    q = wl.sedov_state(N, length=L)
    prob = oracle.uniform_problem((N,) * 3, (0, 0, 0), (L,) * 3, bc=OCTANT)
    return prob, q, oracle.max_dt(prob, q, 0.01)


def pressure(q):
    return 0.4 * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0])


def test_two_stage_step_loses_positivity(start):
    prob, q, dt = start
    assert oracle.physical(oracle.step(prob, q, dt, n_stages=1), 1.4)
    assert oracle.physical(oracle.step(prob, q, 0.5 * dt, n_stages=1), 1.4)
    with np.errstate(all="ignore"):
        q2 = oracle.step(prob, q, dt)
    p = pressure(q2)
    bad = {tuple(int(v) for v in c) for c in np.argwhere(~(p > 0))}
    # exactly the cells two faces away from the energy cell (i + j + k = 2)
    assert bad == {c for c in np.ndindex(3, 3, 3) if sum(c) == 2}, bad


def test_checked_step_is_minimal_halving(start):
    prob, q, dt = start
    q1, taken = oracle.checked_step(prob, q, dt)
    k = np.log2(dt / taken)
    assert k >= 1 and k == int(k)
    assert oracle.physical(q1, 1.4)
    np.testing.assert_array_equal(q1, oracle.step(prob, q, taken))
    with np.errstate(all="ignore"):
        assert not oracle.physical(oracle.step(prob, q, 2 * taken), 1.4)
    assert oracle.checked_step(prob, q, dt, max_halvings=int(k) - 1) == (None, None)


def test_checked_step_keeps_octant_symmetry_and_totals(start):
    prob, q, dt = start
    q1, _ = oracle.checked_step(prob, q, dt)
    # exchanging x and y maps the octant onto itself: state arrays transpose
    # in (j, i) and the x and y momenta swap
    sw = q1[[0, 2, 1, 3, 4]].transpose(0, 1, 3, 2)
    scale = np.abs(q1).max(axis=(1, 2, 3))[:, None, None, None]
    assert np.abs(sw - q1).max() / scale.max() < 1e-13
    assert (np.abs(sw - q1) / scale).max() < 1e-11
    t0, t1 = oracle.totals(prob, q), oracle.totals(prob, q1)
    for v in (0, 4):
        assert abs(t1[v] - t0[v]) < 1e-13 * abs(t0[v]), (v, t1[v] - t0[v])
