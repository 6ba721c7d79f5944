"""Checks of the radial reference solver used by the octant tests: a state
at rest stays at rest, and the spherical Sod solution is converged at the
resolution the tests use (2,000 cells against 4,000)."""

import numpy as np

from tests import radial_reference as rr


def test_rest_state_stays():
    r, rho, u, p = rr.solve(lambda r: np.full_like(r, 1.3), lambda r: np.full_like(r, 0.7), 1.0, 0.1, cells=200)
    assert np.abs(rho - 1.3).max() < 1e-13 and np.abs(u).max() < 1e-13 and np.abs(p - 0.7).max() < 1e-13


def test_spherical_sod_converged():
    rho0 = lambda r: np.where(r < 0.5, 1.0, 0.125)   # noqa: E731
    p0 = lambda r: np.where(r < 0.5, 1.0, 0.1)       # noqa: E731
    r1, d1, _, _ = rr.solve(rho0, p0, 1.0, 0.25, cells=2000)
    r2, d2, _, _ = rr.solve(rho0, p0, 1.0, 0.25, cells=4000)
    assert np.abs(np.interp(r1, r2, d2) - d1).mean() < 1e-3
    # the rarefaction head moves inward at the sound speed sqrt(1.4) of the
    # inner state and has not yet reached r = 0.5 - 1.183 * 0.25 = 0.204;
    # behind the outward shock (near r = 0.88) the gas is compressed
    assert np.abs(d1[r1 < 0.15] - 1.0).max() < 1e-9 and d1[np.searchsorted(r1, 0.22)] < 0.99
    assert d1[(r1 > 0.8) & (r1 < 0.85)].min() > 0.2 and d1[r1 > 0.92].max() < 0.126
