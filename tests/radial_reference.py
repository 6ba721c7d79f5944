"""Reference solution of a spherically symmetric flow: the one-dimensional
Euler equations in r with the geometric source term,
    Q_t + F(Q)_r = -(d - 1)/r (rho U, rho U^2, U (E + p)),  d = 3,
which the paper uses for its spherical Sod problem (Sec. 4).  Solved on a
fine radial grid by a second-order finite-volume scheme written for this
test: minmod-limited linear reconstruction of the primitive variables, HLL
fluxes, the source at the cell centre, two-stage SSP Runge-Kutta; mirror
ghost cells at r = 0 and zero-gradient ghosts at the outer radius.  Test
infrastructure; independent of the HGKS oracle and of the GPU path."""

import numpy as np


def _prim(Q, gamma):
    rho = Q[0]
    u = Q[1] / rho
    p = (gamma - 1.0) * (Q[2] - 0.5 * rho * u * u)
    return rho, u, p


def _flux(rho, u, p, gamma):
    E = p / (gamma - 1.0) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)]), np.array([rho, rho * u, E])


def _minmod(a, b):
    return np.where(a * b > 0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def _rhs(Q, r, dr, gamma):
    rho, u, p = _prim(Q, gamma)
    W = np.array([rho, u, p])
    # ghosts: mirror at r = 0 (u reversed), zero gradient outside
    Wg = np.concatenate([W[:, 1::-1] * np.array([[1], [-1], [1]]), W, W[:, -1:], W[:, -1:]], axis=1)
    s = _minmod(Wg[:, 1:-1] - Wg[:, :-2], Wg[:, 2:] - Wg[:, 1:-1])    # cells -1 .. N
    WL = Wg[:, 1:-2] + 0.5 * s[:, :-1]                                 # left state of faces 0..N
    WR = Wg[:, 2:-1] - 0.5 * s[:, 1:]
    FL, UL = _flux(WL[0], WL[1], WL[2], gamma)
    FR, UR = _flux(WR[0], WR[1], WR[2], gamma)
    cL = np.sqrt(gamma * WL[2] / WL[0])
    cR = np.sqrt(gamma * WR[2] / WR[0])
    sL = np.minimum(WL[1] - cL, WR[1] - cR)
    sR = np.maximum(WL[1] + cL, WR[1] + cR)
    F = np.where(sL >= 0, FL, np.where(sR <= 0, FR, (sR * FL - sL * FR + sL * sR * (UR - UL)) / (sR - sL)))
    F[:, 0] = np.array([0.0, F[1, 0], 0.0])                           # wall at r = 0: no mass or energy flux
    E = p / (gamma - 1.0) + 0.5 * rho * u * u
    src = -(2.0 / r) * np.array([rho * u, rho * u * u, u * (E + p)])
    return -(F[:, 1:] - F[:, :-1]) / dr + src, np.max(np.abs(u) + np.sqrt(gamma * p / rho))


def solve(rho0, p0, r_max, t_end, cells=2000, gamma=1.4, cfl=0.4):
    """Density, velocity and pressure at time t_end on cell centres r from
    initial profiles rho0(r), p0(r) at rest."""
    dr = r_max / cells
    r = (np.arange(cells) + 0.5) * dr
    rho, p = rho0(r), p0(r)
    Q = np.array([rho, np.zeros_like(r), p / (gamma - 1.0)])
    t = 0.0
    while t < t_end - 1e-14:
        k1, smax = _rhs(Q, r, dr, gamma)
        dt = min(cfl * dr / smax, t_end - t)
        Q1 = Q + dt * k1
        k2, _ = _rhs(Q1, r, dr, gamma)
        Q = 0.5 * (Q + Q1 + dt * k2)
        t += dt
    rho, u, p = _prim(Q, gamma)
    return r, rho, u, p
