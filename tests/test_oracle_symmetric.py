"""Pins of the symmetric (mirror) boundary of the oracle (Sec. 4: the
symmetric condition on the planes x = 0, y = 0, z = 0 of the octant
problems).  A mirror-symmetric flow on a doubled domain must give, on its
upper half, exactly what the half domain with a symmetric boundary gives;
a closed box conserves mass and energy; no mass, energy or tangential
momentum crosses a symmetric face."""

import numpy as np
import pytest

import oracle
from oracle import scheme
from paper_1909_01580_amd import workloads as wl
from tests.helpers import nerr

L = 1.0
NX, NY, NZ = 6, 5, 4


def mirror_state(nx, x0, x1, ny, nz, mach=0.3):
    """Cell-centre samples of a smooth state on [x0, x1] x [0,1]^2 that is
    even in x (rho, v, w, p) and odd in x (u), with period 2L in x and
    period 1 in y and z."""
    hx = (x1 - x0) / nx
    x = x0 + (np.arange(nx) + 0.5) * hx
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    c = np.cos(np.pi * X / L)
    s = np.sin(np.pi * X / L)
    cy, cz = np.cos(2 * np.pi * Y), np.sin(2 * np.pi * Z)
    rho = 1.0 + 0.2 * c * cy + 0.1 * cz
    u = mach * s * (1.0 + 0.3 * cy)
    v = mach * 0.5 * c * cz
    w = mach * 0.4 * (1 + c) * cy
    p = 1.0 + 0.1 * c * cz
    return wl.conservative(rho, u, v, w, p)


@pytest.mark.parametrize("mu", [0.0, 2e-3])
def test_half_domain_with_symmetric_ends_equals_periodic_mirror(mu):
    """[-L, L] periodic with data even about x = 0 (and so about x = L)
    against [0, L] with symmetric boundaries at both x-ends."""
    params = oracle.Params(mu=mu)
    full = mirror_state(2 * NX, -L, L, NY, NZ)
    half = mirror_state(NX, 0.0, L, NY, NZ)
    assert np.abs(full[:, :, :, NX:] - half).max() < 1e-14
    pf = oracle.uniform_problem((2 * NX, NY, NZ), (-L, 0, 0), (2 * L, 1, 1), params=params)
    ph = oracle.uniform_problem((NX, NY, NZ), (0, 0, 0), (L, 1, 1),
                                bc=("symmetric", "periodic", "periodic"), params=params)
    dt = 0.5 * oracle.max_dt(pf, full, 0.35)
    rf = oracle.step(pf, full, dt)
    rh = oracle.step(ph, half, dt)
    assert nerr(rh, rf[:, :, :, NX:]).max() < 1e-12


def test_symmetric_low_outflow_high_equals_outflow_mirror():
    """The octant set-up: symmetric at x = 0, outflow at x = L, against the
    mirror-symmetric doubled domain [-L, L] with outflow at both ends."""
    full = mirror_state(2 * NX, -L, L, NY, NZ)
    half = mirror_state(NX, 0.0, L, NY, NZ)
    pf = oracle.uniform_problem((2 * NX, NY, NZ), (-L, 0, 0), (2 * L, 1, 1),
                                bc=("outflow", "periodic", "periodic"))
    ph = oracle.uniform_problem((NX, NY, NZ), (0, 0, 0), (L, 1, 1),
                                bc=(("symmetric", "outflow"), "periodic", "periodic"))
    dt = 0.5 * oracle.max_dt(pf, full, 0.35)
    rf = oracle.step(pf, full, dt)
    rh = oracle.step(ph, half, dt)
    assert nerr(rh, rf[:, :, :, NX:]).max() < 1e-12


def test_closed_box_conserves_mass_and_energy():
    n = (6, 5, 4)
    rng = np.random.default_rng(7)
    x = (np.arange(n[0]) + 0.5) / n[0]
    y = (np.arange(n[1]) + 0.5) / n[1]
    z = (np.arange(n[2]) + 0.5) / n[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    rho = 1.0 + 0.3 * np.exp(-((X - 0.4) ** 2 + (Y - 0.6) ** 2 + (Z - 0.5) ** 2) / 0.05)
    u = 0.2 * np.sin(2 * np.pi * Y) + 0.01 * rng.standard_normal(X.shape)
    v = 0.1 * np.cos(2 * np.pi * Z)
    w = 0.1 * X
    p = 1.0 + 0.2 * Y
    Q = wl.conservative(rho, u, v, w, p)
    prob = oracle.uniform_problem(n, (0, 0, 0), (1, 1, 1), bc=("symmetric",) * 3,
                                  params=oracle.Params(mu=1e-3))
    tot0 = np.array(oracle.totals(prob, Q))
    for _ in range(3):
        Q = oracle.step(prob, Q, 0.5 * oracle.max_dt(prob, Q, 0.35))
    tot = np.array(oracle.totals(prob, Q))
    for v in (0, 4):
        assert abs(tot[v] - tot0[v]) < 1e-13 * abs(tot0[v]), (v, tot[v] - tot0[v])
    # momentum is not conserved: the walls push back
    assert np.abs(tot[1:4] - tot0[1:4]).max() > 1e-6


def test_no_mass_energy_or_tangential_momentum_through_symmetric_faces():
    n = (5, 4, 4)
    Q = mirror_state(n[0], 0.0, L, n[1], n[2])
    prob = oracle.uniform_problem(n, (0, 0, 0), (L, 1, 1),
                                  bc=(("symmetric", "outflow"), "periodic", "periodic"))
    f = oracle.face_fluxes(prob, Q, 0.01)      # [3][nz][ny][nx][2][5]
    wall = f[0, :, :, 0]                         # x-faces at x = 0: (nz, ny, 2, 5)
    scale = np.abs(f[0]).max()
    for var in (0, 2, 3, 4):
        assert np.abs(wall[..., var]).max() < 1e-13 * scale, var
    # the normal momentum flux is the wall pressure (about 1) times the face area
    area = 1.0 / (n[1] * n[2])
    assert np.abs(wall[..., 0, 1]).min() > 0.5 * area


def test_uniform_rest_state_stays_at_rest():
    n = (4, 4, 3)
    Q = np.zeros((5,) + n[::-1])
    Q[0] = 1.3
    Q[4] = 2.0 / 0.4
    prob = oracle.uniform_problem(n, (0, 0, 0), (1, 1, 1), bc=("symmetric", ("symmetric", "outflow"), "symmetric"))
    Q1 = oracle.step(prob, Q, 0.01)
    assert np.abs(Q1 - Q).max() < 1e-14
