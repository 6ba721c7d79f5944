"""Seeded synthetic inputs shaped like the paper's 3D tests.

This module holds input generation only: initial cell averages, vertex
positions of the deforming meshes, and the batch of random smooth problems.
It contains none of the scheme's arithmetic and is the only code that the
library harness and the test oracle both use.

Cell averages of smooth initial data use a 3x3x3 Gauss-Legendre rule on
each cell (through the trilinear cell map on deformed grids); the
discontinuous explosion is sampled at cell centres.  The advection data
use the exact cell average of the sine wave on cubes.
"""

import numpy as np

GAMMA = 1.4

_GL3_X = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)]) / 2.0   # nodes on [-1/2, 1/2]
_GL3_W = np.array([5.0, 8.0, 5.0]) / 18.0


def conservative(rho, u, v, w, p, gamma=GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def _centres(n, origin, length):
    return [origin[d] + (np.arange(n[d]) + 0.5) * (length[d] / n[d]) for d in range(3)]


def _box_average(n, origin, length, point_fn):
    """3x3x3 Gauss average over each box cell of point_fn(x, y, z) -> (5, ...).
    Returns the library layout [5][nz][ny][nx]."""
    h = [length[d] / n[d] for d in range(3)]
    cx, cy, cz = _centres(n, origin, length)
    acc = 0.0
    for a in range(3):
        for b in range(3):
            for c in range(3):
                x = cx + _GL3_X[a] * h[0]
                y = cy + _GL3_X[b] * h[1]
                z = cz + _GL3_X[c] * h[2]
                Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
                acc = acc + _GL3_W[a] * _GL3_W[b] * _GL3_W[c] * point_fn(X, Y, Z)
    return np.ascontiguousarray(acc)


# ------------------------------------------------------------ advection
def advection_exact(n, t=0.0, length=2.0, gamma=GAMMA):
    """Density wave carried by the uniform stream u = v = w = 1, p = 1 on
    [0, length]^3: rho = 1 + 0.2 sin(pi (x+y+z-3t)) (the wave moves with the
    stream; at t = 2 this is the initial field again).  Exact cell averages
    on the uniform cubic grid."""
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    h = [length / n[d] for d in range(3)]
    cx, cy, cz = _centres(n, (0.0, 0.0, 0.0), (length,) * 3)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    s = 1.0
    for d in range(3):
        arg = np.pi * h[d] / 2.0
        s *= np.sin(arg) / arg
    rho = 1.0 + 0.2 * s * np.sin(np.pi * (X + Y + Z - 3.0 * t))
    one = np.ones_like(rho)
    return np.ascontiguousarray(conservative(rho, one, one, one, one, gamma))


# ------------------------------------------------------------ Taylor-Green
def tgv_point(X, Y, Z, mach=0.1, gamma=GAMMA):
    """Taylor-Green vortex with rho0 = V0 = L = 1 and uniform temperature."""
    p0 = 1.0 / (gamma * mach * mach)
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(X)
    p = p0 + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    rho = p / p0
    return conservative(rho, u, v, w, p, gamma)


def tgv_state(n, mach=0.1, gamma=GAMMA):
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    L = 2.0 * np.pi
    return _box_average(n, (-np.pi,) * 3, (L,) * 3,
                        lambda X, Y, Z: tgv_point(X, Y, Z, mach, gamma))


TGV_MU = 1.0 / 1600.0
TGV_PRANDTL = 0.72  # the benchmark configuration's Prandtl number (Sec. 4.6 prints 0.71)


# ------------------------------------------------------------ explosion
def explosion_state(n, radius=0.4, centre=(0.5, 0.5, 0.5), gamma=GAMMA):
    """Spherical Sod-type explosion on [0,1]^3, sampled at cell centres:
    inside rho = 1, p = 1; outside rho = 0.125, p = 0.1; at rest."""
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    cx, cy, cz = _centres(n, (0.0,) * 3, (1.0,) * 3)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    r = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2)
    inside = r < radius
    rho = np.where(inside, 1.0, 0.125)
    p = np.where(inside, 1.0, 0.1)
    zero = np.zeros_like(rho)
    return np.ascontiguousarray(conservative(rho, zero, zero, zero, p, gamma))


def spherical_sod_state(n, gamma=GAMMA):
    """Spherically symmetric Sod problem in the octant [0,1]^3 (symmetric
    planes x = y = z = 0, outflow at 1): rho = 1, p = 1 for r < 0.5,
    rho = 0.125, p = 0.1 beyond, at rest; sampled at cell centres."""
    return explosion_state(n, radius=0.5, centre=(0.0, 0.0, 0.0), gamma=gamma)


SEDOV_ENERGY = 0.106384  # energy released in the octant


def sedov_state(n, length=1.2, energy=SEDOV_ENERGY, p_background=1e-6, gamma=GAMMA):
    """Sedov blast in the octant [0, length]^3 (symmetric planes x = y = z =
    0, outflow at `length`): rho = 1 and p = 1e-6 everywhere except the cell
    at the origin, whose pressure (gamma - 1) energy / V puts the released
    energy into that one cell; at rest."""
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    shape = n[::-1]
    rho = np.ones(shape)
    p = np.full(shape, p_background)
    vol = np.prod([length / n[d] for d in range(3)])
    p[0, 0, 0] = (gamma - 1.0) * energy / vol
    zero = np.zeros(shape)
    return np.ascontiguousarray(conservative(rho, zero, zero, zero, p, gamma))


# ------------------------------------------------ isotropic turbulence
ISO_A0, ISO_K0, ISO_RE_LAMBDA = 1.3e-4, 8.0, 72.0
ISO_PRANDTL, ISO_MU_EXPONENT = 0.71, 0.76


def isotropic_turbulence_params(mach_t, A0=ISO_A0, k0=ISO_K0, re_lambda=ISO_RE_LAMBDA, gamma=GAMMA, rho0=1.0):
    """Scales of the compressible isotropic turbulence of Sec. 4 from the
    spectrum E(k) = A0 k^4 exp(-2 k^2 / k0^2): initial kinetic energy
    K0 = 3 A0 sqrt(2 pi) k0^5 / 64, u_rms = sqrt(2 K0 / 3), the large-eddy
    turnover time sqrt(32 / A0) (2 pi)^(1/4) k0^(-7/2); T0 from
    Ma_t = sqrt(3) u_rms / sqrt(gamma T0) and mu0 from
    Re_lambda = (2 pi)^(1/4) / 4 (rho0 / mu0) sqrt(2 A0) k0^(3/2) (unit gas
    constant, so p = rho T)."""
    K0 = 3.0 * A0 / 64.0 * np.sqrt(2 * np.pi) * k0 ** 5
    u_rms = np.sqrt(2.0 * K0 / 3.0)
    T0 = 3.0 * u_rms ** 2 / (gamma * mach_t ** 2)
    mu0 = (2 * np.pi) ** 0.25 / 4.0 * rho0 * np.sqrt(2.0 * A0) * k0 ** 1.5 / re_lambda
    tau_t0 = np.sqrt(32.0 / A0) * (2 * np.pi) ** 0.25 * k0 ** -3.5
    return {"K0": K0, "u_rms": u_rms, "T0": T0, "p0": rho0 * T0, "rho0": rho0, "mu0": mu0,
            "tau_t0": tau_t0, "mu_exponent": ISO_MU_EXPONENT, "prandtl": ISO_PRANDTL}


def isotropic_turbulence_state(n, mach_t, seed=190901580, A0=ISO_A0, k0=ISO_K0, gamma=GAMMA):
    """Seeded divergence-free random velocity on the periodic box
    [-pi, pi]^3 with the spectrum A0 k^4 exp(-2 k^2 / k0^2) (each Fourier
    mode: Gaussian random complex amplitude, projected normal to its wave
    vector, scaled to the spectrum's energy per mode E(|k|) / (4 pi |k|^2);
    no Nyquist modes), the real part sampled at cell centres and scaled to
    the u_rms of the spectrum; uniform
    density rho0 = 1 and temperature T0 from Ma_t.  Returns the conservative
    state [5][n][n][n] and the parameters."""
    P = isotropic_turbulence_params(mach_t, A0=A0, k0=k0, gamma=gamma)
    rng = np.random.default_rng(seed)
    k1 = np.fft.fftfreq(n, 1.0 / n)
    KZ, KY, KX = np.meshgrid(k1, k1, k1, indexing="ij")
    kk = np.stack([KX, KY, KZ])
    k2 = (kk ** 2).sum(axis=0)
    kmag = np.sqrt(k2)
    a = rng.standard_normal((3, n, n, n)) + 1j * rng.standard_normal((3, n, n, n))
    with np.errstate(invalid="ignore", divide="ignore"):
        a -= kk * (kk * a).sum(axis=0) / np.where(k2 > 0, k2, 1.0)
        norm = np.sqrt((np.abs(a) ** 2).sum(axis=0))
        E = A0 * kmag ** 4 * np.exp(-2.0 * k2 / k0 ** 2)
        amp = np.where(k2 > 0, np.sqrt(E / (4 * np.pi * np.where(k2 > 0, k2, 1.0))) / np.where(norm > 0, norm, 1.0),
                       0.0)
    a *= amp
    # no Nyquist modes: their partner -k is not on the grid
    a[:, np.abs(kk).max(axis=0) >= n // 2] = 0.0
    # the FFT nodes are taken as the cell centres (a translation of a
    # statistically homogeneous field)
    u = np.real(np.fft.ifftn(a, axes=(1, 2, 3))) * n ** 3
    urms = np.sqrt((u ** 2).sum(axis=0).mean() / 3.0)
    u *= P["u_rms"] / urms
    rho = np.full((n, n, n), P["rho0"])
    p = np.full((n, n, n), P["p0"])
    return np.ascontiguousarray(conservative(rho, u[0], u[1], u[2], p, gamma)), P


# ------------------------------------------------------------ deformed grids
def sine_mesh_vertices(n, t, amp=0.1, omega=np.pi, length=2.0, static=False):
    """Vertices x = xi + amp sin(pi xi) sin(pi eta) sin(pi zeta) s(t) (all
    three components), s(t) = sin(omega t), or 1 for the static non-coplanar
    mesh.  Periodic grid on [0, length]^3 with n vertices per axis.
    Library layout [3][nz][ny][nx]."""
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    xi = [np.arange(n[d]) * (length / n[d]) for d in range(3)]
    Z, Y, X = np.meshgrid(xi[2], xi[1], xi[0], indexing="ij")
    s = 1.0 if static else np.sin(omega * t)
    disp = amp * np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z) * s
    return np.ascontiguousarray(np.stack([X + disp, Y + disp, Z + disp]))


def _cell_corners(verts, period):
    """The eight corner arrays (3, i, j, k) of every cell of a periodic
    vertex grid (library layout), keyed by the corner bits (a, b, c)."""
    v = np.transpose(verts, (0, 3, 2, 1))  # (3, i, j, k)
    n = v.shape[1:]
    corners = {}
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                arr = np.roll(v, shift=(-a, -b, -c), axis=(1, 2, 3)).copy()
                for d, bit in enumerate((a, b, c)):
                    if bit:
                        last = [slice(None)] * 3
                        last[d] = n[d] - 1
                        arr[(d,) + tuple(last)] += period[d]
                corners[(a, b, c)] = arr
    return corners


def _trilinear_points(verts, period, node, corners=None):
    """Physical points and |J| at parametric offsets ``node`` (3,) in every
    cell of a periodic vertex grid (library layout)."""
    if corners is None:
        corners = _cell_corners(verts, period)
    xi, eta, zeta = node
    X = 0.0
    dX = [0.0, 0.0, 0.0]
    for (a, b, c), xm in corners.items():
        sa, sb, sc = (2 * a - 1), (2 * b - 1), (2 * c - 1)
        fa, fb, fc = 1 + 2 * sa * xi, 1 + 2 * sb * eta, 1 + 2 * sc * zeta
        X = X + fa * fb * fc / 8.0 * xm
        dX[0] = dX[0] + 2 * sa * fb * fc / 8.0 * xm
        dX[1] = dX[1] + 2 * sb * fa * fc / 8.0 * xm
        dX[2] = dX[2] + 2 * sc * fa * fb / 8.0 * xm
    J = np.einsum("i...,i...->...", dX[0], np.cross(dX[1], dX[2], axis=0))
    return X, np.abs(J)


def hex_average(verts, period, point_fn):
    """3x3x3 Gauss cell averages on a periodic hexahedral grid.
    Returns the library layout [5][nz][ny][nx]."""
    acc = 0.0
    vol = 0.0
    corners = _cell_corners(verts, period)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                X, J = _trilinear_points(verts, period, (_GL3_X[a], _GL3_X[b], _GL3_X[c]), corners)
                w = _GL3_W[a] * _GL3_W[b] * _GL3_W[c] * J
                acc = acc + w * point_fn(X[0], X[1], X[2])
                vol = vol + w
    out = acc / vol
    return np.ascontiguousarray(np.transpose(out, (0, 3, 2, 1)))


def advection_point(X, Y, Z, t=0.0, gamma=GAMMA):
    rho = 1.0 + 0.2 * np.sin(np.pi * (X + Y + Z - 3.0 * t))
    one = np.ones_like(rho)
    return conservative(rho, one, one, one, one, gamma)


def pulse_point(X, Y, Z, gamma=GAMMA):
    """Uniform stream (1, 0.5, 0.25), p = 1, with a smooth density pulse
    centred at (1, 1, 1)."""
    r2 = (X - 1.0) ** 2 + (Y - 1.0) ** 2 + (Z - 1.0) ** 2
    rho = 1.0 + 0.2 * np.exp(-r2 / 0.04)
    one = np.ones_like(rho)
    return conservative(rho, one, 0.5 * one, 0.25 * one, one, gamma)


def uniform_point(X, Y, Z, gamma=GAMMA):
    one = np.ones_like(X)
    return conservative(one, one, one, one, one, gamma)


# ------------------------------------------------------------ batch
def batch_problems(seed=190901580, count=48, sizes=(32, 48, 64, 96), h=2 * np.pi / 64,
                   gamma=GAMMA, average=False):
    """Independent periodic problems of uneven box sizes with random smooth
    data: four Fourier modes per field with integer wave vectors in
    {-2..2}^3 (fitted to each box) and random phases; rho = 1 + 0.1 phi_rho,
    p = (1 + 0.1 phi_p)/gamma, velocity = Ma phi_u with Ma in [0.1, 0.5];
    even problems inviscid, odd ones viscous with mu = 1/1600.  Values are
    sampled at cell centres (or 3x3x3 Gauss averages with average=True).
    Returns a list of dicts (n, length, mu, mach, state)."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(count):
        n = tuple(int(s) for s in rng.choice(sizes, size=3))
        length = tuple(n[d] * h for d in range(3))
        mach = rng.uniform(0.1, 0.5)
        fields = {}
        for name in ("rho", "p", "u", "v", "w"):
            kv = []
            while len(kv) < 4:
                k = tuple(int(x) for x in rng.integers(-2, 3, size=3))
                if k != (0, 0, 0):
                    kv.append(k)
            ph = rng.uniform(0.0, 2 * np.pi, size=4)
            fields[name] = (kv, ph)

        def point(X, Y, Z, fields=fields, length=length, mach=mach):
            vals = {}
            for name, (kv, ph) in fields.items():
                s = 0.0
                for k, phase in zip(kv, ph):
                    s = s + np.sin(2 * np.pi * (k[0] * X / length[0] + k[1] * Y / length[1]
                                                + k[2] * Z / length[2]) + phase)
                vals[name] = s / 4.0
            rho = 1.0 + 0.1 * vals["rho"]
            p = (1.0 + 0.1 * vals["p"]) / gamma
            return conservative(rho, mach * vals["u"], mach * vals["v"], mach * vals["w"], p, gamma)

        if average:
            state = _box_average(n, (0.0,) * 3, length, point)
        else:
            cx, cy, cz = _centres(n, (0.0,) * 3, length)
            Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
            state = np.ascontiguousarray(point(X, Y, Z))
        out.append({"n": n, "length": length, "mu": 0.0 if g % 2 == 0 else 1.0 / 1600.0,
                    "mach": mach, "state": state})
    return out
