"""Shared helpers of the test suite: cases, comparison norms, device setup."""

import numpy as np

from paper_1909_01580_amd import workloads as wl

GAMMA = 1.4


def nerr(a, b, axis_var=0, mom_scale=False):
    """Normalised max-norm error per conservative variable: max |a - b| over
    cells divided by max |b|; momentum components share one denominator
    (the largest momentum magnitude).  With mom_scale the momentum
    denominator is at least sqrt(max rho * max rho E), the momentum a flow
    at its sound speed would carry, for states (near) at rest where the
    momentum is zero up to rounding."""
    a = np.moveaxis(np.asarray(a), axis_var, 0)
    b = np.moveaxis(np.asarray(b), axis_var, 0)
    den = [np.abs(b[v]).max() for v in range(5)]
    mom = max(den[1:4])
    if mom_scale:
        mom = max(mom, np.sqrt(den[0] * den[4]))
    out = []
    for v in range(5):
        d = den[v] if v in (0, 4) else mom
        out.append(np.abs(a[v] - b[v]).max() / max(d, 1e-300))
    return np.array(out)


def smooth_state(n, L, seed, mach=0.4, amp=0.2):
    """Seeded smooth periodic data on a box: rho, p, velocity from a few
    Fourier modes (library layout [5][nz][ny][nx])."""
    rng = np.random.default_rng(seed)
    c = [(np.arange(n[d]) + 0.5) * L[d] / n[d] for d in range(3)]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    f = []
    for _ in range(5):
        k = rng.integers(1, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        f.append(np.sin(2 * np.pi * (k[0] * X / L[0] + k[1] * Y / L[1] + k[2] * Z / L[2]) + ph))
    rho = 1 + amp * f[0]
    p = 1 + amp * f[1]
    return wl.conservative(rho, mach * f[2], mach * f[3], mach * f[4], p)


def blast_state(n, L=(1.0, 1.0, 1.0), centre=(0.45, 0.5, 0.55), radius=0.3, p_out=0.1, rho_out=0.125):
    """Discontinuous sphere (Sod-type jump) sampled at cell centres."""
    c = [(np.arange(n[d]) + 0.5) * L[d] / n[d] for d in range(3)]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    r = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2)
    inside = r < radius
    rho = np.where(inside, 1.0, rho_out)
    p = np.where(inside, 1.0, p_out)
    zero = np.zeros_like(rho)
    return wl.conservative(rho, zero, zero, zero, p)
