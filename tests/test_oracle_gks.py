"""Pins for the oracle gas-kinetic flux (Sec. 3).

* one-dimensional Maxwellian moments (full and half line) against adaptive
  numerical integration;
* micro-slopes against a closed-form inverse of the moment system derived
  by hand, and the round trip <a psi> = b by velocity-space quadrature;
* the whole flux against an independent brute-force evaluation of the
  paper's definition: slopes, equilibrium state and every moment by
  Gauss-Hermite / Gauss-Legendre velocity quadrature, time factors by
  adaptive quadrature in t, then the two-interval linear fit;
* closed forms: a uniform state gives the Euler flux with dF = 0; a weak
  linear shear gives the Navier-Stokes stress -mu dV/dx with mu = tau p
  (first-order Chapman-Enskog truncation, Sec. 3);
* symmetries: mirror (swap sides, reverse the normal) and rotation of the
  tangential axes about the normal.
"""

import numpy as np
import pytest
from scipy import integrate

from oracle import gks

GAMMA = 1.4
K = (5 - 3 * GAMMA) / (GAMMA - 1)


def test_one_dimensional_moments():
    for U, lam in ((0.3, 0.7), (-1.2, 2.5), (0.0, 40.0)):
        m = gks.Moments(np.array(U), np.array(0.1), np.array(-0.2), np.array(lam), K)
        mp = gks.Moments(np.array(U), np.array(0.1), np.array(-0.2), np.array(lam), K, half="+")
        mn = gks.Moments(np.array(U), np.array(0.1), np.array(-0.2), np.array(lam), K, half="-")
        pdf = lambda u: np.sqrt(lam / np.pi) * np.exp(-lam * (u - U) ** 2)  # noqa: E731
        for k in range(7):
            full = integrate.quad(lambda u: u ** k * pdf(u), -np.inf, np.inf, epsabs=1e-14, epsrel=1e-13)[0]
            pos = integrate.quad(lambda u: u ** k * pdf(u), 0, np.inf, epsabs=1e-14, epsrel=1e-13)[0]
            neg = integrate.quad(lambda u: u ** k * pdf(u), -np.inf, 0, epsabs=1e-14, epsrel=1e-13)[0]
            scale = max(1.0, abs(full))
            assert abs(m.u[k] - full) < 1e-12 * scale
            assert abs(mp.u[k] - pos) < 1e-12 * scale
            assert abs(mn.u[k] - neg) < 1e-12 * scale


def test_internal_moments_two_dimensional_gauss_hermite():
    """K = 2 at gamma = 1.4: xi^2 = xi_1^2 + xi_2^2 with two Gaussians."""
    lam = 1.7
    x, w = np.polynomial.hermite.hermgauss(6)
    X1, X2 = np.meshgrid(x / np.sqrt(lam), x / np.sqrt(lam))
    W = np.outer(w, w) / np.pi
    xi2 = X1 ** 2 + X2 ** 2
    m = gks.Moments(np.array(0.0), np.array(0.0), np.array(0.0), np.array(lam), K)
    assert abs((W * xi2).sum() - m.x[1]) < 1e-14
    assert abs((W * xi2 ** 2).sum() - m.x[2]) < 1e-14


def closed_form_slope(b, U, V, W, lam):
    """Inverse of <a psi> = b (b = dW/rho) for a = a1 + a2 u + a3 v + a4 w +
    a5 (u^2+v^2+w^2+xi^2)/2, worked out by hand from the Gaussian moments."""
    q = U * U + V * V + W * W + (K + 3.0) / (2.0 * lam)
    R2, R3, R4 = b[1] - U * b[0], b[2] - V * b[0], b[3] - W * b[0]
    R5 = 2.0 * b[4] - q * b[0]
    a5 = 4.0 * lam * lam / (K + 3.0) * (R5 - 2 * U * R2 - 2 * V * R3 - 2 * W * R4)
    a4 = 2 * lam * R4 - W * a5
    a3 = 2 * lam * R3 - V * a5
    a2 = 2 * lam * R2 - U * a5
    a1 = b[0] - U * a2 - V * a3 - W * a4 - 0.5 * a5 * q
    return np.array([a1, a2, a3, a4, a5])


def test_micro_slope_closed_form():
    rng = np.random.default_rng(20)
    for _ in range(5):
        U, V, W = rng.standard_normal(3)
        lam = rng.uniform(0.3, 3.0)
        b = rng.standard_normal(5)
        m = gks.Moments(np.array([U]), np.array([V]), np.array([W]), np.array([lam]), K)
        a = gks.solve5(gks.moment_matrix(m), b[:, None])[:, 0]
        assert np.allclose(a, closed_form_slope(b, U, V, W, lam), rtol=1e-12, atol=1e-12)


# ------------------------------------------------------- brute force
class Quad:
    """Velocity-space quadrature for one Maxwellian: a list of nodes
    (u, v, w, xi^2) with weights (including rho), over the full space or a
    half line in u."""

    def __init__(self, rho, U, V, W, lam, half=None, nh=10, ngl=160, nxi=4):
        xh, wh = np.polynomial.hermite.hermgauss(nh)
        s = 1.0 / np.sqrt(lam)
        tv, wv = V + xh * s, wh / np.sqrt(np.pi)
        tw, ww = W + xh * s, wh / np.sqrt(np.pi)
        if half is None:
            tu, wu = U + xh * s, wh / np.sqrt(np.pi)
        else:
            lo, hi = (0.0, max(U, 0.0) + 14 * s) if half == "+" else (min(U, 0.0) - 14 * s, 0.0)
            xg, wg = np.polynomial.legendre.leggauss(ngl)
            tu = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
            wu = 0.5 * (hi - lo) * wg * np.sqrt(lam / np.pi) * np.exp(-lam * (tu - U) ** 2)
        xx, wx = np.polynomial.hermite.hermgauss(nxi)
        x1, x2 = np.meshgrid(xx * s, xx * s)
        xi2 = (x1 ** 2 + x2 ** 2).ravel()
        wxi = (np.outer(wx, wx) / np.pi).ravel()
        grids = np.meshgrid(tu, tv, tw, xi2, indexing="ij")
        wts = np.einsum("a,b,c,d->abcd", wu, wv, ww, wxi)
        self.u, self.v, self.w, self.xi2 = (g.ravel() for g in grids)
        self.wt = rho * wts.ravel()

    def psi(self):
        return np.stack([np.ones_like(self.u), self.u, self.v, self.w,
                         0.5 * (self.u ** 2 + self.v ** 2 + self.w ** 2 + self.xi2)])

    def vel(self, j):
        return (self.u, self.v, self.w)[j]

    def moments(self, weight):
        """int psi * weight * g  -> (5,)."""
        return (self.psi() * weight * self.wt).sum(axis=1)

    def integral(self, weight):
        """int weight * g (scalar)."""
        return (weight * self.wt).sum()


def prim(Wc):
    rho = Wc[0]
    U, V, W = Wc[1:4] / rho
    p = (GAMMA - 1) * (Wc[4] - 0.5 * rho * (U * U + V * V + W * W))
    return rho, U, V, W, p, rho / (2 * p)


def brute_flux(Wl, dWl, Wr, dWr, dt, mu, tau_eps=0.01, tau_C=1.0, prandtl=1.0, mu_T0=1.0, mu_exponent=0.0):
    sides = []
    for Wc, dWc, half in ((Wl, dWl, "+"), (Wr, dWr, "-")):
        rho, U, V, W, p, lam = prim(Wc)
        full = Quad(rho, U, V, W, lam)
        part = Quad(rho, U, V, W, lam, half=half)
        psi = full.psi()
        M = np.einsum("ai,bi,i->ab", psi, psi, full.wt)          # int psi psi g
        a = [np.linalg.solve(M, dWc[j]) for j in range(3)]
        rhsA = -sum(full.moments((a[j] @ psi) * full.vel(j)) for j in range(3))
        A = np.linalg.solve(M, rhsA)
        sides.append({"p": p, "part": part, "a": a, "A": A})
    Q0 = sum(s["part"].moments(1.0) for s in sides)
    dQ0 = [sum(s["part"].moments(s["a"][j] @ s["part"].psi()) for s in sides) for j in range(3)]
    r0, U0, V0, W0, p0, lam0 = prim(Q0)
    g0 = Quad(r0, U0, V0, W0, lam0)
    psi0 = g0.psi()
    M0 = np.einsum("ai,bi,i->ab", psi0, psi0, g0.wt)
    ab = [np.linalg.solve(M0, dQ0[j]) for j in range(3)]
    Ab = np.linalg.solve(M0, -sum(g0.moments((ab[j] @ psi0) * g0.vel(j)) for j in range(3)))
    pl, pr = sides[0]["p"], sides[1]["p"]
    jump = abs((pl - pr) / (pl + pr)) * dt
    mu_g = mu * ((p0 / r0) / mu_T0) ** mu_exponent
    tau = mu_g / p0 + tau_C * jump if mu > 0 else tau_eps * dt + tau_C * jump

    u0 = g0.u
    m_eq = g0.moments(u0)
    m_ab = g0.moments(u0 * sum((ab[j] @ psi0) * g0.vel(j) for j in range(3)))
    m_Ab = g0.moments(u0 * (Ab @ psi0))
    m_ne = sum(s["part"].moments(s["part"].u) for s in sides)
    m_nea = sum(s["part"].moments(s["part"].u * sum((s["a"][j] @ s["part"].psi()) * s["part"].vel(j)
                                                      for j in range(3))) for s in sides)
    m_neA = sum(s["part"].moments(s["part"].u * (s["A"] @ s["part"].psi())) for s in sides)

    # heat flux carried by each particle, relative to the velocity of g_0
    def hq(qd):
        return 0.5 * (qd.u - U0) * ((qd.u - U0) ** 2 + (qd.v - V0) ** 2 + (qd.w - W0) ** 2 + qd.xi2)
    y = [g0.integral(hq(g0)),
         g0.integral(hq(g0) * sum((ab[j] @ psi0) * g0.vel(j) for j in range(3))),
         g0.integral(hq(g0) * (Ab @ psi0)),
         sum(s["part"].integral(hq(s["part"])) for s in sides),
         sum(s["part"].integral(hq(s["part"]) * sum((s["a"][j] @ s["part"].psi()) * s["part"].vel(j)
                                                     for j in range(3))) for s in sides),
         sum(s["part"].integral(hq(s["part"]) * (s["A"] @ s["part"].psi())) for s in sides)]
    heat = np.zeros(5)
    heat[4] = 1.0 / prandtl - 1.0
    m_eq, m_ab, m_Ab, m_ne, m_nea, m_neA = (m + heat * yk for m, yk in
                                            zip((m_eq, m_ab, m_Ab, m_ne, m_nea, m_neA), y))

    def tint(fn, delta):
        return integrate.quad(fn, 0.0, delta, epsabs=0.0, epsrel=1e-13, limit=200,
                              points=[min(delta, tau)])[0]

    def Fhat(delta):
        e = lambda t: np.exp(-t / tau)  # noqa: E731
        return (tint(lambda t: 1 - e(t), delta) * m_eq
                + tint(lambda t: (t + tau) * e(t) - tau, delta) * m_ab
                + tint(lambda t: t - tau + tau * e(t), delta) * m_Ab
                + tint(e, delta) * m_ne
                - tint(lambda t: (tau + t) * e(t), delta) * m_nea
                - tint(lambda t: tau * e(t), delta) * m_neA)

    F1, F2 = Fhat(dt), Fhat(0.5 * dt)
    F = (4 * F2 - F1) / dt
    dF = 4 * (F1 - 2 * F2) / dt ** 2
    return F, dF, Q0


def random_state(rng, rho=1.0, p=1.0, umag=0.6):
    U = umag * rng.standard_normal(3)
    r = rho * (1 + 0.2 * rng.uniform(-1, 1))
    pp = p * (1 + 0.2 * rng.uniform(-1, 1))
    return np.array([r, r * U[0], r * U[1], r * U[2], pp / (GAMMA - 1) + 0.5 * r * U @ U])


@pytest.mark.parametrize("case", [0, 1, 2, 3])
def test_flux_against_brute_force(case):
    rng = np.random.default_rng(30 + case)
    Wl, Wr = random_state(rng), random_state(rng)
    if case == 2:
        Wr = Wl * (1 + 1e-3)                         # smooth interface
    dWl = 0.5 * rng.standard_normal((3, 5))
    dWr = 0.5 * rng.standard_normal((3, 5))
    dt = 0.01
    mu = 0.0 if case not in (1, 3) else 2e-4
    # case 3: the viscosity law and Prandtl number of the isotropic-turbulence
    # test (mu (T/T0)^0.76, Pr 0.71): the heat-flux moments by quadrature
    extra = dict(prandtl=0.71, mu_T0=0.8, mu_exponent=0.76) if case == 3 else {}
    F, dF, Q0 = gks.gks_flux(Wl[:, None], dWl[:, :, None], Wr[:, None], dWr[:, :, None], dt, GAMMA, mu, **extra)
    Fb, dFb, Q0b = brute_flux(Wl, dWl, Wr, dWr, dt, mu, **extra)
    assert np.allclose(Q0[:, 0], Q0b, rtol=1e-11, atol=1e-12)
    assert np.allclose(F[:, 0], Fb, rtol=1e-9, atol=1e-10)
    scale = np.abs(dFb).max()
    assert np.allclose(dF[:, 0], dFb, rtol=1e-7, atol=1e-8 * scale)


def test_time_coefficients_against_quadrature():
    for delta, tau in ((0.01, 1e-4), (0.01, 0.005), (1.0, 3.0)):
        T = gks.time_coefficients(delta, tau)
        e = lambda t: np.exp(-t / tau)  # noqa: E731
        fns = [lambda t: 1 - e(t), lambda t: (t + tau) * e(t) - tau, lambda t: t - tau + tau * e(t),
               e, lambda t: (t + tau) * e(t)]
        for Tk, fn in zip(T, fns):
            ref = integrate.quad(fn, 0, delta, epsabs=0, epsrel=1e-13, limit=200)[0]
            assert abs(Tk - ref) <= 1e-12 * max(abs(ref), delta * tau)


def test_time_fit_exact_for_quadratic_integrals():
    a, b, dt = np.array([1.5, -2.0]), np.array([0.3, 7.0]), 0.02
    Fh = lambda d: a * d + 0.5 * b * d * d  # noqa: E731
    F, dF = gks.time_fit(Fh(dt), Fh(0.5 * dt), dt)
    assert np.allclose(F, a, rtol=1e-13) and np.allclose(dF, b, rtol=1e-11)


def test_uniform_state_gives_euler_flux():
    rng = np.random.default_rng(40)
    for _ in range(3):
        Wc = random_state(rng)
        rho, U, V, W, p, _ = prim(Wc)
        zero = np.zeros((3, 5, 1))
        for mu in (0.0, 1e-3):
            F, dF, Q0 = gks.gks_flux(Wc[:, None], zero, Wc[:, None], zero, 0.013, GAMMA, mu)
            euler = np.array([rho * U, rho * U * U + p, rho * U * V, rho * U * W, U * (Wc[4] + p)])
            assert np.allclose(F[:, 0], euler, rtol=1e-13, atol=1e-14)
            assert np.allclose(dF[:, 0], 0.0, atol=1e-10)
            assert np.allclose(Q0[:, 0], Wc, rtol=1e-14)


def test_shear_stress_navier_stokes_limit():
    """rho = p = 1 at rest, V varying linearly along the normal: the flux of
    tangential momentum is -mu dV/dx with mu = tau p (Pr = 1 BGK)."""
    s = 0.2
    Wc = np.array([1.0, 0.0, 0.0, 0.0, 1.0 / (GAMMA - 1)])
    dW = np.zeros((3, 5))
    dW[0, 2] = s                          # d(rho V)/dn_x
    mu, dt = 1e-5, 1e-2                   # tau = mu/p << dt
    F, _, _ = gks.gks_flux(Wc[:, None], dW[:, :, None], Wc[:, None], dW[:, :, None], dt, GAMMA, mu)
    assert abs(F[2, 0] - (-mu * s)) < 1e-3 * mu * s


@pytest.mark.parametrize("prandtl", [1.0, 0.71])
@pytest.mark.parametrize("T", [1.0, 2.5])
def test_heat_flux_navier_stokes_limit(prandtl, T):
    """At rest with uniform pressure and a linear temperature profile along
    the normal the energy flux is Fourier's -kappa dT/dx with
    kappa = c_p mu / Pr, c_p = gamma / (gamma - 1) (unit gas constant), mu from
    the power law mu0 (T/T0)^0.76 (Chapman-Enskog of the BGK model, with
    the Prandtl correction)."""
    s, p, T0, mu0 = 0.2, 1.0, 0.6, 1e-5
    Wc = np.array([p / T, 0.0, 0.0, 0.0, p / (GAMMA - 1)])
    dW = np.zeros((3, 5))
    dW[0, 0] = -p / T ** 2 * s                  # d rho / dn_x with p fixed
    F, _, _ = gks.gks_flux(Wc[:, None], dW[:, :, None], Wc[:, None], dW[:, :, None], 1e-2, GAMMA, mu0,
                           prandtl=prandtl, mu_T0=T0, mu_exponent=0.76)
    kappa = GAMMA / (GAMMA - 1) * mu0 * (T / T0) ** 0.76 / prandtl
    assert abs(F[4, 0] - (-kappa * s)) < 1e-6 * kappa * s
    assert np.abs(F[1:4, 0] - np.array([p, 0.0, 0.0])).max() < 1e-12


def mirror(Wc, dW):
    """Reverse the normal: u -> -u for the states; the derivative along the
    normal changes sign as well."""
    S = np.diag([1.0, -1.0, 1.0, 1.0, 1.0])
    dWm = np.stack([-(S @ dW[0]), S @ dW[1], S @ dW[2]])
    return S @ Wc, dWm


def test_mirror_symmetry():
    rng = np.random.default_rng(50)
    Wl, Wr = random_state(rng), random_state(rng)
    dWl, dWr = rng.standard_normal((3, 5)), rng.standard_normal((3, 5))
    F, dF, _ = gks.gks_flux(Wl[:, None], dWl[:, :, None], Wr[:, None], dWr[:, :, None], 0.01, GAMMA)
    ml, mdl = mirror(Wr, dWr)
    mr, mdr = mirror(Wl, dWl)
    Fm, dFm, _ = gks.gks_flux(ml[:, None], mdl[:, :, None], mr[:, None], mdr[:, :, None], 0.01, GAMMA)
    S = np.diag([1.0, -1.0, 1.0, 1.0, 1.0])
    assert np.allclose(Fm[:, 0], -(S @ F[:, 0]), rtol=1e-11, atol=1e-12)
    assert np.allclose(dFm[:, 0], -(S @ dF[:, 0]), rtol=1e-9, atol=1e-10)


def test_rotation_about_normal():
    """(v, w) -> (w, -v): rotate momenta, derivative directions and flux."""
    rng = np.random.default_rng(51)
    Wl, Wr = random_state(rng), random_state(rng)
    dWl, dWr = rng.standard_normal((3, 5)), rng.standard_normal((3, 5))
    R = np.eye(5)
    R[2:4, 2:4] = [[0, 1], [-1, 0]]

    def rot(Wc, dW):
        d = np.stack([R @ dW[0], R @ dW[2], -(R @ dW[1])])
        return R @ Wc, d
    F, dF, _ = gks.gks_flux(Wl[:, None], dWl[:, :, None], Wr[:, None], dWr[:, :, None], 0.01, GAMMA)
    a, da = rot(Wl, dWl)
    b, db = rot(Wr, dWr)
    Fr, dFr, _ = gks.gks_flux(a[:, None], da[:, :, None], b[:, None], db[:, :, None], 0.01, GAMMA)
    assert np.allclose(Fr[:, 0], R @ F[:, 0], rtol=1e-11, atol=1e-12)
    assert np.allclose(dFr[:, 0], R @ dF[:, 0], rtol=1e-9, atol=1e-10)
