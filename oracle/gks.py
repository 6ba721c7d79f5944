"""Oracle gas-kinetic BGK flux at a face Gauss point (Sec. 3 of the paper).

Test infrastructure only (see the package docstring).

Everything is written in the local frame of the Gauss point: u is the
particle velocity along n_x (the face normal), v and w along n_y and n_z.
Moments are taken against Maxwellians
    g = rho (lam/pi)^((K+3)/2) exp(-lam((u-U)^2 + (v-V)^2 + (w-W)^2 + xi^2)),
K = (5 - 3 gamma)/(gamma - 1) internal degrees of freedom, with the
collision invariants psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2) (Sec. 3).

The algebra is generic and deliberately plain: polynomials in
(u, v, w, xi^2) are dicts {exponents: coefficient array}; an expectation is a
sum of products of one-dimensional moments; every micro-slope is a 5x5
``numpy.linalg.solve`` against the moment matrix <psi psi^T>.

Readings where the paper is silent or inconsistent:
* Eq. (15) attaches H(u) to g_r; the compatibility condition that follows it
  takes u > 0 from the left state, so H(u) goes with g_l and 1 - H(u) with
  g_r (n_x points from the left cell to the right cell).
* One collision time tau (Sec. 4) is used in every term; Delta t inside tau
  is the full time step in both stages; p in the viscous tau is the pressure
  of the equilibrium state g_0; p_l and p_r are the Gauss-point pressures.
"""

import numpy as np
from scipy.special import erfc

# ---------------------------------------------------------------- polynomials
ONE = {(0, 0, 0, 0): 1.0}
UJ = [{(1, 0, 0, 0): 1.0}, {(0, 1, 0, 0): 1.0}, {(0, 0, 1, 0): 1.0}]
PSI = [
    {(0, 0, 0, 0): 1.0},
    {(1, 0, 0, 0): 1.0},
    {(0, 1, 0, 0): 1.0},
    {(0, 0, 1, 0): 1.0},
    {(2, 0, 0, 0): 0.5, (0, 2, 0, 0): 0.5, (0, 0, 2, 0): 0.5, (0, 0, 0, 1): 0.5},
]


def pmul(P, Q):
    out = {}
    for ep, cp in P.items():
        for eq, cq in Q.items():
            e = tuple(x + y for x, y in zip(ep, eq))
            out[e] = out.get(e, 0.0) + cp * cq
    return out


def slope_poly(a):
    """a_1 + a_2 u + a_3 v + a_4 w + a_5 (u^2+v^2+w^2+xi^2)/2 for a (5, ...)."""
    out = {}
    for beta in range(5):
        for e, cf in PSI[beta].items():
            out[e] = out.get(e, 0.0) + a[beta] * cf
    return out


# ----------------------------------------------------------------- moments
class Moments:
    """One-dimensional moments of a normalised Maxwellian.

    u-moments are over the full line, over u > 0 (``half='+'``) or over
    u < 0 (``half='-'``); v, w and xi^2 moments are always full.
    """

    NU = 8  # <u^0> .. <u^7>

    def __init__(self, U, V, W, lam, K, half=None):
        self.u = self._umoments(U, lam, half)
        self.v = self._full(V, lam, 6)
        self.w = self._full(W, lam, 6)
        self.x = [np.ones_like(lam), K / (2.0 * lam), K * (K + 2.0) / (4.0 * lam ** 2)]

    @staticmethod
    def _full(U, lam, n):
        m = [np.ones_like(U), U]
        for k in range(1, n - 1):
            m.append(U * m[k] + k / (2.0 * lam) * m[k - 1])
        return m

    @classmethod
    def _umoments(cls, U, lam, half):
        if half is None:
            return cls._full(U, lam, cls.NU)
        pos = [0.5 * erfc(-np.sqrt(lam) * U)]
        pos.append(U * pos[0] + 0.5 * np.exp(-lam * U * U) / np.sqrt(np.pi * lam))
        for k in range(1, cls.NU - 1):
            pos.append(U * pos[k] + k / (2.0 * lam) * pos[k - 1])
        if half == "+":
            return pos
        full = cls._full(U, lam, cls.NU)
        return [f - p for f, p in zip(full, pos)]


def expect(P, mom):
    """<P> against the normalised Maxwellian described by ``mom``."""
    tot = 0.0
    for (a, b, c, d), cf in P.items():
        tot = tot + cf * mom.u[a] * mom.v[b] * mom.w[c] * mom.x[d]
    return tot


def psi_moments(P, mom):
    """(<P psi_1>, ..., <P psi_5>) -> array (5, ...)."""
    return np.stack([np.broadcast_to(expect(pmul(P, PSI[al]), mom), mom.u[0].shape)
                     for al in range(5)])


def moment_matrix(mom):
    """M_{alpha beta} = <psi_alpha psi_beta>, returned as (..., 5, 5)."""
    M = np.empty(mom.u[0].shape + (5, 5))
    for al in range(5):
        for be in range(5):
            M[..., al, be] = expect(pmul(PSI[al], PSI[be]), mom)
    return M


def solve5(M, rhs):
    """Solve M x = rhs with M (...,5,5), rhs (5,...) -> (5,...)."""
    r = np.moveaxis(rhs, 0, -1)[..., None]
    return np.moveaxis(np.linalg.solve(M, r)[..., 0], -1, 0)


# -------------------------------------------------------------- primitives
def primitives(W, gamma):
    rho = W[0]
    U, V, Wv = W[1] / rho, W[2] / rho, W[3] / rho
    p = (gamma - 1.0) * (W[4] - 0.5 * rho * (U * U + V * V + Wv * Wv))
    lam = rho / (2.0 * p)
    return rho, U, V, Wv, p, lam


def time_coefficients(delta, tau):
    """Time integrals over [0, delta] of the five time factors of Eq. (15):
    (1 - e), ((t+tau) e - tau), (t - tau + tau e), e, (t + tau) e with
    e = exp(-t/tau)."""
    E = np.exp(-delta / tau)
    T1 = delta - tau * (1.0 - E)
    T2 = 2.0 * tau ** 2 * (1.0 - E) - tau * delta * (1.0 + E)
    T3 = 0.5 * delta ** 2 - tau * delta + tau ** 2 * (1.0 - E)
    T4 = tau * (1.0 - E)
    T5 = 2.0 * tau ** 2 * (1.0 - E) - tau * delta * E
    return T1, T2, T3, T4, T5


def time_fit(Ffull, Fhalf, dt):
    """F and dF/dt of the linear-in-time flux F + dF (t - t_n) whose
    integrals over [0, dt] and [0, dt/2] are Ffull and Fhalf (Eq. (16) and
    the two equations that follow it)."""
    Mfit = np.array([[dt, 0.5 * dt ** 2], [0.5 * dt, 0.125 * dt ** 2]])
    sol = np.linalg.solve(Mfit, np.stack([np.reshape(Ffull, -1), np.reshape(Fhalf, -1)]))
    return sol[0].reshape(np.shape(Ffull)), sol[1].reshape(np.shape(Ffull))


def padd(*Ps):
    out = {}
    for P in Ps:
        for e, cf in P.items():
            out[e] = out.get(e, 0.0) + cf
    return out


def heat_flux_poly(U, V, W):
    """(u - U)((u - U)^2 + (v - V)^2 + (w - W)^2 + xi^2) / 2: the normal heat
    flux carried by a particle, relative to the velocity (U, V, W)."""
    cx = {(1, 0, 0, 0): 1.0, (0, 0, 0, 0): -U}
    cy = {(0, 1, 0, 0): 1.0, (0, 0, 0, 0): -V}
    cz = {(0, 0, 1, 0): 1.0, (0, 0, 0, 0): -W}
    c2 = padd(pmul(cx, cx), pmul(cy, cy), pmul(cz, cz), {(0, 0, 0, 1): 1.0})
    return {e: 0.5 * cf for e, cf in pmul(cx, c2).items()}


def gks_flux(Wl, dWl, Wr, dWr, dt, gamma, mu=0.0, tau_eps=0.01, tau_C=1.0,
             return_parts=False, mu_T0=1.0, mu_exponent=0.0, prandtl=1.0):
    """Gas-kinetic flux F and its time derivative dF at Gauss points.

    Wl, Wr:   conservative variables (5, ...) in the local frame.
    dWl, dWr: their derivatives along n_x, n_y, n_z, shape (3, 5, ...).
    dt:       the full time step Delta t.
    Returns F, dF (5, ...) in the local frame, and Q_0 (5, ...), the
    conservative variables of the equilibrium state g_0.
    """
    K = (5.0 - 3.0 * gamma) / (gamma - 1.0)
    rl, Ul, Vl, Wlv, pl, laml = primitives(Wl, gamma)
    rr, Ur, Vr, Wrv, pr, lamr = primitives(Wr, gamma)
    ml = Moments(Ul, Vl, Wlv, laml, K)
    mr = Moments(Ur, Vr, Wrv, lamr, K)
    mlp = Moments(Ul, Vl, Wlv, laml, K, half="+")
    mrn = Moments(Ur, Vr, Wrv, lamr, K, half="-")
    Ml, Mr = moment_matrix(ml), moment_matrix(mr)

    # Micro-slopes <a_j^k> = dQ_k/dn_j and A^k from the time-derivative
    # compatibility <a_1 u + a_2 v + a_3 w + A> = 0 (Sec. 3).
    al = [solve5(Ml, dWl[j] / rl) for j in range(3)]
    ar = [solve5(Mr, dWr[j] / rr) for j in range(3)]
    Al = solve5(Ml, -sum(psi_moments(pmul(slope_poly(al[j]), UJ[j]), ml) for j in range(3)))
    Ar = solve5(Mr, -sum(psi_moments(pmul(slope_poly(ar[j]), UJ[j]), mr) for j in range(3)))

    # Equilibrium state and its slopes from the compatibility condition:
    # u > 0 from the left, u < 0 from the right.
    Q0 = rl * psi_moments(ONE, mlp) + rr * psi_moments(ONE, mrn)
    dQ0 = [rl * psi_moments(slope_poly(al[j]), mlp) + rr * psi_moments(slope_poly(ar[j]), mrn)
           for j in range(3)]
    r0, U0, V0, W0, p0, lam0 = primitives(Q0, gamma)
    m0 = Moments(U0, V0, W0, lam0, K)
    M0 = moment_matrix(m0)
    ab = [solve5(M0, dQ0[j] / r0) for j in range(3)]
    Ab = solve5(M0, -sum(psi_moments(pmul(slope_poly(ab[j]), UJ[j]), m0) for j in range(3)))

    # Collision time (Sec. 4); on the viscous branch mu may follow the power
    # law mu (T / T0)^omega of the isotropic-turbulence test (Sec. 4), with
    # T = p_0 / rho_0 the temperature of g_0.
    jump = np.abs((pl - pr) / (pl + pr)) * dt
    if mu > 0.0:
        mu_g = mu * ((p0 / r0) / mu_T0) ** mu_exponent if mu_exponent != 0.0 else mu
        tau = mu_g / p0 + tau_C * jump
    else:
        tau = tau_eps * dt + tau_C * jump

    # The six velocity moments the time integral of Eq. (15) needs.
    u = UJ[0]
    X1 = r0 * psi_moments(u, m0)
    X2 = r0 * sum(psi_moments(pmul(u, pmul(slope_poly(ab[j]), UJ[j])), m0) for j in range(3))
    X3 = r0 * psi_moments(pmul(u, slope_poly(Ab)), m0)
    X4 = rl * psi_moments(u, mlp) + rr * psi_moments(u, mrn)
    X5 = rl * sum(psi_moments(pmul(u, pmul(slope_poly(al[j]), UJ[j])), mlp) for j in range(3)) \
        + rr * sum(psi_moments(pmul(u, pmul(slope_poly(ar[j]), UJ[j])), mrn) for j in range(3))
    X6 = rl * psi_moments(pmul(u, slope_poly(Al)), mlp) + rr * psi_moments(pmul(u, slope_poly(Ar)), mrn)

    def Fhat(delta):
        T1, T2, T3, T4, T5 = time_coefficients(delta, tau)
        return T1 * X1 + T2 * X2 + T3 * X3 + T4 * X4 - T5 * X5 - tau * T4 * X6

    # Prandtl number (Pr = 0.71 for the viscous tests of Sec. 4; the BGK
    # flux has Pr = 1): the time-integrated energy flux gains (1/Pr - 1) times
    # the time-integrated heat flux, the moment of the heat-flux polynomial
    # relative to the velocity of g_0 against the same time-dependent
    # distribution, term by term.
    if prandtl != 1.0:
        hq = heat_flux_poly(U0, V0, W0)
        Y1 = r0 * expect(hq, m0)
        Y2 = r0 * sum(expect(pmul(hq, pmul(slope_poly(ab[j]), UJ[j])), m0) for j in range(3))
        Y3 = r0 * expect(pmul(hq, slope_poly(Ab)), m0)
        Y4 = rl * expect(hq, mlp) + rr * expect(hq, mrn)
        Y5 = rl * sum(expect(pmul(hq, pmul(slope_poly(al[j]), UJ[j])), mlp) for j in range(3)) \
            + rr * sum(expect(pmul(hq, pmul(slope_poly(ar[j]), UJ[j])), mrn) for j in range(3))
        Y6 = rl * expect(pmul(hq, slope_poly(Al)), mlp) + rr * expect(pmul(hq, slope_poly(Ar)), mrn)
        Fplain = Fhat

        def Fhat(delta):
            T1, T2, T3, T4, T5 = time_coefficients(delta, tau)
            q = T1 * Y1 + T2 * Y2 + T3 * Y3 + T4 * Y4 - T5 * Y5 - tau * T4 * Y6
            out = Fplain(delta).copy()
            out[4] = out[4] + (1.0 / prandtl - 1.0) * q
            return out

    # Linear-in-time flux fitted to its integrals over [0, dt] and
    # [0, dt/2] (Eq. (16) and the two equations after it).
    F, dF = time_fit(Fhat(dt), Fhat(0.5 * dt), dt)
    if return_parts:
        return F, dF, Q0, {"tau": tau, "al": al, "ar": ar, "Al": Al, "Ar": Ar,
                           "ab": ab, "Ab": Ab, "X": (X1, X2, X3, X4, X5, X6)}
    return F, dF, Q0
