"""Oracle finite-volume stage, two-stage fourth-order stepping and the
moving-mesh update (Sec. 3 of the paper, Eq. (9), the S2O4 formulas and
Remark 2), plus the time-step rule and the conservation totals.

Test infrastructure only (see the package docstring).

A stage computes, for every cell, R = -sum_faces F_p and dR = -sum_faces
dF_p where F_p = sum_G (1/4) ||X_a x X_b||_G F_G is the 2x2 Gauss face
flux of Eq. (11) and dF_p its time derivative.  On a static mesh
L = R / |Omega| (Eq. (9)) and the two stages are
    Q*      = Q + dt/2 L(Q) + dt^2/8 dL(Q)
    Q^{n+1} = Q + dt L(Q) + dt^2/6 (dL(Q) + 2 dL(Q*)).

Moving mesh (Remark 2), readings where the paper is silent:
* vertices move with the constant secant velocity (x^{n+1} - x^n)/dt; the
  stage-1 geometry is at t_n and the stage-2 geometry at t_n + dt/2;
* the Gauss-point flux is the kinetic flux through the moving face, i.e. the
  static flux of the states seen from a frame moving with the grid velocity
  at that Gauss point, transformed back (mass, momentum and energy shift);
* the two-stage formulas act on U = |Omega| Q together with the volume:
  dV/dt = R_V = sum_faces sum_G (1/4) U^g_G . a_G (a_G = X_a x X_b), and
  its time derivative uses the exact rate da_G/dt of the moving face; the
  same rate enters dF_p through -Q_0 (U^g . da_G/dt), so a uniform state
  stays uniform to round-off and |Omega| at t_{n+1} equals the geometric
  volume (the stage update integrates the quadratic-in-time R_V exactly).

Time step (the paper gives only CFL = 0.35): dt = CFL min_cells
h_cell / (||U|| + c), h_cell the smallest distance between the centres
(vertex means) of opposite faces.
"""

from dataclasses import dataclass

import numpy as np

from . import geometry as geo
from . import characteristic
from . import weno
from .gks import gks_flux

PAD = geo.PAD


@dataclass
class Params:
    gamma: float = 1.4
    mu: float = 0.0            # 0: inviscid collision time
    weno_Gamma: float = 0.0025
    weno_eps: float = 1e-8
    tau_eps: float = 0.01
    tau_C: float = 1.0
    characteristic: bool = False   # reconstruct in characteristic variables (Sec. 4)
    mu_T0: float = 1.0             # viscosity law mu (T / mu_T0)^mu_exponent (Sec. 4)
    mu_exponent: float = 0.0       # 0: constant mu
    prandtl: float = 1.0           # 1: the BGK flux as it stands
    stencil: str = "S"             # "S" (Sec. 2) or "S_prime" (Remark 1)


BOUNDARIES = ("periodic", "outflow", "symmetric")


class Problem:
    """Grid description for the oracle.

    ``kind`` is 'uniform' (origin, length, per-axis boundaries) or
    'vertices' (periodic hexahedral grid given by its vertices, library
    layout [3][nz][ny][nx], optional next vertices for a moving mesh).
    A per-axis boundary is 'periodic', 'outflow' (zero-gradient ghosts:
    the non-reflecting condition of Sec. 4), 'symmetric' (mirror ghosts with
    the normal momentum reversed: the symmetric condition of Sec. 4) or a
    pair (low end, high end) of the last two.
    """

    def __init__(self, n, bc, params, kind, origin=None, length=None,
                 verts=None, period=None, verts_next=None):
        self.n = tuple(int(x) for x in n)
        self.bc = tuple(bc)
        self.sides = []
        for b in self.bc:
            lo, hi = (b, b) if isinstance(b, str) else tuple(b)
            assert lo in BOUNDARIES and hi in BOUNDARIES
            assert (lo == "periodic") == (hi == "periodic"), "periodic at both ends or neither"
            self.sides.append((lo, hi))
        self.params = params
        self.kind = kind
        self.origin, self.length = origin, length
        self.period = period
        self.verts = None if verts is None else _to_ijk(np.asarray(verts, float))
        self.verts_next = None if verts_next is None else _to_ijk(np.asarray(verts_next, float))
        if kind == "vertices":
            assert all(self.periodic(d) for d in range(3))

    def periodic(self, d):
        return self.sides[d][0] == "periodic"

    @property
    def moving(self):
        return self.verts_next is not None

    def set_next_vertices(self, verts_next):
        self.verts_next = None if verts_next is None else _to_ijk(np.asarray(verts_next, float))

    def padded_vertices(self, alpha=0.0):
        if self.kind == "uniform":
            return geo.padded_vertices_uniform(self.n, self.origin, self.length)
        v = self.verts
        if self.verts_next is not None and alpha != 0.0:
            v = v + alpha * (self.verts_next - self.verts)
        return geo.padded_vertices_periodic(v, self.period)

    def padded_velocities(self, dt):
        if self.verts_next is None:
            return None
        return geo.padded_vertices_periodic((self.verts_next - self.verts) / dt, (0.0, 0.0, 0.0))

    def pad_state(self, Q):
        """Ghost cells, axis by axis: periodic wrap; zero-gradient copy of
        the nearest interior cell (outflow); or the mirror image across the
        boundary face, ghost g outside <-> interior cell g inside, with the
        momentum component normal to that face reversed (symmetric)."""
        out = Q
        for d in range(3):
            n = self.n[d]
            idx = np.arange(-PAD, n + PAD)
            src = idx.copy()
            sign = np.ones(idx.size)
            lo, hi = self.sides[d]
            if lo == "periodic":
                src = idx % n
            else:
                below, above = idx < 0, idx >= n
                src = np.clip(idx, 0, n - 1)
                if lo == "symmetric":
                    src[below] = -1 - idx[below]
                    sign[below] = -1.0
                if hi == "symmetric":
                    src[above] = 2 * n - 1 - idx[above]
                    sign[above] = -1.0
                # a mirror deeper than the grid (n < PAD) only feeds ghost
                # layers the stencil of Sec. 2 never reads
                src = np.clip(src, 0, n - 1)
            out = np.take(out, src, axis=1 + d)
            if np.any(sign < 0):
                shape = [1, 1, 1]
                shape[d] = idx.size
                out = out.copy()
                out[1 + d] *= sign.reshape(shape)
        return out


def _to_ijk(a):
    """Library layout [c][nz][ny][nx] -> oracle (c, i, j, k)."""
    return np.ascontiguousarray(np.transpose(a, (0, 3, 2, 1)))


def _to_lib(a):
    return np.ascontiguousarray(np.transpose(a, (0, 3, 2, 1)))


def uniform_problem(n, origin, length, bc=("periodic",) * 3, params=None):
    return Problem(n, bc, params or Params(), "uniform", origin=origin, length=length)


def vertex_problem(n, verts, period, params=None, verts_next=None):
    return Problem(n, ("periodic",) * 3, params or Params(), "vertices",
                   verts=verts, period=period, verts_next=verts_next)


# ------------------------------------------------------------------ stage
def _faces(prob, rec, vp, vdot, d, dt, chunk=2048):
    """Fluxes of every face normal to axis d that the real cells need.

    Face f (0 <= f < nf) lies between real cells f-1 and f along d.
    Periodic axes have nf = n_d faces (face n_d is face 0); other axes
    have nf = n_d + 1.
    """
    P = prob.params
    n = prob.n
    a_ax, b_ax = geo.face_axes(d)
    nf = n[d] if prob.periodic(d) else n[d] + 1
    order = [d, a_ax, b_ax]
    inv = list(np.argsort(order))

    def face_array(arr, lead):
        # (lead..., f, NA, NB) in (d,a,b) order -> real range, (x,y,z) order, flat
        arr = arr[(Ellipsis, slice(None), slice(PAD, PAD + n[a_ax]), slice(PAD, PAD + n[b_ax]))]
        L = len(lead)
        arr = np.transpose(arr, list(range(L)) + [L + i for i in inv])
        return arr.reshape(tuple(lead) + (-1,))

    fc = geo.face_corners(vp, d, PAD, PAD + nf)
    fg = geo.face_gauss(fc, None if vdot is None else geo.face_corners(vdot, d, PAD, PAD + nf))
    xG = face_array(fg["x"], (3, 4))
    aG = face_array(fg["a"], (3, 4))
    xb = face_array(fg["xb"], (3, 4))
    # the frame at the face centre (characteristic projection: one per face)
    _, xa_c, xb_c = geo.bilinear(fc, 0.0, 0.0)
    a_c = face_array(np.cross(xa_c, xb_c, axis=0), (3,))
    xb_c = face_array(xb_c, (3,))
    ug = face_array(fg["ug"], (3, 4)) if vdot is not None else None
    adot = face_array(fg["adot"], (3, 4)) if vdot is not None else None

    # Flat indices of the left/right reconstructed cells.
    NR = rec["shape"]
    ii = [np.arange(n[e]) + 1 for e in range(3)]
    fL = list(ii)
    fR = list(ii)
    # Real cell f-1 is reconstructed cell f (for f = 0 the ghost, whose
    # geometry is the periodic image or the extended box); real cell f is
    # reconstructed cell f+1.
    fL[d] = np.arange(nf)
    fR[d] = np.arange(nf) + 1
    IL = np.ravel_multi_index(np.meshgrid(*fL, indexing="ij"), NR).reshape(-1)
    IR = np.ravel_multi_index(np.meshgrid(*fR, indexing="ij"), NR).reshape(-1)

    nfaces = IL.size
    out = {k: np.empty((5, nfaces)) for k in ("F", "dF")}
    out["RV"] = np.zeros(nfaces)
    out["dRV"] = np.zeros(nfaces)
    out["stateL"] = np.empty((4, 5, 4, nfaces))
    out["stateR"] = np.empty((4, 5, 4, nfaces))
    out["trigL"] = np.empty((4, nfaces), bool)
    out["trigR"] = np.empty((4, nfaces), bool)
    for s in range(0, nfaces, chunk):
        sl = slice(s, min(s + chunk, nfaces))
        x = xG[:, :, sl]
        nx_, ny_, nz_ = geo.local_frame(aG[:, :, sl], xb[:, :, sl])
        frame = (nx_, ny_, nz_)
        sels = {side: weno.select(rec, idx[None, :]) for side, idx in (("L", IL[sl]), ("R", IR[sl]))}
        if P.characteristic:
            Qbar = 0.5 * (sels["L"]["Q"] + sels["R"]["Q"])
            cframe = tuple(v[:, None] for v in geo.local_frame(a_c[:, sl], xb_c[:, sl]))
        states = []
        for side in ("L", "R"):
            sel = sels[side]
            vals, grads = weno.eval_polys(sel, x)
            if P.characteristic:
                val, grad = characteristic.point_states(sel, x, Qbar, cframe, P.weno_Gamma, P.weno_eps,
                                                        P.gamma)
            else:
                val, grad = weno.combine(sel, vals, grads)
            trig = weno.positivity_trigger(vals, P.gamma)
            Qc = np.broadcast_to(sel["Q"], val.shape)
            val = np.where(trig[None], Qc, val)
            grad = np.where(trig[None, None], 0.0, grad)
            out["state" + side][:, :, :, sl] = np.concatenate([val[None], grad], axis=0)
            out["trig" + side][:, sl] = trig
            states.append((val, grad))
        u_g = None if ug is None else ug[:, :, sl]

        loc = []
        for val, grad in states:
            if u_g is not None:
                val, grad = _galilean(val, grad, u_g)
            W = _rotate(val, frame)
            dW = np.stack([_rotate(np.einsum("d...,dv...->v...", frame[j], grad), frame)
                           for j in range(3)])
            loc.append((W, dW))
        F, dF, Q0 = gks_flux(loc[0][0], loc[0][1], loc[1][0], loc[1][1], dt,
                             P.gamma, P.mu, P.tau_eps, P.tau_C, mu_T0=P.mu_T0,
                             mu_exponent=P.mu_exponent, prandtl=P.prandtl)
        F, dF, Q0 = (_unrotate(v, frame) for v in (F, dF, Q0))
        if u_g is not None:
            F, dF, Q0 = (_galilean_back(v, u_g) for v in (F, dF, Q0))
        area = np.linalg.norm(aG[:, :, sl], axis=0)
        out["F"][:, sl] = 0.25 * (area[None] * F).sum(axis=1)
        dsum = area[None] * dF
        if u_g is not None:
            rate = (u_g * adot[:, :, sl]).sum(axis=0)             # U^g . da/dt
            dsum = dsum - Q0 * rate[None]
            out["RV"][sl] = 0.25 * (u_g * aG[:, :, sl]).sum(axis=0).sum(axis=0)
            out["dRV"][sl] = 0.25 * rate.sum(axis=0)
        out["dF"][:, sl] = 0.25 * dsum.sum(axis=1)

    shape = [n[0], n[1], n[2]]
    shape[d] = nf
    res = {}
    for k, v in out.items():
        res[k] = v.reshape(v.shape[:-1] + tuple(shape))
    return res


def _galilean(val, grad, ug):
    """Conservative variables seen from a frame moving with ug (a constant
    velocity at the point): M - rho ug, E - M.ug + rho |ug|^2 / 2; the same
    linear map applies to the gradients."""
    def tr(w, ug_):
        rho, M, E = w[0], w[1:4], w[4]
        Mn = M - rho[None] * ug_
        En = E - (M * ug_).sum(axis=0) + 0.5 * rho * (ug_ * ug_).sum(axis=0)
        return np.concatenate([rho[None], Mn, En[None]])
    return tr(val, ug), np.stack([tr(grad[d], ug) for d in range(3)])


def _galilean_back(f, ug):
    rho, M, E = f[0], f[1:4], f[4]
    Mn = M + rho[None] * ug
    En = E + (M * ug).sum(axis=0) + 0.5 * rho * (ug * ug).sum(axis=0)
    return np.concatenate([rho[None], Mn, En[None]])


def _rotate(w, frame):
    """(rho, M, E) -> (rho, M.n_x, M.n_y, M.n_z, E)."""
    M = w[1:4]
    return np.concatenate([w[:1]] + [(M * n).sum(axis=0)[None] for n in frame] + [w[4:]])


def _unrotate(f, frame):
    """Local-frame momentum back to global components (Eq. (14) with an
    orthonormal frame)."""
    M = frame[0] * f[1][None] + frame[1] * f[2][None] + frame[2] * f[3][None]
    return np.concatenate([f[:1], M, f[4:]])


def residual(prob, Q, dt, alpha=0.0, keep_faces=False):
    """One stage: R, dR (5,nx,ny,nz), R_V, dR_V and the cell volumes.

    Q is in oracle layout (5, nx, ny, nz).  ``alpha`` places the stage
    geometry at t_n + alpha dt on a moving mesh.
    """
    P = prob.params
    vp = prob.padded_vertices(alpha)
    vdot = prob.padded_velocities(dt) if prob.moving else None
    xq, wj = geo.cell_quadrature(vp)
    V, c, h = geo.cell_volume_centroid(xq, wj)
    rec = weno.reconstruct(xq, wj, V, c, h, prob.pad_state(Q), P.weno_Gamma, P.weno_eps, P.stencil)
    n = prob.n
    R = np.zeros((5,) + n)
    dR = np.zeros((5,) + n)
    RV = np.zeros(n)
    dRV = np.zeros(n)
    faces = []
    for d in range(3):
        fd = _faces(prob, rec, vp, vdot, d, dt)
        faces.append(fd)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[d] = slice(0, n[d])
        if prob.periodic(d):
            hi_idx = (np.arange(n[d]) + 1) % n[d]
        else:
            hi_idx = np.arange(n[d]) + 1
        for key, acc in (("F", R), ("dF", dR)):
            f = fd[key]
            acc -= np.take(f, hi_idx, axis=1 + d) - f[(slice(None),) + tuple(lo)]
        for key, acc in (("RV", RV), ("dRV", dRV)):
            f = fd[key]
            acc += np.take(f, hi_idx, axis=d) - f[tuple(lo)]
    Vr = V[PAD:PAD + n[0], PAD:PAD + n[1], PAD:PAD + n[2]]
    out = {"R": R, "dR": dR, "RV": RV, "dRV": dRV, "V": Vr}
    if keep_faces:
        out["faces"] = faces
    return out


def s2o4(Y, op, dt, n_stages=2):
    """Two-stage fourth-order time stepping for dY/dt = L(Y) given an
    operator op(Y, stage) -> (L, dL/dt) (Sec. 3).  n_stages = 1 is the
    one-stage update Y + dt L + dt^2/2 dL."""
    L, dL = op(Y, 0)
    if n_stages == 1:
        return Y + dt * L + 0.5 * dt * dt * dL
    Ys = Y + 0.5 * dt * L + 0.125 * dt * dt * dL
    L2, dL2 = op(Ys, 1)
    return Y + dt * L + dt * dt / 6.0 * (dL + 2.0 * dL2)


def step(prob, Q_lib, dt, n_stages=2, return_volume=False):
    """Advance the library-layout state Q [5][nz][ny][nx] by one step.
    On a moving mesh ``return_volume`` also returns the updated cell
    volumes [nz][ny][nx]."""
    Q = _to_ijk(np.asarray(Q_lib, float))
    if not prob.moving:
        def op(Y, stage):
            r = residual(prob, Y, dt)
            return r["R"] / r["V"], r["dR"] / r["V"]
        return _to_lib(s2o4(Q, op, dt, n_stages))

    # Moving mesh: Y = (|Omega| Q, |Omega|).
    r0 = residual(prob, Q, dt, 0.0)
    Y0 = np.concatenate([r0["V"][None] * Q, r0["V"][None]])
    cache = {0: r0}

    def op(Y, stage):
        if stage == 0:
            r = cache[0]
        else:
            r = residual(prob, Y[:5] / Y[5][None], dt, 0.5)
        return (np.concatenate([r["R"], r["RV"][None]]),
                np.concatenate([r["dR"], r["dRV"][None]]))

    Y1 = s2o4(Y0, op, dt, n_stages)
    Qn = _to_lib(Y1[:5] / Y1[5][None])
    if return_volume:
        return Qn, _to_lib(Y1[5][None])[0]
    return Qn


def physical(Q_lib, gamma):
    """True when every cell has rho > 0 and p > 0 (NaN counts as not)."""
    Q = np.asarray(Q_lib, float)
    with np.errstate(all="ignore"):
        p = (gamma - 1.0) * (Q[4] - 0.5 * (Q[1] ** 2 + Q[2] ** 2 + Q[3] ** 2) / Q[0])
        return bool(np.all(Q[0] > 0.0) and np.all(p > 0.0))


def checked_step(prob, Q_lib, dt, n_stages=2, max_halvings=8):
    """Step-rejection rule around ``step`` on a static grid: the step is
    taken with dt / 2^k for the smallest k <= max_halvings whose result is
    physical.  Returns (state, dt taken), or (None, None) when even
    dt / 2^max_halvings fails.

    Not part of the method: the paper prints only the CFL number, and for
    the singular start of the Sedov problem (Sec. 4) a small CFL of 0.01.
    At that CFL the two-stage step still drives the pressure of the cells
    two faces away from the energy cell negative in the first step, through the
    dt^2/3 dL(Q*) term of the second stage (the flux into those cells is
    switched on only at the intermediate state, so the first stage gives it
    no weight); halving the step removes it, since that term scales as
    dt^2 while the cells' energy does not."""
    assert not prob.moving
    for _ in range(max_halvings + 1):
        with np.errstate(all="ignore"):
            Qn = step(prob, Q_lib, dt, n_stages)
        if physical(Qn, prob.params.gamma):
            return Qn, dt
        dt = 0.5 * dt
    return None, None


def stage_volumes(prob, alpha=0.0):
    vp = prob.padded_vertices(alpha)
    xq, wj = geo.cell_quadrature(vp)
    V, _, _ = geo.cell_volume_centroid(xq, wj)
    n = prob.n
    return _to_lib(V[None, PAD:PAD + n[0], PAD:PAD + n[1], PAD:PAD + n[2]])[0]


def totals(prob, Q_lib):
    """sum over cells of |Omega| Q for the five conservative variables."""
    V = stage_volumes(prob)
    return np.array([np.sum(V * Q_lib[v]) for v in range(5)])


def kinetic_energy(prob, Q_lib, rho0=1.0):
    """Volume-averaged kinetic energy of the Taylor-Green test (Sec. 4),
    E_k = (1 / (rho0 |Omega|)) int rho |U|^2 / 2 dOmega, with the integrand
    taken on the cell averages: sum_i |Omega_i| |M_i|^2 / (2 rho_i) divided
    by rho0 sum_i |Omega_i|."""
    V = stage_volumes(prob)
    Q = np.asarray(Q_lib, float)
    ke = 0.5 * (Q[1] ** 2 + Q[2] ** 2 + Q[3] ** 2) / Q[0]
    return float(np.sum(V * ke) / (rho0 * np.sum(V)))


def max_dt(prob, Q_lib, cfl):
    Q = _to_ijk(np.asarray(Q_lib, float))
    P = prob.params
    vp = prob.padded_vertices(0.0)
    n = prob.n
    real = vp[:, PAD:PAD + n[0] + 1, PAD:PAD + n[1] + 1, PAD:PAD + n[2] + 1]
    corners = geo.cell_corners(real)
    hmin = None
    for d in range(3):
        bit = 4 >> d  # corner bit of axis d in m = 4a + 2b + c
        lo = np.mean([corners[:, m] for m in range(8) if not (m & bit)], axis=0)
        up = np.mean([corners[:, m] for m in range(8) if (m & bit)], axis=0)
        dist = np.linalg.norm(up - lo, axis=0)
        hmin = dist if hmin is None else np.minimum(hmin, dist)
    rho = Q[0]
    U = Q[1:4] / rho
    p = (P.gamma - 1.0) * (Q[4] - 0.5 * rho * (U * U).sum(axis=0))
    c = np.sqrt(P.gamma * p / rho)
    return cfl * float(np.min(hmin / (np.linalg.norm(U, axis=0) + c)))


# ------------------------------------------------------------ debug views
def gp_states(prob, Q_lib, dt, alpha=0.0):
    """Per cell and Gauss point: value and (x, y, z) gradient of the five
    conservative variables after the positivity fallback, in the global
    frame.  Layout [nz][ny][nx][24][5][4]; Gauss point 4*face + g with faces
    (-x, +x, -y, +y, -z, +z) and g = 2*[a>0] + [b>0] in the face's cyclic
    parameters."""
    Q = _to_ijk(np.asarray(Q_lib, float))
    r = residual(prob, Q, dt, alpha, keep_faces=True)
    n = prob.n
    out = np.empty(n + (24, 5, 4))
    for d in range(3):
        fd = r["faces"][d]
        sR = fd["stateR"]           # (4 val/grad, 5, 4 gp, faces...)
        sL = fd["stateL"]
        lo = [slice(None)] * 3
        lo[d] = slice(0, n[d])
        hi_idx = (np.arange(n[d]) + 1) % n[d] if prob.periodic(d) else np.arange(n[d]) + 1
        minus = sR[(Ellipsis,) + tuple(lo)]
        plus = np.take(sL, hi_idx, axis=3 + d)
        for face, arr in ((2 * d, minus), (2 * d + 1, plus)):
            # (4, 5, 4gp, i, j, k) -> (i, j, k, 4gp, 5, 4)
            out[:, :, :, 4 * face:4 * face + 4] = np.transpose(arr, (3, 4, 5, 2, 1, 0))
    return np.ascontiguousarray(np.transpose(out, (2, 1, 0, 3, 4, 5)))


def fallback_mask(prob, Q_lib, dt, alpha=0.0):
    """Per real cell, bit 4*face + g set where that Gauss point used the
    first-order fallback; layout [nz][ny][nx], same numbering as gp_states."""
    Q = _to_ijk(np.asarray(Q_lib, float))
    r = residual(prob, Q, dt, alpha, keep_faces=True)
    n = prob.n
    mask = np.zeros(n, dtype=np.uint32)
    for d in range(3):
        fd = r["faces"][d]
        lo = [slice(None)] * 3
        lo[d] = slice(0, n[d])
        hi_idx = (np.arange(n[d]) + 1) % n[d] if prob.periodic(d) else np.arange(n[d]) + 1
        minus = fd["trigR"][(slice(None),) + tuple(lo)]          # (4gp, i, j, k)
        plus = np.take(fd["trigL"], hi_idx, axis=1 + d)
        for face, arr in ((2 * d, minus), (2 * d + 1, plus)):
            for g in range(4):
                mask |= arr[g].astype(np.uint32) << np.uint32(4 * face + g)
    return np.ascontiguousarray(np.transpose(mask, (2, 1, 0)))


def face_fluxes(prob, Q_lib, dt, alpha=0.0):
    """Face sums on the lower face of every real cell along each axis:
    layout [3][nz][ny][nx][2][5] holding (F_p, dF_p)."""
    Q = _to_ijk(np.asarray(Q_lib, float))
    r = residual(prob, Q, dt, alpha, keep_faces=True)
    n = prob.n
    out = np.empty((3,) + n + (2, 5))
    for d in range(3):
        fd = r["faces"][d]
        lo = [slice(None)] * 3
        lo[d] = slice(0, n[d])
        for k, key in enumerate(("F", "dF")):
            arr = fd[key][(slice(None),) + tuple(lo)]       # (5, i, j, k)
            out[d, :, :, :, k, :] = np.moveaxis(arr, 0, -1)
    return np.ascontiguousarray(np.transpose(out, (0, 3, 2, 1, 4, 5)))
