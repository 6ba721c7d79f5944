"""Oracle reconstruction in characteristic variables (Sec. 4: the option
stated after the limiting procedure).

Test infrastructure only (see the package docstring).

At a face Gauss point with unit normal n the conservative data of a cell's
stencil are projected to U = L Q, L = R^-1, R the right eigenvectors of the
Euler Jacobian n_x dF/dQ + n_y dG/dQ + n_z dH/dQ.  WENO-AO (Sec. 2) runs on
each component of U -- its 25 polynomials are those of the conservative
data projected by L, since the least squares are linear, while the
smoothness indicators and nonlinear weights are recomputed per
characteristic component -- and the point value and gradient are projected
back with R.  The positivity test of Sec. 4 is unchanged: it looks at the
25 conservative polynomials.

Readings: R is taken at the arithmetic mean of the two cell averages that
share the face, along the frame (n_x, n_y, n_z) of Sec. 3 at the face's
centre, the two tangential (shear) eigenvectors being n_y and n_z (on a box
face normal to axis d, the axes d+1 and d+2 in cyclic order, the frame of
every Gauss point of the face; on a bilinear face of a hexahedral grid the
one projection serves the face's four Gauss points).  The reconstruction is
in the laboratory frame.
"""

import numpy as np

from . import weno


def primitives(Q, gamma):
    rho = Q[0]
    V = Q[1:4] / rho
    p = (gamma - 1.0) * (Q[4] - 0.5 * rho * (V ** 2).sum(axis=0))
    return rho, V, p


def euler_flux_n(Q, n, gamma):
    """n . (F, G, H) of the Euler equations at conservative Q."""
    rho, V, p = primitives(Q, gamma)
    un = (V * n).sum(axis=0)
    return np.concatenate([(rho * un)[None],
                           Q[1:4] * un + p * n,
                           ((Q[4] + p) * un)[None]])


def eigensystem(Qbar, n, t1, t2, gamma):
    """Right eigenvectors R (5,5,...) (columns), L = R^-1 and the eigenvalues
    (5,...) of the Euler Jacobian along the unit normal n at Qbar; t1, t2
    complete (n, t1, t2) to an orthonormal frame.  Column order: u_n - c,
    entropy, shear along t1, shear along t2, u_n + c."""
    shp = np.broadcast_shapes(Qbar.shape[1:], n.shape[1:], t1.shape[1:], t2.shape[1:])
    Qbar = np.broadcast_to(Qbar, (5,) + shp)
    n, t1, t2 = (np.broadcast_to(v, (3,) + shp) for v in (n, t1, t2))
    rho, V, p = primitives(Qbar, gamma)
    c = np.sqrt(gamma * p / rho)
    H = (Qbar[4] + p) / rho
    un = (V * n).sum(axis=0)
    v1 = (V * t1).sum(axis=0)
    v2 = (V * t2).sum(axis=0)
    one = np.ones_like(rho)
    zero = np.zeros_like(rho)
    cols = [
        np.concatenate([one[None], V - c * n, (H - c * un)[None]]),
        np.concatenate([one[None], V, (0.5 * (V ** 2).sum(axis=0))[None]]),
        np.concatenate([zero[None], t1 * one, v1[None]]),
        np.concatenate([zero[None], t2 * one, v2[None]]),
        np.concatenate([one[None], V + c * n, (H + c * un)[None]]),
    ]
    R = np.stack(cols, axis=1)                            # (5 rows, 5 cols, ...)
    Rm = np.moveaxis(R, (0, 1), (-2, -1))
    L = np.moveaxis(np.linalg.inv(Rm), (-2, -1), (0, 1))
    lam = np.stack([un - c, un, un, un, un + c])
    return R, L, lam


def indicators(a, b, X, wg, h, V):
    """Smoothness indicators (Eq. (4)) of P_0 with coefficients a (9,k,...)
    and of P_1..P_24 with coefficients b (24,3,k,...), over a cell with
    scaled Gauss points X (3,8,...), weights wg (8,...), scale h and
    volume V.  Returns beta (M+1,k,...) for M sub-stencils."""
    G = weno.mono_grad(X)                                 # (9,3,8,...)
    Hs = weno.mono_hess()                                 # (9,6)
    ex = (slice(None),) * 3 + (None,)
    d1 = (G[ex] * a[:, None, None]).sum(axis=0) / h       # (3,8,k,...)
    d2 = np.einsum("ns,nk...->sk...", Hs, a) / h ** 2     # (6,k,...)
    int1 = (d1 ** 2 * wg[None, :, None]).sum(axis=(0, 1))
    int2 = (d2 ** 2).sum(axis=0) * V
    M = b.shape[0]
    beta = np.empty((M + 1,) + int1.shape)
    beta[0] = V ** (2.0 / 3.0 - 1.0) * int1 + V ** (4.0 / 3.0 - 1.0) * int2
    wsum = wg.sum(axis=0)
    for m in range(M):
        beta[1 + m] = V ** (2.0 / 3.0 - 1.0) * ((b[m] / h) ** 2).sum(axis=0) * wsum
    return beta


def nonlinear_weights(beta, Gamma, eps):
    """Normalised weights of Eqs. (3) and (5) from the indicators."""
    M = beta.shape[0] - 1
    gam = weno.linear_weights(Gamma, M)
    gshape = (M + 1,) + (1,) * (beta.ndim - 1)
    tau = np.abs(beta[0][None] - beta[1:]).sum(axis=0) / M
    omega = gam.reshape(gshape) * (1.0 + tau[None] / (beta + eps))
    return omega / omega.sum(axis=0)[None]


def _project(M, arr, vaxis):
    """sum_v M[k, v] arr[..., v, ...] with v at position vaxis of arr; the
    matrix M (5,5,T...) broadcasts against the trailing axes T of arr."""
    a = np.moveaxis(arr, vaxis, 0)                        # (5, E..., T...)
    extra = a.ndim - 1 - (M.ndim - 2)
    Mx = M.reshape(M.shape[:2] + (1,) * extra + M.shape[2:])
    return np.moveaxis((Mx * a[None]).sum(axis=1), 0, vaxis)


def point_states(sel, x, Qbar, frame, Gamma, eps, gamma):
    """Value (5,...) and physical gradient (3,5,...) of the characteristic
    reconstruction of the selected cells at points x, for faces whose mean
    state is Qbar and whose projection frame is (n, t1, t2)."""
    R, L, _ = eigensystem(Qbar, *frame, gamma)
    selU = dict(sel)
    selU["Q"] = _project(L, sel["Q"], 0)
    selU["a"] = _project(L, sel["a"], 1)
    selU["b"] = _project(L, sel["b"], 2)
    beta = indicators(selU["a"], selU["b"], sel["xg"], sel["wg"], sel["h"], sel["V"])
    selU["wbar"] = nonlinear_weights(beta, Gamma, eps)
    vals, grads = weno.eval_polys(selU, x)
    valU, gradU = weno.combine(selU, vals, grads)
    return _project(R, valU, 0), _project(R, gradU, 1)
