"""Oracle WENO-AO reconstruction (Sec. 2 of the paper) and the positivity
fallback (Sec. 4, limiting procedure).

Test infrastructure only (see the package docstring).

Per cell and per conserved variable (component-wise):
* P_0: quadratic Q + sum_{1<=|n|<=2} a_n p_n with the zero-mean basis
  p_n = x^n - (cell mean of x^n)  (Eq. (1)); a_n by unweighted least squares
  over the 18 neighbours of the big stencil S (3x3x3 block without its
  eight corners).
* P_m, m = 1..24: linear polynomials (Eq. (2)) fitted by least squares over
  the four non-central cells of each sub-stencil.
* beta_m: smoothness indicators (Eq. (4)); tau = mean |beta_0 - beta_m|
  (Eq. (5)); omega_m = gamma_m (1 + tau / (beta_m + eps)) (Eq. (3)) and
  their normalisation.
* The point value and gradient at a Gauss point combine the 25 polynomials
  as printed in Sec. 2 (the rearranged P_0 with nonlinear weights).

The monomials are written in the cell's scaled coordinate X = (x - c) / h,
c the cell centroid and h = |Omega|^(1/3); the least-squares problem and the
polynomial it returns are unchanged by this affine change of variable
(same function space, same constraints).  Where the paper is silent, the
readings are: unweighted least squares with the cell-mean constraint held
exactly by the zero-mean basis; the sub-stencil constraint integrates over
the cell volume (the printed "dxdy" is read as dV); in S_4 and S_8 the
printed Omega_{i,j+1,k} is read as Omega_{i,j-1,k} so that the eight
stencils are the eight sign quadrants; the other sixteen come from the two
cyclic permutations of the axes; each multi-index in beta appears once.
"""

import numpy as np

from .geometry import PAD

# Monomials x^n with 1 <= |n| <= 2, as exponent triples.
MONO = [(1, 0, 0), (0, 1, 0), (0, 0, 1),
        (2, 0, 0), (0, 2, 0), (0, 0, 2),
        (1, 1, 0), (0, 1, 1), (1, 0, 1)]

# Big stencil S without the centre: offsets in {-1,0,1}^3 whose product is
# not +-1 (the eight corners are excluded).
BIG_OFFSETS = [(i, j, k)
               for k in (-1, 0, 1) for j in (-1, 0, 1) for i in (-1, 0, 1)
               if (i, j, k) != (0, 0, 0) and i * j * k == 0]


def _unit(axis, sign):
    e = [0, 0, 0]
    e[axis] = sign
    return tuple(e)


def _add(p, q):
    return tuple(x + y for x, y in zip(p, q))


def sub_stencil_offsets():
    """The 24 sub-stencils as lists of their four non-central offsets.

    For the axis triples (a, b; c) = (x, y; z), (y, z; x), (z, x; y) and signs
    s_c, s_b, s_a in (+1, -1): {s_a e_a, s_b e_b, s_a e_a + s_b e_b, s_c e_c}.
    The first eight are S_1..S_8 of Sec. 2 in the printed order.
    """
    out = []
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        for sc in (1, -1):
            for sb in (1, -1):
                for sa in (1, -1):
                    ea, eb, ec = _unit(a, sa), _unit(b, sb), _unit(c, sc)
                    out.append([ea, eb, _add(ea, eb), ec])
    return out


SUB_OFFSETS = sub_stencil_offsets()

# The alternative of Remark 1 (Sec. 2): big stencil S' = S plus the six
# cells two steps away along the axes, and eight sub-stencils S'_1..S'_8,
# each the centre and one face neighbour per axis, one per sign octant
# (the printed S'_4 and S'_8 repeat S'_2 and S'_6; read as the two
# remaining octants, as for S_4 and S_8).  The octant set is closed under
# permutations of the axes, so there are no further sub-stencils.
BIG_OFFSETS_WIDE = BIG_OFFSETS + [_unit(ax, 2 * sg) for ax in range(3) for sg in (-1, 1)]
SUB_OFFSETS_WIDE = [[_unit(0, sx), _unit(1, sy), _unit(2, sz)]
                    for sz in (1, -1) for sy in (1, -1) for sx in (1, -1)]
STENCILS = {"S": (BIG_OFFSETS, SUB_OFFSETS), "S_prime": (BIG_OFFSETS_WIDE, SUB_OFFSETS_WIDE)}


def linear_weights(Gamma, M=24):
    """gamma_0 = 1 - M Gamma, gamma_m = Gamma for the M sub-stencils
    (Sec. 2: M = 24)."""
    g = np.full(M + 1, Gamma)
    g[0] = 1.0 - M * Gamma
    return g


def mono_values(X):
    """The nine monomials at scaled points X (3, ...) -> (9, ...)."""
    return np.stack([X[0] ** e[0] * X[1] ** e[1] * X[2] ** e[2] for e in MONO])


def _pow(x, e):
    return x ** e if e > 0 else np.ones_like(x)


def mono_grad(X):
    """d/dX_d of each monomial -> (9, 3, ...)."""
    out = []
    for e in MONO:
        comps = []
        for d in range(3):
            if e[d] == 0:
                comps.append(np.zeros_like(X[0]))
            else:
                f = float(e[d])
                for dd in range(3):
                    f = f * (_pow(X[dd], e[dd] - 1) if dd == d else _pow(X[dd], e[dd]))
                comps.append(f)
        out.append(np.stack(comps))
    return np.stack(out)


# Second-derivative multi-indices |l| = 2, each once.
HESS_IDX = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]


def mono_hess():
    """d^2/dX_p dX_q of each monomial for (p, q) in HESS_IDX -> (9, 6);
    constants because the monomials are at most quadratic."""
    H = np.zeros((9, 6))
    for n, e in enumerate(MONO):
        for s, (p, q) in enumerate(HESS_IDX):
            if p == q:
                H[n, s] = 2.0 if e[p] == 2 else 0.0
            else:
                ee = [0, 0, 0]
                ee[p] += 1
                ee[q] += 1
                H[n, s] = 1.0 if tuple(ee) == e else 0.0
    return H


def _shift(arr, off, N):
    """Slice of a padded array at the reconstructed cells shifted by off.
    Reconstructed cells are the real cells and one ghost layer, padded
    indices [PAD-1, N-PAD+1) along each axis."""
    g = PAD - 1
    sl = tuple(slice(g + off[d], N[d] - g + off[d]) for d in range(3))
    return arr[(Ellipsis,) + sl]


def reconstruct(xq, wj, V, c, h, Qp, Gamma, eps, stencil="S"):
    """WENO-AO reconstruction for every cell with a full big stencil.

    Inputs are per padded cell: Gauss points xq (3,8,...), weights wj (8,...),
    volume V, centroid c (3,...), scale h, cell averages Qp (5,...).
    Returns a dict of per-reconstructed-cell arrays (padded indices
    [PAD-1, N-PAD+1) along each axis).  ``stencil`` is "S" (Sec. 2) or
    "S_prime" (Remark 1).
    """
    big_offs, sub_offs = STENCILS[stencil]
    M = len(sub_offs)
    N = V.shape
    ci = _shift(c, (0, 0, 0), N)
    hi = _shift(h, (0, 0, 0), N)
    Qi = _shift(Qp, (0, 0, 0), N)

    def mean_mono(off):
        xo = _shift(xq, off, N)
        wo = _shift(wj, off, N)
        Vo = _shift(V, off, N)
        X = (xo - ci[:, None]) / hi
        return (mono_values(X) * wo[None]).sum(axis=1) / Vo

    avg_i = mean_mono((0, 0, 0))
    rows = {off: mean_mono(off) - avg_i for off in big_offs}
    diffs = {off: _shift(Qp, off, N) - Qi for off in big_offs}
    shp = ci.shape[1:]
    nr = int(np.prod(shp))

    # P_0: 18 x 9 least squares per cell (Eq. (1) and the big-stencil
    # constraints).
    A = np.stack([rows[o].reshape(9, nr).T for o in big_offs], axis=1)         # (nr,18,9)
    D = np.stack([diffs[o].reshape(5, nr).T for o in big_offs], axis=1)        # (nr,18,5)
    a = np.linalg.pinv(A) @ D                                                  # (nr,9,5)

    # P_m: 4 x 3 least squares on the linear monomials (Eq. (2)); 3 x 3 for
    # the sub-stencils of Remark 1.
    b = np.empty((nr, M, 3, 5))
    for m, offs in enumerate(sub_offs):
        Am = np.stack([rows[o][:3].reshape(3, nr).T for o in offs], axis=1)     # (nr,4,3)
        Dm = np.stack([diffs[o].reshape(5, nr).T for o in offs], axis=1)        # (nr,4,5)
        b[:, m] = np.linalg.pinv(Am) @ Dm

    # Smoothness indicators, Eq. (4), integrals by the cell's Gauss rule.
    xo = _shift(xq, (0, 0, 0), N).reshape(3, 8, nr)
    wo = _shift(wj, (0, 0, 0), N).reshape(8, nr)
    Vi = _shift(V, (0, 0, 0), N).reshape(nr)
    hf = hi.reshape(nr)
    X = (xo - ci.reshape(3, 1, nr)) / hf
    G = mono_grad(X)                                     # (9,3,8,nr) d/dX
    Hs = mono_hess()                                     # (9,6)
    # P_0: first derivatives (physical) at the Gauss points, per variable.
    d1 = np.einsum("ndqr,rnv->dqvr", G, a) / hf          # (3,8,5,nr)
    d2 = np.einsum("ns,rnv->svr", Hs, a) / hf ** 2       # (6,5,nr)
    int1 = (d1 ** 2 * wo[None, :, None, :]).sum(axis=(0, 1))            # (5,nr)
    int2 = (d2 ** 2).sum(axis=0) * Vi                                   # (5,nr)
    beta = np.empty((M + 1, 5, nr))
    beta[0] = Vi ** (2.0 / 3.0 - 1.0) * int1 + Vi ** (4.0 / 3.0 - 1.0) * int2
    for m in range(M):
        g = b[:, m] / hf[:, None, None]                  # (nr,3,5) physical gradient
        intm = (g ** 2).sum(axis=1).T * wo.sum(axis=0)   # (5,nr)
        beta[1 + m] = Vi ** (2.0 / 3.0 - 1.0) * intm

    # Nonlinear weights, Eqs. (3) and (5).
    gam = linear_weights(Gamma, M)
    tau = np.abs(beta[0][None] - beta[1:]).sum(axis=0) / M
    omega = gam[:, None, None] * (1.0 + tau[None] / (beta + eps))
    wbar = omega / omega.sum(axis=0)[None]

    return {
        "shape": shp,
        "c": ci.reshape(3, nr), "h": hf, "V": Vi,
        "xg": X, "wg": wo,
        "avg": avg_i.reshape(9, nr),
        "Q": Qi.reshape(5, nr),
        "a": a, "b": b,
        "beta": beta, "tau": tau, "wbar": wbar, "gamma": gam,
    }


def select(rec, index):
    """Restrict a reconstruction dict to the flat cell indices ``index``
    (an integer array of any shape); the cell axis becomes index.shape."""
    out = {}
    shp = index.shape
    flat = index.reshape(-1)
    for key in ("c", "avg", "Q"):
        out[key] = rec[key][:, flat].reshape(rec[key].shape[:1] + shp)
    for key in ("h", "V"):
        out[key] = rec[key][flat].reshape(shp)
    out["xg"] = rec["xg"][:, :, flat].reshape((3, 8) + shp)
    out["wg"] = rec["wg"][:, flat].reshape((8,) + shp)
    out["a"] = np.moveaxis(rec["a"][flat], 0, -1).reshape((9, 5) + shp)
    M = rec["b"].shape[1]
    out["b"] = np.moveaxis(rec["b"][flat], 0, -1).reshape((M, 3, 5) + shp)
    out["wbar"] = rec["wbar"][:, :, flat].reshape((M + 1, 5) + shp)
    out["gamma"] = rec["gamma"]
    return out


def eval_polys(sel, x):
    """Values (M+1,5,...) and physical gradients (M+1,3,5,...) of P_0..P_M
    of the selected cells at physical points x (3, ...)."""
    X = (x - sel["c"]) / sel["h"]
    mv = mono_values(X) - sel["avg"]                     # (9,...)
    mg = mono_grad(X)                                    # (9,3,...)
    Q = sel["Q"]
    shp = np.broadcast_shapes(Q.shape[1:], X.shape[1:])
    M = sel["b"].shape[0]
    vals = np.empty((M + 1, 5) + shp)
    grads = np.empty((M + 1, 3, 5) + shp)
    vals[0] = Q + np.einsum("n...,nv...->v...", mv, sel["a"])
    grads[0] = np.einsum("nd...,nv...->dv...", mg, sel["a"]) / sel["h"]
    for m in range(M):
        bm = sel["b"][m]                                 # (3,5,...)
        vals[1 + m] = Q + np.einsum("d...,dv...->v...", mv[:3], bm)
        grads[1 + m] = bm / sel["h"]
    return vals, grads


def combine(sel, vals, grads):
    """Point value and gradient of the WENO-AO reconstruction (Sec. 2):
    wbar_0 (P_0/gamma_0 - sum gamma_m/gamma_0 P_m) + sum wbar_m P_m."""
    gam = sel["gamma"]
    w = sel["wbar"]
    K = len(gam)
    val = w[0] * (vals[0] / gam[0] - sum(gam[m] / gam[0] * vals[m] for m in range(1, K))) \
        + sum(w[m] * vals[m] for m in range(1, K))
    grad = w[0][None] * (grads[0] / gam[0] - sum(gam[m] / gam[0] * grads[m] for m in range(1, K))) \
        + sum(w[m][None] * grads[m] for m in range(1, K))
    return val, grad


def positivity_trigger(vals, gamma):
    """True where any of the polynomials (25, or 9 with the stencils of
    Remark 1) gives a non-positive density or a negative pressure at the
    point (Sec. 4 limiting procedure)."""
    rho = vals[:, 0]
    bad_rho = rho <= 0.0
    rs = np.where(bad_rho, 1.0, rho)
    p = (gamma - 1.0) * (vals[:, 4] - 0.5 * (vals[:, 1] ** 2 + vals[:, 2] ** 2 + vals[:, 3] ** 2) / rs)
    bad = bad_rho | (p < 0.0)
    return bad.any(axis=0)
