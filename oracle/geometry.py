"""Oracle geometry: trilinear hexahedra, 2x2x2 Gauss moments, bilinear faces.

Test infrastructure only (see the package docstring).

Sources in the paper:
* Sec. 2, final part: a hexahedron with non-coplanar vertices is the
  trilinear image of [-1/2, 1/2]^3 with the eight base functions psi_1..psi_8;
  cell integrals of x^a y^b z^c use the 2x2x2 Gauss rule with |J|.
* Sec. 3, Eq. (10): a face is the bilinear image of [-1/2, 1/2]^2 with
  phi_1..phi_4; Eq. (11): 2x2 Gauss rule on the face with the area element
  ||X_eta x X_zeta||; the local frame n_x, n_y, n_z at each Gauss point.
* Sec. 3, Remark 2: grid velocity at a face Gauss point is the bilinear
  interpolation of the four vertex velocities.

Arrays are indexed (component, i, j, k) with i along x.
"""

import numpy as np

# Two-point Gauss rule on [-1/2, 1/2]: nodes -+ 1/(2 sqrt 3), weights 1/2.
GNODE = 0.5 / np.sqrt(3.0)
GAUSS = (-GNODE, GNODE)
GWEIGHT = 0.5

PAD = 3  # ghost layers kept around the real cells in every direction (the
         # wide stencil of Remark 1 reaches two cells beyond the ghost layer)


def padded_vertices_uniform(n, origin, length, pad=PAD):
    """Vertices of a uniform box grid, extended by ``pad`` cells per side.

    Returns an array (3, nx+2p+1, ny+2p+1, nz+2p+1); vertex index p along an
    axis sits at origin + (p - pad) * h.
    """
    axes = []
    for d in range(3):
        h = length[d] / n[d]
        axes.append(origin[d] + (np.arange(n[d] + 2 * pad + 1) - pad) * h)
    X, Y, Z = np.meshgrid(axes[0], axes[1], axes[2], indexing="ij")
    return np.stack([X, Y, Z])


def padded_vertices_periodic(verts, period, pad=PAD):
    """Periodic vertex grid: ``verts`` is (3, nx, ny, nz) (one vertex per
    cell and axis); vertex index v outside [0, n) is the image of v mod n
    shifted by the period along that axis."""
    n = verts.shape[1:]
    idx = [np.arange(-pad, n[d] + pad + 1) for d in range(3)]
    out = verts[:, idx[0] % n[0]][:, :, idx[1] % n[1]][:, :, :, idx[2] % n[2]].copy()
    for d in range(3):
        shift = np.floor_divide(idx[d], n[d]) * period[d]
        shape = [1, 1, 1]
        shape[d] = -1
        out[d] += shift.reshape(shape)
    return out


def _signs(bit):
    return -1.0 if bit == 0 else 1.0


def cell_corners(vp):
    """The eight corners of every cell, in the order of psi_1..psi_8:
    corner m = 4*[xi>0] + 2*[eta>0] + [zeta>0].  Shape (3, 8, NX, NY, NZ)."""
    NX, NY, NZ = (s - 1 for s in vp.shape[1:])
    out = np.empty((3, 8, NX, NY, NZ))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                out[:, 4 * a + 2 * b + c] = vp[:, a:a + NX, b:b + NY, c:c + NZ]
    return out


def trilinear(corners, xi, eta, zeta):
    """X(xi, eta, zeta) and its three parametric derivatives for every cell."""
    X = 0.0
    dX = [0.0, 0.0, 0.0]
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                sa, sb, sc = _signs(a), _signs(b), _signs(c)
                fa, fb, fc = 1 + 2 * sa * xi, 1 + 2 * sb * eta, 1 + 2 * sc * zeta
                xm = corners[:, 4 * a + 2 * b + c]
                X = X + (fa * fb * fc / 8.0) * xm
                dX[0] = dX[0] + (2 * sa * fb * fc / 8.0) * xm
                dX[1] = dX[1] + (2 * sb * fa * fc / 8.0) * xm
                dX[2] = dX[2] + (2 * sc * fa * fb / 8.0) * xm
    return X, dX


def cell_quadrature(vp):
    """2x2x2 Gauss points of every cell and their weights w*|J|.

    Returns xq (3, 8, NX, NY, NZ) and wj (8, NX, NY, NZ); Gauss point q is
    4*[xi>0] + 2*[eta>0] + [zeta>0].
    """
    corners = cell_corners(vp)
    shp = corners.shape[2:]
    xq = np.empty((3, 8) + shp)
    wj = np.empty((8,) + shp)
    for qa in (0, 1):
        for qb in (0, 1):
            for qc in (0, 1):
                q = 4 * qa + 2 * qb + qc
                X, dX = trilinear(corners, GAUSS[qa], GAUSS[qb], GAUSS[qc])
                J = np.einsum("i...,i...->...", dX[0], np.cross(dX[1], dX[2], axis=0))
                xq[:, q] = X
                wj[q] = GWEIGHT ** 3 * np.abs(J)
    return xq, wj


def cell_volume_centroid(xq, wj):
    V = wj.sum(axis=0)
    c = (xq * wj[None]).sum(axis=1) / V
    h = np.cbrt(V)
    return V, c, h


# Face parameterisation.  A face normal to axis d is parameterised by the two
# other axes in cyclic order (a, b) = (d+1, d+2) mod 3, so that X_a x X_b
# points towards increasing index along d.  Gauss point g = 2*[a>0] + [b>0].
def face_axes(d):
    return (d + 1) % 3, (d + 2) % 3


def face_corners(vp, d, lo, hi):
    """Corners of every face normal to axis d on the vertex planes lo..hi-1.

    The result is ordered (component, corner, plane, a, b) with (a, b) the
    cyclic face axes; corner m = 2*[a>0] + [b>0].
    """
    a, b = face_axes(d)
    v = np.moveaxis(vp, (1 + d, 1 + a, 1 + b), (1, 2, 3))
    v = v[:, lo:hi]
    NA, NB = v.shape[2] - 1, v.shape[3] - 1
    out = np.empty((3, 4, v.shape[1], NA, NB))
    for ia in (0, 1):
        for ib in (0, 1):
            out[:, 2 * ia + ib] = v[:, :, ia:ia + NA, ib:ib + NB]
    return out  # axes: (comp, corner, along d, along a, along b)


def bilinear(fc, sa, sb):
    """Bilinear face map of Eq. (10) at parameters (sa, sb) and its two
    parametric derivatives."""
    X = 0.0
    Xa = 0.0
    Xb = 0.0
    for ia in (0, 1):
        for ib in (0, 1):
            ea, eb = _signs(ia), _signs(ib)
            fa, fb = 1 + 2 * ea * sa, 1 + 2 * eb * sb
            xm = fc[:, 2 * ia + ib]
            X = X + (fa * fb / 4.0) * xm
            Xa = Xa + (2 * ea * fb / 4.0) * xm
            Xb = Xb + (2 * eb * fa / 4.0) * xm
    return X, Xa, Xb


def face_gauss(fc, fcdot=None):
    """Per face Gauss point: position, area vector X_a x X_b, its time rate
    and the grid velocity (when vertex velocities ``fcdot`` are given).

    Returns dicts of arrays with a leading Gauss-point axis of length 4.
    """
    xs, avec, adot, ug, xb = [], [], [], [], []
    for ga in (0, 1):
        for gb in (0, 1):
            X, Xa, Xb = bilinear(fc, GAUSS[ga], GAUSS[gb])
            xs.append(X)
            xb.append(Xb)
            avec.append(np.cross(Xa, Xb, axis=0))
            if fcdot is not None:
                U, Ua, Ub = bilinear(fcdot, GAUSS[ga], GAUSS[gb])
                ug.append(U)
                adot.append(np.cross(Ua, Xb, axis=0) + np.cross(Xa, Ub, axis=0))
    out = {"x": np.stack(xs, axis=1), "a": np.stack(avec, axis=1), "xb": np.stack(xb, axis=1)}
    if fcdot is not None:
        out["ug"] = np.stack(ug, axis=1)
        out["adot"] = np.stack(adot, axis=1)
    return out


def local_frame(avec, xb):
    """Orthonormal frame of Sec. 3: n_x along X_a x X_b, n_z along X_b,
    n_y = n_z x n_x."""
    nx = avec / np.linalg.norm(avec, axis=0)
    nz = xb / np.linalg.norm(xb, axis=0)
    ny = np.cross(nz, nx, axis=0)
    return nx, ny, nz
