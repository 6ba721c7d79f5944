"""Pins for the oracle geometry (trilinear cells and bilinear faces, Sec. 2
final part and Sec. 3, Eqs. (10)-(11)).

The cell rule (2x2x2 Gauss with |J|) and the face rule (2x2 Gauss of
X_a x X_b) are separate code paths; the divergence theorem ties them:
|Omega| = (1/3) sum_faces int X . dA and int x_d dV = (1/2) sum_faces
int x_d^2 dA_d, both integrated exactly by the face rule because the
integrands are of degree <= 3 per face parameter.
"""

import numpy as np
import pytest

from oracle import geometry as geo


def random_hex_vertices(rng, n=3, amp=0.15):
    """A small padded vertex array of a perturbed grid (every vertex moved)."""
    vp = geo.padded_vertices_uniform((n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), pad=0)
    return vp + amp / n * rng.uniform(-1, 1, size=vp.shape)


def face_integrals(vp):
    """Per cell: (1/3) sum_faces int X . dA and (1/2) sum_faces int x_d^2 dA_d,
    with outward orientation (+ on the upper face, - on the lower face)."""
    n = [s - 1 for s in vp.shape[1:]]
    vol = np.zeros(n)
    mom = np.zeros([3] + n)
    for d in range(3):
        fc = geo.face_corners(vp, d, 0, n[d] + 1)
        fg = geo.face_gauss(fc)
        dotx = 0.25 * (fg["x"] * fg["a"]).sum(axis=0).sum(axis=0)          # (planes, a, b)
        sq = 0.25 * (fg["x"] ** 2 * fg["a"]).sum(axis=1)                    # (3, planes, a, b)
        a, b = geo.face_axes(d)
        inv = list(np.argsort([d, a, b]))
        dotx = np.transpose(dotx, inv)
        sq = np.transpose(sq, [0] + [1 + i for i in inv])
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[d] = slice(1, None)
        lo[d] = slice(0, -1)
        vol += (dotx[tuple(hi)] - dotx[tuple(lo)]) / 3.0
        mom += 0.5 * (sq[(slice(None),) + tuple(hi)] - sq[(slice(None),) + tuple(lo)])
    return vol, mom


def test_uniform_cells():
    vp = geo.padded_vertices_uniform((4, 3, 2), (0.5, -1.0, 2.0), (2.0, 1.5, 1.0), pad=0)
    xq, wj = geo.cell_quadrature(vp)
    V, c, h = geo.cell_volume_centroid(xq, wj)
    assert np.allclose(V, 0.5 * 0.5 * 0.5, rtol=0, atol=1e-15)
    assert np.allclose(c[0, :, 0, 0], 0.5 + 0.25 + 0.5 * np.arange(4), atol=1e-14)
    assert np.allclose(c[2, 0, 0, :], 2.0 + 0.25 + 0.5 * np.arange(2), atol=1e-14)


def test_affine_cell_volume_and_centroid():
    rng = np.random.default_rng(1)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    vp = geo.padded_vertices_uniform((1, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), pad=0)
    vp = np.einsum("ij,j...->i...", A, vp) + b[:, None, None, None]
    xq, wj = geo.cell_quadrature(vp)
    V, c, _ = geo.cell_volume_centroid(xq, wj)
    assert abs(V[0, 0, 0] - abs(np.linalg.det(A))) < 1e-14
    assert np.allclose(c[:, 0, 0, 0], A @ np.full(3, 0.5) + b, atol=1e-14)


def test_divergence_theorem_ties_cell_and_face_rules():
    rng = np.random.default_rng(2)
    vp = random_hex_vertices(rng)
    xq, wj = geo.cell_quadrature(vp)
    V, c, _ = geo.cell_volume_centroid(xq, wj)
    vol, mom = face_integrals(vp)
    assert np.allclose(V, vol, rtol=0, atol=1e-15)
    assert np.allclose(c * V[None], mom, rtol=0, atol=1e-15)


def test_closed_surface_and_face_vector_area():
    rng = np.random.default_rng(3)
    vp = random_hex_vertices(rng)
    total = 0.0
    for d in range(3):
        fc = geo.face_corners(vp, d, 0, vp.shape[1 + d])
        fg = geo.face_gauss(fc)
        area = 0.25 * fg["a"].sum(axis=1)              # (3, planes, a, b)
        # Vector area of a bilinear face is half the cross product of its
        # diagonals (corner 0 -> 3 crossed with corner 2 -> 1).
        diag = 0.5 * np.cross(fc[:, 3] - fc[:, 0], fc[:, 1] - fc[:, 2], axis=0)
        assert np.allclose(area, diag, rtol=0, atol=1e-15)
        # Closed surface of the first cell: upper minus lower face.
        total = total + area[:, 1, 0, 0] - area[:, 0, 0, 0]
    assert np.allclose(total, 0.0, atol=1e-15)


def test_local_frame_orthonormal_and_axis_aligned_on_boxes():
    rng = np.random.default_rng(4)
    vp = random_hex_vertices(rng)
    fc = geo.face_corners(vp, 1, 0, 3)
    fg = geo.face_gauss(fc)
    nx, ny, nz = geo.local_frame(fg["a"], fg["xb"])
    for u in (nx, ny, nz):
        assert np.allclose((u * u).sum(axis=0), 1.0, atol=1e-14)
    for u, v in ((nx, ny), (ny, nz), (nx, nz)):
        assert np.allclose((u * v).sum(axis=0), 0.0, atol=1e-14)
    assert np.allclose(np.cross(nx, ny, axis=0), nz, atol=1e-14)
    box = geo.padded_vertices_uniform((2, 2, 2), (0.0,) * 3, (1.0,) * 3, pad=0)
    for d in range(3):
        fg = geo.face_gauss(geo.face_corners(box, d, 0, 3))
        nx, ny, nz = geo.local_frame(fg["a"], fg["xb"])
        e = np.zeros(3)
        e[d] = 1.0
        assert np.allclose(nx, e[:, None, None, None, None], atol=1e-15)
        e2 = np.zeros(3)
        e2[(d + 1) % 3] = 1.0
        assert np.allclose(ny, e2[:, None, None, None, None], atol=1e-15)


def test_area_rate_matches_finite_difference():
    """a_G(t) is quadratic in t for linearly moving vertices, so a central
    difference reproduces da_G/dt up to round-off."""
    rng = np.random.default_rng(5)
    vp = random_hex_vertices(rng)
    vel = rng.standard_normal(vp.shape)
    fc, fv = geo.face_corners(vp, 2, 0, 4), geo.face_corners(vel, 2, 0, 4)
    fg = geo.face_gauss(fc, fv)
    s = 1e-3
    ap = geo.face_gauss(fc + s * fv)["a"]
    am = geo.face_gauss(fc - s * fv)["a"]
    assert np.allclose((ap - am) / (2 * s), fg["adot"], rtol=0, atol=1e-10)
    # Grid velocity is the bilinear interpolation of the vertex velocities.
    assert np.allclose(fg["ug"], geo.face_gauss(fv)["x"], atol=1e-15)


@pytest.mark.parametrize("n", [(3, 4, 5)])
def test_periodic_padding_images(n):
    rng = np.random.default_rng(6)
    verts = rng.standard_normal((3,) + n)
    period = (2.0, 3.0, 5.0)
    vp = geo.padded_vertices_periodic(verts, period, pad=2)
    # Vertex p = -1 along x is vertex n-1 shifted by -period in x only.
    assert np.allclose(vp[:, 1, 2, 2], verts[:, n[0] - 1, 0, 0] - np.array([2.0, 0, 0]))
    assert np.allclose(vp[:, 2 + n[0], 2, 2], verts[:, 0, 0, 0] + np.array([2.0, 0, 0]))
