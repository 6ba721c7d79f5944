"""The full-size moving-mesh GPU test checks sampled cells against oracle
steps of 13^3 vertex patches treated as periodic (the patch's own period:
13 nominal cells).  The seam cell of such a patch is distorted, but a
two-stage step at a cell depends only on cells within 4 of it (two stages,
each a one-cell reconstruction stencil and the face between), and the seam
is 6 cells from the centre.  Pinned here on a small periodic moving mesh:
the patch centre equals the full oracle step exactly."""

import time

import numpy as np

import oracle
from paper_1909_01580_amd import workloads as wl


def test_patch_centre_equals_full_step():
    n, P, t0, dt = 16, (2.0, 2.0, 2.0), 0.1, 4e-3
    V0 = wl.sine_mesh_vertices(n, t0, amp=0.05, omega=2 * np.pi)
    V1 = wl.sine_mesh_vertices(n, t0 + dt, amp=0.05, omega=2 * np.pi)
    q0 = wl.hex_average(V0, P, wl.pulse_point)
    start = time.time()
    full = oracle.step(oracle.vertex_problem((n, n, n), V0, P, verts_next=V1), q0, dt)
    for c in [(8, 7, 9), (6, 9, 6)]:
        sl = (slice(None),) + tuple(slice(x - 6, x + 7) for x in c[::-1])
        va, vb, q = (np.ascontiguousarray(a[sl]) for a in (V0, V1, q0))
        patch = oracle.step(oracle.vertex_problem((13, 13, 13), va, (13 * 2.0 / n,) * 3, verts_next=vb), q, dt)
        assert np.array_equal(patch[:, 6, 6, 6], full[:, c[2], c[1], c[0]]), c
        # the seam corrupts cells next to it: the patch is not the grid
        assert np.abs(patch[:, 6, 6, 12] - full[:, c[2], c[1], c[0] + 6]).max() > 1e-10
    assert time.time() - start < 120
