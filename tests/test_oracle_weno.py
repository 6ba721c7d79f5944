"""Pins for the oracle WENO-AO reconstruction (Sec. 2) and the positivity
fallback (Sec. 4).

* exactness: quadratic cell averages are reproduced by P_0 on boxes and on
  deformed hexahedra (data averaged with the cell rule the method uses);
  linear data make every indicator equal, so the weights are the linear
  weights and the WENO value is exact; constants give zero slopes;
* closed forms derived by hand on unit cubes (normal equations of the 18x9
  system, the indicator of a quadratic) against the generic least squares;
* a hand-worked step: beta_0 = 4/3, twelve sub-stencils with beta = 1 and
  twelve with beta = 0, tau = 5/6;
* the fallback mask of a linear pressure ramp, known in closed form.
"""

import os

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import weno

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def build(vp, avg_fn, Gamma=0.0025, eps=1e-8):
    xq, wj = geo.cell_quadrature(vp)
    V, c, h = geo.cell_volume_centroid(xq, wj)
    Qp = avg_fn(xq, wj, V, c)
    return weno.reconstruct(xq, wj, V, c, h, Qp, Gamma, eps), (xq, wj, V, c, h)


def box(n=5, h=1.0):
    return geo.padded_vertices_uniform((n, n, n), (0.0,) * 3, (n * h,) * 3, pad=0)


def quad_fn(rng):
    c0 = rng.standard_normal()
    lin = rng.standard_normal(3)
    Qm = rng.standard_normal((3, 3))
    Qm = 0.5 * (Qm + Qm.T)

    def f(x):
        return c0 + np.einsum("d,d...->...", lin, x) + np.einsum("de,d...,e...->...", Qm, x, x)
    return f, (c0, lin, Qm)


def rule_average(f):
    """Cell averages of a scalar field by the cell's own 2x2x2 rule,
    replicated into five 'variables' with different offsets."""
    def avg(xq, wj, V, c):
        s = (f(xq) * wj).sum(axis=0) / V
        return np.stack([s + k for k in range(5)])
    return avg


def centre(rec):
    """Flat index of the central reconstructed cell."""
    shp = rec["shape"]
    return np.ravel_multi_index(tuple(s // 2 for s in shp), shp)


def eval_at(rec, idx, x):
    sel = weno.select(rec, np.array([[idx]]))
    return weno.eval_polys(sel, x[:, None, None])


def test_stencil_structure():
    offs = weno.BIG_OFFSETS
    assert len(offs) == 18 and len(set(offs)) == 18
    assert sum(1 for o in offs if sum(map(abs, o)) == 1) == 6
    assert sum(1 for o in offs if sum(map(abs, o)) == 2) == 12
    subs = weno.SUB_OFFSETS
    assert len(subs) == 24
    assert len({frozenset(s) for s in subs}) == 24
    for s in subs:
        assert all(o in offs for o in s)
    # The first eight are the printed S_1..S_8 (with the S_4/S_8 reading).
    rows = np.loadtxt(os.path.join(GOLDEN, "substencils_S1_S8.txt"), dtype=int)
    for m in range(8):
        printed = {tuple(rows[m, 3 * k:3 * k + 3]) for k in range(4)}
        assert printed == set(subs[m])


def test_linear_weights():
    g = weno.linear_weights(0.0025)
    assert np.all(g > 0) and abs(g.sum() - 1.0) < 1e-15 and abs(g[0] - 0.94) < 1e-15


@pytest.mark.parametrize("deformed", [False, True])
def test_quadratic_exactness(deformed):
    rng = np.random.default_rng(10 + deformed)
    vp = box(5, 0.3)
    if deformed:
        vp = vp + 0.05 * rng.uniform(-1, 1, size=vp.shape)
    f, _ = quad_fn(rng)
    rec, _ = build(vp, rule_average(f))
    idx = centre(rec)
    c = rec["c"][:, idx]
    for x in (c, c + 0.1 * rng.standard_normal(3)):
        vals, grads = eval_at(rec, idx, x)
        assert np.allclose(vals[0, 0, 0, 0], f(x), rtol=0, atol=1e-12)
        # Gradient of the quadratic by central difference (exact for quadratics).
        e = 1e-3
        g = np.array([(f(x + e * np.eye(3)[d]) - f(x - e * np.eye(3)[d])) / (2 * e) for d in range(3)])
        assert np.allclose(grads[0, :, 0, 0, 0], g, rtol=0, atol=1e-9)


def test_quadratic_exactness_box_closed_form_averages():
    """Exact cube averages of a quadratic (x_d^2 averages to c_d^2 + h^2/12)."""
    rng = np.random.default_rng(12)
    h = 0.25
    vp = box(5, h)
    f, (c0, lin, Qm) = quad_fn(rng)

    def avg(xq, wj, V, c):
        s = c0 + np.einsum("d,d...->...", lin, c) + np.einsum("de,d...,e...->...", Qm, c, c) \
            + np.trace(Qm) * h * h / 12.0
        return np.stack([s] * 5)
    rec, _ = build(vp, avg)
    idx = centre(rec)
    x = rec["c"][:, idx] + np.array([0.5 * h, 0.1, -0.05])
    vals, _ = eval_at(rec, idx, x)
    assert abs(vals[0, 0, 0, 0] - f(x)) < 1e-13


def test_linear_data_gives_linear_weights_and_exact_value():
    rng = np.random.default_rng(13)
    vp = box(5, 0.2) + 0.03 * rng.uniform(-1, 1, size=box(5, 0.2).shape)
    lin = rng.standard_normal(3)
    rec, _ = build(vp, rule_average(lambda x: 2.0 + np.einsum("d,d...->...", lin, x)))
    idx = centre(rec)
    beta = rec["beta"][:, 0, idx]
    assert np.allclose(beta, beta[0], rtol=1e-12)
    assert np.allclose(rec["wbar"][:, 0, idx], weno.linear_weights(0.0025), rtol=1e-10)
    x = rec["c"][:, idx] + 0.05
    sel = weno.select(rec, np.array([[idx]]))
    vals, grads = weno.eval_polys(sel, x[:, None, None])
    val, grad = weno.combine(sel, vals, grads)
    assert abs(val[0, 0, 0] - (2.0 + lin @ x)) < 1e-13
    assert np.allclose(grad[:, 0, 0, 0], lin, atol=1e-12)


def test_constant_data():
    rec, _ = build(box(5, 0.2), lambda xq, wj, V, c: np.ones((5,) + V.shape) * 3.0)
    assert np.allclose(rec["a"], 0.0, atol=1e-13) and np.allclose(rec["b"], 0.0, atol=1e-13)
    assert np.allclose(rec["beta"], 0.0, atol=1e-25)
    assert np.allclose(rec["wbar"][:, 0, 0], weno.linear_weights(0.0025), rtol=1e-14)


def test_closed_forms_on_unit_cubes():
    """Normal equations of the 18x9 system on unit cubes, solved by hand:
    a_d = (1/10) sum o_d d_o; a_de = (1/4) sum o_d o_e d_o over edge cells;
    a_dd = (r_d - (2/9)(r_x + r_y + r_z))/6 with r_d = sum o_d^2 d_o; and the
    indicator beta_0 = sum a_d^2 + (13/3) sum a_dd^2 + (7/6) sum a_de^2;
    sub-stencil (a, b; c): b_c = s_c d_c, s_a b_a = (2 d_a - d_b + d_ab)/3."""
    rng = np.random.default_rng(14)
    vp = box(5, 1.0)
    data = rng.standard_normal((5, 5, 5, 5))
    rec, _ = build(vp, lambda xq, wj, V, c: data)
    idx = centre(rec)
    Qc = data[:, 2, 2, 2]
    d = {o: data[:, 2 + o[0], 2 + o[1], 2 + o[2]] - Qc for o in weno.BIG_OFFSETS}
    a = rec["a"][idx]                                     # (9, 5)
    for ax in range(3):
        ad = sum(o[ax] * d[o] for o in weno.BIG_OFFSETS) / 10.0
        assert np.allclose(a[ax], ad, atol=1e-13)
    r = [sum(o[ax] ** 2 * d[o] for o in weno.BIG_OFFSETS) for ax in range(3)]
    for ax in range(3):
        add = (r[ax] - 2.0 / 9.0 * (r[0] + r[1] + r[2])) / 6.0
        assert np.allclose(a[3 + ax], add, atol=1e-13)
    for k, (p, q) in enumerate(((0, 1), (1, 2), (0, 2))):
        ade = sum(o[p] * o[q] * d[o] for o in weno.BIG_OFFSETS if o[p] and o[q]) / 4.0
        assert np.allclose(a[6 + k], ade, atol=1e-13)
    beta0 = (a[:3] ** 2).sum(0) + 13.0 / 3.0 * (a[3:6] ** 2).sum(0) + 7.0 / 6.0 * (a[6:] ** 2).sum(0)
    assert np.allclose(rec["beta"][0, :, idx], beta0, rtol=1e-12)
    for m, offs in enumerate(weno.SUB_OFFSETS):
        ea, eb, eab, ec = offs
        ax_a = next(i for i in range(3) if ea[i])
        ax_b = next(i for i in range(3) if eb[i])
        ax_c = next(i for i in range(3) if ec[i])
        sa, sb, sc = ea[ax_a], eb[ax_b], ec[ax_c]
        b = rec["b"][idx, m]
        assert np.allclose(b[ax_c], sc * d[ec], atol=1e-13)
        assert np.allclose(sa * b[ax_a], (2 * d[ea] - d[eb] + d[eab]) / 3.0, atol=1e-13)
        assert np.allclose(sb * b[ax_b], (2 * d[eb] - d[ea] + d[eab]) / 3.0, atol=1e-13)
        assert np.allclose(rec["beta"][1 + m, :, idx], (b ** 2).sum(0), rtol=1e-12)


def test_hand_worked_step():
    """Unit cubes, centre value 0, every neighbour with o_x = +1 equal to 1:
    P_0 = X/2 + (X^2 - 1/12)/2 gives beta_0 = 1/4 + (13/3)/4 = 4/3; the
    sub-stencils reaching +x have slope 1 (beta = 1), the others are flat."""
    vp = box(5, 1.0)
    data = np.zeros((5, 5, 5, 5))
    data[:, 3:, :, :] = 1.0
    eps = 1e-8
    rec, _ = build(vp, lambda xq, wj, V, c: data, eps=eps)
    idx = centre(rec)
    beta = rec["beta"][:, 0, idx]
    assert abs(beta[0] - 4.0 / 3.0) < 1e-13
    assert sorted(np.round(beta[1:], 12)) == [0.0] * 12 + [1.0] * 12
    assert abs(rec["tau"][0, idx] - 5.0 / 6.0) < 1e-13
    # The flat stencils dominate: the WENO value at the -x face centre is
    # close to the centre value 0, while P_0 alone gives -1/4 + 1/12 = -1/6.
    x = rec["c"][:, idx] + np.array([-0.5, 0.0, 0.0])
    sel = weno.select(rec, np.array([[idx]]))
    vals, grads = weno.eval_polys(sel, x[:, None, None])
    val, _ = weno.combine(sel, vals, grads)
    assert abs(vals[0, 0, 0, 0] + 1.0 / 6.0) < 1e-13
    assert abs(val[0, 0, 0]) < 1e-6


def test_positivity_mask_of_linear_pressure_ramp():
    """Density 1, no momentum, energy linear in x with p(x_c) = 0.4 and slope
    -1 per cell: every polynomial is exact, so p < 0 exactly at the Gauss
    points with x - x_c > 0.4, i.e. the four points of the +x face
    (x - x_c = 1/2) and none of the others (|x - x_c| <= 1/(2 sqrt 3))."""
    vp = box(5, 1.0)
    gamma = 1.4

    def avg(xq, wj, V, c):
        p = 0.4 - (c[0] - 2.5)
        return np.stack([np.ones_like(p), 0 * p, 0 * p, 0 * p, p / (gamma - 1.0)])
    rec, _ = build(vp, avg)
    idx = centre(rec)
    sel = weno.select(rec, np.array([[idx]]))
    cc = rec["c"][:, idx]
    g = geo.GNODE
    for d in range(3):
        for side in (-1, 1):
            for ga in (-g, g):
                for gb in (-g, g):
                    off = np.zeros(3)
                    off[d] = 0.5 * side
                    off[(d + 1) % 3] = ga
                    off[(d + 2) % 3] = gb
                    vals, _ = weno.eval_polys(sel, (cc + off)[:, None, None])
                    trig = weno.positivity_trigger(vals, gamma)[0, 0]
                    assert trig == (d == 0 and side == 1)
