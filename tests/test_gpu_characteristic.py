"""Reconstruction in characteristic variables (Sec. 4) on the GPU FP64 path
against the oracle, element by element through the C ABI: Gauss-point
states after the fallback, face fluxes, one- and two-stage steps, on ragged
grids with periodic, outflow and symmetric ends, smooth and discontinuous
data (the fallback active).  Bar as for the component-wise path: normalised
max-norm error <= 1e-12 per variable, momentum measured against the scale
sqrt(max rho * max rho E) where the data start at rest.  Also: an entropy wave keeps velocity
and pressure constant at every Gauss point, and the FP32 mode stays within
1e-5 (L1 of density) of FP64."""

import numpy as np
import pytest
import torch

import oracle
from oracle import scheme
from tests.helpers import blast_state, nerr, smooth_state

pytestmark = pytest.mark.gpu

TOL = 1e-12

CASES = {
    "periodic_smooth": dict(n=(12, 10, 9), L=(1.2, 1.0, 0.9), bc=("periodic",) * 3, mu=0.0,
                            state=lambda n, L: smooth_state(n, L, 1, mach=0.6)),
    "outflow_blast_viscous": dict(n=(14, 11, 10), L=(1.0, 1.0, 1.0), bc=("outflow",) * 3, mu=1e-3,
                                  state=lambda n, L: blast_state(n, L)),
    "symmetric_octant_blast": dict(n=(13, 11, 10), L=(1.0, 1.0, 1.0), bc=(("symmetric", "outflow"),) * 3, mu=0.0,
                                   state=lambda n, L: blast_state(n, L, centre=(0.0, 0.0, 0.0), radius=0.5)),
    "mixed_ends": dict(n=(9, 12, 10), L=(0.9, 1.2, 1.0),
                       bc=(("symmetric", "outflow"), "periodic", ("outflow", "symmetric")), mu=0.0,
                       state=lambda n, L: smooth_state(n, L, 5, mach=0.5)),
    # longer than one 64-cell tile row along x, ragged in every direction
    "long_x_mixed": dict(n=(67, 5, 3), L=(3.35, 0.5, 0.3), bc=(("outflow", "symmetric"), "periodic", "symmetric"),
                         mu=5e-4, state=lambda n, L: blast_state(n, L, centre=(1.6, 0.25, 0.0), radius=0.4)),
}


@pytest.fixture(scope="module")
def hg():
    from paper_1909_01580_amd import hgks
    hgks.load()
    return hgks


def setup(hg, case, precision="fp64"):
    c = CASES[case]
    Q = c["state"](c["n"], c["L"])
    prob = oracle.uniform_problem(c["n"], (0.0, 0.0, 0.0), c["L"], bc=c["bc"],
                                  params=oracle.Params(mu=c["mu"], characteristic=True))
    ctx = hg.Context(c["n"], bc=c["bc"], mu=c["mu"], precision=precision, characteristic=True)
    ctx.set_uniform_grid((0.0, 0.0, 0.0), c["L"])
    ctx.set_state(torch.tensor(Q, device="cuda:0"))
    return Q, prob, ctx


@pytest.mark.parametrize("case", list(CASES))
def test_gp_states(hg, case):
    Q, prob, ctx = setup(hg, case)
    dt = oracle.max_dt(prob, Q, 0.35)
    gpu = ctx.debug_gp_states(dt).cpu().numpy()
    ref = scheme.gp_states(prob, Q, dt)
    for k in range(4):
        # at rest the momentum is zero up to the rounding of R (L Q)
        e = nerr(gpu[..., k], ref[..., k], axis_var=4, mom_scale=True)
        assert e.max() < TOL * (1 if k == 0 else 10), (k, e)
    if "blast" in case:
        _, count = ctx.check()
        assert count > 100


@pytest.mark.parametrize("case", list(CASES))
def test_face_flux(hg, case):
    Q, prob, ctx = setup(hg, case)
    dt = oracle.max_dt(prob, Q, 0.35)
    gpu = ctx.debug_face_flux(dt).cpu().numpy()
    ref = scheme.face_fluxes(prob, Q, dt)
    for k in range(2):
        scale = np.abs(ref[..., k, :]).max()
        err = np.abs(gpu[..., k, :] - ref[..., k, :]).max() / scale
        assert err < TOL * (1 if k == 0 else 100), (k, err)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("n_stages", [1, 2])
def test_step(hg, case, n_stages):
    Q, prob, ctx = setup(hg, case)
    ref = Q
    for _ in range(2 if n_stages == 2 else 1):
        dt = oracle.max_dt(prob, ref, 0.35)
        ref = oracle.step(prob, ref, dt, n_stages=n_stages)
        ctx.step(dt, n_stages)
    e = nerr(ctx.get_state().cpu().numpy(), ref, mom_scale=True)
    assert e.max() < TOL, e


def test_differs_from_componentwise(hg):
    """The option changes the result on discontinuous data (it is not a
    no-op), and the component-wise path is untouched by it."""
    Q, prob, ctx = setup(hg, "outflow_blast_viscous")
    c = CASES["outflow_blast_viscous"]
    plain = hg.Context(c["n"], bc=c["bc"], mu=c["mu"])
    plain.set_uniform_grid((0.0, 0.0, 0.0), c["L"])
    plain.set_state(torch.tensor(Q, device="cuda:0"))
    dt = oracle.max_dt(prob, Q, 0.35)
    ctx.step(dt, 2)
    plain.step(dt, 2)
    a, b = ctx.get_state().cpu().numpy(), plain.get_state().cpu().numpy()
    assert np.abs(a - b).max() > 1e-6
    prob0 = oracle.uniform_problem(c["n"], (0.0, 0.0, 0.0), c["L"], bc=c["bc"], params=oracle.Params(mu=c["mu"]))
    assert nerr(b, oracle.step(prob0, Q, dt)).max() < TOL


def test_entropy_wave_keeps_velocity_and_pressure(hg):
    n, L = (17, 9, 7), (1.0, 1.0, 1.0)
    x = (np.arange(n[0]) + 0.5) / n[0]
    y = (np.arange(n[1]) + 0.5) / n[1]
    Z, Y, X = np.meshgrid(np.arange(n[2]), y, x, indexing="ij")
    rho = 1.0 + 0.8 * (X > 0.45) + 0.1 * np.sin(2 * np.pi * Y)
    u = np.array([0.7, -0.3, 0.2])
    Q = np.concatenate([rho[None], u[:, None, None, None] * rho, (1.0 / 0.4 + 0.5 * rho * (u @ u))[None]])
    ctx = hg.Context(n, weno_eps=1e-3, characteristic=True)
    ctx.set_uniform_grid((0.0, 0.0, 0.0), L)
    ctx.set_state(torch.tensor(Q, device="cuda:0"))
    gp = ctx.debug_gp_states(0.01).cpu().numpy()[..., 0]   # values [..., 24, 5]
    V = gp[..., 1:4] / gp[..., 0:1]
    p = 0.4 * (gp[..., 4] - 0.5 * (gp[..., 1:4] ** 2).sum(axis=-1) / gp[..., 0])
    assert np.abs(V - u).max() < 1e-13 and np.abs(p - 1.0).max() < 1e-13


def test_mixed_precision_close_to_fp64(hg):
    Q, prob, c64 = setup(hg, "periodic_smooth")
    _, _, c32 = setup(hg, "periodic_smooth", precision="mixed")
    for _ in range(5):
        dt = c64.max_dt(0.35)
        c64.step(dt, 2)
        c32.step(dt, 2)
    a, b = c64.get_state().cpu().numpy()[0], c32.get_state().cpu().numpy()[0]
    assert np.abs(a - b).sum() / np.abs(a).sum() < 1e-5


# ------------------------------------------------------------ hexahedral grids
HEX_PERIOD = (2.0, 2.0, 2.0)


def hex_blast(X, Y, Z, gamma=1.4):
    from paper_1909_01580_amd import workloads as wl
    r = np.sqrt((X - 0.9) ** 2 + (Y - 1.0) ** 2 + (Z - 1.1) ** 2)
    inside = r < 0.6
    rho = np.where(inside, 1.0, 0.125)
    p = np.where(inside, 1.0, 0.1)
    zero = np.zeros_like(rho)
    return wl.conservative(rho, zero + 0.3, zero, zero - 0.2, p, gamma)


def hex_setup(hg, kind, precision="fp64", mu=0.0):
    from paper_1909_01580_amd import workloads as wl
    n = (10, 9, 8)
    moving = kind.startswith("moving")
    t, dt = 0.1, 0.03
    v0 = wl.sine_mesh_vertices(n, t, amp=0.1, omega=np.pi, static=not moving)
    v1 = wl.sine_mesh_vertices(n, t + dt, amp=0.1, omega=np.pi) if moving else None
    Q = wl.hex_average(v0, HEX_PERIOD, hex_blast if "blast" in kind else wl.pulse_point)
    params = oracle.Params(mu=mu, characteristic=True)
    ctx = hg.Context(n, moving=True, characteristic=True, precision=precision, mu=mu)
    ctx.set_vertices(torch.tensor(v0, device="cuda:0"), HEX_PERIOD)
    ctx.set_state(torch.tensor(Q, device="cuda:0"))
    static = oracle.vertex_problem(n, v0, HEX_PERIOD, params=params)
    if "blast" in kind:
        dt = oracle.max_dt(static, Q, 0.35)
    prob = oracle.vertex_problem(n, v0, HEX_PERIOD, params=params, verts_next=v1)
    return ctx, Q, static, prob, v1, dt


@pytest.mark.parametrize("kind", ["static_smooth", "static_blast", "moving_smooth", "moving_blast_viscous"])
def test_hex_characteristic(hg, kind):
    """Characteristic reconstruction on the non-coplanar static mesh and the
    moving mesh (projection frame at each face centre): Gauss-point states,
    fallback words (bit for bit), face fluxes and a two-stage step against
    the oracle, FP64, 1e-12 (momentum against sqrt(max rho max rho E))."""
    ctx, Q, static, prob, v1, dt = hex_setup(hg, kind, mu=1e-3 if "viscous" in kind else 0.0)
    gpu = ctx.debug_gp_states(dt).cpu().numpy()
    ref = scheme.gp_states(static, Q, dt)
    for k in range(4):
        e = nerr(gpu[..., k], ref[..., k], axis_var=4, mom_scale=True)
        assert e.max() < TOL * (1 if k == 0 else 10), (k, e)
    mask = scheme.fallback_mask(static, Q, dt)
    assert np.array_equal(ctx.debug_fallback_mask(dt).cpu().numpy().astype(np.uint32), mask)
    gf = ctx.debug_face_flux(dt).cpu().numpy()
    rf = scheme.face_fluxes(static, Q, dt)
    for k in range(2):
        err = np.abs(gf[..., k, :] - rf[..., k, :]).max() / np.abs(rf[..., k, :]).max()
        assert err < TOL * (1 if k == 0 else 100), (k, err)
    if v1 is not None:
        ctx.set_next_vertices(torch.tensor(v1, device="cuda:0"))
    ctx.step(dt, 2)
    e = nerr(ctx.get_state().cpu().numpy(), oracle.step(prob, Q, dt), mom_scale=True)
    assert e.max() < TOL, e


def test_hex_characteristic_mixed_and_componentwise(hg):
    """On the moving mesh the FP32 mode stays within 1e-5 (L1 of density) of
    FP64 over three steps, and the option is not the component-wise scheme."""
    from paper_1909_01580_amd import workloads as wl
    n, dt = (10, 9, 8), 0.02
    out = {}
    for label, prec, charv in (("f64", "fp64", True), ("f32", "mixed", True), ("cw", "fp64", False)):
        ctx = hg.Context(n, moving=True, characteristic=charv, precision=prec)
        v0 = wl.sine_mesh_vertices(n, 0.0, amp=0.1, omega=np.pi)
        ctx.set_vertices(torch.tensor(v0, device="cuda:0"), HEX_PERIOD)
        ctx.set_state(torch.tensor(wl.hex_average(v0, HEX_PERIOD, hex_blast), device="cuda:0"))
        for s in range(3):
            ctx.set_next_vertices(torch.tensor(wl.sine_mesh_vertices(n, (s + 1) * dt, amp=0.1, omega=np.pi),
                                               device="cuda:0"))
            ctx.step(dt, 2)
        out[label] = ctx.get_state().cpu().numpy()
        assert ctx.check()[0] == 0
    r = out["f64"][0]
    assert np.abs(out["f32"][0] - r).sum() / np.abs(r).sum() < 1e-5
    assert np.abs(out["cw"][0] - r).max() > 1e-6
