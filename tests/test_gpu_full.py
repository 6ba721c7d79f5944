"""Full-size workloads in the launch configuration the benchmark times:
sampled FP64 parity against the oracle (the oracle advances a 13^3 patch
around each sampled cell; a two-stage step at a cell depends only on cells
within 4 of it), mixed-precision tolerance against FP64, conservation and
positivity.

* 128^3 Taylor-Green vortex (periodic, viscous, Prandtl number 0.72 as
  the benchmark runs it);
* 256^3 spherical explosion (outflow, inviscid) with the fallback active;
* the 48 uneven periodic problems of the batched benchmark (about 1.0e7
  cells) in one batch with persistent launches and a captured graph:
  sampled FP64 parity in viscous and inviscid grids of different shapes,
  and the mixed batch within the FP32 tolerance of the FP64 one;
* 128^3 moving mesh with a density pulse: sampled parity from 13^3 vertex
  patches that the oracle treats as periodic (the seam cell, 6 cells from
  the centre, is distorted, but what it produces cannot reach the centre in
  two stages; a CPU test pins that the patch centre equals the full
  periodic oracle step), plus conservation and the mixed tolerance over 10
  steps.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1909_01580_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    from paper_1909_01580_amd import hgks
    hgks.load()
    return hgks


def patch_step(Q, centre, h, bc, mu, dt, prandtl=1.0):
    """Oracle step of the 13^3 patch around `centre`; returns the centre."""
    n = Q.shape[1:][::-1]
    idx = []
    for d, c in enumerate(centre):
        r = np.arange(c - 6, c + 7)
        idx.append(r % n[d] if bc == "periodic" else np.clip(r, 0, n[d] - 1))
    patch = Q[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]]
    prob = oracle.uniform_problem((13, 13, 13), (0, 0, 0), (13 * h,) * 3, bc=("outflow",) * 3,
                                  params=oracle.Params(mu=mu, prandtl=prandtl))
    return oracle.step(prob, np.ascontiguousarray(patch), dt)[:, 6, 6, 6]


def test_taylor_green_128(hg):
    n = 128
    q0 = wl.tgv_state(n)
    h = 2 * np.pi / n
    runs = {}
    for prec in ("fp64", "mixed"):
        ctx = hg.Context((n, n, n), mu=wl.TGV_MU, precision=prec, prandtl=wl.TGV_PRANDTL)
        ctx.set_uniform_grid((-np.pi,) * 3, (2 * np.pi,) * 3)
        ctx.set_state(torch.tensor(q0, device="cuda:0"))
        dt0 = ctx.max_dt(0.35)
        ctx.step(dt0, 2)
        first = ctx.get_state().cpu().numpy()
        for _ in range(9):
            ctx.step(ctx.max_dt(0.35), 2)
        runs[prec] = (dt0, first, ctx.get_state().cpu().numpy(), ctx.totals())
    dt0, first, _, tot = runs["fp64"]
    for c in [(0, 0, 0), (127, 5, 77), (64, 64, 64), (17, 127, 3)]:
        ref = patch_step(q0, c, h, "periodic", wl.TGV_MU, dt0, wl.TGV_PRANDTL)
        got = first[:, c[2], c[1], c[0]]
        scale = np.array([1.0, 1.0, 1.0, 1.0, np.abs(q0[4]).max()])
        assert np.all(np.abs(got - ref) / scale < 1e-12), (c, got - ref)
    r64, rmx = runs["fp64"][2][0], runs["mixed"][2][0]
    assert np.abs(rmx - r64).sum() / np.abs(r64).sum() < 1e-5
    tot0 = np.array([q0[v].sum() * h ** 3 for v in range(5)])
    assert np.abs(np.array(tot) - tot0).max() < 1e-13 * np.abs(tot0).max()


def test_explosion_256(hg):
    """The 256^3 spherical explosion as configured (outflow, to t = 0.1):
    sampled FP64 parity after the first step, positivity after every step
    in FP64 and mixed, the limiter active throughout, and the mixed run's
    L1 density difference from FP64 at t = 0.1 (reported and bounded)."""
    n = 256
    q0 = wl.explosion_state(n)
    h = 1.0 / n
    ctx = hg.Context((n, n, n), bc=("outflow",) * 3)
    ctx.set_uniform_grid((0, 0, 0), (1, 1, 1))
    ctx.set_state(torch.tensor(q0, device="cuda:0"))
    dt = ctx.max_dt(0.35)
    ctx.step(dt, 2)
    _, fallback = ctx.check()
    assert fallback > 1000                    # the limiter is exercised
    first = ctx.get_state().cpu().numpy()
    i_front = int((0.5 + 0.4) / h)           # on the initial discontinuity
    for c in [(0, 0, 0), (255, 128, 0), (128, 128, 128), (i_front, 128, 128), (i_front - 1, 131, 127)]:
        ref = patch_step(q0, c, h, "outflow", 0.0, dt)
        got = first[:, c[2], c[1], c[0]]
        scale = np.array([1.0, 1.0, 1.0, 1.0, 2.5])
        assert np.all(np.abs(got - ref) / scale < 1e-12), (c, got - ref)

    def run_to(cx, t_end, t0=0.0):
        """Steps to t_end with the positivity check after each; returns the
        steps taken and how many of them used the fallback somewhere."""
        t, steps, active = t0, 0, 0
        while t < t_end * (1 - 1e-12):
            d = min(cx.max_dt(0.35), t_end - t)
            cx.step(d, 2)
            t += d
            steps += 1
            nonphys, fb = cx.check()
            assert nonphys == 0, (t, nonphys)
            active += fb > 0
        return steps, active

    steps64, act64 = run_to(ctx, 0.1, dt)
    mx = hg.Context((n, n, n), bc=("outflow",) * 3, precision="mixed")
    mx.set_uniform_grid((0, 0, 0), (1, 1, 1))
    mx.set_state(torch.tensor(q0, device="cuda:0"))
    steps32, act32 = run_to(mx, 0.1)
    r64 = ctx.get_state()[0]
    r32 = mx.get_state()[0]
    l1 = float((r32 - r64).abs().sum() / r64.abs().sum())
    print(f"explosion 256^3 to t = 0.1: {steps64 + 1} FP64 steps ({act64} more with fallback points), "
          f"{steps32} mixed steps ({act32} with fallback points), mixed vs FP64 L1(rho) {l1:.3e}", flush=True)
    assert act64 > 0 and act32 > 0           # the limiter acts beyond the first step
    assert l1 < 1e-3


def hex_patch_step(V0, V1, Q, centre, dt, n):
    """Oracle step of the 13^3 vertex patch around `centre` (at least 6
    cells from the grid's edges), treated as periodic with the nominal
    period of 13 cells; returns the centre."""
    sl = (slice(None),) + tuple(slice(c - 6, c + 7) for c in centre[::-1])
    va, vb, q = (np.ascontiguousarray(a[sl]) for a in (V0, V1, Q))
    prob = oracle.vertex_problem((13, 13, 13), va, (13 * 2.0 / n,) * 3, verts_next=vb)
    return oracle.step(prob, q, dt)[:, 6, 6, 6]


MOVING_N = 128


def moving_verts(t):
    return wl.sine_mesh_vertices(MOVING_N, t, amp=0.05, omega=2 * np.pi)


@pytest.fixture(scope="module")
def moving_q0():
    return wl.hex_average(moving_verts(0.0), (2.0, 2.0, 2.0), wl.pulse_point)


def test_moving_mesh_128_sampled_parity(hg, moving_q0):
    """One FP64 step of the benchmark's moving mesh from t = 0.1 (the nodes
    displaced and moving) against oracle patches around sampled cells."""
    n = MOVING_N
    t0 = 0.1
    V0 = moving_verts(t0)
    ctx = hg.Context((n, n, n), moving=True, precision="fp64")
    ctx.set_vertices(torch.tensor(V0, device="cuda:0"), (2.0, 2.0, 2.0))
    ctx.set_state(torch.tensor(moving_q0, device="cuda:0"))
    dt = ctx.max_dt(0.35)
    V1 = moving_verts(t0 + dt)
    ctx.set_next_vertices(torch.tensor(V1, device="cuda:0"))
    ctx.step(dt, 2)
    got = ctx.get_state().cpu().numpy()
    scale = np.abs(moving_q0).reshape(5, -1).max(axis=1)
    for c in [(64, 64, 64), (70, 58, 66), (20, 100, 40), (110, 9, 77), (7, 60, 118)]:
        ref = hex_patch_step(V0, V1, moving_q0, c, dt, n)
        err = np.abs(got[:, c[2], c[1], c[0]] - ref) / scale
        assert np.all(err < 1e-12), (c, err)


def test_moving_mesh_128(hg, moving_q0):
    n = MOVING_N
    P = (2.0, 2.0, 2.0)
    verts = moving_verts
    q0 = moving_q0
    out = {}
    for prec in ("fp64", "mixed"):
        ctx = hg.Context((n, n, n), moving=True, precision=prec)
        ctx.set_vertices(torch.tensor(verts(0.0), device="cuda:0"), P)
        ctx.set_state(torch.tensor(q0, device="cuda:0"))
        tot0 = np.array(ctx.totals())
        dt = 0.5 * ctx.max_dt(0.35)
        t = 0.0
        for _ in range(10):
            ctx.set_next_vertices(torch.tensor(verts(t + dt), device="cuda:0"))
            ctx.step(dt, 2)
            t += dt
        out[prec] = ctx.get_state()[0]
        assert np.abs(np.array(ctx.totals()) - tot0).max() < 1e-13 * np.abs(tot0).max()
    assert float((out["mixed"] - out["fp64"]).abs().sum() / out["fp64"].abs().sum()) < 1e-5


def test_batched_48_grids(hg):
    problems = wl.batch_problems()
    grids = [{"n": p["n"], "length": p["length"], "mu": p["mu"]} for p in problems]
    out = {}
    for prec in ("fp64", "mixed"):
        b = hg.Batch(grids, precision=prec)
        for i, p in enumerate(problems):
            b.set_state(i, torch.tensor(p["state"], device="cuda:0"))
        b.sync()
        for phase in range(len(hg.PHASES)):     # persistent launches, as timed
            b.set_launch(phase, 2048)
        b.capture(0.35, 1, 2)
        b.replay()
        b.sync()
        out[prec] = (b.dt(), [b.get_state(i).cpu().numpy() for i in range(b.n)])
    dts, q64 = out["fp64"]
    h = 2 * np.pi / 64
    samples = {0: [(0, 0, 0), (63, 50, 47)], 1: [(47, 31, 95), (20, 3, 40)], 17: [(24, 24, 24)],
               30: [(31, 63, 0), (5, 33, 70)], 47: [(16, 47, 63)]}
    for g, cells in samples.items():
        q0 = problems[g]["state"]
        scale = np.abs(q0).reshape(5, -1).max(axis=1)
        for c in cells:
            ref = patch_step(q0, c, h, "periodic", problems[g]["mu"], dts[g])
            err = np.abs(q64[g][:, c[2], c[1], c[0]] - ref) / scale
            assert np.all(err < 1e-12), (g, c, err)
    for g in range(len(problems)):
        r64, rmx = q64[g][0], out["mixed"][1][g][0]
        assert np.abs(rmx - r64).sum() / np.abs(r64).sum() < 1e-5, g
