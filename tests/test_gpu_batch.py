"""Batched grids (one persistent launch per phase, per-grid dt on device,
HIP graph) against single-grid contexts: the same per-cell and per-face
code must give the same results; graph replays must equal eager steps;
persistence (any workgroup count) must not change results."""

import numpy as np
import pytest
import torch

from tests.helpers import nerr, smooth_state

pytestmark = pytest.mark.gpu

GRIDS = [
    {"n": (12, 10, 9), "length": (1.2, 1.0, 0.9), "mu": 0.0},
    {"n": (8, 14, 11), "length": (0.8, 1.4, 1.1), "mu": 1e-3},
    {"n": (16, 8, 8), "length": (1.6, 0.8, 0.8), "mu": 0.0},
    {"n": (9, 9, 13), "length": (0.9, 0.9, 1.3), "mu": 5e-4},
    {"n": (10, 12, 10), "length": (1.0, 1.2, 1.0), "mu": 0.0},
]


@pytest.fixture(scope="module")
def hg():
    from paper_1909_01580_amd import hgks
    hgks.load()
    return hgks


def states():
    return [smooth_state(g["n"], g["length"], 40 + i, mach=0.5) for i, g in enumerate(GRIDS)]


# reconstruction options of the whole batch: the stencils of Sec. 2, those
# of Remark 1, characteristic variables (Sec. 4)
OPTIONS = {"S": {}, "S_prime": {"stencil": "S_prime"}, "characteristic": {"characteristic": True}}


def make_batch(hg, precision, qs, option="S"):
    kw = dict(OPTIONS[option])
    if "characteristic" in kw:
        kw["characteristic"] = 1
    b = hg.Batch(GRIDS, precision=precision, **kw)
    for i, q in enumerate(qs):
        b.set_state(i, torch.tensor(q, device="cuda:0"))
    return b


def run_single(hg, precision, qs, dts_per_step, option="S"):
    out = []
    for i, g in enumerate(GRIDS):
        ctx = hg.Context(g["n"], mu=g["mu"], precision=precision, **OPTIONS[option])
        ctx.set_uniform_grid((0, 0, 0), g["length"])
        ctx.set_state(torch.tensor(qs[i], device="cuda:0"))
        for dts in dts_per_step:
            ctx.step(dts[i], 2)
        out.append(ctx.get_state().cpu().numpy())
    return out


@pytest.mark.parametrize("option", list(OPTIONS))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_grids(hg, precision, option):
    """option: the reconstruction option of every grid (OPTIONS)."""
    qs = states()
    b = make_batch(hg, precision, qs, option)
    dt = torch.empty(len(GRIDS), dtype=torch.float64, device="cuda:0")
    dts_per_step = []
    for _ in range(3):
        b.max_dt(0.35, dt)
        b.sync()
        dts_per_step.append(dt.cpu().numpy().copy())
        b.step(dt, 2)
    b.sync()
    single = run_single(hg, precision, qs, dts_per_step, option)
    # The batch and single-grid kernels run the same per-face and per-cell
    # code, but the compiler may fuse float operations differently in the
    # two kernels: FP64 agrees to round-off, mixed to float rounding.
    tol = 1e-14 if precision == "fp64" else 1e-6
    for i in range(len(GRIDS)):
        got = b.get_state(i).cpu().numpy()
        err = np.abs(got - single[i]).max() / np.abs(single[i]).max()
        assert err < tol, (i, err)
    # per-grid dt equals the single-grid reduction
    for i, g in enumerate(GRIDS):
        ctx = hg.Context(g["n"], mu=g["mu"], precision=precision, **OPTIONS[option])
        ctx.set_uniform_grid((0, 0, 0), g["length"])
        ctx.set_state(torch.tensor(qs[i], device="cuda:0"))
        assert abs(ctx.max_dt(0.35) - dts_per_step[0][i]) <= 1e-15 * dts_per_step[0][i]


@pytest.mark.parametrize("option", list(OPTIONS))
def test_batch_step_against_oracle(hg, option):
    """One two-stage FP64 step of every grid of the batch against the
    oracle's step of that grid (periodic, its own mu and time step),
    element by element: normalised max-norm error <= 1e-12."""
    import oracle

    qs = states()
    b = make_batch(hg, "fp64", qs, option)
    dt = torch.empty(len(GRIDS), dtype=torch.float64, device="cuda:0")
    b.max_dt(0.35, dt)
    b.sync()
    dts = dt.cpu().numpy().copy()
    b.step(dt, 2)
    b.sync()
    for i, g in enumerate(GRIDS):
        prob = oracle.uniform_problem(g["n"], (0.0, 0.0, 0.0), g["length"], bc=("periodic",) * 3,
                                      params=oracle.Params(mu=g["mu"], **OPTIONS[option]))
        assert abs(oracle.max_dt(prob, qs[i], 0.35) - dts[i]) <= 1e-14 * dts[i]
        ref = oracle.step(prob, qs[i], dts[i], n_stages=2)
        e = nerr(b.get_state(i).cpu().numpy(), ref, mom_scale=True)
        assert e.max() < 1e-12, (i, e)


@pytest.mark.parametrize("option", list(OPTIONS))
def test_graph_replay_equals_eager(hg, option):
    qs = states()
    eager = make_batch(hg, "mixed", qs, option)
    graph = make_batch(hg, "mixed", qs, option)
    graph.capture(0.35, 2, 2)
    dt = torch.empty(len(GRIDS), dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        for _ in range(2):
            eager.max_dt(0.35)            # into the batch's own dt array
            eager.max_dt(0.35, dt)        # and into dt, on the batch's stream
            eager.step(dt, 2)
        eager.sync()
        graph.replay()
        graph.sync()
        # eager work between replays (the replays must not depend on it)
        _ = torch.ones(1000, device="cuda:0").sum().item()
        assert graph.dt() == eager.dt()
        for i in range(len(GRIDS)):
            a = graph.get_state(i).cpu().numpy()
            e = eager.get_state(i).cpu().numpy()
            assert np.array_equal(a, e), (rep, i, np.abs(a - e).max())


@pytest.mark.parametrize("option", list(OPTIONS))
@pytest.mark.parametrize("wg", [8, 64, 1024])
def test_persistent_workgroups_do_not_change_results(hg, wg, option):
    qs = states()
    ref = make_batch(hg, "fp64", qs, option)
    alt = make_batch(hg, "fp64", qs, option)
    for phase in range(5):
        alt.set_launch(phase, wg)
    dt = torch.empty(len(GRIDS), dtype=torch.float64, device="cuda:0")
    for b in (ref, alt):
        b.max_dt(0.35, dt)
        b.step(dt, 2)
        b.sync()
    for i in range(len(GRIDS)):
        assert np.array_equal(ref.get_state(i).cpu().numpy(), alt.get_state(i).cpu().numpy())


@pytest.mark.parametrize("tile,band", [((64, 4, 1), 16), ((16, 16, 1), 4), ((8, 8, 4), 32), ((256, 1, 1), 1)])
def test_tile_shapes_do_not_change_results(hg, tile, band):
    """Cell tiles as boxes of cells and other flux band heights (the
    autotuner's choices) give the same state bit for bit, eager and in a
    graph captured after the change."""
    qs = states()
    ref = make_batch(hg, "fp64", qs)
    alt = make_batch(hg, "fp64", qs)
    alt.set_tiles(tile, band)
    for phase in (0, 3):
        alt.set_launch(phase, 64)            # persistent walk over box tiles too
    dt = torch.empty(len(GRIDS), dtype=torch.float64, device="cuda:0")
    for b in (ref, alt):
        b.max_dt(0.35, dt)
        b.step(dt, 2)
        b.sync()
    for i in range(len(GRIDS)):
        assert np.array_equal(ref.get_state(i).cpu().numpy(), alt.get_state(i).cpu().numpy()), i
    ref.capture(0.35, 2, 2)
    alt.capture(0.35, 2, 2)
    for b in (ref, alt):
        b.replay()
        b.sync()
    assert ref.dt() == alt.dt()
    for i in range(len(GRIDS)):
        assert np.array_equal(ref.get_state(i).cpu().numpy(), alt.get_state(i).cpu().numpy()), i
    with pytest.raises(hg.HGKSError):
        alt.set_tiles((16, 16, 2), 16)       # product is not 256
    with pytest.raises(hg.HGKSError):
        alt.set_tiles((0, 0, 0), 0)


def test_batch_conservation(hg):
    qs = states()
    b = make_batch(hg, "fp64", qs)
    t0 = np.array(b.totals())
    b.capture(0.35, 5, 2)
    b.replay()
    b.sync()
    t1 = np.array(b.totals())
    assert np.abs(t1 - t0).max() < 1e-13 * np.abs(t0).max()


def test_batch_call_order_and_arguments(hg):
    """Refused batch calls return their status, change nothing, and the
    batch then steps exactly as a fresh one does."""
    lib = hg.load()
    qs = states()

    def refused(status, fn, *args):
        with pytest.raises(hg.HGKSError) as e:
            fn(*args)
        assert e.value.status == status, e.value

    b = hg.Batch(GRIDS, precision="fp64")
    dt = torch.full((b.n,), 1e-3, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    refused(hg.HGKS_ESTATE, b.step, dt, 2)                 # no states yet
    refused(hg.HGKS_ESTATE, b.max_dt, 0.35, dt)
    refused(hg.HGKS_ESTATE, b.get_state, 0)
    for i, q in enumerate(qs[:-1]):
        b.set_state(i, torch.tensor(q, device="cuda:0"))
    refused(hg.HGKS_ESTATE, b.step, dt, 2)                 # one grid still without a state
    b.set_state(len(qs) - 1, torch.tensor(qs[-1], device="cuda:0"))
    refused(hg.HGKS_EINVAL, b.step, dt, 3)
    assert lib.hgks_batch_step(b.h, None, 2) == hg.HGKS_EINVAL
    for cfl in (0.0, -1.0, float("nan"), float("inf")):
        refused(hg.HGKS_EINVAL, b.max_dt, cfl, dt)
        refused(hg.HGKS_EINVAL, b.capture, cfl, 2, 2)
    refused(hg.HGKS_EINVAL, b.capture, 0.35, 0, 2)
    refused(hg.HGKS_ESTATE, b.replay)                      # nothing captured
    for phase, wg in ((-1, 0), (99, 0), (1, 12), (1, 4), (1, 1 << 20)):
        refused(hg.HGKS_EINVAL, b.set_launch, phase, wg)
    for i in (-1, b.n):
        refused(hg.HGKS_EINVAL, hg.hgks_batch_set_state, b.h, i, torch.tensor(qs[0], device="cuda:0"))
        refused(hg.HGKS_EINVAL, hg.hgks_batch_set_uniform_grid, b.h, i, (0, 0, 0), (1, 1, 1))
    for length in ((0.0, 1.0, 1.0), (1.0, float("inf"), 1.0), (1.0, 1.0, float("nan"))):
        refused(hg.HGKS_EINVAL, hg.hgks_batch_set_uniform_grid, b.h, 1, (0, 0, 0), length)
    fresh = make_batch(hg, "fp64", qs)
    for bb in (b, fresh):
        bb.max_dt(0.35, dt)
        bb.step(dt, 2)
    for i in range(b.n):
        assert torch.equal(b.get_state(i), fresh.get_state(i)), i
