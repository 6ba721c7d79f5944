"""Call order and argument errors at the C ABI, on a real context: each is
refused with its status and a message, leaves the context's state alone,
and the context keeps working afterwards (a step after the refused calls
equals the same step on a fresh context)."""

import math

import numpy as np
import pytest
import torch

from tests.helpers import smooth_state

pytestmark = pytest.mark.gpu

N = (10, 9, 8)
L = (1.0, 0.9, 0.8)


@pytest.fixture(scope="module")
def hg():
    from paper_1909_01580_amd import hgks
    hgks.load()
    return hgks


def refused(hg, status, fn, *args):
    with pytest.raises(hg.HGKSError) as e:
        fn(*args)
    assert e.value.status == status, e.value
    assert hg.load().hgks_last_error()


def fresh(hg, **kw):
    ctx = hg.Context(N, mu=1e-3, **kw)
    ctx.set_uniform_grid((0.0, 0.0, 0.0), L)
    return ctx


def test_call_order(hg):
    ctx = hg.Context(N)
    q = torch.tensor(smooth_state(N, L, 1), device="cuda:0")
    refused(hg, hg.HGKS_ESTATE, ctx.step, 1e-3, 2)          # no grid, no state
    refused(hg, hg.HGKS_ESTATE, ctx.max_dt, 0.35)
    refused(hg, hg.HGKS_ESTATE, ctx.get_state)
    ctx.set_uniform_grid((0.0, 0.0, 0.0), L)
    refused(hg, hg.HGKS_ESTATE, ctx.step, 1e-3, 2)          # grid, no state
    refused(hg, hg.HGKS_ESTATE, ctx.totals)
    ctx.set_state(q)
    ctx.step(1e-3, 2)


def test_bad_arguments_leave_the_context_usable(hg):
    q0 = torch.tensor(smooth_state(N, L, 2, mach=0.5), device="cuda:0")
    ctx = fresh(hg)
    ctx.set_state(q0)
    lib = hg.load()
    for dt in (0.0, -1e-3, math.nan, math.inf):
        refused(hg, hg.HGKS_EINVAL, ctx.step, dt, 2)
    for n_stages in (0, 3, -1):
        refused(hg, hg.HGKS_EINVAL, ctx.step, 1e-3, n_stages)
    for cfl in (0.0, -0.3, math.nan):
        refused(hg, hg.HGKS_EINVAL, ctx.max_dt, cfl)
    for length in ((0.0, 1.0, 1.0), (1.0, -1.0, 1.0), (1.0, 1.0, math.nan)):
        refused(hg, hg.HGKS_EINVAL, ctx.set_uniform_grid, (0.0, 0.0, 0.0), length)
    refused(hg, hg.HGKS_EINVAL, ctx.set_uniform_grid, (math.inf, 0.0, 0.0), L)
    assert lib.hgks_set_state(ctx.h, None) == hg.HGKS_EINVAL
    assert lib.hgks_get_state(ctx.h, None) == hg.HGKS_EINVAL
    assert lib.hgks_step(None, 1e-3, 2) != hg.HGKS_OK
    # a box context takes no vertices
    refused(hg, hg.HGKS_EINVAL, ctx.set_vertices, q0[:3], (1.0, 1.0, 1.0))
    # nothing above touched the state or the grid: the same step as a fresh context
    dt = ctx.max_dt(0.35)
    ctx.step(dt, 2)
    ref = fresh(hg)
    ref.set_state(q0)
    assert ref.max_dt(0.35) == dt
    ref.step(dt, 2)
    assert torch.equal(ctx.get_state(), ref.get_state())


def test_moving_context_errors(hg):
    n = (8, 8, 8)
    ctx = hg.Context(n, moving=True)
    verts = torch.zeros((3, 8, 8, 8), dtype=torch.float64, device="cuda:0")
    refused(hg, hg.HGKS_EINVAL, ctx.set_uniform_grid, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    refused(hg, hg.HGKS_ESTATE, ctx.set_next_vertices, verts)   # before set_vertices
    for period in ((0.0, 1.0, 1.0), (1.0, -2.0, 1.0), (1.0, 1.0, math.nan)):
        refused(hg, hg.HGKS_EINVAL, ctx.set_vertices, verts, period)
    from paper_1909_01580_amd import workloads as wl
    v0 = wl.sine_mesh_vertices(n, 0.0, amp=0.1, omega=np.pi)
    ctx.set_vertices(torch.tensor(v0, device="cuda:0"), (2.0, 2.0, 2.0))
    one = np.ones(n[::-1])
    ctx.set_state(torch.tensor(wl.conservative(one, one, one, one, one), device="cuda:0"))
    refused(hg, hg.HGKS_EUNSUPPORTED, ctx.step_checked, 1e-3, 2, 4)
    ctx.step(1e-3, 2)
    assert ctx.check()[0] == 0
