"""The step with its time step formed on the device (hgks_step_cfl) through
the C ABI.

* Bit for bit the same states and time steps as hgks_max_dt followed by
  hgks_step (the CFL rule of Sec. 4 and the stage of Sec. 3), in FP64 and
  mixed precision, on a periodic viscous box with the Prandtl correction
  and on an outflow box with a blast (fallback points), over several steps
  queued without a host synchronisation.
* A state with a non-physical cell: dt = 0, the state is left as it was,
  and the next hgks_sync reports HGKS_ENONPHYS once.
* Argument and call-order errors; a moving mesh is refused.
"""

import numpy as np
import pytest
import torch

from paper_1909_01580_amd import workloads as wl
from tests.helpers import blast_state, smooth_state

pytestmark = pytest.mark.gpu

CASES = {
    "periodic_prandtl": dict(n=(12, 10, 9), L=(1.2, 1.0, 0.9), bc=("periodic",) * 3, mu=2e-3, prandtl=0.72,
                             state=lambda n, L: smooth_state(n, L, 31, mach=0.4)),
    "outflow_blast": dict(n=(14, 12, 10), L=(1.0, 1.0, 1.0), bc=("outflow",) * 3, mu=0.0, prandtl=1.0,
                          state=lambda n, L: blast_state(n, L)),
}


@pytest.fixture(scope="module")
def hg():
    from paper_1909_01580_amd import hgks
    hgks.load()
    assert torch.cuda.is_available()
    return hgks


def context(hg, c, precision):
    ctx = hg.Context(c["n"], bc=c["bc"], mu=c["mu"], prandtl=c["prandtl"], precision=precision)
    ctx.set_uniform_grid((0.0, 0.0, 0.0), c["L"])
    return ctx


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_equals_max_dt_and_step(hg, case, precision):
    c = CASES[case]
    q0 = torch.tensor(c["state"](c["n"], c["L"]), device="cuda:0")
    steps = 4
    host = context(hg, c, precision)
    host.set_state(q0)
    dts = []
    for _ in range(steps):
        dts.append(host.max_dt(0.35))
        host.step(dts[-1], 2)
    dev = context(hg, c, precision)
    dev.set_state(q0)
    dt_dev = torch.full((steps,), -1.0, dtype=torch.float64, device="cuda:0")
    for k in range(steps):
        dev.step_cfl(0.35, 2, dt_dev[k:k + 1])
    dev.sync()
    assert dt_dev.cpu().tolist() == dts
    assert torch.equal(dev.get_state(), host.get_state())
    # the one-stage update and no dt output
    host.step(host.max_dt(0.5), 1)
    dev.step_cfl(0.5, 1)
    dev.sync()
    assert torch.equal(dev.get_state(), host.get_state())


def test_nonphysical_state_is_left_and_reported(hg):
    c = CASES["periodic_prandtl"]
    q = c["state"](c["n"], c["L"])
    q[4, 2, 3, 4] = 0.5 * (q[1, 2, 3, 4] ** 2 + q[2, 2, 3, 4] ** 2 + q[3, 2, 3, 4] ** 2) / q[0, 2, 3, 4] - 0.1
    ctx = context(hg, c, "fp64")
    ctx.set_state(torch.tensor(q, device="cuda:0"))
    dt_dev = torch.full((2,), -1.0, dtype=torch.float64, device="cuda:0")
    ctx.step_cfl(0.35, 2, dt_dev[0:1])
    ctx.step_cfl(0.35, 2, dt_dev[1:2])
    with pytest.raises(hg.HGKSError) as e:
        ctx.sync()
    assert e.value.status == hg.HGKS_ENONPHYS
    ctx.sync()                                      # reported once, then clear
    assert dt_dev.cpu().tolist() == [0.0, 0.0]
    assert np.array_equal(ctx.get_state().cpu().numpy(), q)
    # a physical state afterwards steps again, with a fresh status word
    good = c["state"](c["n"], c["L"])
    ctx.set_state(torch.tensor(good, device="cuda:0"))
    ctx.step_cfl(0.35, 2, dt_dev[0:1])
    ctx.sync()
    assert dt_dev[0].item() > 0.0
    assert not np.array_equal(ctx.get_state().cpu().numpy(), good)


def test_errors(hg):
    c = CASES["periodic_prandtl"]
    ctx = context(hg, c, "fp64")
    with pytest.raises(hg.HGKSError) as e:
        ctx.step_cfl(0.35, 2)                       # no state yet
    assert e.value.status == hg.HGKS_ESTATE
    ctx.set_state(torch.tensor(c["state"](c["n"], c["L"]), device="cuda:0"))
    for cfl, stages in ((0.0, 2), (-1.0, 2), (float("inf"), 2), (float("nan"), 2), (0.35, 3), (0.35, 0)):
        with pytest.raises(hg.HGKSError) as e:
            ctx.step_cfl(cfl, stages)
        assert e.value.status == hg.HGKS_EINVAL
    with pytest.raises(ValueError):
        ctx.step_cfl(0.35, 2, torch.zeros(1, dtype=torch.float32, device="cuda:0"))
    ctx.sync()
    n = (8, 8, 8)
    m = hg.Context(n, moving=True)
    m.set_vertices(torch.tensor(wl.sine_mesh_vertices(n, 0.0, amp=0.1, omega=np.pi), device="cuda:0"),
                   (2.0, 2.0, 2.0))
    one = np.ones(n[::-1])
    m.set_state(torch.tensor(wl.conservative(one, one, one, one, one), device="cuda:0"))
    with pytest.raises(hg.HGKSError) as e:
        m.step_cfl(0.35, 2)
    assert e.value.status == hg.HGKS_EUNSUPPORTED
