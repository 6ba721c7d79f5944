"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/hgks.h declares, and its host-only logic
(defaults, configuration validation, workspace sizing) behaves."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgks.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hgks_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1909_01580_amd import hgks
    if not os.path.exists(hgks.LIB_PATH):
        pytest.skip("libhgks.so not built")
    return hgks.load()


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    from paper_1909_01580_amd import hgks
    assert sorted(hgks.EXPORTS) == names


def test_defaults_and_workspace(lib):
    from paper_1909_01580_amd import hgks
    cfg = hgks.hgks_default_config(16, 16, 16)
    assert cfg.gamma == 1.4 and cfg.weno_Gamma == 0.0025 and cfg.tau_eps == 0.01 and cfg.tau_C == 1.0
    n = hgks.hgks_workspace_size(cfg)
    # state x3, coefficients, masks, faces, reductions
    N = 16 ** 3
    assert n >= (15 + 50 + 30) * 8 * N
    cfg.precision = hgks.PREC["mixed"]
    assert hgks.hgks_workspace_size(cfg) < n
    cfg.bc[0] = hgks.BC["outflow"]
    n2 = hgks.hgks_workspace_size(cfg)
    assert n2 > 0


@pytest.mark.parametrize("field,value", [("nx", 1), ("gamma", 1.0), ("weno_Gamma", 0.05),
                                         ("weno_eps", 0.0), ("precision", 7), ("moving", 2),
                                         ("characteristic", 2), ("mu_T0", 0.0), ("prandtl", 0.0),
                                         # 32-bit indices and byte offsets
                                         ("nx", 2 ** 31 - 1), ("nz", 1 << 26)])
def test_invalid_configurations_rejected(lib, field, value):
    from paper_1909_01580_amd import hgks
    cfg = hgks.hgks_default_config(8, 8, 8)
    setattr(cfg, field, value)
    with pytest.raises(hgks.HGKSError) as e:
        hgks.hgks_workspace_size(cfg)
    assert e.value.status == hgks.HGKS_EINVAL


def test_grid_size_limit(lib):
    """Kernels address their arrays with 32-bit byte offsets: every grid,
    box or hexahedral, needs (nx+2)(ny+2)(nz+2) < 2^29."""
    from paper_1909_01580_amd import hgks
    for moving in (0, 1):
        cfg = hgks.hgks_default_config(1022, 1022, 510)        # 2^29 with the layers
        cfg.moving = moving
        with pytest.raises(hgks.HGKSError) as e:
            hgks.hgks_workspace_size(cfg)
        assert e.value.status == hgks.HGKS_EINVAL
        cfg = hgks.hgks_default_config(1022, 1022, 509)
        cfg.moving = moving
        assert hgks.hgks_workspace_size(cfg) > 0


def test_boundary_ends(lib):
    """bc_hi defaults to "as the low end"; symmetric and mixed ends are
    accepted; a periodic end needs a periodic partner; unknown codes fail."""
    from paper_1909_01580_amd import hgks
    cfg = hgks.hgks_default_config(8, 8, 8)
    assert list(cfg.bc_hi) == [hgks.BC["same"]] * 3
    cfg.bc[0] = hgks.BC["symmetric"]
    cfg.bc_hi[0] = hgks.BC["outflow"]
    cfg.bc[1] = hgks.BC["symmetric"]
    assert hgks.hgks_workspace_size(cfg) > 0
    for lo, hi in (("periodic", "outflow"), ("symmetric", "periodic")):
        bad = hgks.hgks_default_config(8, 8, 8)
        bad.bc[2], bad.bc_hi[2] = hgks.BC[lo], hgks.BC[hi]
        with pytest.raises(hgks.HGKSError):
            hgks.hgks_workspace_size(bad)
    bad = hgks.hgks_default_config(8, 8, 8)
    bad.bc_hi[1] = 5
    with pytest.raises(hgks.HGKSError):
        hgks.hgks_workspace_size(bad)


def test_step_checked_workspace(lib):
    """Static grids keep one more copy of the state for the step rejection
    of hgks_step_checked; moving meshes do not offer it."""
    from paper_1909_01580_amd import hgks
    cfg = hgks.hgks_default_config(16, 16, 16)
    n_static = hgks.hgks_workspace_size(cfg)
    assert n_static >= (20 + 50 + 30) * 8 * 16 ** 3


def test_characteristic_workspace_and_limits(lib):
    """Characteristic mode keeps six per-face coefficient arrays beside the
    cell array, on box and hexahedral grids and in batches (box grids)."""
    from paper_1909_01580_amd import hgks
    for moving in (0, 1):
        cfg = hgks.hgks_default_config(16, 12, 10)
        cfg.moving = moving
        assert cfg.characteristic == 0
        n0 = hgks.hgks_workspace_size(cfg)
        cfg.characteristic = 1
        n1 = hgks.hgks_workspace_size(cfg)
        assert n1 - n0 >= 6 * 50 * 8 * 16 * 12 * 10
    with pytest.raises(hgks.HGKSError):
        hgks.hgks_batch_workspace_size([cfg])      # batches take box grids only
    cfg.moving = 0
    assert hgks.hgks_batch_workspace_size([cfg]) > 0


def test_viscosity_law_and_prandtl_limits(lib):
    """Defaults: constant mu, Pr = 1; the law and the correction are offered
    on box grids, on hexahedral (moving) grids and in batches, per grid;
    the law needs mu_T0 > 0 and the Prandtl number must be positive."""
    from paper_1909_01580_amd import hgks
    cfg = hgks.hgks_default_config(8, 8, 8)
    assert (cfg.mu_T0, cfg.mu_exponent, cfg.prandtl) == (1.0, 0.0, 1.0)
    cfg.mu, cfg.mu_exponent, cfg.prandtl = 1e-3, 0.76, 0.71
    assert hgks.hgks_workspace_size(cfg) > 0
    plain = hgks.hgks_default_config(9, 8, 8)
    assert hgks.hgks_batch_workspace_size([cfg, plain]) > 0
    cfg.moving = 1
    assert hgks.hgks_workspace_size(cfg) > 0
    for field, bad in (("mu_T0", 0.0), ("prandtl", 0.0), ("prandtl", float("inf"))):
        c = hgks.hgks_default_config(8, 8, 8)
        setattr(c, field, bad)
        with pytest.raises(hgks.HGKSError):
            hgks.hgks_workspace_size(c)


def test_wide_stencil_limits(lib):
    """The stencils of Remark 1: box and hexahedral grids and batches with
    component-wise reconstruction; a symmetric end needs 3 cells."""
    from paper_1909_01580_amd import hgks
    cfg = hgks.hgks_default_config(8, 8, 8)
    assert cfg.stencil == 0
    cfg.stencil = 1
    assert hgks.hgks_workspace_size(cfg) > 0
    hexa = hgks.hgks_default_config(8, 8, 8)
    hexa.stencil, hexa.moving = 1, 1
    assert hgks.hgks_workspace_size(hexa) > 0
    for field, value in (("characteristic", 1), ("stencil", 2)):
        bad = hgks.hgks_default_config(8, 8, 8)
        bad.stencil = 1
        setattr(bad, field, value)
        with pytest.raises(hgks.HGKSError):
            hgks.hgks_workspace_size(bad)
    thin = hgks.hgks_default_config(2, 8, 8)
    thin.stencil = 1
    assert hgks.hgks_workspace_size(thin) > 0          # periodic: wraps
    thin.bc[0] = hgks.BC["symmetric"]
    with pytest.raises(hgks.HGKSError):
        hgks.hgks_workspace_size(thin)
    assert hgks.hgks_batch_workspace_size([cfg]) > 0


def test_moving_requires_periodic(lib):
    from paper_1909_01580_amd import hgks
    cfg = hgks.hgks_default_config(8, 8, 8)
    cfg.moving = 1
    cfg.bc[2] = hgks.BC["outflow"]
    with pytest.raises(hgks.HGKSError):
        hgks.hgks_workspace_size(cfg)


def test_null_and_small_workspace(lib):
    from paper_1909_01580_amd import hgks
    cfg = hgks.hgks_default_config(8, 8, 8)
    h = ctypes.c_void_p()
    st = lib.hgks_create(ctypes.byref(cfg), None, 0, ctypes.byref(h))
    assert st == hgks.HGKS_EINVAL
    st = lib.hgks_create(ctypes.byref(cfg), ctypes.c_void_p(256), 16, ctypes.byref(h))
    assert st == hgks.HGKS_ENOMEM
    assert b"workspace" in lib.hgks_last_error()


def test_batch_stencil_family(lib):
    """A batch takes the stencils of Sec. 2 or of Remark 1, one family for
    all its grids: a batch that mixes them is refused."""
    from paper_1909_01580_amd import hgks
    cfgs = [hgks.hgks_default_config(12, 10, 9), hgks.hgks_default_config(8, 14, 11)]
    n_s = hgks.hgks_batch_workspace_size(cfgs)
    for c in cfgs:
        c.stencil = hgks.STENCIL["S_prime"]
    assert hgks.hgks_batch_workspace_size(cfgs) == n_s
    cfgs[0].stencil = hgks.STENCIL["S"]
    with pytest.raises(hgks.HGKSError) as e:
        hgks.hgks_batch_workspace_size(cfgs)
    assert e.value.status == hgks.HGKS_EINVAL


def test_batch_characteristic(lib):
    """A batch reconstructs in characteristic variables for all its grids or
    for none: six per-face coefficient arrays per grid beside the
    component-wise one."""
    from paper_1909_01580_amd import hgks
    cfgs = [hgks.hgks_default_config(12, 10, 9), hgks.hgks_default_config(8, 14, 11)]
    n_c = hgks.hgks_batch_workspace_size(cfgs)
    for c in cfgs:
        c.characteristic = 1
    n_f = hgks.hgks_batch_workspace_size(cfgs)
    cells = 12 * 10 * 9 + 8 * 14 * 11
    assert n_f - n_c >= 6 * 50 * 8 * cells
    cfgs[1].characteristic = 0
    with pytest.raises(hgks.HGKSError) as e:
        hgks.hgks_batch_workspace_size(cfgs)
    assert e.value.status == hgks.HGKS_EINVAL
