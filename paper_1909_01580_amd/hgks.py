"""ctypes binding of the HGKS C ABI (include/hgks.h).

Argument marshalling only: every step of the time stage runs in the HIP
library.  PyTorch provides device memory and the stream.  Loading fails
loudly when libhgks.so has not been built.

Module-level functions carry the C names (``hgks_step(ctx, dt, n)`` ...);
``Context`` wraps a context handle with methods of the same names without
the prefix.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgks.so")

HGKS_OK, HGKS_EINVAL, HGKS_ENOMEM, HGKS_EDEVICE, HGKS_ESTATE, HGKS_ENONPHYS, HGKS_EUNSUPPORTED = range(7)
BC = {"same": -1, "periodic": 0, "outflow": 1, "symmetric": 2}
PREC = {"fp64": 0, "mixed": 1}

STENCIL = {"S": 0, "S_prime": 1}
EXPORTS = [
    "hgks_default_config", "hgks_workspace_size", "hgks_create", "hgks_destroy",
    "hgks_set_uniform_grid", "hgks_set_vertices", "hgks_set_next_vertices",
    "hgks_set_state", "hgks_get_state", "hgks_max_dt", "hgks_step", "hgks_step_checked", "hgks_totals",
    "hgks_check", "hgks_debug_gp_states", "hgks_debug_face_flux", "hgks_sync",
    "hgks_last_error", "hgks_profile_begin", "hgks_profile_end",
    "hgks_batch_workspace_size", "hgks_batch_create", "hgks_batch_destroy",
    "hgks_batch_set_uniform_grid", "hgks_batch_set_state", "hgks_batch_get_state",
    "hgks_batch_max_dt", "hgks_batch_step", "hgks_batch_set_launch", "hgks_batch_capture",
    "hgks_batch_replay", "hgks_batch_dt", "hgks_batch_totals", "hgks_batch_sync",
    "hgks_kinetic_energy", "hgks_debug_fallback_mask",
    "hgks_batch_set_tiles", "hgks_step_noalloc", "hgks_noalloc_capacity",
]
PHASES = ("recon", "fallback", "flux", "update", "reduce")


class hgks_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3),
        ("gamma", ctypes.c_double), ("mu", ctypes.c_double),
        ("weno_Gamma", ctypes.c_double), ("weno_eps", ctypes.c_double),
        ("tau_eps", ctypes.c_double), ("tau_C", ctypes.c_double),
        ("precision", ctypes.c_int32), ("moving", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("bc_hi", ctypes.c_int32 * 3),
        ("characteristic", ctypes.c_int32),
        ("mu_T0", ctypes.c_double), ("mu_exponent", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("stencil", ctypes.c_int32),
    ]


class HGKSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hgks status {status}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libhgks.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, D, I32, SZ = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_size_t
    DP = ctypes.POINTER(ctypes.c_double)
    sig = {
        "hgks_default_config": [ctypes.POINTER(hgks_config), I32, I32, I32],
        "hgks_workspace_size": [ctypes.POINTER(hgks_config), ctypes.POINTER(SZ)],
        "hgks_create": [ctypes.POINTER(hgks_config), P, SZ, ctypes.POINTER(P)],
        "hgks_destroy": [P],
        "hgks_set_uniform_grid": [P, DP, DP],
        "hgks_set_vertices": [P, P, DP],
        "hgks_set_next_vertices": [P, P],
        "hgks_set_state": [P, P],
        "hgks_get_state": [P, P],
        "hgks_max_dt": [P, D, DP],
        "hgks_step": [P, D, I32],
        "hgks_step_checked": [P, D, I32, I32, DP],
        "hgks_totals": [P, DP],
        "hgks_check": [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
        "hgks_debug_gp_states": [P, D, P],
        "hgks_debug_face_flux": [P, D, P],
        "hgks_sync": [P],
        "hgks_profile_begin": [P],
        "hgks_profile_end": [P, DP, ctypes.POINTER(ctypes.c_int64)],
        "hgks_batch_workspace_size": [ctypes.POINTER(hgks_config), I32, ctypes.POINTER(SZ)],
        "hgks_batch_create": [ctypes.POINTER(hgks_config), I32, P, SZ, ctypes.POINTER(P)],
        "hgks_batch_destroy": [P],
        "hgks_batch_set_uniform_grid": [P, I32, DP, DP],
        "hgks_batch_set_state": [P, I32, P],
        "hgks_batch_get_state": [P, I32, P],
        "hgks_batch_max_dt": [P, D, P],
        "hgks_batch_step": [P, P, I32],
        "hgks_batch_set_launch": [P, I32, I32],
        "hgks_batch_set_tiles": [P, I32, I32, I32, I32],
        "hgks_batch_capture": [P, D, I32, I32],
        "hgks_batch_replay": [P],
        "hgks_batch_dt": [P, DP],
        "hgks_batch_totals": [P, DP],
        "hgks_batch_sync": [P],
        "hgks_kinetic_energy": [P, D, DP],
        "hgks_debug_fallback_mask": [P, D, P],
        "hgks_step_noalloc": [ctypes.POINTER(hgks_config), DP, DP, P, D, I32],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.hgks_last_error.argtypes = []
    L.hgks_last_error.restype = ctypes.c_char_p
    L.hgks_noalloc_capacity.argtypes = []
    L.hgks_noalloc_capacity.restype = ctypes.c_size_t
    _lib = L
    return L


def _check(status):
    if status != HGKS_OK:
        raise HGKSError(status, load().hgks_last_error().decode())


def _dptr(t, shape=None, dtype=torch.float64):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("expected a contiguous CUDA tensor of dtype %s" % dtype)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _arr3(x):
    return (ctypes.c_double * 3)(*[float(v) for v in x])


# ------------------------------------------------------------ C-named calls
def hgks_default_config(nx, ny, nz):
    cfg = hgks_config()
    _check(load().hgks_default_config(ctypes.byref(cfg), nx, ny, nz))
    return cfg


def hgks_workspace_size(cfg):
    n = ctypes.c_size_t()
    _check(load().hgks_workspace_size(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


def hgks_create(cfg, workspace):
    h = ctypes.c_void_p()
    _check(load().hgks_create(ctypes.byref(cfg), ctypes.c_void_p(workspace.data_ptr()),
                              workspace.numel() * workspace.element_size(), ctypes.byref(h)))
    return h


def hgks_destroy(h):
    _check(load().hgks_destroy(h))


def hgks_set_uniform_grid(h, origin, length):
    _check(load().hgks_set_uniform_grid(h, _arr3(origin), _arr3(length)))


def hgks_set_vertices(h, xyz, period):
    _check(load().hgks_set_vertices(h, _dptr(xyz), _arr3(period)))


def hgks_set_next_vertices(h, xyz):
    _check(load().hgks_set_next_vertices(h, _dptr(xyz)))


def hgks_set_state(h, q):
    _check(load().hgks_set_state(h, _dptr(q)))


def hgks_get_state(h, out):
    _check(load().hgks_get_state(h, _dptr(out)))


def hgks_max_dt(h, cfl):
    dt = ctypes.c_double()
    _check(load().hgks_max_dt(h, cfl, ctypes.byref(dt)))
    return dt.value


def hgks_step(h, dt, n_stages=2):
    _check(load().hgks_step(h, dt, n_stages))


def hgks_step_checked(h, dt, n_stages=2, max_halvings=8):
    taken = ctypes.c_double(0.0)
    _check(load().hgks_step_checked(h, dt, n_stages, max_halvings, ctypes.byref(taken)))
    return taken.value


def hgks_totals(h):
    out = (ctypes.c_double * 5)()
    _check(load().hgks_totals(h, out))
    return list(out)


def hgks_check(h):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load().hgks_check(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def hgks_kinetic_energy(h, rho0=1.0):
    ek = ctypes.c_double()
    _check(load().hgks_kinetic_energy(h, rho0, ctypes.byref(ek)))
    return ek.value


def hgks_debug_fallback_mask(h, dt, out):
    _check(load().hgks_debug_fallback_mask(h, dt, _dptr(out, dtype=torch.int32)))


def hgks_step_noalloc(cfg, origin, length, q, dt, n_stages=2):
    _check(load().hgks_step_noalloc(ctypes.byref(cfg), _arr3(origin), _arr3(length), _dptr(q), dt, n_stages))


def hgks_noalloc_capacity():
    return load().hgks_noalloc_capacity()


def hgks_debug_gp_states(h, dt, out):
    _check(load().hgks_debug_gp_states(h, dt, _dptr(out)))


def hgks_debug_face_flux(h, dt, out):
    _check(load().hgks_debug_face_flux(h, dt, _dptr(out)))


def hgks_sync(h):
    _check(load().hgks_sync(h))


def hgks_profile_begin(h):
    _check(load().hgks_profile_begin(h))


def hgks_profile_end(h):
    """Returns {phase: (total ms, timed launches)}."""
    ms = (ctypes.c_double * 5)()
    cnt = (ctypes.c_int64 * 5)()
    _check(load().hgks_profile_end(h, ms, cnt))
    return {name: (ms[i], cnt[i]) for i, name in enumerate(PHASES)}


# ------------------------------------------------------------ wrapper
def make_config(n, bc=("periodic",) * 3, gamma=1.4, mu=0.0, weno_Gamma=0.0025, weno_eps=1e-8, tau_eps=0.01,
                tau_C=1.0, precision="fp64", moving=False, characteristic=False, mu_T0=1.0, mu_exponent=0.0,
                prandtl=1.0, stencil="S", stream=None):
    """An hgks_config for an n = (nx, ny, nz) grid.  ``bc`` gives per axis
    one of 'periodic', 'outflow', 'symmetric', or a pair (low end, high
    end) of the last two; ``stream`` is a torch stream (None: the default
    stream)."""
    cfg = hgks_default_config(*[int(x) for x in n])
    for d in range(3):
        # one condition for the axis, or (low end, high end)
        lo, hi = (bc[d], "same") if isinstance(bc[d], str) else bc[d]
        cfg.bc[d] = BC[lo]
        cfg.bc_hi[d] = BC[hi]
    cfg.gamma, cfg.mu = gamma, mu
    cfg.weno_Gamma, cfg.weno_eps = weno_Gamma, weno_eps
    cfg.tau_eps, cfg.tau_C = tau_eps, tau_C
    cfg.precision = PREC[precision]
    cfg.moving = 1 if moving else 0
    cfg.characteristic = 1 if characteristic else 0
    cfg.mu_T0, cfg.mu_exponent, cfg.prandtl = mu_T0, mu_exponent, prandtl
    cfg.stencil = STENCIL[stencil]
    cfg.stream = ctypes.c_void_p(None if stream is None else stream.cuda_stream)
    return cfg


class Context:
    """One HGKS context with its workspace held as a torch tensor.

    ``bc`` gives per axis one of 'periodic', 'outflow', 'symmetric', or a
    pair (low end, high end) of the last two."""

    def __init__(self, n, bc=("periodic",) * 3, gamma=1.4, mu=0.0, weno_Gamma=0.0025,
                 weno_eps=1e-8, tau_eps=0.01, tau_C=1.0, precision="fp64", moving=False,
                 characteristic=False, mu_T0=1.0, mu_exponent=0.0, prandtl=1.0, stencil="S", device="cuda:0",
                 stream=None):
        self.n = tuple(int(x) for x in n)
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.cfg = make_config(self.n, bc=bc, gamma=gamma, mu=mu, weno_Gamma=weno_Gamma, weno_eps=weno_eps,
                               tau_eps=tau_eps, tau_C=tau_C, precision=precision, moving=moving,
                               characteristic=characteristic, mu_T0=mu_T0, mu_exponent=mu_exponent,
                               prandtl=prandtl, stencil=stencil, stream=stream)
        cfg = self.cfg
        nbytes = hgks_workspace_size(cfg)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.h = hgks_create(cfg, self._ws)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.hgks_destroy(h)
            self.h = None

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (5, nz, ny, nx)

    def set_uniform_grid(self, origin, length):
        hgks_set_uniform_grid(self.h, origin, length)

    def set_vertices(self, xyz, period):
        hgks_set_vertices(self.h, xyz, period)

    def set_next_vertices(self, xyz):
        hgks_set_next_vertices(self.h, xyz)

    def set_state(self, q):
        hgks_set_state(self.h, q)

    def get_state(self, out=None):
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        hgks_get_state(self.h, out)
        return out

    def max_dt(self, cfl):
        return hgks_max_dt(self.h, cfl)

    def step(self, dt, n_stages=2):
        hgks_step(self.h, dt, n_stages)

    def step_checked(self, dt, n_stages=2, max_halvings=8):
        return hgks_step_checked(self.h, dt, n_stages, max_halvings)

    def totals(self):
        return hgks_totals(self.h)

    def check(self):
        return hgks_check(self.h)

    def kinetic_energy(self, rho0=1.0):
        return hgks_kinetic_energy(self.h, rho0)

    def debug_fallback_mask(self, dt):
        """Fallback words [nz][ny][nx] (uint32 bit patterns held in int32)."""
        nx, ny, nz = self.n
        out = torch.empty((nz, ny, nx), dtype=torch.int32, device=self.device)
        hgks_debug_fallback_mask(self.h, dt, out)
        return out

    def debug_gp_states(self, dt):
        nx, ny, nz = self.n
        out = torch.empty((nz, ny, nx, 24, 5, 4), dtype=torch.float64, device=self.device)
        hgks_debug_gp_states(self.h, dt, out)
        return out

    def debug_face_flux(self, dt):
        nx, ny, nz = self.n
        out = torch.empty((3, nz, ny, nx, 2, 5), dtype=torch.float64, device=self.device)
        hgks_debug_face_flux(self.h, dt, out)
        return out

    def sync(self):
        hgks_sync(self.h)

    def profile_begin(self):
        hgks_profile_begin(self.h)

    def profile_end(self):
        return hgks_profile_end(self.h)


# ------------------------------------------------------------ batches
def hgks_batch_workspace_size(cfgs):
    arr = (hgks_config * len(cfgs))(*cfgs)
    n = ctypes.c_size_t()
    _check(load().hgks_batch_workspace_size(arr, len(cfgs), ctypes.byref(n)))
    return n.value


def hgks_batch_create(cfgs, workspace):
    arr = (hgks_config * len(cfgs))(*cfgs)
    h = ctypes.c_void_p()
    _check(load().hgks_batch_create(arr, len(cfgs), ctypes.c_void_p(workspace.data_ptr()),
                                    workspace.numel() * workspace.element_size(), ctypes.byref(h)))
    return h


def hgks_batch_destroy(h):
    _check(load().hgks_batch_destroy(h))


def hgks_batch_set_uniform_grid(h, i, origin, length):
    _check(load().hgks_batch_set_uniform_grid(h, i, _arr3(origin), _arr3(length)))


def hgks_batch_set_state(h, i, q):
    _check(load().hgks_batch_set_state(h, i, _dptr(q)))


def hgks_batch_get_state(h, i, out):
    _check(load().hgks_batch_get_state(h, i, _dptr(out)))


def hgks_batch_max_dt(h, cfl, dt=None):
    _check(load().hgks_batch_max_dt(h, cfl, None if dt is None else _dptr(dt)))


def hgks_batch_step(h, dt, n_stages=2):
    _check(load().hgks_batch_step(h, _dptr(dt), n_stages))


def hgks_batch_set_launch(h, phase, workgroups):
    _check(load().hgks_batch_set_launch(h, phase, workgroups))


def hgks_batch_set_tiles(h, tile, flux_band):
    _check(load().hgks_batch_set_tiles(h, int(tile[0]), int(tile[1]), int(tile[2]), int(flux_band)))


def hgks_batch_capture(h, cfl, n_steps, n_stages=2):
    _check(load().hgks_batch_capture(h, cfl, n_steps, n_stages))


def hgks_batch_replay(h):
    _check(load().hgks_batch_replay(h))


def hgks_batch_dt(h, n):
    out = (ctypes.c_double * n)()
    _check(load().hgks_batch_dt(h, out))
    return list(out)


def hgks_batch_totals(h, n):
    out = (ctypes.c_double * (5 * n))()
    _check(load().hgks_batch_totals(h, out))
    return [list(out[5 * i:5 * i + 5]) for i in range(n)]


def hgks_batch_sync(h):
    _check(load().hgks_batch_sync(h))


class Batch:
    """Independent periodic box grids advanced together.  ``grids`` is a
    list of dicts with keys n (nx, ny, nz), length (Lx, Ly, Lz) and mu, and
    optionally the grid's own viscosity law and Prandtl number (mu_T0,
    mu_exponent, prandtl); keyword arguments set a field for every grid
    (``stencil="S_prime"``: the stencils of Remark 1 for the whole batch)."""

    def __init__(self, grids, gamma=1.4, precision="mixed", device="cuda:0", stream=None, **kw):
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.Stream(self.device)
        self.stream = stream
        cfgs = []
        for g in grids:
            cfg = hgks_default_config(*g["n"])
            cfg.gamma, cfg.mu = gamma, g.get("mu", 0.0)
            cfg.precision = PREC[precision]
            for k, v in kw.items():
                setattr(cfg, k, STENCIL[v] if k == "stencil" else v)
            for k in ("mu_T0", "mu_exponent", "prandtl"):
                if k in g:
                    setattr(cfg, k, g[k])
            cfg.stream = ctypes.c_void_p(stream.cuda_stream)
            cfgs.append(cfg)
        self.cfgs = cfgs
        self.grids = [dict(g) for g in grids]
        self.n = len(grids)
        nbytes = hgks_batch_workspace_size(cfgs)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.h = hgks_batch_create(cfgs, self._ws)
        for i, g in enumerate(grids):
            hgks_batch_set_uniform_grid(self.h, i, g.get("origin", (0.0, 0.0, 0.0)), g["length"])

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.hgks_batch_destroy(h)
            self.h = None

    def shape(self, i):
        nx, ny, nz = self.grids[i]["n"]
        return (5, nz, ny, nx)

    def set_state(self, i, q):
        # q was produced on the caller's stream; the batch copies on its own,
        # and the allocator must not reuse q's memory before that copy ran.
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        hgks_batch_set_state(self.h, i, q)
        q.record_stream(self.stream)

    def get_state(self, i):
        out = torch.empty(self.shape(i), dtype=torch.float64, device=self.device)
        hgks_batch_get_state(self.h, i, out)
        hgks_batch_sync(self.h)
        return out

    def max_dt(self, cfl, dt=None):
        hgks_batch_max_dt(self.h, cfl, dt)

    def step(self, dt, n_stages=2):
        hgks_batch_step(self.h, dt, n_stages)

    def set_launch(self, phase, workgroups):
        hgks_batch_set_launch(self.h, phase, workgroups)

    def set_tiles(self, tile=(0, 0, 0), flux_band=16):
        """Cell tile shape (0, 0, 0: 256 consecutive cells) and flux band
        height; discards a captured graph."""
        hgks_batch_set_tiles(self.h, tile, flux_band)

    def capture(self, cfl, n_steps, n_stages=2):
        hgks_batch_capture(self.h, cfl, n_steps, n_stages)

    def replay(self):
        hgks_batch_replay(self.h)

    def dt(self):
        return hgks_batch_dt(self.h, self.n)

    def totals(self):
        return hgks_batch_totals(self.h, self.n)

    def sync(self):
        hgks_batch_sync(self.h)
