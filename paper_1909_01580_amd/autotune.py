"""Launch-shape autotuner for batched grids.

It times whole batched steps on the batch's stream while one launch
parameter varies and keeps the fastest value (coordinate descent):

1. the cell tile shape (256 consecutive cells, or a box of cells) and the
   band height of the flux tiles' cell order, with one workgroup per tile;
2. the persistent workgroup count of every phase (reconstruction, fallback
   test, face flux, update, time-step reduction; 0 = one workgroup per
   tile), two sweeps.

The result is a table {"tile": (tx, ty, tz), "flux_band": b, phase:
workgroups, ...}, also applied to the batch.
"""

import torch

from . import hgks

CANDIDATES = (0, 256, 512, 1024, 2048, 4096, 8192)
TILE_SHAPES = ((0, 0, 0), (64, 4, 1), (32, 8, 1), (16, 16, 1), (32, 4, 2), (16, 4, 4), (8, 8, 4))
FLUX_BANDS = (4, 8, 16, 32)


def _time_steps(batch, dt, steps):
    s = batch.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(s)
    for _ in range(steps):
        batch.max_dt(0.35, dt)
        batch.step(dt, 2)
    ev1.record(s)
    ev1.synchronize()
    return ev0.elapsed_time(ev1) / steps


def tune(batch, steps=2, sweeps=2, candidates=CANDIDATES, tiles=TILE_SHAPES, bands=FLUX_BANDS,
         restore_state=True):
    """Autotune the tile shapes and the persistent workgroup count of every
    phase of ``batch``.  The batch's states are saved and restored around
    the timing runs.  Returns (table, timings)."""
    saved = [batch.get_state(i) for i in range(batch.n)] if restore_state else None
    dt = torch.empty(batch.n, dtype=torch.float64, device=batch.device)
    choice = {p: 0 for p in range(len(hgks.PHASES))}
    for p, w in choice.items():
        batch.set_launch(p, w)
    batch.set_tiles((0, 0, 0), 16)
    _time_steps(batch, dt, 1)  # warm up
    timings = {}
    best = None
    for shape in tiles:
        batch.set_tiles(shape, 16)
        t = _time_steps(batch, dt, steps)
        timings[("tile", shape)] = t
        if best is None or t < best[1]:
            best = (shape, t)
    tile = best[0]
    best = None
    for band in bands:
        batch.set_tiles(tile, band)
        t = _time_steps(batch, dt, steps)
        timings[("flux_band", band)] = t
        if best is None or t < best[1]:
            best = (band, t)
    band = best[0]
    batch.set_tiles(tile, band)
    for _ in range(sweeps):
        for p in range(len(hgks.PHASES)):
            best = None
            for w in candidates:
                batch.set_launch(p, w)
                t = _time_steps(batch, dt, steps)
                timings[(p, w)] = t
                if best is None or t < best[1]:
                    best = (w, t)
            choice[p] = best[0]
            batch.set_launch(p, best[0])
    if saved is not None:
        for i, q in enumerate(saved):
            batch.set_state(i, q)
        batch.sync()
    table = {"tile": tuple(tile), "flux_band": band}
    table.update({hgks.PHASES[p]: w for p, w in choice.items()})
    return table, timings
