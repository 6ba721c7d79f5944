"""Launch-shape autotuner for batched grids.

For each phase of the batched stage (reconstruction, fallback test, face
flux, update, time-step reduction) it tries a set of persistent workgroup
counts, timing whole steps on the batch's stream while one phase varies
(coordinate descent, two sweeps), and keeps the fastest.  The result is a
table {phase: workgroups}, also applied to the batch.
"""

import torch

from . import hgks

CANDIDATES = (0, 256, 512, 1024, 2048, 4096, 8192)


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


def tune(batch, steps=2, sweeps=2, candidates=CANDIDATES, restore_state=True):
    """Autotune the persistent workgroup count of every phase of ``batch``.
    The batch's states are saved and restored around the timing runs."""
    saved = [batch.get_state(i) for i in range(batch.n)] if restore_state else None
    dt = torch.empty(batch.n, dtype=torch.float64, device=batch.device)
    choice = {p: 0 for p in range(len(hgks.PHASES))}
    for p, w in choice.items():
        batch.set_launch(p, w)
    _time_steps(batch, dt, 1)  # warm up
    timings = {}
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
    return {hgks.PHASES[p]: w for p, w in choice.items()}, timings
