"""Throughput of the HGKS time step on the 128^3 Taylor-Green vortex.

One step = one two-stage fourth-order time step of the whole hot path
(WENO-AO reconstruction, gas-kinetic face flux, stage update) over the
128^3 periodic grid on [-pi, pi]^3 (Re 1600, Ma 0.1, Prandtl number 0.72
through the heat-flux correction), including the per-step time-step
reduction.  The FP64 path gives ``value``; the mixed
path (FP32 reconstruction and flux, FP64 accumulation) is reported beside
it with its error against the FP64 result.

Prints one JSON line.  Inputs are synthetic (the analytic initial field);
they are resident in device memory before the timed region starts.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3}      # TFLOP/s, MI355X vector
HBM_PEAK = 8000.0                         # GB/s
BYTES_PER_CELL_STAGE = 120.0              # algorithmic HBM bytes (FP64 state)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "flux_box_tgv128_traffic.json")


# The device code of the box-grid flux kernel whose HBM traffic the counter
# runs measured (its launch shape is set in box_kernels.h as well).
FLUX_SOURCES = ("common.h", "gks_flux.h", "weno_box.h", "box_kernels.h")


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1909_01580_amd", "csrc")
    for name in FLUX_SOURCES:
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def op_counts():
    with open(os.path.join(ROOT, "paper_1909_01580_amd", "opcount.json")) as f:
        return json.load(f)


def measured_traffic(precision):
    """HBM bytes per flux launch from the committed rocprofv3 counter runs,
    or None when they were taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    entry = t.get(precision)
    if not entry or t.get("source_hash") != source_hash():
        return None
    return entry["bytes_per_launch"]


def run_gpu(n, steps, warmup, precision, cfl=0.35, record_first=False, characteristic=False, stencil="S"):
    import torch
    from paper_1909_01580_amd import hgks
    from paper_1909_01580_amd import workloads as wl

    q0 = torch.tensor(wl.tgv_state(n), device="cuda:0")
    ctx = hgks.Context((n, n, n), mu=wl.TGV_MU, precision=precision, characteristic=characteristic, stencil=stencil,
                       prandtl=wl.TGV_PRANDTL)
    ctx.set_uniform_grid((-np.pi,) * 3, (2 * np.pi,) * 3)
    ctx.set_state(q0)
    first = None
    for i in range(warmup):
        dt = ctx.max_dt(cfl)
        ctx.step(dt, 2)
        if i == 0 and record_first:
            first = (dt, ctx.get_state().cpu().numpy())
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.profile_begin()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        dt = ctx.max_dt(cfl)
        ctx.step(dt, 2)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = ctx.profile_end()
    ms = ev0.elapsed_time(ev1)
    state = ctx.get_state().cpu().numpy()
    totals = ctx.totals()
    return {"ms": ms, "wall": wall, "prof": prof, "state": state, "totals": totals,
            "first": first, "q0": q0.cpu().numpy()}


def run_batched(steps, precision="mixed", tune=True, unbatched_steps=2):
    """48 independent periodic problems of uneven sizes (32..96 per axis,
    about 1.0e7 cells): autotuned persistent launches, a HIP graph of
    ``steps`` steps (per-grid dt reduction inside), timed by replay."""
    import torch
    from paper_1909_01580_amd import autotune, hgks
    from paper_1909_01580_amd import workloads as wl

    problems = wl.batch_problems()
    grids = [{"n": p["n"], "length": p["length"], "mu": p["mu"]} for p in problems]
    cells = sum(int(np.prod(g["n"])) for g in grids)
    b = hgks.Batch(grids, precision=precision)
    for i, p in enumerate(problems):
        b.set_state(i, torch.tensor(p["state"], device="cuda:0"))
    b.sync()
    table = None
    if tune:
        table, _ = autotune.tune(b)
    b.capture(0.35, steps, 2)
    b.replay()                      # warm-up replay
    b.sync()
    for i, p in enumerate(problems):  # time from the initial states
        b.set_state(i, torch.tensor(p["state"], device="cuda:0"))
    b.sync()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(b.stream)
    b.replay()
    ev1.record(b.stream)
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1)
    rho = [b.get_state(i)[0].cpu().numpy() for i in range(b.n)]
    out = {"cells": cells, "grids": len(grids), "ms": ms, "steps": steps,
           "value": cells * 2 * steps / (ms / 1e3), "launch_table": table, "rho": rho}
    if unbatched_steps:
        # The same problems one context at a time (same precision).
        ctxs = []
        for i, (g, p) in enumerate(zip(grids, problems)):
            c = hgks.Context(g["n"], mu=g["mu"], precision=precision)
            c.set_uniform_grid((0, 0, 0), g["length"])
            c.set_state(torch.tensor(p["state"], device="cuda:0"))
            ctxs.append(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(unbatched_steps):
            for c in ctxs:
                c.step(c.max_dt(0.35), 2)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["unbatched_value"] = cells * 2 * unbatched_steps / el
        del ctxs
    del b
    torch.cuda.empty_cache()
    return out


def moving_initial(n):
    """Node positions at t = 0 and the initial cell averages (3x3x3 Gauss
    on the hexahedra) of the moving-mesh workload."""
    import math
    from paper_1909_01580_amd import workloads as wl
    v0 = wl.sine_mesh_vertices(n, 0.0, amp=0.05, omega=2 * math.pi)
    return v0, wl.hex_average(v0, (2.0, 2.0, 2.0), wl.pulse_point)


def run_moving(n, steps, warmup, precision, v0, q0, cfl=0.35):
    """Moving hexahedral mesh on [0,2]^3 (periodic): nodes
    x = xi + 0.05 sin(2 pi t) sin(pi xi) sin(pi eta) sin(pi zeta) on every
    component, grid velocity the secant over each step, a density pulse on a
    uniform stream.  The node positions of t_{n+1} are formed on the GPU
    inside the timed region (one elementwise kernel per step)."""
    import math
    import torch
    from paper_1909_01580_amd import hgks
    from paper_1909_01580_amd import workloads as wl

    P = (2.0, 2.0, 2.0)
    amp, omega = 0.05, 2 * math.pi
    xi = torch.tensor(wl.sine_mesh_vertices(n, 0.0, amp=0.0, static=True), device="cuda:0")
    shape = torch.tensor(wl.sine_mesh_vertices(n, 0.0, amp=1.0, static=True), device="cuda:0") - xi
    nxt = torch.empty_like(xi)
    ctx = hgks.Context((n, n, n), moving=True, precision=precision)
    ctx.set_vertices(torch.tensor(v0, device="cuda:0"), P)
    ctx.set_state(torch.tensor(q0, device="cuda:0"))
    tot0 = np.array(ctx.totals())
    t = 0.0

    def one_step(t):
        dt = ctx.max_dt(cfl)
        torch.add(xi, shape, alpha=amp * math.sin(omega * (t + dt)), out=nxt)
        ctx.set_next_vertices(nxt)
        ctx.step(dt, 2)
        return t + dt
    for _ in range(warmup):
        t = one_step(t)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.profile_begin()
    ev0.record()
    for _ in range(steps):
        t = one_step(t)
    ev1.record()
    torch.cuda.synchronize()
    prof = ctx.profile_end()
    ms = ev0.elapsed_time(ev1)
    drift = float(np.abs(np.array(ctx.totals()) - tot0).max() / np.abs(tot0).max())
    return {"ms": ms, "prof": prof, "rho": ctx.get_state()[0].cpu().numpy(), "drift": drift}


def run_turbulence(n, steps, warmup, precision, mach_t):
    """Compressible isotropic turbulence (Sec. 4) on [-pi, pi]^3, periodic:
    seeded divergence-free field with the spectrum A0 k^4 exp(-2 k^2/k0^2)
    (A0 1.3e-4, k0 8), Re_lambda 72, the given Ma_t, viscosity
    mu0 (T/T0)^0.76 and Prandtl number 0.71, CFL 0.35."""
    import torch
    from paper_1909_01580_amd import hgks
    from paper_1909_01580_amd import workloads as wl

    q0, P = wl.isotropic_turbulence_state(n, mach_t)
    ctx = hgks.Context((n, n, n), mu=P["mu0"], precision=precision, mu_T0=P["T0"],
                       mu_exponent=P["mu_exponent"], prandtl=P["prandtl"])
    ctx.set_uniform_grid((-np.pi,) * 3, (2 * np.pi,) * 3)
    ctx.set_state(torch.tensor(q0, device="cuda:0"))
    for _ in range(warmup):
        ctx.step(ctx.max_dt(0.35), 2)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.profile_begin()
    ev0.record()
    for _ in range(steps):
        ctx.step(ctx.max_dt(0.35), 2)
    ev1.record()
    torch.cuda.synchronize()
    prof = ctx.profile_end()
    return {"ms": ev0.elapsed_time(ev1), "prof": prof, "rho": ctx.get_state()[0].cpu().numpy(),
            "nonphysical": ctx.check()[0]}


def run_octant(n, steps, warmup, precision):
    """Sedov blast in the octant [0,1.2]^3 (Sec. 4): symmetric planes at
    x, y, z = 0, outflow at 1.2, the released energy in the corner cell,
    CFL 0.01 (the singular start), steps taken through the step-rejection
    entry point, which checks every step and halves a rejected one."""
    import torch
    from paper_1909_01580_amd import hgks
    from paper_1909_01580_amd import workloads as wl

    ctx = hgks.Context((n, n, n), bc=(("symmetric", "outflow"),) * 3, precision=precision)
    ctx.set_uniform_grid((0.0, 0.0, 0.0), (1.2, 1.2, 1.2))
    ctx.set_state(torch.tensor(wl.sedov_state(n), device="cuda:0"))
    tot0 = np.array(ctx.totals())
    halved = 0
    for _ in range(warmup):
        dt = ctx.max_dt(0.01)
        halved += ctx.step_checked(dt) < dt
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.profile_begin()
    ev0.record()
    for _ in range(steps):
        dt = ctx.max_dt(0.01)
        halved += ctx.step_checked(dt) < dt
    ev1.record()
    torch.cuda.synchronize()
    prof = ctx.profile_end()
    drift = np.abs(np.array(ctx.totals()) - tot0)[[0, 4]] / np.abs(tot0)[[0, 4]]
    return {"ms": ev0.elapsed_time(ev1), "prof": prof, "halved": int(halved), "drift": float(drift.max()),
            "nonphysical": ctx.check()[0]}


def sampled_oracle_error(q0, first, n):
    """Error of the first GPU FP64 step against the oracle at sampled cells:
    the oracle advances a 13^3 periodic patch around each sampled cell (the
    two-stage step at a cell depends on cells within 4 of it).  Part of the
    CPU-baseline leg (its only caller), the one place the benchmark runs the
    oracle."""
    import oracle
    from paper_1909_01580_amd import workloads as wl
    dt, gpu = first
    h = 2 * np.pi / n
    worst = np.zeros(5)
    samples = [(0, 0, 0), (n - 1, 5, 77), (64, 64, 64), (17, n - 1, 3)]
    for (i, j, k) in samples:
        idx = [np.arange(c - 6, c + 7) % n for c in (i, j, k)]
        patch = q0[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]]
        prob = oracle.uniform_problem((13, 13, 13), (0, 0, 0), (13 * h,) * 3, bc=("outflow",) * 3,
                                      params=oracle.Params(mu=wl.TGV_MU, prandtl=wl.TGV_PRANDTL))
        ref = oracle.step(prob, patch, dt)[:, 6, 6, 6]
        got = gpu[:, k, j, i]
        scale = np.array([1.0, 1.0, 1.0, 1.0, np.abs(q0[4]).max()])
        worst = np.maximum(worst, np.abs(got - ref) / scale)
    return float(worst.max()), len(samples)


def cpu_baseline(q0, n, first=None, budget_cells=32):
    """The oracle leg of the benchmark, the only part that runs the oracle:
    its throughput on a bounded sample of the same workload (one two-stage
    step of a 32^3 block of the 128^3 Taylor-Green state, outflow at the
    block faces, single-threaded; about 10-15 s of CPU work) and, when the
    first FP64 GPU step is given, that step's error at sampled cells.
    Returns (baseline record, error record or None)."""
    check = None
    if first is not None:
        err, ns = sampled_oracle_error(q0, first, n)
        check = {"max_normalised": err, "sampled_cells": ns, "steps": 1}
    import oracle
    from paper_1909_01580_amd import workloads as wl
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except ImportError:  # pragma: no cover
        limiter = None
    m = budget_cells
    h = 2 * np.pi / n
    block = np.ascontiguousarray(q0[:, :m, :m, :m])
    prob = oracle.uniform_problem((m, m, m), (0, 0, 0), (m * h,) * 3, bc=("outflow",) * 3,
                                  params=oracle.Params(mu=wl.TGV_MU, prandtl=wl.TGV_PRANDTL))
    dt = oracle.max_dt(prob, block, 0.35)
    t0 = time.perf_counter()
    oracle.step(prob, block, dt)
    el = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister()
    return {"value": m ** 3 * 2 / el, "unit": "cell-stage updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one two-stage step of a {m}^3 block of the 128^3 Taylor-Green state, "
                      f"outflow block faces, NumPy FP64, one thread ({el:.1f} s)"}, check


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--precision", choices=("both", "fp64", "mixed"), default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--no-moving", action="store_true")
    ap.add_argument("--moving-steps", type=int, default=10)
    ap.add_argument("--no-octant", action="store_true")
    ap.add_argument("--no-characteristic", action="store_true")
    ap.add_argument("--no-turbulence", action="store_true")
    ap.add_argument("--no-wide-stencil", action="store_true")
    ap.add_argument("--turbulence-steps", type=int, default=5)
    ap.add_argument("--characteristic-steps", type=int, default=5)
    ap.add_argument("--octant-steps", type=int, default=10)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also copy this many MiB once (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design only, described in the documentation)", file=sys.stderr)
        sys.exit(2)
    import torch
    n = args.n
    ops = op_counts()
    results = {}
    for prec in (("fp64", "mixed") if args.precision == "both" else (args.precision,)):
        results[prec] = run_gpu(n, args.steps, max(args.warmup, 1), prec, record_first=(prec == "fp64"))
    if args.copy_calibration:
        nb = args.copy_calibration * (1 << 20)
        a = torch.empty(nb // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    cells = n ** 3
    head = results.get("fp64") or results["mixed"]
    head_prec = "fp64" if "fp64" in results else "mixed"
    ms_step = head["ms"] / args.steps
    value = cells * 2 * args.steps / (head["ms"] / 1e3)
    fl_ms, fl_n = head["prof"]["flux"]
    launch_ms = fl_ms / max(fl_n, 1)
    # the Taylor-Green flux runs the Prandtl-corrected instantiation
    flops_per_launch = 12 * cells * ops["flux_gp_ops_prandtl"]
    achieved = flops_per_launch / (launch_ms / 1e3) / 1e12
    peak = PEAK["fp64" if head_prec == "fp64" else "fp32"]
    out = {
        "metric": "cell-stage updates/sec (128^3 Taylor-Green, FP64; FP32-mixed beside)",
        "value": value,
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_prec == "fp64" else "f32 (f64 accumulation)",
        "data": "synthetic",
        "config": {"workload": "taylor-green-vortex 128^3 periodic [-pi,pi]^3, Re 1600, Ma 0.1, Pr 0.72, "
                               "gamma 1.4, CFL 0.35, two-stage steps with per-step dt reduction",
                   "cells": cells, "precision": head_prec},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(head_prec),
                     "kernel": "k_flux_box<double, true, false> (Prandtl-corrected)", "launch_ms": launch_ms,
                     "ops_per_launch": flops_per_launch},
        "hbm": {"algorithmic_GBps": BYTES_PER_CELL_STAGE * value / 1e9,
                "frac_of_8TBps": BYTES_PER_CELL_STAGE * value / 1e9 / HBM_PEAK},
        "phases_ms_per_step": {k: v[0] / args.steps for k, v in head["prof"].items()},
        "conservation_rel_drift": float(np.abs(np.array(head["totals"]) - np.array(
            [np.sum(head["q0"][v]) * (2 * np.pi / n) ** 3 for v in range(5)])).max()
            / np.abs(head["totals"]).max()),
    }
    if "mixed" in results and "fp64" in results:
        mx = results["mixed"]
        r64 = results["fp64"]["state"][0]
        out["mixed"] = {
            "value": cells * 2 * args.steps / (mx["ms"] / 1e3),
            "ms_per_step": mx["ms"] / args.steps,
            "speedup_vs_fp64": results["fp64"]["ms"] / mx["ms"],
            "l1_rho_rel_error_vs_fp64": float(np.abs(mx["state"][0] - r64).sum() / np.abs(r64).sum()),
            "flux_launch_ms": mx["prof"]["flux"][0] / max(mx["prof"]["flux"][1], 1),
            "roofline_frac_fp32": (flops_per_launch / (mx["prof"]["flux"][0] / max(mx["prof"]["flux"][1], 1) / 1e3)
                                   / 1e12) / PEAK["fp32"],
        }
    if not args.no_batched:
        bm = run_batched(args.batched_steps, "mixed")
        b64 = run_batched(args.batched_steps, "fp64", tune=False, unbatched_steps=0)
        num = sum(np.abs(a - r).sum() for a, r in zip(bm["rho"], b64["rho"]))
        den = sum(np.abs(r).sum() for r in b64["rho"])
        out["batched"] = {
            "workload": f"{bm['grids']} periodic Euler/NS boxes, edges in {{32,48,64,96}}, "
                        f"{bm['cells']} cells, seeded Fourier-mode data, Ma 0.1-0.5",
            "value": bm["value"], "unit": "cell-stage updates/s", "dtype": "f32 (f64 accumulation)",
            "ms_per_step": bm["ms"] / bm["steps"], "steps_per_graph": bm["steps"],
            "unbatched_value": bm.get("unbatched_value"),
            "speedup_vs_unbatched": bm["value"] / bm["unbatched_value"] if bm.get("unbatched_value") else None,
            "speedup_vs_plain_fp64": bm["value"] / value if head_prec == "fp64" else None,
            "fp64_batched_value": b64["value"],
            "l1_rho_rel_error_vs_fp64": float(num / den),
            "launch_table": bm["launch_table"],
        }
    if not args.no_moving:
        v0, q0m = moving_initial(args.n)
        mv = {p: run_moving(args.n, args.moving_steps, 2, p, v0, q0m) for p in ("fp64", "mixed")}
        r64 = mv["fp64"]["rho"]
        out["moving"] = {
            "workload": f"moving hexahedral mesh {n}^3 periodic [0,2]^3, nodes xi + 0.05 sin(2 pi t) "
                        "sin(pi xi) sin(pi eta) sin(pi zeta), density pulse on a (1, 0.5, 0.25) stream, "
                        "CFL 0.35, per-step dt reduction and node update on the GPU",
            "value": cells * 2 * args.moving_steps / (mv["fp64"]["ms"] / 1e3),
            "unit": "cell-stage updates/s", "dtype": "f64",
            "ms_per_step": mv["fp64"]["ms"] / args.moving_steps,
            "phases_ms_per_step": {k: v[0] / args.moving_steps for k, v in mv["fp64"]["prof"].items()},
            "mixed_value": cells * 2 * args.moving_steps / (mv["mixed"]["ms"] / 1e3),
            "mixed_phases_ms_per_step": {k: v[0] / args.moving_steps for k, v in mv["mixed"]["prof"].items()},
            "l1_rho_rel_error_mixed_vs_fp64": float(np.abs(mv["mixed"]["rho"] - r64).sum() / np.abs(r64).sum()),
            "conservation_rel_drift": max(mv["fp64"]["drift"], mv["mixed"]["drift"]),
        }
    if not args.no_octant:
        oc = {p: run_octant(args.n, args.octant_steps, 2, p) for p in ("fp64", "mixed")}
        out["octant"] = {
            "workload": f"Sedov blast {n}^3 in the octant [0,1.2]^3, symmetric planes x,y,z = 0, outflow at 1.2, "
                        "energy 0.106384 in the corner cell, CFL 0.01, every step checked for positivity",
            "value": cells * 2 * args.octant_steps / (oc["fp64"]["ms"] / 1e3),
            "unit": "cell-stage updates/s", "dtype": "f64",
            "ms_per_step": oc["fp64"]["ms"] / args.octant_steps,
            "phases_ms_per_step": {k: v[0] / args.octant_steps for k, v in oc["fp64"]["prof"].items()},
            "mixed_value": cells * 2 * args.octant_steps / (oc["mixed"]["ms"] / 1e3),
            "steps_halved": {p: oc[p]["halved"] for p in oc},
            "nonphysical_cells": {p: oc[p]["nonphysical"] for p in oc},
            "mass_energy_rel_drift": max(oc["fp64"]["drift"], oc["mixed"]["drift"]),
        }
    if not args.no_characteristic:
        cr = {p: run_gpu(n, args.characteristic_steps, 1, p, characteristic=True) for p in ("fp64", "mixed")}
        cs = args.characteristic_steps
        out["characteristic"] = {
            "workload": f"the same {n}^3 Taylor-Green steps with reconstruction in characteristic variables "
                        "(six per-face quadratics per cell)",
            "value": cells * 2 * cs / (cr["fp64"]["ms"] / 1e3), "unit": "cell-stage updates/s", "dtype": "f64",
            "ms_per_step": cr["fp64"]["ms"] / cs,
            "phases_ms_per_step": {k: v[0] / cs for k, v in cr["fp64"]["prof"].items()},
            "mixed_value": cells * 2 * cs / (cr["mixed"]["ms"] / 1e3),
            "mixed_phases_ms_per_step": {k: v[0] / cs for k, v in cr["mixed"]["prof"].items()},
            "cost_vs_componentwise_fp64": (cr["fp64"]["ms"] / cs) / ms_step,
        }
    if not args.no_wide_stencil:
        ws = args.characteristic_steps
        wr = {p: run_gpu(n, ws, 1, p, stencil="S_prime") for p in ("fp64", "mixed")}
        out["wide_stencil"] = {
            "workload": f"the same {n}^3 Taylor-Green steps with the stencils of Remark 1 (S' with the cells two "
                        "steps away along the axes, eight octant sub-stencils)",
            "value": cells * 2 * ws / (wr["fp64"]["ms"] / 1e3), "unit": "cell-stage updates/s", "dtype": "f64",
            "ms_per_step": wr["fp64"]["ms"] / ws,
            "phases_ms_per_step": {k: v[0] / ws for k, v in wr["fp64"]["prof"].items()},
            "mixed_value": cells * 2 * ws / (wr["mixed"]["ms"] / 1e3),
        }
    if not args.no_turbulence:
        ts = args.turbulence_steps
        tb = {p: run_turbulence(n, ts, 1, p, 0.5) for p in ("fp64", "mixed")}
        r64 = tb["fp64"]["rho"]
        out["turbulence"] = {
            "workload": f"compressible isotropic turbulence {n}^3 periodic [-pi,pi]^3, Ma_t 0.5, Re_lambda 72, "
                        "spectrum A0 k^4 exp(-2k^2/k0^2) (A0 1.3e-4, k0 8), mu0 (T/T0)^0.76, Pr 0.71 "
                        "(heat-flux correction), CFL 0.35",
            "value": cells * 2 * ts / (tb["fp64"]["ms"] / 1e3), "unit": "cell-stage updates/s", "dtype": "f64",
            "ms_per_step": tb["fp64"]["ms"] / ts,
            "phases_ms_per_step": {k: v[0] / ts for k, v in tb["fp64"]["prof"].items()},
            "mixed_value": cells * 2 * ts / (tb["mixed"]["ms"] / 1e3),
            "l1_rho_rel_error_mixed_vs_fp64": float(np.abs(tb["mixed"]["rho"] - r64).sum() / np.abs(r64).sum()),
            "nonphysical_cells": {p: tb[p]["nonphysical"] for p in tb},
        }
    if not args.no_cpu_baseline:
        first = None if args.no_oracle_check else head.get("first")
        out["cpu_baseline"], check = cpu_baseline(head["q0"], n, first)
        if check is not None:
            out["fp64_error_vs_oracle"] = check
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
