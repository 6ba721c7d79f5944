"""Summaries of rocprofv3 output: the figures the roofline record uses.

Reads the CSV files rocprofv3 writes (``--kernel-trace --stats`` and
``--pmc``) and prints short markdown tables, or writes the JSON records
that ``bench.py`` reads back:

* ``flops``: floating-point operations one flux launch executes, from the
  instruction counters, 64 lanes x (2 FMA + ADD + MUL + TRANS) per wave,
  in the path's own precision;
* ``traffic``: HBM bytes per launch from FETCH_SIZE and WRITE_SIZE (KiB
  per dispatch), each scaled by what the same counter reads for a plain
  device copy of known size, taken in the same run.

Each record carries a hash of the flux sources it was taken on; bench.py
ignores a record whose hash no longer matches.

    python -m paper_1909_01580_amd.counters table <counter_collection.csv>
    python -m paper_1909_01580_amd.counters stats <kernel_stats.csv>
    python -m paper_1909_01580_amd.counters flops --fp64 A.csv --mixed B.csv -o out.json --command ...
    python -m paper_1909_01580_amd.counters traffic --fetch A.csv --write B.csv --copy-mib 1024 -o out.json

(the traffic runs hold both precisions' launches and the calibration copy).
"""

import argparse
import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
FLUX_SOURCES = ("common.h", "gks_flux.h", "weno_box.h", "box_kernels.h")
FLUX_KERNEL = "k_flux_box"
COPY_KERNELS = ("copy", "Copy", "elementwise_kernel")  # torch's device copy
SIMDS = 1024            # 256 compute units x 4 SIMDs
CYCLES_PER_VALU = 4     # a wave64 VALU instruction on a 16-lane SIMD
XCDS = 8                # GRBM_GUI_ACTIVE sums the eight XCDs' busy cycles


def code_only(text):
    """C++ source without its comments and with whitespace runs collapsed:
    what the compiler sees, so that a comment edit keeps a record valid."""
    out, i, n = [], 0, len(text)
    while i < n:
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif text[i] == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(text[i])
            i += 1
    return " ".join("".join(out).split())


def source_hash(names=FLUX_SOURCES):
    """Hash of the code (comments excluded) of the flux kernel's sources."""
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(HERE, "csrc", name), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()[:16]


def short_name(kernel):
    s = kernel.split("(")[0]
    for p in ("void ", "__amd_rocclr_"):
        s = s.replace(p, "")
    return s.strip()


def read_counters(path):
    """{kernel: {dispatch id: {counter: value summed over instances}}}."""
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    with open(path) as f:
        for r in csv.DictReader(f):
            per[r["Kernel_Name"]][r["Dispatch_Id"]][r["Counter_Name"]] += float(r["Counter_Value"])
    return per


def averages(per, match):
    """{kernel: (counter averages per dispatch, dispatches)} over the
    kernels whose name contains ``match``."""
    out = {}
    for k, ds in per.items():
        if match not in k:
            continue
        cs = collections.defaultdict(list)
        for d in ds.values():
            for c, v in d.items():
                cs[c].append(v)
        out[k] = ({c: sum(v) / len(v) for c, v in cs.items()}, len(ds))
    return out


def pick(per, match, args_match):
    """The one kernel whose name contains ``match`` and ``args_match``."""
    cand = {k: v for k, v in averages(per, match).items() if args_match in k}
    if len(cand) != 1:
        raise SystemExit(f"expected one kernel matching {match!r} / {args_match!r}, found {sorted(cand)}")
    (k, v), = cand.items()
    return k, v[0], v[1]


def flux_args(prec):
    # the Taylor-Green benchmark's instantiation: Prandtl correction, no per-face arrays
    return "<double, true, false>" if prec == "fp64" else "<float, true, false>"


def flops_entry(path, prec):
    per = read_counters(path)
    k, c, n = pick(per, FLUX_KERNEL, flux_args(prec))
    sfx = "F64" if prec == "fp64" else "F32"
    waves = c["SQ_WAVES"]
    fma, mul, add, trans = (c[f"SQ_INSTS_VALU_{op}_{sfx}"] for op in ("FMA", "MUL", "ADD", "TRANS"))
    flop = 64.0 * (2 * fma + add + mul + trans)
    e = {"kernel": short_name(k), "dispatches": n, "waves_per_launch": waves,
         "valu_per_wave": c["SQ_INSTS_VALU"] / waves,
         f"fma_{sfx.lower()}_per_wave": fma / waves, f"mul_{sfx.lower()}_per_wave": mul / waves,
         f"add_{sfx.lower()}_per_wave": add / waves, f"trans_{sfx.lower()}_per_wave": trans / waves,
         "flop_per_launch": flop}
    if "GRBM_GUI_ACTIVE" in c and c["GRBM_GUI_ACTIVE"] > 0:
        cycles = c["GRBM_GUI_ACTIVE"] / XCDS
        e["kernel_cycles"] = cycles
        e["issue_rate"] = c["SQ_INSTS_VALU"] * CYCLES_PER_VALU / (cycles * SIMDS)
    return e


def copy_factor(per, counter, nbytes):
    """Bytes per counted KiB for a plain copy of nbytes (read nbytes, write nbytes)."""
    best = None
    for k, ds in per.items():
        if not any(p in k for p in COPY_KERNELS):
            continue
        for d in ds.values():
            v = d.get(counter, 0.0)
            # the calibration copy is the largest copy dispatch of the run
            if best is None or v > best:
                best = v
    if not best:
        raise SystemExit(f"no copy dispatch with {counter} found")
    return nbytes / (best * 1024.0), best


def traffic_entry(fetch_csv, write_csv, prec, ff, wf):
    pf, pw = read_counters(fetch_csv), read_counters(write_csv)
    _, cf, _ = pick(pf, FLUX_KERNEL, flux_args(prec))
    _, cw, _ = pick(pw, FLUX_KERNEL, flux_args(prec))
    return {"bytes_per_launch": cf["FETCH_SIZE"] * 1024.0 * ff + cw["WRITE_SIZE"] * 1024.0 * wf,
            "fetch_kib_raw": cf["FETCH_SIZE"], "write_kib_raw": cw["WRITE_SIZE"]}


def table(path, out=sys.stdout):
    per = read_counters(path)
    rows = averages(per, "")
    counters = sorted({c for v, _ in rows.values() for c in v})
    out.write("| kernel | dispatches | " + " | ".join(counters) + " |\n")
    out.write("|---|---|" + "---|" * len(counters) + "\n")
    for k in sorted(rows):
        v, n = rows[k]
        out.write(f"| `{short_name(k)}` | {n} | " + " | ".join(f"{v.get(c, 0):.4g}" for c in counters) + " |\n")
    if "SQ_WAVES" in counters and "SQ_INSTS_VALU" in counters:
        out.write("\nVALU instructions per wave:\n\n| kernel | VALU/wave |\n|---|---|\n")
        for k in sorted(rows):
            v, _ = rows[k]
            if v.get("SQ_WAVES"):
                out.write(f"| `{short_name(k)}` | {v['SQ_INSTS_VALU'] / v['SQ_WAVES']:.1f} |\n")


def stats(path, out=sys.stdout, top=25):
    with open(path) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out.write("| kernel | calls | average (us) | total (ms) | share |\n|---|---|---|---|---|\n")
    for r in rows[:top]:
        out.write(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.1f}% |\n")


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1909_01580_amd.counters")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("table")
    t.add_argument("csv")
    s = sub.add_parser("stats")
    s.add_argument("csv")
    fl = sub.add_parser("flops")
    fl.add_argument("--fp64")
    fl.add_argument("--mixed")
    fl.add_argument("-o", "--output", required=True)
    fl.add_argument("--command", action="append", default=[])
    tr = sub.add_parser("traffic")
    tr.add_argument("--fetch", required=True)
    tr.add_argument("--write", required=True)
    tr.add_argument("--copy-mib", type=int, required=True)
    tr.add_argument("-o", "--output", required=True)
    tr.add_argument("--command", action="append", default=[])
    a = ap.parse_args(argv)
    if a.cmd == "table":
        table(a.csv)
    elif a.cmd == "stats":
        stats(a.csv)
    elif a.cmd == "flops":
        rec = {"source_hash": source_hash(), "sources": list(FLUX_SOURCES),
               "definition": "flop_per_launch = 64 x (2 FMA + ADD + MUL + TRANS) VALU instructions of the path's "
                             "precision, summed over the launch's waves; issue_rate = VALU instructions x 4 "
                             "cycles / (kernel cycles x 1024 SIMDs), kernel cycles = GRBM_GUI_ACTIVE / 8 (the "
                             "counter sums the eight XCDs)",
               "commands": a.command}
        for prec, path in (("fp64", a.fp64), ("mixed", a.mixed)):
            if path:
                rec[prec] = flops_entry(path, prec)
        with open(a.output, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))
    elif a.cmd == "traffic":
        nb = a.copy_mib * (1 << 20)
        ff, fraw = copy_factor(read_counters(a.fetch), "FETCH_SIZE", nb)
        wf, wraw = copy_factor(read_counters(a.write), "WRITE_SIZE", nb)
        rec = {"source_hash": source_hash(), "sources": list(FLUX_SOURCES),
               "fetch_factor": ff, "write_factor": wf,
               "calibration": f"{a.copy_mib} MiB device-to-device copy: FETCH_SIZE {fraw:.0f} KiB, "
                              f"WRITE_SIZE {wraw:.0f} KiB",
               "kernel": "k_flux_box<T, true, false> (Prandtl-corrected, the Taylor-Green benchmark's)",
               "commands": a.command}
        for prec in ("fp64", "mixed"):
            try:
                rec[prec] = traffic_entry(a.fetch, a.write, prec, ff, wf)
            except SystemExit as e:
                print(f"{prec}: {e}", file=sys.stderr)
        with open(a.output, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
