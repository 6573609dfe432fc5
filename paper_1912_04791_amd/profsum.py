"""Summarise rocprofv3 output of bench.py runs into the text files kept under profiles/.

    python -m paper_1912_04791_amd.profsum --name k_step_c2_fp64 --kernel "k_step<3, 0>" \
        --trace DIR --fetch DIR --write DIR [--flops DIR] --calib-mib 256 \
        --workload c2 --precision fp64 --cmd "<full profiling command>"

Reads the CSV outputs (``*_kernel_stats.csv`` of a ``--kernel-trace --stats`` run and
``*_counter_collection.csv`` of ``--pmc`` runs), and writes ``profiles/<name>.md`` with the
figures used (average kernel duration, HBM bytes per launch scaled by the plain-copy
calibration, hardware FLOP counts), plus an entry in ``profiles/traffic.json`` keyed by
workload and precision and stamped with the hash of the kernel sources it was taken on.

The calibration: bench.py --calib-copy-mib M first copies M MiB device-to-device (one
``__amd_rocclr_copyBuffer`` dispatch reading and writing exactly M MiB, the run's first copy);
the ratio of the known bytes to what FETCH_SIZE / WRITE_SIZE report for that dispatch scales
the step kernel's readings.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def kernel_stats(trace_dir: str, kernel: str):
    path = _one(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    for r in csv.DictReader(open(path)):
        if kernel in r["Name"]:
            return {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                    "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"])}
    raise KeyError(kernel)


def counters(pmc_dir: str, kernel: str):
    """Per-counter list of per-dispatch values for the kernel, and per counter the value of the
    calibration copy: the first copy dispatch of the run, since bench.py issues it before any
    other copy (later copies, such as the state copied back after an odd step count, can be
    larger than it)."""
    path = _one(os.path.join(pmc_dir, "**", "*counter_collection.csv"))
    out, copies = {}, {}
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        v = float(r["Counter_Value"])
        if kernel in name:
            out.setdefault(r["Counter_Name"], []).append(v)
        elif "copyBuffer" in name:
            copies.setdefault(r["Counter_Name"], []).append((int(r["Dispatch_Id"]), v))
    first = {k: min(vs)[1] for k, vs in copies.items()}
    return out, first


def timing_note(events_us: str, traced_us: float) -> str:
    """How the traced average relates to bench.py's events figure (a value or a range)."""
    top = max(float(x) for x in events_us.replace("\u2013", "-").split("-") if x.strip())
    head = (f"`bench.py` times this kernel at {events_us} us per step with HIP events over "
            "graph-replayed steps on the stream it runs on (a range spans several boxes); the "
            "roofline it reports uses that figure.")
    if traced_us > 1.02 * top:
        return head + (f" The traced average above ({traced_us:.2f} us) is higher because under "
                       "the kernel trace each dispatch is timestamped on its own and consecutive "
                       "dispatches run back to back, which removes the overlap of one kernel's "
                       "tail with the next kernel's start that graph replays otherwise get.")
    return head + (f" The traced average above ({traced_us:.2f} us) agrees with it within 2%: at "
                   "this step length the overlap of one kernel's tail with the next kernel's "
                   "start, which the trace removes, is too small to show.")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--flops")
    ap.add_argument("--calib-mib", type=int, default=256)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--precision", required=True)
    ap.add_argument("--cmd", required=True, help="the profiling commands, verbatim")
    ap.add_argument("--algorithmic-bytes", type=float, default=None)
    ap.add_argument("--edges", type=int, default=None)
    ap.add_argument("--events-us", default=None,
                    help="the kernel's step time from bench.py's HIP events, e.g. 26.5-28.5")
    args = ap.parse_args()

    import sys
    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash, ops_per_edge_update

    st = kernel_stats(args.trace, args.kernel)
    lines = [f"# {args.name}", "", f"Kernel `{args.kernel}`, workload `{args.workload}`, "
             f"precision `{args.precision}`.", "", "Commands (run from the repository root):", "",
             "```", args.cmd.strip(), "```", "",
             f"Kernel sources hash: `{kernel_source_hash()}`", "",
             "## Kernel trace (`--kernel-trace --stats`)", "",
             f"- calls: {st['calls']}",
             f"- average duration: {st['avg_ns'] / 1e3:.2f} us "
             f"(min {st['min_ns'] / 1e3:.2f}, max {st['max_ns'] / 1e3:.2f})"]
    entry = {"avg_ns": st["avg_ns"], "kernel_hash": kernel_source_hash()}
    known = args.calib_mib * 1024.0   # KiB
    if args.fetch and args.write:
        f, fc = counters(args.fetch, args.kernel)
        w, wc = counters(args.write, args.kernel)
        f_copy = fc["FETCH_SIZE"]
        w_copy = wc["WRITE_SIZE"]
        sf, sw = known / f_copy, known / w_copy
        fk = statistics.median(f["FETCH_SIZE"])
        wk = statistics.median(w["WRITE_SIZE"])
        fb, wb = fk * sf * 1024.0, wk * sw * 1024.0
        entry.update({"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                      "fetch_scale": sf, "write_scale": sw})
        lines += ["", "## HBM traffic (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`)", "",
                  f"- calibration copy of {args.calib_mib} MiB: FETCH_SIZE read {f_copy:.0f} KiB, "
                  f"WRITE_SIZE read {w_copy:.0f} KiB -> scale factors {sf:.3f} (fetch), "
                  f"{sw:.3f} (write)",
                  f"- step kernel, median over {len(f['FETCH_SIZE'])} dispatches: FETCH_SIZE "
                  f"{fk:.0f} KiB, WRITE_SIZE {wk:.0f} KiB",
                  f"- scaled: {fb / 1e6:.2f} MB read + {wb / 1e6:.2f} MB written = "
                  f"{(fb + wb) / 1e6:.2f} MB per launch",
                  f"- achieved HBM bandwidth at the traced duration: "
                  f"{(fb + wb) / (st['avg_ns'] * 1e-9) / 1e9:.1f} GB/s (of 8000)"]
        if args.algorithmic_bytes:
            lines.append(f"- algorithmic bytes per launch: {args.algorithmic_bytes / 1e6:.2f} MB "
                         f"(measured / algorithmic = {(fb + wb) / args.algorithmic_bytes:.3f})")
    if args.flops:
        c, _ = counters(args.flops, args.kernel)
        lines += ["", "## VALU counters (`--pmc`), median per dispatch", ""]
        for k in sorted(c):
            lines.append(f"- {k}: {statistics.median(c[k]):.6g}")
        if "SQ_INSTS_VALU_FLOPS_FP64" in c:
            f64 = statistics.median(c["SQ_INSTS_VALU_FLOPS_FP64"]) * 64
            f32 = statistics.median(c.get("SQ_INSTS_VALU_FLOPS_FP32", [0.0])) * 64
            rate = (f64 + f32) / (st["avg_ns"] * 1e-9) / 1e12
            entry.update({"hw_flops_fp64": f64, "hw_flops_fp32": f32, "hw_tflops": rate})
            lines.append(f"- hardware FLOPs per launch (counter x 64 lanes): FP64 {f64:.4g}, "
                         f"FP32 {f32:.4g}; rate {rate:.2f} TFLOP/s at the traced duration")
        if args.edges and "SQ_INSTS_VALU" in c:
            per = statistics.median(c["SQ_INSTS_VALU"]) * 64 / args.edges
            entry["valu_insts_per_edge"] = per
            lines.append(f"- VALU instructions per edge update: {per:.0f} "
                         f"(algorithmic operation count {ops_per_edge_update()})")
        if args.edges and "SQ_ACTIVE_INST_VALU" in c:
            # cycles the waves spend issuing VALU instructions, in units of 4 cycles: above the
            # instruction count where quarter-rate (transcendental) instructions hold the SIMD
            act = statistics.median(c["SQ_ACTIVE_INST_VALU"]) * 64 / args.edges
            entry["valu_active_per_edge"] = act
            lines.append(f"- VALU-active 4-cycle units per edge update: {act:.0f}")
    if args.events_us:
        lines += ["", "## Timing note", "", timing_note(args.events_us, st["avg_ns"] / 1e3)]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"{args.name}.md"), "w") as fo:
        fo.write("\n".join(lines) + "\n")
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        allt = json.load(open(tpath))
    except (OSError, ValueError):
        allt = {}
    allt[f"{args.workload}:{args.precision}"] = entry
    with open(tpath, "w") as fo:
        json.dump(allt, fo, indent=1, sort_keys=True)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
