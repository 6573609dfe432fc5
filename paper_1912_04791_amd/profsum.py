"""Summarise rocprofv3 output of bench.py runs into the text files kept under profiles/.

    python -m paper_1912_04791_amd.profsum --name k_step_c5_fp64 --kernel "k_step<3, 0, 0, false>" \
        --workload c5 --precision fp64 --trace DIR --bench-log FILE --bench-json FILE \
        [--fetch DIR --write DIR --calib-mib 256] [--flops DIR] [--valu DIR] [--stall DIR ...] \
        [--clock DIR] \
        --cmd "<the profiling commands>"

Kernel trace (``--kernel-trace``): every GPU run bench.py makes is one ``k_cfl`` dispatch (the
CFL maximum of the initial state) followed by its step-kernel dispatches, and bench.py logs each
run to stderr as a ``[run]`` line (workload, precision, solver, steps, kind) in the order it
makes them.  The trace's runs are matched to those lines in order, so the durations of the
timed run of one workload and precision are read apart from its warm-up run, from its
full-length run and from the other workloads that run the same kernel.

Counters (``--pmc``, bench.py runs of the one workload): per-dispatch values of the step kernel,
median over its dispatches.  HBM bytes from FETCH_SIZE and WRITE_SIZE, scaled by what they read
for a plain device copy of known size (bench.py --calib-copy-mib M issues it as the run's first
copy); VALU FLOPs from SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F64,F32} (wave instructions) x 64
lanes, an FMA counted twice; VALU instructions and VALU-active cycles per edge update; wave-cycle
shares of the stall counters.

Writes ``profiles/<name>.md`` and an entry in ``profiles/traffic.json`` keyed by workload and
precision, stamped with the hash of the kernel sources and the launch it was taken at.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

FLOP_COUNTERS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                 "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32",
                 "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_TRANS_F32")


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def read_runs(log_path: str):
    """The [run] lines bench.py printed, in order: dicts of workload, precision, solver, steps,
    kind."""
    runs = []
    for line in open(log_path, errors="replace"):
        if not line.startswith("[run] "):
            continue
        d = dict(kv.split("=", 1) for kv in line[6:].split())
        d["steps"] = int(d["steps"])
        runs.append(d)
    return runs


def trace_runs(trace_dir: str):
    """The trace's dispatches in order, grouped into runs: each k_cfl dispatch opens a run, and
    the step-kernel dispatches after it belong to it.  Returns a list of (step kernel name,
    [durations in ns]) for the runs with at least one step dispatch."""
    path = _one(os.path.join(trace_dir, "**", "*kernel_trace.csv"))
    rows = list(csv.DictReader(open(path)))
    key = "Dispatch_Id" if rows and "Dispatch_Id" in rows[0] else "Correlation_Id"
    rows.sort(key=lambda r: (int(r["Start_Timestamp"]), int(r[key])))
    out, cur = [], None
    for r in rows:
        name = r["Kernel_Name"]
        if "k_cfl<" in name:
            if cur and cur[1]:
                out.append(cur)
            cur = [None, []]
        elif "k_step<" in name and cur is not None:
            if cur[0] is None:
                cur[0] = name
            cur[1].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    if cur and cur[1]:
        out.append(cur)
    return out


def match_runs(logged, traced):
    """Pair the logged runs with the traced ones, in order; their step counts must agree."""
    if len(logged) != len(traced):
        raise ValueError(f"{len(logged)} logged runs, {len(traced)} traced runs with step kernels")
    for lg, (name, durs) in zip(logged, traced):
        if lg["steps"] != len(durs):
            raise ValueError(f"run {lg} has {len(durs)} step dispatches in the trace ({name})")
    return list(zip(logged, traced))


def dispatch_stats(durs_ns):
    s = sorted(durs_ns)
    return {"n": len(s), "mean_us": statistics.fmean(s) / 1e3, "median_us": statistics.median(s) / 1e3,
            "min_us": s[0] / 1e3, "max_us": s[-1] / 1e3}


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


def clock_per_dispatch(run_dir: str, kernel: str, n_xcd: int = 8):
    """Effective shader clock of each dispatch of the kernel from a run that took the kernel trace
    and GRBM_GUI_ACTIVE (GPU-busy cycles, summed over the XCDs) together: cycles / XCDs /
    duration.  Returns a list of (duration in s, clock in Hz, counters of the dispatch)."""
    tr = list(csv.DictReader(open(_one(os.path.join(run_dir, "**", "*kernel_trace.csv")))))
    cc = list(csv.DictReader(open(_one(os.path.join(run_dir, "**", "*counter_collection.csv")))))
    dur = {int(r["Dispatch_Id"]): (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
           for r in tr if kernel in r["Kernel_Name"]}
    per = {}
    for r in cc:
        if kernel in r["Kernel_Name"]:
            per.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    out = []
    for d, c in sorted(per.items()):
        if d in dur and "GRBM_GUI_ACTIVE" in c and dur[d] > 0:
            out.append((dur[d], c["GRBM_GUI_ACTIVE"] / n_xcd / dur[d], c))
    return out


def valu_flops(c):
    """FP64 and FP32 VALU FLOPs per dispatch from the instruction counters: 64 lanes per wave
    instruction, an FMA counted twice (medians over the dispatches)."""
    med = {k: statistics.median(v) for k, v in c.items()}
    f64 = 64.0 * (med.get("SQ_INSTS_VALU_ADD_F64", 0.0) + med.get("SQ_INSTS_VALU_MUL_F64", 0.0) +
                  2.0 * med.get("SQ_INSTS_VALU_FMA_F64", 0.0) + med.get("SQ_INSTS_VALU_TRANS_F64", 0.0))
    f32 = 64.0 * (med.get("SQ_INSTS_VALU_ADD_F32", 0.0) + med.get("SQ_INSTS_VALU_MUL_F32", 0.0) +
                  2.0 * med.get("SQ_INSTS_VALU_FMA_F32", 0.0) + med.get("SQ_INSTS_VALU_TRANS_F32", 0.0))
    return f64, f32


def timing_note(events_us: float, traced_us: float) -> str:
    """How the traced mean of the timed dispatches relates to bench.py's events figure."""
    head = (f"`bench.py` timed this run at {events_us:.2f} us per step with HIP events on the "
            "stream the kernels run on (graph replays; the figure includes the gaps between "
            "dispatches and the run's CFL prologue).")
    if traced_us <= events_us:
        return head + (f" The traced mean of the same run's step dispatches, {traced_us:.2f} us, "
                       f"is {100.0 * (1.0 - traced_us / events_us):.1f}% below it: the kernel's own "
                       "time, without the gaps.")
    return head + (f" The traced mean of the same run's step dispatches, {traced_us:.2f} us, is "
                   f"{100.0 * (traced_us / events_us - 1.0):.1f}% above it: under the kernel trace each "
                   "dispatch is timestamped on its own, which serialises the dispatches the graph "
                   "replays otherwise overlap (one kernel's tail with the next one's start).")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--precision", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--bench-log", required=True, help="stderr of the traced bench.py run")
    ap.add_argument("--bench-json", required=True, help="stdout (the JSON line) of that run")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--flops")
    ap.add_argument("--valu")
    ap.add_argument("--stall", nargs="*", default=[],
                    help="counter runs (directories) whose counters are merged for the cycle shares")
    ap.add_argument("--clock", help="a run with --kernel-trace and --pmc GRBM_GUI_ACTIVE together")
    ap.add_argument("--calib-mib", type=int, default=256)
    ap.add_argument("--cmd", required=True, help="the profiling commands, verbatim")
    args = ap.parse_args()

    import sys
    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash, ops_per_edge_update

    bj = json.loads(open(args.bench_json).read().strip().splitlines()[-1])
    if bj["config"]["workload"].startswith(args.workload + ":"):
        legd, edges, n_cells = (bj if args.precision == bj["config"]["precision"] else bj[args.precision]), \
            bj["config"]["edges_per_step"], bj["config"]["n_cells"]
    else:
        sec = bj[args.workload]
        legd, edges, n_cells = sec[args.precision], sec["edges_per_step"], sec["n_cells"]
    launch = legd["launch"] if "launch" in legd else bj["config"]["launch"]
    events_us = legd["ms_per_step"] * 1e3
    graph = legd.get("graph") or bj["config"].get("graph")

    pairs = match_runs(read_runs(args.bench_log), trace_runs(args.trace))
    mine = [(lg, tr) for lg, tr in pairs
            if lg["workload"] == args.workload and lg["precision"] == args.precision
            and lg["solver"] == "adot" and args.kernel in tr[0]]
    timed = [tr for lg, tr in mine if lg["kind"] == "timed"]
    full = [tr for lg, tr in mine if lg["kind"] == "full"]
    if len(timed) != 1:
        raise ValueError(f"{len(timed)} timed runs of {args.workload} {args.precision} in the trace")
    ts = dispatch_stats(timed[0][1])
    kernel_full = timed[0][0]

    h = kernel_source_hash()
    lines = [f"# {args.name}", "",
             f"Kernel `{kernel_full}`, workload `{args.workload}` ({n_cells} cells, {edges} edge "
             f"updates per step), precision `{args.precision}`, launch tile {launch['tile']}, "
             f"{launch['blocks_per_cu']} workgroups per CU, {launch['cfl_split']} CFL sub-slot(s), "
             f"graphs of {launch['graph_steps']} steps.", "",
             "Commands (run from the repository root):", "", "```", args.cmd.strip(), "```", "",
             f"Kernel sources hash: `{h}`", "",
             "## Kernel trace (`--kernel-trace --stats`) of the bench command", "",
             f"- timed run ({ts['n']} steps; graph replays {graph}): mean {ts['mean_us']:.2f} us, "
             f"median {ts['median_us']:.2f}, min {ts['min_us']:.2f}, max {ts['max_us']:.2f} per dispatch"]
    entry = {"kernel_hash": h, "launch": [launch["tile"], launch["blocks_per_cu"], launch["cfl_split"]],
             "trace_timed_mean_ns": ts["mean_us"] * 1e3, "events_ms_per_step": legd["ms_per_step"]}
    if full:
        fs = dispatch_stats(full[0][1])
        entry["trace_full_mean_ns"] = fs["mean_us"] * 1e3
        lines.append(f"- full-length run ({fs['n']} steps): mean {fs['mean_us']:.2f} us, median "
                     f"{fs['median_us']:.2f}, min {fs['min_us']:.2f}, max {fs['max_us']:.2f} per dispatch")
    lines += ["", "## Timing note", "", timing_note(events_us, ts["mean_us"])]

    sec_s = legd["ms_per_step"] * 1e-3
    if args.fetch and args.write:
        known = args.calib_mib * 1024.0   # KiB
        f, fc = counters(args.fetch, args.kernel)
        w, wc = counters(args.write, args.kernel)
        sf, sw = known / fc["FETCH_SIZE"], known / wc["WRITE_SIZE"]
        fk, wk = statistics.median(f["FETCH_SIZE"]), statistics.median(w["WRITE_SIZE"])
        fb, wb = fk * sf * 1024.0, wk * sw * 1024.0
        alg = 48.0 * n_cells
        entry.update({"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                      "fetch_scale": sf, "write_scale": sw})
        lines += ["", "## HBM traffic (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`)", "",
                  f"- calibration copy of {args.calib_mib} MiB: FETCH_SIZE read {fc['FETCH_SIZE']:.0f} "
                  f"KiB, WRITE_SIZE read {wc['WRITE_SIZE']:.0f} KiB -> scale factors {sf:.3f} "
                  f"(fetch), {sw:.3f} (write)",
                  f"- step kernel, median over {len(f['FETCH_SIZE'])} dispatches: FETCH_SIZE "
                  f"{fk:.0f} KiB, WRITE_SIZE {wk:.0f} KiB",
                  f"- scaled: {fb / 1e6:.2f} MB read + {wb / 1e6:.2f} MB written = "
                  f"{(fb + wb) / 1e6:.2f} MB per launch; algorithmic 48 B per cell = {alg / 1e6:.2f} MB "
                  f"(measured / algorithmic = {(fb + wb) / alg:.3f})",
                  f"- at the events step time: {(fb + wb) / sec_s / 1e9:.1f} GB/s (of 8000)"]
    if args.flops:
        c, _ = counters(args.flops, args.kernel)
        f64, f32 = valu_flops(c)
        tf = (f64 + f32) / sec_s / 1e12
        entry.update({"flops_f64": f64, "flops_f32": f32})
        lines += ["", "## VALU FLOPs (`--pmc` SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F64,F32})", ""]
        for k in FLOP_COUNTERS:
            if k in c:
                lines.append(f"- {k}: {statistics.median(c[k]):.6g} wave instructions per dispatch")
        lines += [f"- FLOPs per launch (x 64 lanes, FMA x 2): FP64 {f64:.4g}, FP32 {f32:.4g}; "
                  f"{(f64 + f32) / edges:.0f} per edge update (algorithmic operation count "
                  f"{ops_per_edge_update()})",
                  f"- at the events step time: {tf:.2f} TFLOP/s = {tf / 78.6:.3f} of the 78.6 TFLOP/s "
                  "VALU peak (FP64; non-packed FP32 issues at the same rate)"]
    if args.valu:
        c, _ = counters(args.valu, args.kernel)
        lines += ["", "## VALU instructions and activity (`--pmc`)", ""]
        for k in sorted(c):
            lines.append(f"- {k}: {statistics.median(c[k]):.6g} per dispatch")
        if "SQ_INSTS_VALU" in c:
            per = statistics.median(c["SQ_INSTS_VALU"]) * 64 / edges
            entry["valu_insts_per_edge"] = per
            lines.append(f"- VALU instructions per edge update: {per:.0f}")
        if "SQ_ACTIVE_INST_VALU" in c:
            # cycles the waves spend issuing VALU instructions, in units of 4 cycles: above the
            # instruction count where quarter-rate (transcendental) instructions hold the SIMD
            act = statistics.median(c["SQ_ACTIVE_INST_VALU"]) * 64 / edges
            entry["valu_active_per_edge"] = act
            lines.append(f"- VALU-active 4-cycle units per edge update: {act:.0f}")
    if args.stall:
        med = {}
        for d in args.stall:
            c, _ = counters(d, args.kernel)
            med.update({k: statistics.median(v) for k, v in c.items()})
        lines += ["", "## Where the waves' cycles go (`--pmc`, quad-cycles summed over waves)", ""]
        for k in sorted(med):
            lines.append(f"- {k}: {med[k]:.6g}")
        wc_ = med.get("SQ_WAVE_CYCLES")
        if wc_:
            shares = {k: med[k] / wc_ for k in ("SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU",
                                                "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY",
                                                "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_LDS",
                                                "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_VMEM",
                                                "SQ_ACTIVE_INST_MISC")
                      if k in med}
            entry["wave_cycle_shares"] = shares
            lines.append("- shares of the wave-cycles: " +
                         ", ".join(f"{k[3:]} {v:.3f}" for k, v in shares.items()))
            if "SQ_ACTIVE_INST_VALU" in med:
                busy = med["SQ_ACTIVE_INST_VALU"] / (1024 * sec_s * 2.4e9 / 4.0)
                entry["valu_busy"] = busy
                lines.append(f"- VALU busy: {busy:.3f} of the 1024 SIMDs' 4-cycle issue slots at "
                             "the events step time")
    if args.clock:
        rows = clock_per_dispatch(args.clock, args.kernel)
        if rows:
            clk = statistics.median(r[1] for r in rows)
            dur_ = statistics.median(r[0] for r in rows)
            entry["clock_ghz"] = clk / 1e9
            lines += ["", "## Effective clock (`--kernel-trace` with `--pmc GRBM_GUI_ACTIVE` in one run)", "",
                      f"- {len(rows)} dispatches, median duration {dur_ * 1e6:.1f} us under the counters; "
                      f"GRBM_GUI_ACTIVE / 8 XCDs / duration: median {clk / 1e9:.3f} GHz (min "
                      f"{min(r[1] for r in rows) / 1e9:.3f}, max {max(r[1] for r in rows) / 1e9:.3f}), "
                      "against the 2.4 GHz of the published peaks"]
            act = [r[2].get("SQ_ACTIVE_INST_VALU") for r in rows]
            if all(a is not None for a in act):
                busy = statistics.median(a * 4.0 / (1024 * d * f) for a, (d, f, _) in zip(act, rows))
                entry["valu_busy_at_clock"] = busy
                lines.append(f"- VALU busy at that clock: {busy:.3f} of the 1024 SIMDs' cycles "
                             "(SQ_ACTIVE_INST_VALU x 4 / (1024 x duration x clock))")
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
