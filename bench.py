"""Benchmark of the A-DOT hot path on one MI355X: edge updates per second.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

A "step" is one time step of the whole hot path over the workload: ghost cells,
CFL time step, DOT fluctuation at every edge, cell update, next CFL maximum
(one fused kernel).  W untimed warm-up steps, then exactly K timed steps with
the state already resident in HBM; the timed region is bracketed by device
synchronisation and measured with HIP events on the stream the kernels run on.

Prints ONE JSON line (rank 0) with the FP64 figure as ``value``, the mixed form
beside it, the roofline of the fused step kernel, and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "A-DOT edge updates/s, FP64 vs FP32-mixed at stated L1 err; % VALU peak"
UNIT = "edge-updates/s"
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 2.4 GHz x 64 lanes x 2 (FMA)
FP32_VALU_PEAK_TFLOPS = 157.3  # the published FP32 vector peak (packed FP32: two per lane)
FP32_NONPACKED_PEAK_TFLOPS = 78.6   # the rate without packed FP32, which these kernels are
                                    # built without: the FP64 rate

# Algorithmic operation count of one edge update (each +, -, *, / and each sqrt, arccos,
# cosine counted as one): the matrix-vector form of the DOT fluctuation costs about 150 flops,
# 9 divisions, 3 square roots, 1 arccos and 3 cosines per quadrature node (166 operations),
# and each updated cell about 51 for its CFL speed plus 9 for the update.  At G = 3 that is
# 558 operations per edge update.  A fixed count of the method, not of the kernel's
# instruction stream (which the VALU counters report separately).
OPS_PER_NODE = 166
OPS_PER_CELL = 60


def ops_per_edge_update(G: int = 3) -> int:
    return G * OPS_PER_NODE + OPS_PER_CELL


def _code_only(text: str) -> str:
    """C/C++ source without comments and whitespace (string literals kept as they are)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            if not c.isspace():
                out.append(c)
            i += 1
    return "".join(out)


def kernel_source_hash() -> str:
    """Hash of the code (comments and whitespace removed) of the device sources (`.hip` and
    the headers they include) and the build flags: a counter summary stays valid across edits
    that change no kernel code.  The host `.cpp` is left out: it chooses launches, which each
    summary records, and compiles no device code."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1912_04791_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), encoding="utf-8") as f:
                h.update(_code_only(f.read()).encode())
    with open(os.path.join(ROOT, "paper_1912_04791_amd", "build.py"), encoding="utf-8") as f:
        h.update(f.read().encode())
    return h.hexdigest()[:16]


def _profile_entry(workload: str, precision: str):
    """Committed counter summary of the step kernel, if it was taken on the current kernel
    code (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    ent = d.get(f"{workload}:{precision}")
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    return ent


def measured_traffic(workload: str, precision: str):
    """HBM bytes per step-kernel launch from the committed counter summary (or None)."""
    ent = _profile_entry(workload, precision)
    return None if ent is None else ent.get("bytes_per_launch")


# VALU issue: every wave64 VALU instruction holds a 16-lane SIMD for 4 cycles (FP64 or FP32,
# packed FP32 being off); 256 compute units x 4 SIMDs at 2.4 GHz
SIMDS = 1024
CLOCK_HZ = 2.4e9
CYCLES_PER_WAVE_INST = 4


def valu_issue(workload: str, precision: str, edges: int, ms_per_step: float):
    """Share of the chip's VALU issue slots the step kernel's instruction stream fills at the
    measured step time, from the committed VALU counter (instructions per edge update), or None."""
    ent = _profile_entry(workload, precision)
    if ent is None or "valu_insts_per_edge" not in ent:
        return None
    per_edge = ent["valu_insts_per_edge"]
    busy_s = per_edge * edges / 64.0 * CYCLES_PER_WAVE_INST / SIMDS / CLOCK_HZ
    out = {"insts_per_edge": per_edge, "frac": busy_s / (ms_per_step * 1e-3)}
    if "valu_active_per_edge" in ent:
        # the VALU-active counter (4-cycle units), which also counts the extra cycles of
        # quarter-rate instructions: the share of the SIMDs' cycles spent issuing VALU work
        act_s = ent["valu_active_per_edge"] * edges / 64.0 * CYCLES_PER_WAVE_INST / SIMDS / CLOCK_HZ
        out["active_per_edge"] = ent["valu_active_per_edge"]
        out["active_frac"] = act_s / (ms_per_step * 1e-3)
    return out


def alu_roofline(precision: str, achieved_tflops: float) -> dict:
    """ALU roofline of the step kernel: FP64 against the FP64 vector peak; the mixed form against
    the published FP32 vector peak, with the non-packed rate it can actually issue at beside it."""
    if precision == "mixed":
        return {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VALU_PEAK_TFLOPS,
                "peak_nonpacked": FP32_NONPACKED_PEAK_TFLOPS,
                "frac_nonpacked": achieved_tflops / FP32_NONPACKED_PEAK_TFLOPS}
    return {"bound": "alu", "achieved": achieved_tflops, "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved_tflops / FP64_VALU_PEAK_TFLOPS}


def make_workload(name: str):
    from paper_1912_04791_amd import inputs
    return inputs.MAKERS[name]()


def _descriptions():
    from paper_1912_04791_amd import inputs
    return inputs.DESCRIPTIONS


def time_gpu(wl, precision: str, steps: int, warmup: int, launch=None, solver: str = "adot"):
    import torch
    from paper_1912_04791_amd import dsve

    stream = torch.cuda.current_stream()
    ctx = dsve.Context.from_workload(wl, precision=precision, stream=stream, solver=solver)
    if launch:
        ctx.set_launch(*launch[:3])
        ctx.set_cfl_split(launch[3])
    h, q, z, t = dsve.upload(wl)
    if launch is None:
        # pick tile and persistent grid size on a scratch copy (outside the timed region)
        ctx.autotune(h, q, z, trial_steps=20)
    if warmup > 0:
        ctx.adot_step(h, q, z, warmup, t)
    ctx.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    ctx.adot_step(h, q, z, steps, t)
    e1.record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    res = {"ms_total": ms, "wall_s": wall, "launch": (*ctx.get_launch(), ctx.get_cfl_split()),
           "cus": ctx.device_cus(), "resident": ctx.get_resident()}
    ctx.close()
    return res


def gpu_state_after(wl, precision: str, steps: int):
    import torch
    from paper_1912_04791_amd import dsve
    ctx = dsve.Context.from_workload(wl, precision=precision)
    h, q, z, t = dsve.upload(wl)
    ctx.adot_step(h, q, z, steps, t)
    ctx.sync()
    torch.cuda.synchronize()
    out = (h.cpu().numpy(), q.cpu().numpy(), z.cpu().numpy())
    ctx.close()
    return out


def rel_l1_max(got, ref) -> float:
    hs = np.abs(ref[0]).sum()
    return float(max(np.abs(g - r).sum() / max(np.abs(r).sum(), 1e-3 * hs)
                     for g, r in zip(got, ref)))


def oracle_sample(wl):
    """The sample of the workload the oracle runs: the whole channel for a single-channel
    workload, every k-th channel (at least 8 channels, about 2e5 cells) for a batched one."""
    if wl.n_channels == 1:
        return wl, None
    stride = max(1, int(wl.n_cells // 200_000))
    stride = min(stride, max(1, wl.n_channels // 8))
    chans = np.arange(0, wl.n_channels, stride)
    return wl.subset(chans), chans


# Algorithmic figures of the standalone entry points: operations per unit as counted for the step
# kernel (a node 166, a cell's CFL speed 51), HBM bytes per unit from their argument layouts.
FLUCT_OPS_PER_EDGE = 3 * OPS_PER_NODE   # pairwise D+- at G = 3
FLUCT_BYTES_PER_EDGE = 96               # six states read, six fluctuation components written
CFL_OPS_PER_CELL = 51
CFL_BYTES_PER_CELL = 16                 # h and q read (the speeds do not depend on z)
UPDATE_BYTES_PER_CELL = 96              # h, q, z read and written, D- and D+ read (3 rows each)
HBM_PEAK_GBS = 8000.0


def entry_point_rates(reps: int = 20):
    """The C ABI's standalone calls (dot_edge_fluct, cfl_reduce, cell_update), each timed alone
    with HIP events on the stream they run on, on device-resident synthetic inputs: 2^22 random
    edge pairs, and a single FP64 channel of 2^24 cells."""
    import torch
    from paper_1912_04791_amd import dsve, inputs
    f64 = dict(dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def seconds_per_call(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    def valu(units, ops, secs):
        tf = units * ops / secs / 1e12
        return {"bound": "alu", "achieved": tf, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / FP64_VALU_PEAK_TFLOPS}

    def hbm(units, nbytes, secs):
        gbs = units * nbytes / secs / 1e9
        return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS}

    out = {}
    n = 1 << 22
    WL, WR = inputs.make_random_edges(n, seed=5)
    ctx = dsve.Context.single(16, porosity=0.4, A_g=0.005, dx=1.0, stream=stream)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (*WL, *WR)]
    Dm, Dp = torch.empty(3, n, **f64), torch.empty(3, n, **f64)
    t = seconds_per_call(lambda: ctx.dot_edge_fluct(*dev, Dm, Dp))
    ctx.sync()
    ctx.close()
    out["dot_edge_fluct"] = {"edges": n, "us_per_call": t * 1e6, "edges_per_s": n / t,
                             "roofline": valu(n, FLUCT_OPS_PER_EDGE, t),
                             "hbm_GB_per_s": n * FLUCT_BYTES_PER_EDGE / t / 1e9}
    del dev, Dm, Dp

    N = 1 << 24
    rng = np.random.default_rng(6)
    h = torch.from_numpy(1.0 + 0.1 * rng.random(N)).cuda()
    q = 0.4 * h
    z = torch.zeros(N, **f64)
    ctx = dsve.Context.single(N, porosity=0.4, A_g=0.005, dx=0.01, stream=stream)
    amax, dt = torch.zeros(1, **f64), torch.zeros(1, **f64)
    t = seconds_per_call(lambda: ctx.cfl_reduce(h, q, z, amax, dt))
    out["cfl_reduce"] = {"cells": N, "us_per_call": t * 1e6, "cells_per_s": N / t,
                         "roofline": valu(N, CFL_OPS_PER_CELL, t),
                         "hbm_GB_per_s": N * CFL_BYTES_PER_CELL / t / 1e9}
    Dm = torch.from_numpy(1e-3 * rng.standard_normal((3, N + 1))).cuda()
    Dp = torch.from_numpy(1e-3 * rng.standard_normal((3, N + 1))).cuda()
    dt.fill_(1e-6)
    t = seconds_per_call(lambda: ctx.cell_update(Dm, Dp, dt, h, q, z))
    ctx.sync()
    ctx.close()
    out["cell_update"] = {"cells": N, "us_per_call": t * 1e6, "cells_per_s": N / t,
                          "roofline": hbm(N, UPDATE_BYTES_PER_CELL, t)}
    return out


def cpu_baseline(wl, budget_s: float = 12.0):
    """The oracle as it stands, on this host's cores, on a bounded sample of the same
    workload.  Returns the baseline dict, the oracle state and the sample description."""
    import oracle
    sample, chans = oracle_sample(wl)
    threads = oracle.default_threads()
    specs = [oracle.ChannelSpec(n_cells=int(sample.lengths()[c]), dx=float(sample.dx[c]),
                                Ag=float(sample.Ag[c]), porosity=float(sample.porosity[c]), g=wl.g,
                                n_gauss=wl.n_gauss, cfl=wl.cfl, bc_left=int(sample.bc_left[c]),
                                bc_right=int(sample.bc_right[c]), q_in=float(sample.q_in[c]),
                                h_in=float(sample.h_in[c]), h_out=float(sample.h_out[c]),
                                law=int(sample.law), par=tuple(float(v) for v in sample.law_par[c]),
                                ks=float(sample.ks[c]),
                                dir_left=tuple(float(v) for v in sample.dir_left[c]),
                                dir_right=tuple(float(v) for v in sample.dir_right[c]))
             for c in range(sample.n_channels)]

    def run(n):
        if chans is None:
            return oracle.run(specs[0], sample.h, sample.q, sample.z, n, nthreads=threads)[:3]
        return oracle.run_batched(specs, sample.offsets, sample.h, sample.q, sample.z, n,
                                  nthreads=threads)[:3]

    t0 = time.perf_counter()
    run(1)
    one = time.perf_counter() - t0
    n = int(max(1, min(wl.steps, budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    ref = run(n)
    el = time.perf_counter() - t0
    eu = sample.edges_per_step() * n
    what = (f"{wl.name}: first {n} of {wl.steps} steps at full size ({wl.n_cells} cells)"
            if chans is None else
            f"{wl.name}: {sample.n_channels} of {wl.n_channels} channels (every "
            f"{chans[1] - chans[0] if chans.size > 1 else 1}th, {sample.n_cells} cells), first {n} "
            f"of {wl.steps} steps")
    base = {"value": eu / el, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{what}; {el:.1f} s on {threads} threads"}
    return base, ref, n, chans


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--workload", default="c2",
                    choices=["c1", "c2", "c3", "c4", "c5", "soni", "bellal_mpm", "bellal_vanrijn",
                             "bellal_thr"])
    ap.add_argument("--precisions", default=None,
                    help="comma list; default fp64,mixed (mixed,fp64 for the mixed workloads)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--dot-steps", type=int, default=100,
                    help="steps timed for the original DOT (numerical eigensolver) baseline; 0 skips it")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=-1)
    ap.add_argument("--graph-steps", type=int, default=-1)
    ap.add_argument("--cfl-split", type=int, default=0,
                    help="CFL sub-slots per channel with an explicit launch (0 = automatic)")
    ap.add_argument("--no-entry", action="store_true",
                    help="skip timing the standalone entry points")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding over "
              "several GPUs is described in the design notes but not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.calib_copy_mib > 0:
        # a plain device copy of known size, the first copy of the run (counter summaries
        # scale FETCH_SIZE / WRITE_SIZE by what they read for it)
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {n * 8} bytes read, {n * 8} bytes written",
              file=sys.stderr, flush=True)
        del src, dst

    wl = make_workload(args.workload)
    DESCRIPTIONS = _descriptions()
    edges = wl.edges_per_step()
    launch = None
    if args.tile or args.blocks_per_cu >= 0 or args.graph_steps >= 0:
        launch = (args.tile or 256, max(args.blocks_per_cu, 0),
                  60 if args.graph_steps < 0 else args.graph_steps, args.cfl_split)

    if args.precisions is None:
        args.precisions = "mixed,fp64" if wl.precision == "mixed" else "fp64,mixed"
    precisions = [p for p in args.precisions.split(",") if p]
    results = {}
    for prec in precisions:
        r = time_gpu(wl, prec, args.steps, args.warmup, launch)
        r["edge_updates_per_s"] = edges * args.steps / (r["ms_total"] * 1e-3)
        r["ms_per_step"] = r["ms_total"] / args.steps
        print(f"[bench] {wl.name} {prec}: {r['ms_per_step'] * 1e3:.2f} us/step, "
              f"{r['edge_updates_per_s']:.4e} edge-updates/s", file=sys.stderr, flush=True)
        results[prec] = r

    main_prec = precisions[0]
    main = results[main_prec]
    ops = ops_per_edge_update(wl.n_gauss)
    form = "GRASS" if wl.law == 0 else "LAW"
    achieved_tflops = edges * ops / (main["ms_per_step"] * 1e-3) / 1e12
    traffic = measured_traffic(wl.name, main_prec)

    out = {
        "metric": METRIC,
        "value": main["edge_updates_per_s"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS[wl.name],
                   "n_cells": wl.n_cells, "n_channels": wl.n_channels,
                   "edges_per_step": edges, "precision": main_prec,
                   "launch": {"tile": main["launch"][0], "blocks_per_cu": main["launch"][1],
                              "graph_steps": main["launch"][2],
                              "cfl_split": main["launch"][3]},
                   "parallelism": "single GPU"},
        "roofline": {**alu_roofline(main_prec, achieved_tflops),
                     "traffic": traffic,
                     "kernel": (f"{'k_resident' if main['resident'] else 'k_step'}<{wl.n_gauss}, "
                                f"{'FP64' if main_prec == 'fp64' else 'MIXED'}, {form}>"),
                     "ops_per_edge_update": ops,
                     "valu_issue": valu_issue(wl.name, main_prec, edges, main["ms_per_step"])},
    }
    if wl.law != 0:
        out["roofline"]["note"] = ("ops count the scheme only; the closure's powers and roots "
                                   "per node are extra work, so frac is a lower bound")
    for prec in precisions[1:]:
        r = results[prec]
        achieved_p = edges * ops / (r["ms_per_step"] * 1e-3) / 1e12
        out[prec] = {"value": r["edge_updates_per_s"], "ms_per_step": r["ms_per_step"],
                     "speedup_vs_" + main_prec: r["edge_updates_per_s"] / main["edge_updates_per_s"],
                     "launch": {"tile": r["launch"][0], "blocks_per_cu": r["launch"][1],
                                "graph_steps": r["launch"][2], "cfl_split": r["launch"][3]},
                     "roofline": {**alu_roofline(prec, achieved_p),
                                  "traffic": measured_traffic(wl.name, prec),
                                  "valu_issue": valu_issue(wl.name, prec, edges, r["ms_per_step"])}}

    if args.dot_steps > 0:
        # the paper's own baseline: the same scheme with the numerical eigen-decomposition
        r = time_gpu(wl, "fp64", args.dot_steps, min(args.warmup, 6), launch, solver="dot")
        v = edges * args.dot_steps / (r["ms_total"] * 1e-3)
        print(f"[bench] {wl.name} dot fp64: {r['ms_total'] / args.dot_steps * 1e3:.2f} us/step, "
              f"{v:.4e} edge-updates/s", file=sys.stderr, flush=True)
        adot64 = results.get("fp64")
        out["dot_fp64"] = {"value": v, "ms_per_step": r["ms_total"] / args.dot_steps,
                           "steps": args.dot_steps,
                           "launch": {"tile": r["launch"][0], "blocks_per_cu": r["launch"][1],
                                      "graph_steps": r["launch"][2], "cfl_split": r["launch"][3]},
                           "adot_fp64_speedup": (adot64["edge_updates_per_s"] / v) if adot64 else None}

    if not args.no_entry:
        out["entry_points"] = entry_point_rates()
        for k, v in out["entry_points"].items():
            r = v["roofline"]
            print(f"[bench] {k}: {v['us_per_call']:.1f} us/call, {r['achieved']:.2f} {r['unit']} "
                  f"({r['frac']:.2f} of {r['bound']} peak)", file=sys.stderr, flush=True)

    if not args.no_cpu:
        base, ref, n, chans = cpu_baseline(wl)
        out["cpu_baseline"] = base
        errs = {}
        for prec in precisions:
            got = gpu_state_after(wl, prec, n)
            if chans is None:
                errs[prec] = rel_l1_max(got, ref)
            else:
                sample, _ = oracle_sample(wl)
                worst = 0.0
                for j, c in enumerate(chans):
                    lo, hi = int(wl.offsets[c]), int(wl.offsets[c + 1])
                    slo, shi = int(sample.offsets[j]), int(sample.offsets[j + 1])
                    worst = max(worst, rel_l1_max([g[lo:hi] for g in got],
                                                  [r[slo:shi] for r in ref]))
                errs[prec] = worst
        out["l1_vs_oracle"] = {"steps": n, "per": "channel" if chans is not None else "run",
                               "channels_compared": None if chans is None else int(len(chans)),
                               **errs}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
