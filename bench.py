"""Benchmark of the A-DOT hot path on one MI355X: edge updates per second.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5]

A "step" is one time step of the whole hot path over the workload: ghost cells,
CFL time step, DOT fluctuation at every edge, cell update, next CFL maximum
(one fused kernel).  W untimed warm-up steps, then exactly K timed steps with
the state already resident in HBM and the HIP graphs they replay captured
beforehand; the timed region is bracketed by device synchronisation and
measured with HIP events on the stream the kernels run on.

The headline workload is c5, the largest single-GPU configuration: 65 536
batched channels of 512-4096 cells (1.51e8 cells), FP64.  Prints ONE JSON line
with the FP64 figure as ``value``; the mixed form beside it (speed-up, per-channel
L1 against the oracle over all 5000 steps on sampled channels); the rooflines of
the fused step kernel, algorithmic and from the committed VALU counters; the
other workloads (c4, c2) with their own rooflines; the original numerical-
eigensolver DOT; the standalone entry points; and the CPU oracle timed on a
bounded sample of c5 on this host's cores.  Every GPU run is logged to stderr as
a ``[run]`` line, so a kernel trace of this command can be matched to its legs.
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
HBM_PEAK_GBS = 8000.0
# Launches chosen by the autotuner on an MI355X, keyed by device, precision, law and problem
# shape; a hit sets the launch without trials (the profiles under profiles/ were taken at them)
TUNE_CACHE = os.path.join(ROOT, "paper_1912_04791_amd", "tuned_launch.json")
# Seconds of warm-up rounds before the timed steps of a workload timed beside the headline (its
# timed region can be a fraction of a millisecond); the headline warms up for its W steps alone.
EXTRA_WARM_S = 0.2

# Algorithmic operation count of one edge update (each +, -, *, / and each sqrt, arccos,
# cosine counted as one): the matrix-vector form of the DOT fluctuation costs about 150 flops,
# 9 divisions, 3 square roots, 1 arccos and 3 cosines per quadrature node (166 operations),
# and each updated cell about 51 for its CFL speed plus 9 for the update.  At G = 3 that is
# 558 operations per edge update.  A fixed count of the method, not of the kernel's
# instruction stream (which the VALU counters report separately).
OPS_PER_NODE = 166
OPS_PER_CELL = 60

# The paper's own CPU times (Secs. 4.1-4.3, 5.1): serial double-precision runs on hardware,
# language and compiler it does not state; context, not a target.
PAPER_CPU = {
    "hardware": "unstated",
    "precision": "fp64",
    "test1_adot_nc500_s": 0.1,          # Sec. 4.1 (also DOT at nc = 100, PRICE-C at nc = 500)
    "test2_adot_nc300_s": 1.3,          # Sec. 4.2 (also DOT at nc = 100, PRICE-C at nc = 300)
    "test3_adot_nc1200_s": 10.0,        # Sec. 4.3 (also DOT at nc = 300, PRICE-C at nc = 1200)
    "sec51_2400s_nc100_s": {"adot": 1.50, "dot": 14.97, "price_c": 1.48},   # Sec. 5.1
    "adot_vs_dot": "about 10x at equal error (Secs. 4.1-4.3, 6)",
}


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
    that change no kernel code.  The host `.cpp`, which chooses launches (each summary records
    the launch it was taken at), compiles no device code and is left out."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1912_04791_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), encoding="utf-8") as f:
                h.update(_code_only(f.read()).encode())
    with open(os.path.join(ROOT, "paper_1912_04791_amd", "build.py"), encoding="utf-8") as f:
        h.update(f.read().encode())
    return h.hexdigest()[:16]


def _profile_entry(workload: str, precision: str, launch=None):
    """Committed counter summary of the step kernel for this workload and precision, if it was
    taken on the current kernel code and (when `launch` is given) at the same launch
    (tile, blocks per CU, CFL sub-slots); else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    ent = d.get(f"{workload}:{precision}")
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    if launch is not None and ent.get("launch") is not None and \
            list(ent["launch"]) != [launch[0], launch[1], launch[3]]:
        return None
    return ent


# VALU issue: every wave64 VALU instruction holds a 16-lane SIMD for 4 cycles (FP64 or FP32,
# packed FP32 being off); 256 compute units x 4 SIMDs at 2.4 GHz
SIMDS = 1024
CLOCK_HZ = 2.4e9
CYCLES_PER_WAVE_INST = 4


def counter_figures(workload: str, precision: str, edges: int, ms_per_step: float, launch):
    """Figures from the committed counter summary of the step kernel (same kernel code, same
    launch), at the measured step time:
      traffic       HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy)
      counter_flops VALU FLOPs per launch from SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F64,F32} x 64
                    lanes, an FMA counted twice, as a rate and a fraction of the VALU peak
      valu_issue    share of the chip's VALU issue slots the instruction stream fills.
    Each is None when no matching summary is committed."""
    ent = _profile_entry(workload, precision, launch)
    out = {"traffic": None, "counter_flops": None, "valu_issue": None}
    if ent is None:
        return out
    out["traffic"] = ent.get("bytes_per_launch")
    sec = ms_per_step * 1e-3
    if "flops_f64" in ent:
        f64, f32 = ent["flops_f64"], ent.get("flops_f32", 0.0)
        tf = (f64 + f32) / sec / 1e12
        peak = FP64_VALU_PEAK_TFLOPS if precision == "fp64" else FP32_NONPACKED_PEAK_TFLOPS
        out["counter_flops"] = {"flops_per_launch_f64": f64, "flops_per_launch_f32": f32,
                                "tflops": tf, "peak": peak, "frac": tf / peak,
                                "per_edge_update": (f64 + f32) / edges}
    if "valu_insts_per_edge" in ent:
        per_edge = ent["valu_insts_per_edge"]
        busy_s = per_edge * edges / 64.0 * CYCLES_PER_WAVE_INST / SIMDS / CLOCK_HZ
        vi = {"insts_per_edge": per_edge, "frac": busy_s / sec}
        if "valu_active_per_edge" in ent:
            # the VALU-active counter (4-cycle units) also counts the extra cycles of
            # quarter-rate (transcendental) instructions
            act_s = ent["valu_active_per_edge"] * edges / 64.0 * CYCLES_PER_WAVE_INST / SIMDS / CLOCK_HZ
            vi["active_per_edge"] = ent["valu_active_per_edge"]
            vi["active_frac"] = act_s / sec
        out["valu_issue"] = vi
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


def log_run(wl_name: str, precision: str, solver: str, steps: int, kind: str):
    """One line per GPU run on stderr: a kernel trace of this command is matched to its legs
    by these lines (each run is one k_cfl dispatch followed by its step kernels)."""
    print(f"[run] workload={wl_name} precision={precision} solver={solver} steps={steps} "
          f"kind={kind}", file=sys.stderr, flush=True)


def make_context(wl, precision: str, stream, launch=None, solver: str = "adot",
                 tune_cache: str | None = TUNE_CACHE):
    """Context and device state for a workload; the launch is set explicitly, or by the
    autotuner (its cache first; trials on a scratch copy of the state on a miss)."""
    from paper_1912_04791_amd import dsve
    ctx = dsve.Context.from_workload(wl, precision=precision, stream=stream, solver=solver)
    h, q, z, t = dsve.upload(wl)
    if launch:
        ctx.set_launch(*launch[:3])
        ctx.set_cfl_split(launch[3])
    else:
        ctx.autotune(h, q, z, trial_steps=20, cache_path=tune_cache)
    return ctx, (h, q, z, t)


def time_gpu(wl, precision: str, steps: int, warmup: int, launch=None, solver: str = "adot",
             tune_cache: str | None = TUNE_CACHE, warm_s: float = 0.0):
    """W warm-up steps, then K steps timed with HIP events on the context's stream.  The graphs
    of both runs are captured first, so the warm-up ends where the timed steps begin, with no
    host wait between them.  With warm_s > 0 (the workloads timed beside the headline), warm-up
    rounds of about 20 ms each run for warm_s seconds before that, so that a short timed region
    (20 c2 steps take 0.5 ms) starts at the clock the load holds rather than at an idle GPU's."""
    import torch
    stream = torch.cuda.current_stream()
    ctx, (h, q, z, t) = make_context(wl, precision, stream, launch, solver, tune_cache)
    if warmup > 0:
        ctx.prepare_run(h, q, z, warmup, t)
    ctx.prepare_run(h, q, z, steps, t)
    ctx.sync()
    torch.cuda.synchronize()
    if warmup > 0:
        if warm_s > 0:
            # rounds of about 20 ms each, sized from one round of W steps
            log_run(wl.name, precision, solver, warmup, "warmup")
            t0 = time.perf_counter()
            ctx.adot_step(h, q, z, warmup, t)
            ctx.sync()
            per_step = max((time.perf_counter() - t0) / warmup, 1e-6)
            n_round = int(min(max(warmup, 0.02 / per_step), 5000))
            t_end = time.perf_counter() + warm_s
            while time.perf_counter() < t_end:
                log_run(wl.name, precision, solver, n_round, "warmup")
                ctx.adot_step(h, q, z, n_round, t)
                ctx.sync()
        log_run(wl.name, precision, solver, warmup, "warmup")
        ctx.adot_step(h, q, z, warmup, t)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    log_run(wl.name, precision, solver, steps, "timed")
    e0.record(stream)
    ctx.adot_step(h, q, z, steps, t)
    e1.record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    glaunch, gsteps, direct = ctx.last_run()
    tile, bpc, gsz = ctx.get_launch()
    res = {"ms_total": ms, "wall_s": wall, "launch": (tile, bpc, gsz, ctx.get_cfl_split()),
           "cus": ctx.device_cus(), "resident": ctx.get_resident(),
           "graph": {"replays": glaunch, "steps_replayed": gsteps, "direct_launches": direct}}
    ctx.close()
    return res


def gpu_state_after(wl, precision: str, steps: int, cells=None, tune_cache: str | None = TUNE_CACHE):
    """State after `steps` steps of the whole workload on the GPU (at the tuned launch), as host
    arrays (only the cells in `cells`, an index array, when given), and the run's step time."""
    import torch
    stream = torch.cuda.current_stream()
    ctx, (h, q, z, t) = make_context(wl, precision, stream, None, "adot", tune_cache)
    ctx.prepare_run(h, q, z, steps, t)
    ctx.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    log_run(wl.name, precision, "adot", steps, "full")
    e0.record(stream)
    ctx.adot_step(h, q, z, steps, t)
    e1.record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    if cells is not None:
        idx = torch.from_numpy(np.asarray(cells, dtype=np.int64)).cuda()
        out = tuple(a.index_select(0, idx).cpu().numpy() for a in (h, q, z))
    else:
        out = (h.cpu().numpy(), q.cpu().numpy(), z.cpu().numpy())
    ctx.close()
    return out, ms / max(steps, 1)


def rel_l1_max(got, ref, g: float = 9.81) -> float:
    """Largest relative L1 over h, q, z: ||got - ref||_1 / max(||ref||_1, 1e-3 ||s||_1), s the
    variable's natural size in its units (the depth for h and z, the critical discharge
    h sqrt(g h) for q)."""
    h = np.abs(ref[0])
    scales = (h, h * np.sqrt(g * h), h)
    return float(max(np.abs(a - r).sum() / max(np.abs(r).sum(), 1e-3 * s.sum())
                     for a, r, s in zip(got, ref, scales)))


# Algorithmic figures of the standalone entry points: operations per unit as counted for the step
# kernel (a node 166, a cell's CFL speed 51), HBM bytes per unit from their argument layouts.
FLUCT_OPS_PER_EDGE = 3 * OPS_PER_NODE   # pairwise D+- at G = 3
FLUCT_BYTES_PER_EDGE = 96               # six states read, six fluctuation components written
CFL_OPS_PER_CELL = 51
CFL_BYTES_PER_CELL = 16                 # h and q read (the speeds do not depend on z)
UPDATE_BYTES_PER_CELL = 96              # h, q, z read and written, D- and D+ read (3 rows each)


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


def host_cpu():
    """This host's CPU: model name, logical CPUs, CPUs this process may run on, and the thread
    count the oracle uses (the CPUs it may run on, capped by OMP_NUM_THREADS when set, the CPU
    share a job on this host is given)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = nproc
    threads = avail
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        threads = min(threads, int(omp))
    return {"model": model, "nproc": nproc, "affinity": avail,
            "omp_num_threads": int(omp) if omp.isdigit() else None, "threads": threads}


def _specs(sample, wl):
    import oracle
    return [oracle.ChannelSpec(n_cells=int(sample.lengths()[c]), dx=float(sample.dx[c]),
                               Ag=float(sample.Ag[c]), porosity=float(sample.porosity[c]), g=wl.g,
                               n_gauss=wl.n_gauss, cfl=wl.cfl, bc_left=int(sample.bc_left[c]),
                               bc_right=int(sample.bc_right[c]), q_in=float(sample.q_in[c]),
                               h_in=float(sample.h_in[c]), h_out=float(sample.h_out[c]),
                               law=int(sample.law), par=tuple(float(v) for v in sample.law_par[c]),
                               ks=float(sample.ks[c]),
                               dir_left=tuple(float(v) for v in sample.dir_left[c]),
                               dir_right=tuple(float(v) for v in sample.dir_right[c]))
            for c in range(sample.n_channels)]


def oracle_run(sample, wl, steps: int, threads: int):
    import oracle
    specs = _specs(sample, wl)
    if sample.n_channels == 1:
        return oracle.run(specs[0], sample.h, sample.q, sample.z, steps, nthreads=threads)[:3]
    return oracle.run_batched(specs, sample.offsets, sample.h, sample.q, sample.z, steps,
                              nthreads=threads)[:3]


def cpu_baseline(wl, chan_stride: int, single_channels: int):
    """The oracle as it stands, on this host's cores, over all of the workload's steps on a
    deterministic sample of its channels (every `chan_stride`-th), with the oracle's thread count
    (host_cpu) and again with one thread on the first `single_channels` of them.  Returns the
    baseline dict, the sampled channels and the oracle state of the sample."""
    cpu = host_cpu()
    chans = np.arange(0, wl.n_channels, chan_stride)
    sample = wl.subset(chans)
    t0 = time.perf_counter()
    ref = oracle_run(sample, wl, wl.steps, cpu["threads"])
    el = time.perf_counter() - t0
    eu = sample.edges_per_step() * wl.steps
    one = wl.subset(chans[:single_channels])
    t0 = time.perf_counter()
    oracle_run(one, wl, wl.steps, 1)
    el1 = time.perf_counter() - t0
    eu1 = one.edges_per_step() * wl.steps
    base = {"value": eu / el, "unit": UNIT, "cores": cpu["threads"], "kind": "oracle",
            "sample": (f"{wl.name}: {sample.n_channels} of {wl.n_channels} channels (every "
                       f"{chan_stride}th, {sample.n_cells} cells), all {wl.steps} steps; "
                       f"{el:.1f} s on {cpu['threads']} threads"),
            "one_thread": {"value": eu1 / el1, "unit": UNIT, "cores": 1,
                           "sample": (f"{wl.name}: the first {one.n_channels} of those channels "
                                      f"({one.n_cells} cells), all {wl.steps} steps; {el1:.1f} s")},
            "cpu_model": cpu["model"], "nproc": cpu["nproc"], "affinity": cpu["affinity"],
            "omp_num_threads": cpu["omp_num_threads"],
            "paper_cpu": PAPER_CPU}
    return base, chans, sample, ref


def per_channel_l1(got, ref, sample) -> float:
    worst = 0.0
    for j in range(sample.n_channels):
        lo, hi = int(sample.offsets[j]), int(sample.offsets[j + 1])
        worst = max(worst, rel_l1_max([g[lo:hi] for g in got], [r[lo:hi] for r in ref]))
    return worst


def leg(wl, precisions, steps, warmup, launch, tune_cache, warm_s: float = 0.0):
    """Timed runs of one workload in each precision, with their rooflines."""
    edges = wl.edges_per_step()
    ops = ops_per_edge_update(wl.n_gauss)
    out = {}
    for prec in precisions:
        r = time_gpu(wl, prec, steps, warmup, launch, tune_cache=tune_cache, warm_s=warm_s)
        v = edges * steps / (r["ms_total"] * 1e-3)
        msps = r["ms_total"] / steps
        print(f"[bench] {wl.name} {prec}: {msps * 1e3:.2f} us/step, {v:.4e} edge-updates/s",
              file=sys.stderr, flush=True)
        achieved = edges * ops / (msps * 1e-3) / 1e12
        form = "GRASS" if wl.law == 0 else "LAW"
        kernel = (f"{'k_resident' if r['resident'] else 'k_step'}<{wl.n_gauss}, "
                  f"{'FP64' if prec == 'fp64' else 'MIXED'}, {form}>")
        cf = counter_figures(wl.name, prec, edges, msps, r["launch"])
        roof = {**alu_roofline(prec, achieved), "traffic": cf["traffic"], "kernel": kernel,
                "ops_per_edge_update": ops, "counter_flops": cf["counter_flops"],
                "valu_issue": cf["valu_issue"]}
        if wl.law != 0:
            roof["note"] = ("ops count the scheme only; the closure's powers and roots per node "
                            "are extra work, so frac is a lower bound")
        out[prec] = {"value": v, "ms_per_step": msps, "steps": steps, "warmup": warmup,
                     **({"warm_s": warm_s} if warm_s > 0 else {}),
                     "launch": {"tile": r["launch"][0], "blocks_per_cu": r["launch"][1],
                                "graph_steps": r["launch"][2], "cfl_split": r["launch"][3]},
                     "graph": r["graph"], "roofline": roof}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c5",
                    choices=["c1", "c2", "c3", "c4", "c5", "soni", "bellal_mpm", "bellal_vanrijn",
                             "bellal_thr"])
    ap.add_argument("--precisions", default="fp64,mixed",
                    help="comma list; the first is the headline value")
    ap.add_argument("--extra", default=None,
                    help="comma list of further workloads timed beside the headline (default "
                         "c4,c2 for the c5 headline, none otherwise; 'none' for none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline and L1")
    ap.add_argument("--dot-steps", type=int, default=10,
                    help="steps timed for the original DOT (numerical eigensolver) baseline on "
                         "the headline workload; 0 skips it")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=-1)
    ap.add_argument("--graph-steps", type=int, default=-1)
    ap.add_argument("--cfl-split", type=int, default=0,
                    help="CFL sub-slots per channel with an explicit launch (0 = automatic)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuner cache (read, and written on a miss); 'none' tunes afresh")
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
    tune_cache = None if args.tune_cache == "none" else args.tune_cache

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

    launch = None
    if args.tile or args.blocks_per_cu >= 0 or args.graph_steps >= 0:
        launch = (args.tile or 256, max(args.blocks_per_cu, 0),
                  60 if args.graph_steps < 0 else args.graph_steps, args.cfl_split)
    precisions = [p for p in args.precisions.split(",") if p]
    extra = (["c4", "c2"] if args.workload == "c5" else []) if args.extra is None else \
        [w for w in args.extra.split(",") if w and w != "none"]
    DESCRIPTIONS = _descriptions()

    wl = make_workload(args.workload)
    edges = wl.edges_per_step()
    res = leg(wl, precisions, args.steps, args.warmup, launch, tune_cache)
    main_prec = precisions[0]
    m = res[main_prec]
    out = {
        "metric": METRIC,
        "value": m["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS[wl.name],
                   "n_cells": wl.n_cells, "n_channels": wl.n_channels,
                   "edges_per_step": edges, "precision": main_prec,
                   "launch": m["launch"], "graph": m["graph"],
                   "parallelism": "single GPU"},
        "roofline": m["roofline"],
    }
    for prec in precisions[1:]:
        r = res[prec]
        out[prec] = {**r, "speedup_vs_" + main_prec: r["value"] / m["value"]}

    for name in extra:
        w2 = make_workload(name)
        r2 = leg(w2, precisions, args.steps, args.warmup, launch, tune_cache, warm_s=EXTRA_WARM_S)
        out[name] = {"workload": DESCRIPTIONS[w2.name], "n_cells": w2.n_cells,
                     "n_channels": w2.n_channels, "edges_per_step": w2.edges_per_step(), **r2}
        if len(precisions) > 1:
            out[name]["speedup_" + precisions[1] + "_vs_" + main_prec] = \
                r2[precisions[1]]["value"] / r2[main_prec]["value"]
        del w2

    if args.dot_steps > 0:
        # the paper's own baseline: the same scheme with the numerical eigen-decomposition, at
        # the FP64 form's launch
        fl = res.get("fp64", m)["launch"]
        dl = (fl["tile"], fl["blocks_per_cu"], fl["graph_steps"], fl["cfl_split"])
        r = time_gpu(wl, "fp64", args.dot_steps, 1, dl, solver="dot")
        v = edges * args.dot_steps / (r["ms_total"] * 1e-3)
        print(f"[bench] {wl.name} dot fp64: {r['ms_total'] / args.dot_steps * 1e3:.2f} us/step, "
              f"{v:.4e} edge-updates/s", file=sys.stderr, flush=True)
        adot64 = res.get("fp64")
        out["dot_fp64"] = {"value": v, "ms_per_step": r["ms_total"] / args.dot_steps,
                           "steps": args.dot_steps, "graph": r["graph"],
                           "launch": {"tile": r["launch"][0], "blocks_per_cu": r["launch"][1],
                                      "graph_steps": r["launch"][2], "cfl_split": r["launch"][3]},
                           "adot_fp64_speedup": (adot64["value"] / v) if adot64 else None}

    if not args.no_entry:
        out["entry_points"] = entry_point_rates()
        for k, v in out["entry_points"].items():
            r = v["roofline"]
            print(f"[bench] {k}: {v['us_per_call']:.1f} us/call, {r['achieved']:.2f} {r['unit']} "
                  f"({r['frac']:.2f} of {r['bound']} peak)", file=sys.stderr, flush=True)

    if not args.no_cpu:
        # the oracle over all steps: on sampled channels of a batched workload (every 1024th of
        # c5, 64 channels), on the whole channel of a single-channel one
        batched = wl.n_channels > 1
        stride = max(1, wl.n_channels // 64) if batched else 1
        base, chans, sample, ref = cpu_baseline(wl, stride, 2 if batched else 1)
        out["cpu_baseline"] = base
        print(f"[bench] cpu oracle: {base['value']:.4e} edge-updates/s on {base['cores']} "
              f"threads, {base['one_thread']['value']:.4e} on one", file=sys.stderr, flush=True)
        cells = np.concatenate([np.arange(wl.offsets[c], wl.offsets[c + 1]) for c in chans])
        l1 = {"steps": wl.steps, "per": "channel" if batched else "run",
              "channels_compared": int(len(chans))}
        for prec in precisions:
            got, msps = gpu_state_after(wl, prec, wl.steps, cells, tune_cache)
            l1[prec] = per_channel_l1(got, ref, sample)
            l1[prec + "_run_ms_per_step"] = msps
        out["l1_vs_oracle"] = l1
        # the single-channel extra workload over all its steps, whole channel
        for name in extra:
            w2 = make_workload(name)
            if w2.n_channels != 1:
                continue
            t0 = time.perf_counter()
            ref2 = oracle_run(w2, w2, w2.steps, host_cpu()["threads"])
            el = time.perf_counter() - t0
            e2 = {"steps": w2.steps, "per": "run", "oracle_s": el}
            for prec in precisions:
                got, _ = gpu_state_after(w2, prec, w2.steps, None, tune_cache)
                e2[prec] = rel_l1_max(got, ref2)
            out["l1_vs_oracle_" + name] = e2
            print(f"[bench] {name} L1 over {w2.steps} steps: " +
                  ", ".join(f"{p} {e2[p]:.2e}" for p in precisions), file=sys.stderr, flush=True)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
