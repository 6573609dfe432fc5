"""Full-size, full-length parity of the workloads, run by hand on a GPU host:

    python tests/full_length_parity.py c2 c3 c5

Each workload runs on the GPU for all its steps in both forms (autotuned launch, as the
benchmark times it), then in the oracle.  A single channel runs in the oracle in chunks of
50 steps that print their progress (chunked oracle runs are bitwise those of one run: the
state and clock carry over).  A batched workload is compared on 64 evenly spaced channels,
which is exact sampling since channels are independent.  One JSON line per form gives the
largest relative L1 error over h, q, z (per channel for batched runs) and the largest
relative error of the clocks.  The oracle needs about 13 minutes on 16 threads for c3
(2^24 cells, 2000 steps).  Not collected by pytest; the GPU tests cover the same paths on
shorter runs or fewer channels.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from paper_1912_04791_amd import dsve, inputs  # noqa: E402
from common import max_rel_l1, oracle_run, per_channel_rel_l1, spec_of  # noqa: E402

import numpy as np  # noqa: E402

CHUNK = 50
SAMPLED_CHANNELS = 64


def gpu_run(wl, precision):
    ctx = dsve.Context.from_workload(wl, precision=precision)
    h, q, z, t = dsve.upload(wl)
    ctx.autotune(h, q, z, trial_steps=12)
    t0 = time.time()
    ctx.adot_step(h, q, z, wl.steps, t)
    ctx.sync()
    secs = time.time() - t0
    out = tuple(x.cpu().numpy() for x in (h, q, z, t))
    ctx.close()
    print(f"gpu {wl.name} {precision}: {wl.steps} steps in {secs:.2f} s", flush=True)
    return out


def oracle_run_chunked(wl):
    spec = spec_of(wl)
    h, q, z, t = wl.h, wl.q, wl.z, 0.0
    done, t0 = 0, time.time()
    while done < wl.steps:
        n = min(CHUNK, wl.steps - done)
        h, q, z, t = oracle.run(spec, h, q, z, n, t0=t)
        done += n
        print(f"oracle {wl.name}: {done}/{wl.steps} steps, {time.time() - t0:.0f} s", flush=True)
    return h, q, z, t


def main(names):
    for name in names:
        wl = inputs.MAKERS[name]()
        got = {p: gpu_run(wl, p) for p in ("fp64", "mixed")}
        line = {"workload": name, "n_cells": wl.n_cells, "n_channels": wl.n_channels,
                "steps": wl.steps}
        if wl.n_channels == 1:
            h, q, z, t = oracle_run_chunked(wl)
            for p, g in got.items():
                print(json.dumps({**line, "precision": p, "rel_l1_max": max_rel_l1(g, (h, q, z)),
                                  "clock_rel": abs(g[3][0] / t - 1.0)}), flush=True)
            continue
        chans = np.arange(0, wl.n_channels, max(1, wl.n_channels // SAMPLED_CHANNELS))
        sub = wl.subset(chans)
        t0 = time.time()
        ref = oracle_run(sub)
        print(f"oracle {name}: {len(chans)} channels, {time.time() - t0:.0f} s", flush=True)
        sel = np.concatenate([np.arange(wl.offsets[c], wl.offsets[c + 1]) for c in chans])
        for p, g in got.items():
            per = per_channel_rel_l1(tuple(x[sel] for x in g[:3]), ref, sub.offsets)
            clock = float(np.max(np.abs(g[3][chans] / ref[3] - 1.0)))
            print(json.dumps({**line, "precision": p, "channels_compared": int(len(chans)),
                              "rel_l1_max": float(per.max()),
                              "rel_l1_median": float(np.median(per)), "clock_rel": clock}),
                  flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2"])
