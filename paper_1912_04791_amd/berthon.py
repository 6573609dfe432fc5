"""Grid-convergence run of the smooth analytical solution of Sec. 4.2 (Test 2) on the GPU.

    python -m paper_1912_04791_amd.berthon [--n 100,300,600,900,1800,7200,28800] [--precisions fp64,mixed]

For each grid of N cells: the exact solution as initial state, Dirichlet ghost cells carrying
it, time steps of the fused A-DOT kernel up to t_end = 10 s (the step count is fixed after a
first chunk of steps from the constant time step of this steady flow, so the run ends within
one time step of t_end), then the normalised root-square errors E_phi of Eq. Eg for
phi = h, q, z against the closed form at the run's final clock.  Prints one JSON line per
(N, precision) with the errors, the step count and the GPU time to solution (HIP events on
the context's stream).
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import inputs


def e_phi(got: np.ndarray, ref: np.ndarray) -> float:
    """Normalised root-square error of Eq. Eg."""
    return float(np.sqrt(np.sum((got - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))


def run(n_cells: int, precision: str = "fp64", t_end: float | None = None, first: int = 60):
    import torch
    from . import dsve

    t_end = inputs.BERTHON["t_end"] if t_end is None else t_end
    wl = inputs.make_berthon(n_cells)
    stream = torch.cuda.current_stream()
    ctx = dsve.Context.from_workload(wl, precision=precision, stream=stream)
    h, q, z, t = dsve.upload(wl)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.adot_step(h, q, z, first, t)
    ctx.sync()
    dt = float(t[0]) / first                     # the time step of the steady flow
    total = max(first, int(round(t_end / dt)))
    ctx.adot_step(h, q, z, total - first, t)
    e1.record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    tf = float(t[0])
    he, qe, ze = inputs.berthon_exact(wl.meta["x"], tf, wl.g)
    got = [a.cpu().numpy() for a in (h, q, z)]
    ctx.close()
    return {"n_cells": n_cells, "precision": precision, "steps": total, "t_final": tf,
            "E_h": e_phi(got[0], he), "E_q": e_phi(got[1], qe), "E_z": e_phi(got[2], ze),
            "gpu_s": e0.elapsed_time(e1) * 1e-3}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", default="100,300,600,900,1800,7200,28800")
    ap.add_argument("--precisions", default="fp64,mixed")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("needs a GPU", file=sys.stderr)
        sys.exit(1)
    for n in (int(v) for v in args.n.split(",") if v):
        for prec in (p for p in args.precisions.split(",") if p):
            print(json.dumps(run(n, prec)), flush=True)


if __name__ == "__main__":
    main()
