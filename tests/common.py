"""Shared helpers for the tests (no method arithmetic here)."""
import numpy as np

import oracle
from paper_1912_04791_amd import inputs


def spec_of(wl: inputs.Workload, c: int = 0) -> "oracle.ChannelSpec":
    return oracle.ChannelSpec(n_cells=int(wl.lengths()[c]), dx=float(wl.dx[c]), Ag=float(wl.Ag[c]),
                              porosity=float(wl.porosity[c]), g=wl.g, n_gauss=wl.n_gauss,
                              cfl=wl.cfl, bc_left=int(wl.bc_left[c]), bc_right=int(wl.bc_right[c]),
                              q_in=float(wl.q_in[c]), h_out=float(wl.h_out[c]),
                              h_in=float(wl.h_in[c]), law=int(wl.law),
                              par=tuple(float(v) for v in wl.law_par[c]), ks=float(wl.ks[c]),
                              dir_left=tuple(float(v) for v in wl.dir_left[c]),
                              dir_right=tuple(float(v) for v in wl.dir_right[c]))


def oracle_run(wl: inputs.Workload, steps: int | None = None, nthreads: int | None = None):
    """Oracle result of a workload: (h, q, z, t[C])."""
    n = wl.steps if steps is None else steps
    if wl.n_channels == 1:
        h, q, z, t = oracle.run(spec_of(wl), wl.h, wl.q, wl.z, n, nthreads=nthreads)
        return h, q, z, np.array([t])
    specs = [spec_of(wl, c) for c in range(wl.n_channels)]
    return oracle.run_batched(specs, wl.offsets, wl.h, wl.q, wl.z, n, nthreads=nthreads)


def rel_l1(a: np.ndarray, ref: np.ndarray, scale: np.ndarray) -> float:
    """||a - ref||_1 / max(||ref||_1, 1e-3 ||scale||_1) (per variable; `scale` is the variable's
    natural size in its own units, see l1_scales)."""
    den = max(np.abs(ref).sum(), 1e-3 * np.abs(scale).sum())
    return float(np.abs(a - ref).sum() / den)


def l1_scales(h_ref: np.ndarray, g: float = inputs.G_ACC):
    """Scales of the floor of the relative L1 for h, q, z: the depth for h and z, and for q the
    critical discharge h c = h sqrt(g h) (q / (h c) is the Froude number, the non-dimensional
    discharge of Sec. 3.3)."""
    h = np.abs(h_ref)
    return h, h * np.sqrt(g * h), h


def max_rel_l1(got, ref) -> float:
    """Largest relative L1 error over h, q, z."""
    return max(rel_l1(g, r, s) for g, r, s in zip(got[:3], ref[:3], l1_scales(ref[0])))


def per_channel_rel_l1(got, ref, offsets) -> np.ndarray:
    C = len(offsets) - 1
    out = np.zeros(C)
    for c in range(C):
        lo, hi = offsets[c], offsets[c + 1]
        out[c] = max(rel_l1(g[lo:hi], r[lo:hi], s)
                     for g, r, s in zip(got[:3], ref[:3], l1_scales(ref[0][lo:hi])))
    return out
