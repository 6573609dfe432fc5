"""Seeded synthetic inputs for the A-DOT hot path.

This module builds initial states and per-channel parameters only; it holds
none of the scheme's arithmetic (no eigenstructure, no fluctuations, no
update, no time step).  Both the HIP path and the CPU oracle are fed from
here, so it imports neither.

Workloads (all synthetic; the paper's own test data are not used):

* ``c1`` -- Riemann problem on [0, 10] m, N = 250, left (h, u, z) = (2.0, 0.5, 0.0),
  right (1.0, 0.3, 0.2), A_g = 0.01, porosity 0.4, transmissive, 200 steps.
  Shaped like the paper's movable-bed Riemann test (Sec. 4.1).
* ``c2`` -- one periodic channel, N = 2^20, L = 1000 m, h = 1 + 0.1 sin(2 pi k x / L)
  with k drawn from {1..8}, u = 0.4 + 0.05 n(x) where n is unit-variance periodic Gaussian
  noise limited to Fourier modes 0..64 (a random Fourier series with complex Gaussian
  coefficients, mean removed), z = 0.05 cos(2 pi x / L),
  A_g = 0.005, porosity 0.4, 1000 steps.
* ``c3`` -- transcritical flow over a Gaussian bed bump, N = 2^24, L = 100 m,
  z = 0.2 exp(-((x-50)/5)^2), q = 0.5, h the frictionless Bernoulli profile
  through critical depth at the crest (subcritical upstream, supercritical
  downstream) times (1 + 0.01 U[-1, 1]); inflow q = 0.5 on the left,
  transmissive on the right, A_g = 0.001, porosity 0.4, 2000 steps.
  Shaped like the paper's flow over a movable hump (Sec. 4.3).
* ``c4`` -- 4096 independent channels, lengths log-uniform in [256, 65536],
  dx = 0.04, Riemann states h ~ U[0.5, 3], u ~ U[-1, 1], z_L = 0, z_R ~ U[-0.3, 0.3],
  A_g ~ U[0.001, 0.05], porosity ~ U[0.3, 0.45], transmissive, 500 steps.
* ``c5`` -- 65536 channels, lengths uniform in {512..4096}; half (a seeded
  permutation) smooth periodic channels built with the ``c2`` recipe on
  L_c = N_c * 1000 / 2^20 with modes |m| <= 8, half Riemann channels built with
  the ``c4`` recipe; A_g and porosity drawn per channel as in ``c4``; 5000 steps.

Every generator takes scale parameters so the same recipe can be built at a
size the oracle finishes in seconds.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

G_ACC = 9.81

BC_TRANSMISSIVE = 0
BC_PERIODIC = 1
BC_INFLOW_Q = 2


@dataclass
class Workload:
    """Initial state and parameters of one or more channels (concatenated SoA)."""
    name: str
    h: np.ndarray
    q: np.ndarray
    z: np.ndarray
    offsets: np.ndarray          # int64 [C+1]
    dx: np.ndarray               # float64 [C]
    Ag: np.ndarray               # float64 [C]
    porosity: np.ndarray         # float64 [C]
    bc_left: np.ndarray          # int32 [C]
    bc_right: np.ndarray         # int32 [C]
    q_in: np.ndarray             # float64 [C]
    steps: int
    g: float = G_ACC
    cfl: float = 0.9
    n_gauss: int = 3
    precision: str = "fp64"
    seed: int | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_channels(self) -> int:
        return int(self.offsets.size - 1)

    @property
    def n_cells(self) -> int:
        return int(self.offsets[-1])

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def edges_per_step(self) -> int:
        """Edge updates per step: N_c + 1 per channel, N_c for a periodic channel."""
        n = self.lengths()
        per = np.where(self.bc_left == BC_PERIODIC, n, n + 1)
        return int(per.sum())

    def channel(self, c: int) -> "Workload":
        """The single-channel workload of channel c (copies of its arrays)."""
        lo, hi = int(self.offsets[c]), int(self.offsets[c + 1])
        return Workload(
            name=f"{self.name}[{c}]", h=self.h[lo:hi].copy(), q=self.q[lo:hi].copy(),
            z=self.z[lo:hi].copy(), offsets=np.array([0, hi - lo], dtype=np.int64),
            dx=self.dx[c:c + 1].copy(), Ag=self.Ag[c:c + 1].copy(),
            porosity=self.porosity[c:c + 1].copy(), bc_left=self.bc_left[c:c + 1].copy(),
            bc_right=self.bc_right[c:c + 1].copy(), q_in=self.q_in[c:c + 1].copy(),
            steps=self.steps, g=self.g, cfl=self.cfl, n_gauss=self.n_gauss,
            precision=self.precision, seed=self.seed, meta=dict(self.meta))

    def subset(self, channels) -> "Workload":
        """A workload made of the listed channels (copies)."""
        channels = np.asarray(channels, dtype=np.int64)
        parts = [(int(self.offsets[c]), int(self.offsets[c + 1])) for c in channels]
        lens = np.array([hi - lo for lo, hi in parts], dtype=np.int64)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        cat = lambda a: np.concatenate([a[lo:hi] for lo, hi in parts]) if parts else a[:0]
        return Workload(
            name=f"{self.name}[subset {channels.size}]", h=cat(self.h), q=cat(self.q),
            z=cat(self.z), offsets=off, dx=self.dx[channels].copy(), Ag=self.Ag[channels].copy(),
            porosity=self.porosity[channels].copy(), bc_left=self.bc_left[channels].copy(),
            bc_right=self.bc_right[channels].copy(), q_in=self.q_in[channels].copy(),
            steps=self.steps, g=self.g, cfl=self.cfl, n_gauss=self.n_gauss,
            precision=self.precision, seed=self.seed,
            meta=dict(self.meta, subset=channels.tolist()[:16]))


def _single(name, h, q, z, dx, Ag, porosity, bc_l, bc_r, q_in, steps, **kw) -> Workload:
    n = h.size
    return Workload(
        name=name, h=np.ascontiguousarray(h, dtype=np.float64),
        q=np.ascontiguousarray(q, dtype=np.float64), z=np.ascontiguousarray(z, dtype=np.float64),
        offsets=np.array([0, n], dtype=np.int64), dx=np.array([dx], dtype=np.float64),
        Ag=np.array([Ag], dtype=np.float64), porosity=np.array([porosity], dtype=np.float64),
        bc_left=np.array([bc_l], dtype=np.int32), bc_right=np.array([bc_r], dtype=np.int32),
        q_in=np.array([q_in], dtype=np.float64), steps=steps, **kw)


def cell_centres(n: int, length: float, x0: float = 0.0) -> np.ndarray:
    dx = length / n
    return x0 + (np.arange(n, dtype=np.float64) + 0.5) * dx


# ---------------------------------------------------------------------------
def make_c1(n_cells: int = 250, steps: int = 200) -> Workload:
    """Riemann problem on [0, 10] m (left cells x < 5)."""
    L = 10.0
    x = cell_centres(n_cells, L)
    left = x < 5.0
    h = np.where(left, 2.0, 1.0)
    u = np.where(left, 0.5, 0.3)
    z = np.where(left, 0.0, 0.2)
    return _single("c1", h, h * u, z, L / n_cells, 0.01, 0.4, BC_TRANSMISSIVE, BC_TRANSMISSIVE,
                   0.0, steps, meta={"L": L})


def _fourier_noise(coefs: np.ndarray, n: int) -> np.ndarray:
    """Rows of sum_{m=0..M} Re(c_m exp(2 pi i m x)), x = (j + 1/2)/n, each rescaled to unit
    standard deviation: periodic Gaussian noise limited to Fourier modes m <= M."""
    coefs = np.atleast_2d(coefs)
    x = (np.arange(n, dtype=np.float64) + 0.5) / n
    z = np.exp(2j * np.pi * x)
    zm = np.ones(n, dtype=np.complex128)
    out = np.zeros((coefs.shape[0], n))
    for m in range(coefs.shape[1]):
        out += (coefs[:, m:m + 1] * zm[None, :]).real
        zm = zm * z
    out -= out.mean(axis=1, keepdims=True)
    sd = out.std(axis=1, keepdims=True)
    return out / np.where(sd > 0, sd, 1.0)


def _noise_coefs(rng: np.random.Generator, max_mode: int) -> np.ndarray:
    return rng.standard_normal(max_mode + 1) + 1j * rng.standard_normal(max_mode + 1)


def smooth_periodic_state(rng: np.random.Generator, n: int, length: float, max_mode: int):
    """h = 1 + 0.1 sin(2 pi k x/L), u = 0.4 + 0.05 noise, z = 0.05 cos(2 pi x/L)."""
    x = cell_centres(n, length)
    k = int(rng.integers(1, 9))
    h = 1.0 + 0.1 * np.sin(2.0 * np.pi * k * x / length)
    u = 0.4 + 0.05 * _fourier_noise(_noise_coefs(rng, max_mode), n)[0]
    z = 0.05 * np.cos(2.0 * np.pi * x / length)
    return h, h * u, z, k


def make_c2(n_cells: int = 1 << 20, steps: int = 1000, seed: int = 2, length: float = 1000.0,
            max_mode: int = 64) -> Workload:
    rng = np.random.default_rng(seed)
    h, q, z, k = smooth_periodic_state(rng, n_cells, length, max_mode)
    return _single("c2", h, q, z, length / n_cells, 0.005, 0.4, BC_PERIODIC, BC_PERIODIC, 0.0,
                   steps, seed=seed, meta={"L": length, "k": k})


def bernoulli_depth(z: np.ndarray, q: float, H: float, g: float, supercritical: np.ndarray,
                    iters: int = 80) -> np.ndarray:
    """Depth h solving h + q^2/(2 g h^2) + z = H, on the chosen branch (Newton, FP64).

    Physics of the initial condition only (frictionless steady energy balance).
    Cells whose iterate has stopped moving leave the active set.
    """
    hc = (q * q / g) ** (1.0 / 3.0)
    E = H - z
    h = np.where(supercritical, 0.5 * hc, np.maximum(E, 1.5 * hc))
    idx = np.arange(h.size)
    for _ in range(iters):
        if idx.size == 0:
            break
        hh, EE, sup = h[idx], E[idx], supercritical[idx]
        f = hh + q * q / (2.0 * g * hh * hh) - EE
        df = 1.0 - q * q / (g * hh ** 3)
        step = f / np.where(np.abs(df) > 1e-14, df, 1e-14)
        h_new = hh - step
        # stay on the branch: subcritical h >= hc, supercritical h <= hc
        h_new = np.where(sup, np.clip(h_new, 1e-6, hc), np.maximum(h_new, hc))
        moving = np.abs(h_new - hh) > 1e-15 * hc
        h[idx] = h_new
        idx = idx[moving]
    return h


def make_c3(n_cells: int = 1 << 24, steps: int = 2000, seed: int = 3, length: float = 100.0,
            q0: float = 0.5, Ag: float = 0.001) -> Workload:
    rng = np.random.default_rng(seed)
    x = cell_centres(n_cells, length)
    z = 0.2 * np.exp(-((x - 50.0) / 5.0) ** 2)
    hc = (q0 * q0 / G_ACC) ** (1.0 / 3.0)
    H = 0.2 + 1.5 * hc
    h = bernoulli_depth(z, q0, H, G_ACC, supercritical=(x >= 50.0))
    h = h * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, n_cells))
    q = np.full(n_cells, q0)
    return _single("c3", h, q, z, length / n_cells, Ag, 0.4, BC_INFLOW_Q, BC_TRANSMISSIVE, q0,
                   steps, seed=seed, precision="mixed", meta={"L": length, "hc": hc, "H": H})


def riemann_state(rng: np.random.Generator, n: int):
    """Centre-jump Riemann data: h ~ U[0.5,3], u ~ U[-1,1] each side, z_L = 0, z_R ~ U[-0.3,0.3]."""
    hL, hR = rng.uniform(0.5, 3.0, 2)
    uL, uR = rng.uniform(-1.0, 1.0, 2)
    zR = rng.uniform(-0.3, 0.3)
    left = np.arange(n) < n // 2
    h = np.where(left, hL, hR)
    u = np.where(left, uL, uR)
    z = np.where(left, 0.0, zR)
    return h, h * u, z


def _assemble(name, parts, dx, Ag, por, bcl, bcr, steps, seed, **kw) -> Workload:
    lens = np.array([p[0].size for p in parts], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    C = lens.size
    return Workload(
        name=name, h=np.concatenate([p[0] for p in parts]),
        q=np.concatenate([p[1] for p in parts]), z=np.concatenate([p[2] for p in parts]),
        offsets=off, dx=np.asarray(dx, dtype=np.float64), Ag=np.asarray(Ag, dtype=np.float64),
        porosity=np.asarray(por, dtype=np.float64), bc_left=np.asarray(bcl, dtype=np.int32),
        bc_right=np.asarray(bcr, dtype=np.int32), q_in=np.zeros(C), steps=steps, seed=seed, **kw)


def make_c4(n_channels: int = 4096, len_lo: int = 256, len_hi: int = 65536, steps: int = 500,
            seed: int = 4) -> Workload:
    ss = np.random.SeedSequence(seed)
    top = np.random.default_rng(ss.spawn(1)[0])
    lens = np.rint(np.exp(top.uniform(np.log(len_lo), np.log(len_hi), n_channels))).astype(np.int64)
    Ag = top.uniform(0.001, 0.05, n_channels)
    por = top.uniform(0.3, 0.45, n_channels)
    children = ss.spawn(n_channels + 1)[1:]
    parts = [riemann_state(np.random.default_rng(children[c]), int(lens[c]))
             for c in range(n_channels)]
    dx = np.full(n_channels, 0.04)
    bc = np.full(n_channels, BC_TRANSMISSIVE)
    return _assemble("c4", parts, dx, Ag, por, bc, bc, steps, seed)


def make_c5(n_channels: int = 65536, len_lo: int = 512, len_hi: int = 4096, steps: int = 5000,
            seed: int = 5) -> Workload:
    ss = np.random.SeedSequence(seed)
    top = np.random.default_rng(ss.spawn(1)[0])
    lens = top.integers(len_lo, len_hi + 1, n_channels).astype(np.int64)
    Ag = top.uniform(0.001, 0.05, n_channels)
    por = top.uniform(0.3, 0.45, n_channels)
    kind = top.permutation(np.arange(n_channels) % 2)  # 0 smooth, 1 Riemann
    children = ss.spawn(n_channels + 1)[1:]
    parts = [None] * n_channels
    dx, bcl = np.zeros(n_channels), np.zeros(n_channels, dtype=np.int32)
    smooth_k, smooth_coefs = {}, {}
    for c in range(n_channels):
        rng = np.random.default_rng(children[c])
        n = int(lens[c])
        if kind[c] == 0:
            # same draws, in the same order, as smooth_periodic_state (k, then the coefficients)
            smooth_k[c] = int(rng.integers(1, 9))
            smooth_coefs[c] = _noise_coefs(rng, 8)
            dx[c] = (n * 1000.0 / float(1 << 20)) / n
            bcl[c] = BC_PERIODIC
        else:
            parts[c] = riemann_state(rng, n)
            dx[c] = 0.04
            bcl[c] = BC_TRANSMISSIVE
    # smooth channels, synthesised in groups of equal length
    smooth = np.array(sorted(smooth_k), dtype=np.int64)
    for n in np.unique(lens[smooth]) if smooth.size else []:
        grp = smooth[lens[smooth] == n]
        noise = _fourier_noise(np.stack([smooth_coefs[c] for c in grp]), int(n))
        Lc = n * 1000.0 / float(1 << 20)
        x = cell_centres(int(n), Lc)
        z = 0.05 * np.cos(2.0 * np.pi * x / Lc)
        for j, c in enumerate(grp):
            h = 1.0 + 0.1 * np.sin(2.0 * np.pi * smooth_k[c] * x / Lc)
            parts[c] = (h, h * (0.4 + 0.05 * noise[j]), z.copy())
    return _assemble("c5", parts, dx, Ag, por, bcl, bcl.copy(), steps, seed, precision="mixed",
                     meta={"kind": kind})


def make_lake_at_rest(n_cells: int = 400, length: float = 10.0, level: float = 1.0,
                      Ag: float = 0.01, steps: int = 200, seed: int = 7) -> Workload:
    """Still water over a rough bed: u = 0, h + z = level (periodic)."""
    rng = np.random.default_rng(seed)
    x = cell_centres(n_cells, length)
    z = 0.2 * np.sin(2 * np.pi * x / length) + 0.05 * rng.uniform(-1, 1, n_cells)
    h = level - z
    return _single("lake", h, np.zeros(n_cells), z, length / n_cells, Ag, 0.4, BC_PERIODIC,
                   BC_PERIODIC, 0.0, steps, seed=seed)


def make_random_edges(n: int, seed: int = 11, h_range=(0.05, 5.0), u_range=(-3.0, 3.0),
                      rel_jump: float = 0.3):
    """Random edge pairs (W-, W+) with moderate jumps, for pairwise fluctuation tests."""
    rng = np.random.default_rng(seed)
    hL = rng.uniform(*h_range, n)
    uL = rng.uniform(*u_range, n)
    zL = rng.uniform(-1.0, 1.0, n)
    hR = hL * (1.0 + rel_jump * rng.uniform(-1.0, 1.0, n))
    uR = uL + rel_jump * rng.uniform(-1.0, 1.0, n)
    zR = zL + rel_jump * rng.uniform(-1.0, 1.0, n)
    return (hL, hL * uL, zL), (hR, hR * uR, zR)


MAKERS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4, "c5": make_c5}

DESCRIPTIONS = {
    "c1": "c1: Riemann problem on [0, 10] m, N=250, A_g=0.01, porosity 0.4, G=3, CFL 0.9, "
          "transmissive, 200 steps",
    "c2": "c2: periodic single channel, N=2^20 cells, L=1000 m, smooth seeded state, "
          "A_g=0.005, porosity 0.4, G=3, CFL 0.9, 1000 steps",
    "c3": "c3: transcritical flow over a bed bump, N=2^24 cells, L=100 m, q=0.5, "
          "Fr 0.33-2.46, A_g=0.001, porosity 0.4, G=3, CFL 0.9, 2000 steps",
    "c4": "c4: 4096 channels, lengths log-uniform in [256, 65536] (4.8e7 cells), seeded "
          "Riemann states, per-channel A_g and porosity, G=3, CFL 0.9, 500 steps",
    "c5": "c5: 65536 channels, lengths uniform in [512, 4096] (1.5e8 cells), half smooth "
          "periodic, half Riemann, per-channel A_g and porosity, G=3, CFL 0.9, 5000 steps",
}
