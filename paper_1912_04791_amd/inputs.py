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

Workloads of the other closures, the friction source and the experiment boundary conditions,
shaped like the paper's laboratory cases (their measured data are not used):

* ``soni`` -- aggradation by sediment overfeeding (Sec. 5.1): flume of 30 m, uniform flow
  h0 = 0.05 m, q0 = 0.02 m^2/s on the bed slope s0 = 3.56e-3 (z = 1.2 - s0 x), power law
  q_s = 1.45e-3 u^5, porosity 0.4, K_s = 49.4; upstream inflow-(q, h) with q0 and
  h_in = 5^(-1/5) h0 (the depth at which the power law carries five times the equilibrium
  solid discharge at q0), downstream fixed depth h0.  The batched form draws per channel
  N_c in {512..4096}, q0 ~ U[0.015, 0.025], s0 ~ U[3e-3, 4e-3], K_s ~ U[45, 55], an
  overfeeding factor F ~ U[2, 5] (h_in = F^(-1/5) h0) and h0 = (q0^2 / (K_s^2 s0))^(3/10),
  the uniform-flow depth of the friction law.
* ``berthon`` -- the smooth analytical solution of Sec. 4.2 (Test 2) on N cells, Dirichlet
  ghost cells carrying the exact solution, for the error E_phi of Eq. Eg against the closed form.
* ``bellal_<law>`` -- sediment bore in a steep flume (Sec. 5.2): 6.9 m, s0 = 3.02e-2,
  q0 = 0.024 m^2/s (12 l/s over 0.5 m), d50 = 1.65 mm, porosity 0.42, K_s = 62, S_g = 2.6,
  nu = 1e-6, theta_cr = 0.03; start from the uniform flow h0 = (q0^2 / (K_s^2 s0))^(3/10)
  (supercritical) and raise the downstream depth to 0.2093 m (fixed depth) at t = 0, with the
  upstream discharges held at their equilibrium values (inflow-(q, h) with h0).  Laws:
  ``mpm`` (Meyer-Peter & Mueller), ``vanrijn`` (Van Rijn), ``thr`` (Grass with threshold,
  A_g = 0.0024, u_cr = 0.3).  The batched form draws per channel N_c in {512..4096},
  q0 ~ U[0.02, 0.028], s0 ~ U[0.025, 0.035], d50 ~ U[1.2, 2.0] mm, K_s ~ U[55, 70] and the
  downstream depth ~ U[0.07, 0.11] m: 1.2 to 2 times the depth conjugate to the inflow, so
  that, as in the experiment, a bore advances slowly upstream (a 0.21 m step over a 2.6 cm
  supercritical flow instead floods the flume backwards within seconds, with q changing sign).

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
BC_FIXED_DEPTH = 3
BC_INFLOW_QH = 4
BC_DIRICHLET = 5

LAW_GRASS = 0
LAW_GRASS_THR = 1
LAW_POWER = 2
LAW_MPM = 3
LAW_VANRIJN = 4

# per-channel array fields of a Workload, in the order channel()/subset() copy them
PER_CHANNEL = ("dx", "Ag", "porosity", "bc_left", "bc_right", "q_in", "h_in", "h_out", "ks",
               "law_par", "dir_left", "dir_right")


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
    law: int = LAW_GRASS         # closure, common to all channels
    law_par: np.ndarray | None = None   # float64 [C, 4] parameters of the law per channel
    ks: np.ndarray | None = None        # float64 [C] Strickler coefficient (0: no friction)
    h_in: np.ndarray | None = None      # float64 [C] depth of an inflow-(q, h) boundary
    h_out: np.ndarray | None = None     # float64 [C] depth of a fixed-depth boundary
    dir_left: np.ndarray | None = None  # float64 [C, 4] Dirichlet ghost (h, q, z, dz/dt), left
    dir_right: np.ndarray | None = None  # float64 [C, 4] the same, right

    def __post_init__(self):
        C = self.offsets.size - 1
        for f in ("law_par", "dir_left", "dir_right"):
            v = getattr(self, f)
            v = np.zeros((C, 4)) if v is None else np.asarray(v, dtype=np.float64).reshape(C, 4)
            setattr(self, f, np.ascontiguousarray(v))
        for f in ("ks", "h_in", "h_out"):
            v = getattr(self, f)
            setattr(self, f, np.zeros(C) if v is None else np.asarray(v, dtype=np.float64).reshape(C))

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
        return self.subset([c], name=f"{self.name}[{c}]")

    def subset(self, channels, name: str | None = None) -> "Workload":
        """A workload made of the listed channels (copies)."""
        channels = np.asarray(channels, dtype=np.int64)
        parts = [(int(self.offsets[c]), int(self.offsets[c + 1])) for c in channels]
        lens = np.array([hi - lo for lo, hi in parts], dtype=np.int64)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        cat = lambda a: np.concatenate([a[lo:hi] for lo, hi in parts]) if parts else a[:0]
        per = {f: getattr(self, f)[channels].copy() for f in PER_CHANNEL}
        meta = dict(self.meta) if channels.size == 1 else dict(self.meta, subset=channels.tolist()[:16])
        return Workload(
            name=name or f"{self.name}[subset {channels.size}]", h=cat(self.h), q=cat(self.q),
            z=cat(self.z), offsets=off, steps=self.steps, g=self.g, cfl=self.cfl,
            n_gauss=self.n_gauss, precision=self.precision, seed=self.seed, meta=meta,
            law=self.law, **per)


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


def make_riemann(n_cells: int, length: float, x_jump: float, left: dict, right: dict,
                 A_g: float, porosity: float, steps: int = 0) -> Workload:
    """Riemann problem on [0, length] with the jump at x_jump: conservative states
    ``{"h", "q", "z"}`` left and right, transmissive ends (the set-up of Sec. 4.1)."""
    x = cell_centres(n_cells, length)
    lm = x < x_jump
    h = np.where(lm, left["h"], right["h"])
    q = np.where(lm, left["q"], right["q"])
    z = np.where(lm, left["z"], right["z"])
    return _single("riemann", h, q, z, length / n_cells, A_g, porosity, BC_TRANSMISSIVE,
                   BC_TRANSMISSIVE, 0.0, steps, meta={"L": length, "x_jump": x_jump})


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


def _assemble(name, parts, dx, Ag, por, bcl, bcr, steps, seed, q_in=None, **kw) -> Workload:
    lens = np.array([p[0].size for p in parts], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    C = lens.size
    return Workload(
        name=name, h=np.concatenate([p[0] for p in parts]),
        q=np.concatenate([p[1] for p in parts]), z=np.concatenate([p[2] for p in parts]),
        offsets=off, dx=np.asarray(dx, dtype=np.float64), Ag=np.asarray(Ag, dtype=np.float64),
        porosity=np.asarray(por, dtype=np.float64), bc_left=np.asarray(bcl, dtype=np.int32),
        bc_right=np.asarray(bcr, dtype=np.int32),
        q_in=np.zeros(C) if q_in is None else np.asarray(q_in, dtype=np.float64), steps=steps,
        seed=seed, **kw)


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


# ---------------------------------------------------------------------------
def uniform_flow_depth(q: np.ndarray, ks: np.ndarray, slope: np.ndarray) -> np.ndarray:
    """Depth at which the friction slope q^2 / (K_s^2 h^(10/3)) equals the bed slope."""
    return (np.asarray(q) ** 2 / (np.asarray(ks) ** 2 * np.asarray(slope))) ** 0.3


def _sloped_channel(n: int, length: float, h0: float, q0: float, slope: float, z0: float):
    x = cell_centres(n, length)
    return np.full(n, h0), np.full(n, q0), z0 - slope * x


def make_soni(n_channels: int = 8192, len_lo: int = 512, len_hi: int = 4096, steps: int = 2000,
              seed: int = 21, n_cells: int | None = None) -> Workload:
    """Sec. 5.1-shaped aggradation runs (power law, friction, inflow-(q, h), fixed depth).

    With n_channels = 1 and n_cells given: the paper's single flume with its stated values."""
    L, beta, alpha, por = 30.0, 5.0, 1.45e-3, 0.4
    if n_channels == 1:
        n = n_cells or 100
        h0, q0, s0, ks, feed = 0.05, 0.02, 3.56e-3, 49.4, 5.0
        lens = np.array([n])
        q0v, s0v, ksv, feedv, h0v = [np.array([v]) for v in (q0, s0, ks, feed, h0)]
    else:
        ss = np.random.SeedSequence(seed)
        top = np.random.default_rng(ss.spawn(1)[0])
        lens = top.integers(len_lo, len_hi + 1, n_channels).astype(np.int64)
        q0v = top.uniform(0.015, 0.025, n_channels)
        s0v = top.uniform(3e-3, 4e-3, n_channels)
        ksv = top.uniform(45.0, 55.0, n_channels)
        feedv = top.uniform(2.0, 5.0, n_channels)
        h0v = uniform_flow_depth(q0v, ksv, s0v)
    C = lens.size
    parts = [_sloped_channel(int(lens[c]), L, h0v[c], q0v[c], s0v[c], 1.2) for c in range(C)]
    par = np.zeros((C, 4))
    par[:, 0] = beta
    return _assemble("soni", parts, L / lens, np.full(C, alpha), np.full(C, por),
                     np.full(C, BC_INFLOW_QH), np.full(C, BC_FIXED_DEPTH), steps, seed, q_in=q0v,
                     law=LAW_POWER, law_par=par, ks=ksv, h_in=h0v * feedv ** (-1.0 / beta),
                     h_out=h0v)


BELLAL_LAWS = {"mpm": LAW_MPM, "vanrijn": LAW_VANRIJN, "thr": LAW_GRASS_THR}


def make_bellal(law: str = "mpm", n_channels: int = 8192, len_lo: int = 512, len_hi: int = 4096,
                steps: int = 2000, seed: int = 22, n_cells: int | None = None) -> Workload:
    """Sec. 5.2-shaped sediment-bore runs with one of the three closures of that section.

    With n_channels = 1 and n_cells given: the paper's single flume with its stated values."""
    L, por, Sg, nu, theta_cr = 6.9, 0.42, 2.6, 1e-6, 0.03
    code = BELLAL_LAWS[law]
    if n_channels == 1:
        lens = np.array([n_cells or 200])
        q0v, s0v, d50v, ksv, houtv = [np.array([v]) for v in (0.024, 0.0302, 1.65e-3, 62.0, 0.2093)]
    else:
        ss = np.random.SeedSequence(seed)
        top = np.random.default_rng(ss.spawn(1)[0])
        lens = top.integers(len_lo, len_hi + 1, n_channels).astype(np.int64)
        q0v = top.uniform(0.02, 0.028, n_channels)
        s0v = top.uniform(0.025, 0.035, n_channels)
        d50v = top.uniform(1.2e-3, 2.0e-3, n_channels)
        ksv = top.uniform(55.0, 70.0, n_channels)
        houtv = top.uniform(0.07, 0.11, n_channels)
    C = lens.size
    h0v = uniform_flow_depth(q0v, ksv, s0v)
    parts = [_sloped_channel(int(lens[c]), L, h0v[c], q0v[c], s0v[c], s0v[c] * L) for c in range(C)]
    par = np.zeros((C, 4))
    Ag = np.zeros(C)
    if code == LAW_GRASS_THR:
        Ag[:] = 0.0024
        par[:, 0] = 0.3
    else:
        par[:, 0] = d50v
        par[:, 1] = Sg
        if code == LAW_VANRIJN:
            par[:, 2] = nu
            par[:, 3] = theta_cr
    return _assemble(f"bellal_{law}", parts, L / lens, Ag, np.full(C, por),
                     np.full(C, BC_INFLOW_QH), np.full(C, BC_FIXED_DEPTH), steps, seed, q_in=q0v,
                     law=code, law_par=par, ks=ksv, h_in=h0v, h_out=houtv)


# ---------------------------------------------------------------------------
# Smooth analytical solution of Sec. 4.2 (Test 2): steady subcritical flow over a bed eroding
# linearly in time.  alpha = beta = A_g = 0.005, C = 1, L = 7 m, t_end = 10 s are printed in
# the paper; q0 is not, and q0 = 1 m^2/s (subcritical on [0, L]) is a reading; xi = 1
# (porosity 0), which the printed bed law z(x, t) = z(x, 0) - alpha t requires.
BERTHON = {"alpha": 0.005, "beta": 0.005, "A_g": 0.005, "C": 1.0, "L": 7.0, "t_end": 10.0,
           "q0": 1.0}


def berthon_exact(x, t: float, g: float = G_ACC):
    """(h, q, z) of the analytical solution at positions x and time t."""
    a, b, Ag, C, q0 = (BERTHON[k] for k in ("alpha", "beta", "A_g", "C", "q0"))
    u = ((a * np.asarray(x, dtype=np.float64) + b) / Ag) ** (1.0 / 3.0)
    return q0 / u, np.full_like(u, q0), -(u ** 3 + 2.0 * g * q0) / (2.0 * g * u) + C - a * t


def make_berthon(n_cells: int = 300, steps: int = 0) -> Workload:
    """Test 2 on N cells: the exact solution at t = 0 as initial state, Dirichlet ghost cells
    carrying the exact solution at the ghost centres (the bed falling at the rate alpha).
    ``steps`` 0 gives an estimate of the steps to t_end (CFL 0.9 with max |u| + c)."""
    L = BERTHON["L"]
    dx = L / n_cells
    x = cell_centres(n_cells, L)
    h, q, z = berthon_exact(x, 0.0)
    gh, gq, gz = berthon_exact(np.array([-0.5 * dx, L + 0.5 * dx]), 0.0)
    rate = -BERTHON["alpha"]
    if steps <= 0:
        speed = np.max(np.abs(q / h) + np.sqrt(G_ACC * h))
        steps = int(np.ceil(BERTHON["t_end"] / (0.9 * dx / speed)))
    wl = _single("berthon", h, q, z, dx, BERTHON["A_g"], 0.0, BC_DIRICHLET, BC_DIRICHLET, 0.0,
                 steps, dir_left=np.array([[gh[0], gq[0], gz[0], rate]]),
                 dir_right=np.array([[gh[1], gq[1], gz[1], rate]]))
    wl.meta["x"] = x
    return wl


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


MAKERS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4, "c5": make_c5,
          "soni": make_soni, "bellal_mpm": lambda **kw: make_bellal("mpm", **kw),
          "bellal_vanrijn": lambda **kw: make_bellal("vanrijn", **kw),
          "bellal_thr": lambda **kw: make_bellal("thr", **kw)}

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
    "soni": "soni: 8192 overfed 30 m flumes, lengths uniform in [512, 4096], power law "
            "1.45e-3 u^5, Strickler friction, inflow-(q, h) and fixed-depth ends, per-channel "
            "q0, slope, K_s and feed, G=3, CFL 0.9, 2000 steps",
    "bellal_mpm": "bellal_mpm: 8192 steep 6.9 m flumes with a downstream depth step, lengths "
                  "uniform in [512, 4096], Meyer-Peter & Mueller, Strickler friction, per-channel "
                  "q0, slope, d50, K_s, outlet depth 0.07-0.11 m, G=3, CFL 0.9, 2000 steps",
    "bellal_vanrijn": "bellal_vanrijn: as bellal_mpm with the Van Rijn closure",
    "bellal_thr": "bellal_thr: as bellal_mpm with Grass with threshold (A_g 0.0024, u_cr 0.3)",
}
