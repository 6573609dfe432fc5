"""CPU FP64 oracle for the A-DOT scheme (ctypes binding to ``adot_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does.
It shares no code with the HIP path; inputs come from the seeded generators
in ``paper_1912_04791_amd.inputs`` (which hold none of the method's arithmetic).

Every function documents the passage of the paper it follows; the C file
holds the arithmetic.  Array conventions: states are SoA float64 arrays
``h, q, z``; fluctuations are ``[3, n]`` arrays (row r = component r).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adot_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK = 0
E_ARG = -1
E_NONFINITE = -3
E_NONHYPERBOLIC = -4

BC_TRANSMISSIVE = 0
BC_PERIODIC = 1
BC_INFLOW_Q = 2
BC_FIXED_DEPTH = 3
BC_INFLOW_QH = 4
BC_DIRICHLET = 5

LAW_GRASS = 0       # q_s = A_g u^3                                   (Sec. 2, Eq. Grass)
LAW_GRASS_THR = 1   # q_s = A_g (u - u_cr)^3, par = (u_cr,)           (Sec. 2, Eq. GrassThr)
LAW_POWER = 2       # q_s = A_g u^beta, par = (beta,)                 (Sec. 5.1)
LAW_MPM = 3         # Meyer-Peter & Mueller, par = (d50, S_g)         (Sec. 2, Eqs. MPM, Shields)
LAW_VANRIJN = 4     # Van Rijn, par = (d50, S_g, nu, theta_cr)        (Sec. 2, Eqs. vanRijn, u_star)

_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c99",
           "-Wall", "-Wextra", "-pthread"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = f"{_LIB_PATH}.{os.getpid()}.tmp"
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Channel(ctypes.Structure):
    """One channel of the scheme (mirrors ``or_channel`` in the C file)."""
    _fields_ = [
        ("n_cells", ctypes.c_int64),
        ("g", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("Ag", ctypes.c_double),
        ("n_gauss", ctypes.c_int),
        ("cfl", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("bc_left", ctypes.c_int),
        ("bc_right", ctypes.c_int),
        ("q_in", ctypes.c_double),
        ("h_out", ctypes.c_double),
        ("h_in", ctypes.c_double),
        ("dir_l", ctypes.c_double * 4),
        ("dir_r", ctypes.c_double * 4),
        ("law", ctypes.c_int),
        ("par", ctypes.c_double * 4),
        ("ks", ctypes.c_double),
    ]


class Phys(ctypes.Structure):
    """Physical parameters (mirrors ``or_phys``): g, xi, A_g, closure law and its parameters,
    Strickler coefficient of the friction slope (0 = no friction)."""
    _fields_ = [("g", ctypes.c_double), ("xi", ctypes.c_double), ("Ag", ctypes.c_double),
                ("law", ctypes.c_int), ("par", ctypes.c_double * 4), ("ks", ctypes.c_double)]


def make_phys(g: float, xi: float, Ag: float, law: int = LAW_GRASS, par=(), ks: float = 0.0) -> Phys:
    pr = list(par) + [0.0] * (4 - len(par))
    return Phys(g, xi, Ag, law, (ctypes.c_double * 4)(*pr), ks)


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def _load(lib_path: str | None = None):
    global _lib
    if _lib is not None and lib_path is None:
        return _lib
    path = lib_path or _LIB_PATH
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(path)
    lib.or_gauss.argtypes = [ctypes.c_int, _dp, _dp]
    _pp = ctypes.POINTER(Phys)
    lib.or_eig_batch.argtypes = [_i64, _dp, _dp, _dp, _pp, _dp, _dp, _dp, _dp, _dp]
    lib.or_fluct_batch.argtypes = [_i64, _dp, _dp, _dp, _dp, _dp, _dp, _pp, ctypes.c_int, _dp, _dp,
                                   ctypes.c_int]
    lib.or_cfl_amax.argtypes = [_i64, _dp, _dp, _dp, _pp, _dp, ctypes.c_int]
    lib.or_step.argtypes = [_i64, _dp, _dp, _dp, _dp, _dp, _pp, ctypes.c_int, ctypes.c_double,
                            ctypes.c_double, _dp, _dp, _dp, ctypes.c_int]
    lib.or_run.argtypes = [ctypes.POINTER(Channel), _dp, _dp, _dp, ctypes.c_int, _dp, _dp,
                           ctypes.c_int]
    lib.or_run_batched.argtypes = [_i64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(Channel),
                                   _dp, _dp, _dp, ctypes.c_int, _dp, ctypes.c_int]
    lib.or_channel_size.restype = ctypes.c_int
    lib.or_phys_size.restype = ctypes.c_int
    assert lib.or_channel_size() == ctypes.sizeof(Channel), "or_channel layout mismatch"
    assert lib.or_phys_size() == ctypes.sizeof(Phys), "or_phys layout mismatch"
    if lib_path is None:
        _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


# --------------------------------------------------------------------------
def gauss(G: int, lib=None):
    """Gauss-Legendre nodes and weights on [0, 1] (Sec. 3.1, Eq. DOTjumpN); weights sum to 1."""
    lib = lib or _load()
    s = np.zeros(G)
    w = np.zeros(G)
    st = lib.or_gauss(G, _ptr(s), _ptr(w))
    if st != OK:
        raise OracleError(st, "gauss")
    return s, w


def eigensystem(h, q, z, g: float, xi: float, Ag: float, lib=None, check: bool = True,
                law: int = LAW_GRASS, par=(), ks: float = 0.0):
    """Closed-form eigenstructure at each state (Sec. 3.3 steps 1-5).

    Returns dict with ``lam`` [n,3] (lambda_1 <= lambda_2 <= lambda_3), ``R`` [n,3,3]
    (right eigenvectors as columns, Eq. RR), ``Rinv`` [n,3,3] (left eigenvectors as rows,
    Eq. RR-1), ``A`` [n,3,3] (Eq. W&A_definition) and ``absA`` [n,3,3] (Eq. ExAbsA).
    """
    lib = lib or _load()
    h, q, z = _f64(h).ravel(), _f64(q).ravel(), _f64(z).ravel()
    n = h.size
    lam = np.zeros((n, 3))
    R = np.zeros((n, 3, 3))
    Rinv = np.zeros((n, 3, 3))
    A = np.zeros((n, 3, 3))
    absA = np.zeros((n, 3, 3))
    ph = make_phys(g, xi, Ag, law, par, ks)
    st = lib.or_eig_batch(n, _ptr(h), _ptr(q), _ptr(z), ctypes.byref(ph), _ptr(lam), _ptr(R),
                          _ptr(Rinv), _ptr(A), _ptr(absA))
    if check and st != OK:
        raise OracleError(st, "eigensystem")
    return {"lam": lam, "R": R, "Rinv": Rinv, "A": A, "absA": absA, "status": st}


def fluct(WL, WR, g: float, xi: float, Ag: float, G: int = 3, nthreads: int | None = None,
          lib=None, check: bool = True, law: int = LAW_GRASS, par=(), ks: float = 0.0):
    """DOT fluctuations for n independent edges (Sec. 3.1, Eq. DOTjumpN).

    ``WL``/``WR`` are (h, q, z) tuples of length-n arrays (left / right states).
    Returns ``(Dm, Dp)`` as [3, n] arrays.
    """
    lib = lib or _load()
    hL, qL, zL = (_f64(a).ravel() for a in WL)
    hR, qR, zR = (_f64(a).ravel() for a in WR)
    n = hL.size
    Dm = np.zeros((3, n))
    Dp = np.zeros((3, n))
    ph = make_phys(g, xi, Ag, law, par, ks)
    st = lib.or_fluct_batch(n, _ptr(hL), _ptr(qL), _ptr(zL), _ptr(hR), _ptr(qR), _ptr(zR),
                            ctypes.byref(ph), G, _ptr(Dm), _ptr(Dp), nthreads or default_threads())
    if check and st != OK:
        raise OracleError(st, "fluct")
    return Dm, Dp


def cfl_amax(h, q, z, g: float, xi: float, Ag: float, nthreads: int | None = None, lib=None,
             law: int = LAW_GRASS, par=(), ks: float = 0.0):
    """max over cells of max_m |lambda_m(W_i)| (the CFL reduction)."""
    lib = lib or _load()
    h, q, z = _f64(h).ravel(), _f64(q).ravel(), _f64(z).ravel()
    out = ctypes.c_double(0.0)
    ph = make_phys(g, xi, Ag, law, par, ks)
    st = lib.or_cfl_amax(h.size, _ptr(h), _ptr(q), _ptr(z), ctypes.byref(ph), ctypes.byref(out),
                         nthreads or default_threads())
    if st != OK:
        raise OracleError(st, "cfl_amax")
    return out.value


def step(h, q, z, ghost_l, ghost_r, g: float, xi: float, Ag: float, G: int, dt: float, dx: float,
         nthreads: int | None = None, lib=None, law: int = LAW_GRASS, par=(), ks: float = 0.0):
    """One path-conservative update (Sec. 3, Eq. scheme; friction point source if ks > 0)
    with given ghosts and dt."""
    lib = lib or _load()
    h, q, z = _f64(h).ravel(), _f64(q).ravel(), _f64(z).ravel()
    gl, gr = _f64(ghost_l), _f64(ghost_r)
    hn, qn, zn = np.zeros_like(h), np.zeros_like(q), np.zeros_like(z)
    ph = make_phys(g, xi, Ag, law, par, ks)
    st = lib.or_step(h.size, _ptr(h), _ptr(q), _ptr(z), _ptr(gl), _ptr(gr), ctypes.byref(ph), G, dt,
                     dx, _ptr(hn), _ptr(qn), _ptr(zn), nthreads or default_threads())
    if st != OK:
        raise OracleError(st, "step")
    return hn, qn, zn


@dataclass
class ChannelSpec:
    """Parameters of one channel; ``porosity`` p gives xi = 1/(1-p) (Sec. 2)."""
    n_cells: int
    dx: float
    Ag: float
    porosity: float = 0.4
    g: float = 9.81
    n_gauss: int = 3
    cfl: float = 0.9
    bc_left: int = BC_TRANSMISSIVE
    bc_right: int = BC_TRANSMISSIVE
    q_in: float = 0.0
    h_out: float = 0.0
    h_in: float = 0.0
    dir_left: tuple = (0.0, 0.0, 0.0, 0.0)    # Dirichlet ghost (h, q, z at t = 0, dz/dt)
    dir_right: tuple = (0.0, 0.0, 0.0, 0.0)
    law: int = LAW_GRASS
    par: tuple = ()
    ks: float = 0.0

    def to_c(self) -> Channel:
        pr = list(self.par) + [0.0] * (4 - len(self.par))
        return Channel(self.n_cells, self.g, 1.0 / (1.0 - self.porosity), self.Ag, self.n_gauss,
                       self.cfl, self.dx, self.bc_left, self.bc_right, self.q_in, self.h_out,
                       self.h_in, (ctypes.c_double * 4)(*self.dir_left),
                       (ctypes.c_double * 4)(*self.dir_right), self.law, (ctypes.c_double * 4)(*pr), self.ks)


def run(spec: ChannelSpec, h, q, z, n_steps: int, t0: float = 0.0, nthreads: int | None = None,
        lib=None, return_dt: bool = False):
    """Time loop of one channel: ghosts, CFL dt, update; returns (h, q, z, t[, dts])."""
    lib = lib or _load()
    h, q, z = _f64(h).copy(), _f64(q).copy(), _f64(z).copy()
    assert h.size == spec.n_cells
    t = ctypes.c_double(t0)
    dts = np.zeros(max(n_steps, 1))
    ch = spec.to_c()
    st = lib.or_run(ctypes.byref(ch), _ptr(h), _ptr(q), _ptr(z), n_steps, ctypes.byref(t), _ptr(dts),
                    nthreads or default_threads())
    if st != OK:
        raise OracleError(st, "run")
    if return_dt:
        return h, q, z, t.value, dts[:n_steps]
    return h, q, z, t.value


def run_batched(specs, offsets, h, q, z, n_steps: int, t0=None, nthreads: int | None = None,
                lib=None):
    """Many independent channels, each with its own dt (channels over threads)."""
    lib = lib or _load()
    h, q, z = _f64(h).copy(), _f64(q).copy(), _f64(z).copy()
    C = len(specs)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    assert off.size == C + 1 and off[-1] == h.size
    chs = (Channel * C)(*[s.to_c() for s in specs])
    t = _f64(np.zeros(C) if t0 is None else t0).copy()
    st = lib.or_run_batched(C, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), chs, _ptr(h),
                            _ptr(q), _ptr(z), n_steps, _ptr(t), nthreads or default_threads())
    if st != OK:
        raise OracleError(st, "run_batched")
    return h, q, z, t
