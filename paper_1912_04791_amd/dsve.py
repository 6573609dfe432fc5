"""ctypes binding to libdsve.so (the C ABI of include/dsve.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch provides device memory (float64 CUDA tensors) and the
stream; nothing here computes any part of the scheme.  If the library is not
built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DSVE_LIBRARY") or os.path.join(_HERE, "libdsve.so")

OK = 0
E_ARG = -1
E_HIP = -2
E_NONFINITE = -3
E_NONHYPERBOLIC = -4
E_UNSUPPORTED = -5

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
FP64 = 0
MIXED = 1
PRECISIONS = {"fp64": FP64, "mixed": MIXED}
SOLVER_ADOT = 0
SOLVER_DOT = 1

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1912_04791_amd.build` "
        "(there is no fallback path)")


class Params(ctypes.Structure):
    """Mirror of ``dsve_params``."""
    _fields_ = [
        ("g", ctypes.c_double),
        ("porosity", ctypes.c_double),
        ("law", ctypes.c_int),
        ("A_g", ctypes.c_double),
        ("law_extra", ctypes.c_double * 4),
        ("n_gauss", ctypes.c_int),
        ("cfl", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("bc_left", ctypes.c_int),
        ("bc_right", ctypes.c_int),
        ("q_in", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("h_in", ctypes.c_double),
        ("h_out", ctypes.c_double),
        ("ks", ctypes.c_double),
        ("dir_left", ctypes.c_double * 4),
        ("dir_right", ctypes.c_double * 4),
        ("solver", ctypes.c_int),
    ]


class Channel(ctypes.Structure):
    """Mirror of ``dsve_channel``."""
    _fields_ = [
        ("A_g", ctypes.c_double),
        ("porosity", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("q_in", ctypes.c_double),
        ("h_in", ctypes.c_double),
        ("h_out", ctypes.c_double),
        ("ks", ctypes.c_double),
        ("law_extra", ctypes.c_double * 4),
        ("dir_left", ctypes.c_double * 4),
        ("dir_right", ctypes.c_double * 4),
        ("bc_left", ctypes.c_int),
        ("bc_right", ctypes.c_int),
    ]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_ctxp = ctypes.c_void_p

# PyTorch brings its own HIP runtime.  It is loaded first so that the library binds to that
# same runtime: loaded before it, the library would pull in the system runtime beside torch's,
# and the streams and memory that torch hands over would be unknown to the runtime the library
# calls (dsve_init then fails on the stream).
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)
lib.dsve_abi_version.restype = ctypes.c_int
lib.dsve_init.argtypes = [ctypes.POINTER(_ctxp), ctypes.POINTER(Params), _i64, _vp]
lib.dsve_batch_init.argtypes = [ctypes.POINTER(_ctxp), _i64, _vp, ctypes.POINTER(Channel),
                                ctypes.POINTER(Params), _vp]
lib.dsve_destroy.argtypes = [_ctxp]
lib.dot_edge_fluct.argtypes = [_ctxp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp]
lib.cell_update.argtypes = [_ctxp, _vp, _vp, _vp, _vp, _vp, _vp]
lib.cfl_reduce.argtypes = [_ctxp, _vp, _vp, _vp, _vp, _vp]
lib.adot_step.argtypes = [_ctxp, _vp, _vp, _vp, ctypes.c_int, _vp]
lib.adot_step_batched.argtypes = [_ctxp, _vp, _vp, _vp, ctypes.c_int, _vp]
lib.dsve_sync.argtypes = [_ctxp]
lib.dsve_last_error.argtypes = [_ctxp]
lib.dsve_last_error.restype = ctypes.c_char_p
lib.dsve_clear_error.argtypes = [_ctxp]
lib.dsve_set_launch.argtypes = [_ctxp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
lib.dsve_get_launch.argtypes = [_ctxp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]
lib.dsve_autotune.argtypes = [_ctxp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_char_p]
lib.dsve_set_cfl_split.argtypes = [_ctxp, ctypes.c_int]
lib.dsve_get_cfl_split.argtypes = [_ctxp, ctypes.POINTER(ctypes.c_int)]
lib.dsve_set_resident.argtypes = [_ctxp, ctypes.c_int]
lib.dsve_get_resident.argtypes = [_ctxp, ctypes.POINTER(ctypes.c_int)]
lib.dsve_device_cus.argtypes = [_ctxp]
lib.dsve_device_cus.restype = ctypes.c_int
lib.dsve_prepare_run.argtypes = [_ctxp, _vp, _vp, _vp, ctypes.c_int, _vp]
lib.adot_step_noalloc.argtypes = [_ctxp, _vp, _vp, _vp, ctypes.c_int, _vp]
lib.dsve_get_last_run.argtypes = [_ctxp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int)]
assert lib.dsve_abi_version() == 5, "libdsve ABI version mismatch"

ENTRY_POINTS = ("dsve_abi_version", "dsve_init", "dsve_batch_init", "dsve_destroy",
                "dot_edge_fluct", "cell_update", "cfl_reduce", "adot_step", "adot_step_batched",
                "dsve_sync", "dsve_last_error", "dsve_clear_error", "dsve_set_launch",
                "dsve_get_launch", "dsve_set_cfl_split", "dsve_get_cfl_split", "dsve_set_resident",
                "dsve_get_resident", "dsve_autotune", "dsve_device_cus", "dsve_prepare_run",
                "dsve_get_last_run", "adot_step_noalloc")


class DsveError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dsve status {status}: {msg}")
        self.status = status


def _ptr(t, numel: int | None = None, at_least: int | None = None, device: int | None = None) -> int:
    """Device pointer of a contiguous float64 CUDA tensor, after checking its element count
    (exactly ``numel``, or at least ``at_least``) and its device: the library takes raw
    pointers and trusts the sizes it was given."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    if at_least is not None and t.numel() < at_least:
        raise ValueError(f"expected at least {at_least} elements, got {t.numel()}")
    if device is not None and t.device.index != device:
        raise ValueError(f"tensor on cuda:{t.device.index}, context on cuda:{device}")
    return t.data_ptr()


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_params(g=9.81, porosity=0.4, A_g=0.01, n_gauss=3, cfl=0.9, dx=1.0,
                bc_left=BC_TRANSMISSIVE, bc_right=BC_TRANSMISSIVE, q_in=0.0,
                precision="fp64", law=LAW_GRASS, law_extra=(), h_in=0.0, h_out=0.0,
                ks=0.0, dir_left=(0.0, 0.0, 0.0, 0.0), dir_right=(0.0, 0.0, 0.0, 0.0),
                solver=SOLVER_ADOT) -> Params:
    """``precision`` "fp64" | "mixed" (or the code); ``solver`` SOLVER_ADOT | SOLVER_DOT
    (or "adot" | "dot")."""
    p = Params()
    p.g = g
    p.porosity = porosity
    p.law = int(law)
    p.A_g = A_g
    ex = list(law_extra) + [0.0] * (4 - len(law_extra))
    for k in range(4):
        p.law_extra[k] = float(ex[k])
    p.n_gauss = n_gauss
    p.cfl = cfl
    p.dx = dx
    p.bc_left = bc_left
    p.bc_right = bc_right
    p.q_in = q_in
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.h_in = h_in
    p.h_out = h_out
    p.ks = ks
    for k in range(4):
        p.dir_left[k] = float(dir_left[k])
        p.dir_right[k] = float(dir_right[k])
    p.solver = {"adot": SOLVER_ADOT, "dot": SOLVER_DOT}[solver] if isinstance(solver, str) else int(solver)
    return p


def make_channels(A_g, porosity, dx, bc_left, bc_right, q_in=None, h_in=None, h_out=None,
                  ks=None, law_extra=None, dir_left=None, dir_right=None):
    """A ``dsve_channel`` array from per-channel arrays (missing ones are zero)."""
    C = len(A_g)
    z = np.zeros(C)
    cols = [np.asarray(a if a is not None else z, dtype=np.float64)
            for a in (A_g, porosity, dx, q_in, h_in, h_out, ks)]
    four = lambda a: np.zeros((C, 4)) if a is None else np.asarray(a, dtype=np.float64).reshape(C, 4)
    ex, dl, dr = four(law_extra), four(dir_left), four(dir_right)
    bcl = np.asarray(bc_left, dtype=np.int32)
    bcr = np.asarray(bc_right, dtype=np.int32)
    for a in (*cols, bcl, bcr):
        assert a.shape[0] == C
    arr = (Channel * C)()
    for c in range(C):
        ch = arr[c]
        ch.A_g, ch.porosity, ch.dx, ch.q_in, ch.h_in, ch.h_out, ch.ks = (float(a[c]) for a in cols)
        for k in range(4):
            ch.law_extra[k] = float(ex[c, k])
            ch.dir_left[k] = float(dl[c, k])
            ch.dir_right[k] = float(dr[c, k])
        ch.bc_left = int(bcl[c])
        ch.bc_right = int(bcr[c])
    return arr


class Context:
    """One libdsve context (single channel or batched).  Methods map 1:1 to entry points."""

    def __init__(self, handle, n_cells: int, n_channels: int, batched: bool):
        import torch
        self._h = handle
        self.n_cells = n_cells
        self.n_channels = n_channels
        self.batched = batched
        self.device = torch.cuda.current_device()   # the device the library bound it to

    def _state(self, h, q, z):
        n, d = self.n_cells, self.device
        return _ptr(h, n, device=d), _ptr(q, n, device=d), _ptr(z, n, device=d)

    # -- construction -----------------------------------------------------
    @classmethod
    def single(cls, n_cells: int, stream=None, **params) -> "Context":
        p = make_params(**params)
        h = _ctxp()
        st = lib.dsve_init(ctypes.byref(h), ctypes.byref(p), int(n_cells), _stream_handle(stream))
        if st != OK:
            raise DsveError(st, "dsve_init failed")
        return cls(h, int(n_cells), 1, False)

    @classmethod
    def batch(cls, offsets, A_g, porosity, dx, bc_left, bc_right, q_in=None, stream=None,
              h_in=None, h_out=None, ks=None, law_extra=None, dir_left=None, dir_right=None,
              **common) -> "Context":
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        C = off.size - 1
        chans = make_channels(A_g, porosity, dx, bc_left, bc_right, q_in, h_in, h_out, ks,
                              law_extra, dir_left, dir_right)
        assert len(chans) == C
        p = make_params(**common)
        h = _ctxp()
        st = lib.dsve_batch_init(ctypes.byref(h), C, off.ctypes.data, chans, ctypes.byref(p),
                                 _stream_handle(stream))
        if st != OK:
            raise DsveError(st, "dsve_batch_init failed")
        return cls(h, int(off[-1]), C, True)

    @classmethod
    def from_workload(cls, wl, precision=None, stream=None, solver="adot") -> "Context":
        """Context for an ``inputs.Workload`` (single channel when it has one channel)."""
        prec = precision or wl.precision
        if wl.n_channels == 1:
            return cls.single(wl.n_cells, stream=stream, g=wl.g, porosity=float(wl.porosity[0]),
                              A_g=float(wl.Ag[0]), n_gauss=wl.n_gauss, cfl=wl.cfl,
                              dx=float(wl.dx[0]), bc_left=int(wl.bc_left[0]),
                              bc_right=int(wl.bc_right[0]), q_in=float(wl.q_in[0]),
                              precision=prec, law=wl.law, law_extra=tuple(wl.law_par[0]),
                              h_in=float(wl.h_in[0]), h_out=float(wl.h_out[0]),
                              ks=float(wl.ks[0]), dir_left=tuple(wl.dir_left[0]),
                              dir_right=tuple(wl.dir_right[0]), solver=solver)
        return cls.batch(wl.offsets, wl.Ag, wl.porosity, wl.dx, wl.bc_left, wl.bc_right, wl.q_in,
                         stream=stream, h_in=wl.h_in, h_out=wl.h_out, ks=wl.ks,
                         law_extra=wl.law_par, dir_left=wl.dir_left, dir_right=wl.dir_right,
                         g=wl.g, n_gauss=wl.n_gauss, cfl=wl.cfl, precision=prec, law=wl.law,
                         solver=solver)

    # -- helpers ----------------------------------------------------------
    def _check(self, st: int, what: str):
        if st != OK:
            msg = lib.dsve_last_error(self._h)
            raise DsveError(st, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if self._h:
            lib.dsve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points -----------------------------------------------------
    def dot_edge_fluct(self, hL, qL, zL, hR, qR, zR, Dm, Dp):
        """n edges: six states of n elements each; Dm, Dp hold [3][n]."""
        n, d = hL.numel(), self.device
        ins = [_ptr(x, n, device=d) for x in (hL, qL, zL, hR, qR, zR)]
        self._check(lib.dot_edge_fluct(self._h, *ins, n, _ptr(Dm, 3 * n, device=d),
                                       _ptr(Dp, 3 * n, device=d)), "dot_edge_fluct")

    def cell_update(self, Dm, Dp, dt, h, q, z):
        """Dm, Dp hold [3][N+1] edge fluctuations of an N-cell channel; dt one value."""
        e, d = 3 * (self.n_cells + 1), self.device
        self._check(lib.cell_update(self._h, _ptr(Dm, e, device=d), _ptr(Dp, e, device=d),
                                    _ptr(dt, at_least=1, device=d), *self._state(h, q, z)),
                    "cell_update")

    def cfl_reduce(self, h, q, z, amax, dt):
        d = self.device
        self._check(lib.cfl_reduce(self._h, *self._state(h, q, z), _ptr(amax, at_least=1, device=d),
                                   _ptr(dt, at_least=1, device=d)), "cfl_reduce")

    def adot_step(self, h, q, z, n_steps: int, t):
        """n_steps steps in place; t holds one clock per channel."""
        fn = lib.adot_step_batched if self.batched else lib.adot_step
        self._check(fn(self._h, *self._state(h, q, z), int(n_steps),
                       _ptr(t, self.n_channels, device=self.device)), "adot_step")

    def adot_step_noalloc(self, h, q, z, n_steps: int, t):
        """adot_step without allocation (static device scratch; at most 2^20 cells, 4096 channels)."""
        self._check(lib.adot_step_noalloc(self._h, *self._state(h, q, z), int(n_steps),
                                          _ptr(t, self.n_channels, device=self.device)),
                    "adot_step_noalloc")

    def prepare_run(self, h, q, z, n_steps: int, t):
        """Capture the graphs a run of n_steps on these tensors replays (no work enqueued)."""
        self._check(lib.dsve_prepare_run(self._h, *self._state(h, q, z), int(n_steps),
                                         _ptr(t, self.n_channels, device=self.device)),
                    "dsve_prepare_run")

    def last_run(self):
        """(graph replays, steps they ran, kernels launched directly) of the last run."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(lib.dsve_get_last_run(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
                    "dsve_get_last_run")
        return a.value, b.value, c.value

    def sync(self):
        self._check(lib.dsve_sync(self._h), "dsve_sync")

    def sync_status(self) -> int:
        return lib.dsve_sync(self._h)

    def last_error(self) -> str:
        m = lib.dsve_last_error(self._h)
        return m.decode() if m else ""

    def clear_error(self):
        self._check(lib.dsve_clear_error(self._h), "dsve_clear_error")

    def set_launch(self, tile: int = 256, blocks_per_cu: int = 0, graph_steps: int = 60):
        self._check(lib.dsve_set_launch(self._h, tile, blocks_per_cu, graph_steps), "dsve_set_launch")

    def get_launch(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(lib.dsve_get_launch(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
                    "dsve_get_launch")
        return a.value, b.value, c.value

    def set_cfl_split(self, split: int):
        """CFL sub-slots per channel (1, 2 or 4; 0 = chosen from the launch shape)."""
        self._check(lib.dsve_set_cfl_split(self._h, split), "dsve_set_cfl_split")

    def get_cfl_split(self) -> int:
        v = ctypes.c_int()
        self._check(lib.dsve_get_cfl_split(self._h, ctypes.byref(v)), "dsve_get_cfl_split")
        return v.value

    def set_resident(self, mode: int):
        """0: channel-resident runs when every channel has at most 511 cells; 1: never."""
        self._check(lib.dsve_set_resident(self._h, mode), "dsve_set_resident")

    def get_resident(self) -> bool:
        v = ctypes.c_int()
        self._check(lib.dsve_get_resident(self._h, ctypes.byref(v)), "dsve_get_resident")
        return bool(v.value)

    def autotune(self, h, q, z, trial_steps: int = 10, cache_path: str | None = None):
        cp = cache_path.encode() if cache_path else None
        self._check(lib.dsve_autotune(self._h, *self._state(h, q, z), trial_steps, cp),
                    "dsve_autotune")

    def device_cus(self) -> int:
        return lib.dsve_device_cus(self._h)


def upload(wl, device="cuda"):
    """Device float64 copies of a workload's state and a zeroed clock per channel."""
    import torch
    h = torch.from_numpy(np.ascontiguousarray(wl.h)).to(device)
    q = torch.from_numpy(np.ascontiguousarray(wl.q)).to(device)
    z = torch.from_numpy(np.ascontiguousarray(wl.z)).to(device)
    t = torch.zeros(wl.n_channels, dtype=torch.float64, device=device)
    return h, q, z, t
