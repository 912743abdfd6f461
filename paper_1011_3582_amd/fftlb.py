"""Python binding of libfftlb.so (ctypes).  Argument marshalling only: every step of the
solver runs in the HIP kernels of the library; PyTorch provides device memory and streams.

Importing this module loads the library and raises if it is not built or not loadable;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import re

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfftlb.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "fftlb.h")

FFTLB_OK, FFTLB_EINVAL, FFTLB_ENOSPC, FFTLB_EHIP, FFTLB_EUNSTABLE = 0, -1, -2, -3, -4
Q = 33
NGLOBALS = 8
GLOBAL_NAMES = ("mass", "px", "py", "energy", "residual", "umax", "nonfinite", "steps")


class FFTLBError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = _lib.fftlb_strerror(code).decode() if _lib is not None else str(code)
        detail = _lib.fftlb_last_error().decode() if (_lib is not None and code == FFTLB_EHIP) else ""
        super().__init__(f"{what}: {msg} ({code}){' - ' + detail if detail else ''}")


class Config(ctypes.Structure):
    """Mirror of struct fftlb_config in include/fftlb.h."""
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
                ("tau", ctypes.c_double), ("K", ctypes.c_double), ("H", ctypes.c_double),
                ("zeta", ctypes.c_double), ("q", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("filter_order", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("convection", ctypes.c_int32)]


# convection schemes (fftlb_config.convection)
CONV_SPECTRAL, CONV_LW, CONV_MLW1, CONV_MLW2, CONV_FL = 0, 1, 2, 3, 4


class Plan(ctypes.Structure):
    """Mirror of struct fftlb_plan: column-pass tile widths and radices."""
    _fields_ = [("conv_cols", ctypes.c_int32), ("multi_cols", ctypes.c_int32), ("conv_radix", ctypes.c_int32),
                ("multi_radix", ctypes.c_int32)]

    def as_tuple(self):
        return (self.conv_cols, self.multi_cols, self.conv_radix, self.multi_radix)


@dataclasses.dataclass
class Params:
    """Model parameters; defaults are the paper's (Sec. 3.5 list, k4 window) with the
    van der Waals constants of the benchmark fluid (a = 2, b = 0.4)."""
    dx: float = 1.0 / 256.0
    dy: float = 1.0 / 256.0
    dt: float = 1e-5
    tau: float = 1e-2
    K: float = 1e-5
    H: float = 0.0
    zeta: float = 0.0
    q: float = -0.004
    a: float = 2.0
    b: float = 0.4
    m: int = 4
    precision: int = 0   # 0: f stored in FP32; 1: compensated hi + lo (see fftlb_config)
    convection: int = 0  # CONV_SPECTRAL, or the finite-difference scheme CONV_LW / CONV_MLW1 / CONV_MLW2 / CONV_FL

    def config(self, nx: int, ny: int) -> Config:
        return Config(nx, ny, self.dx, self.dy, self.dt, self.tau, self.K, self.H, self.zeta, self.q,
                      self.a, self.b, self.m, self.precision, self.convection)


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1011_3582_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    cfgp = ctypes.POINTER(Config)
    planp = ctypes.POINTER(Plan)
    fpp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "fftlb_get_plan": (ctypes.c_int, [vp, planp]),
        "fftlb_set_plan": (ctypes.c_int, [vp, planp]),
        "fftlb_autotune": (ctypes.c_int, [vp, i32, ctypes.c_char_p, vp, planp]),
        "fftlb_batch_workspace_bytes": (ctypes.c_int, [i32, cfgp, ctypes.POINTER(sz)]),
        "fftlb_batch_create": (ctypes.c_int, [i32, cfgp, vp, sz, fpp, fpp, fpp, fpp, vp, ctypes.POINTER(vp)]),
        "fftlb_batch_autotune": (ctypes.c_int, [vp, i32, ctypes.c_char_p, vp]),
        "fftlb_batch_run": (ctypes.c_int, [vp, ctypes.c_double, i32, i32, i64, vp]),
        "fftlb_batch_status": (ctypes.c_int, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]),
        "fftlb_batch_instance": (ctypes.c_int, [vp, i32, ctypes.POINTER(vp)]),
        "fftlb_batch_destroy": (ctypes.c_int, [vp]),
        "fftlb_workspace_bytes": (ctypes.c_int, [cfgp, ctypes.POINTER(sz)]),
        "fftlb_init": (ctypes.c_int, [cfgp, vp, sz, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]),
        "fftlb_step": (ctypes.c_int, [vp, i64, vp]),
        "fftlb_moments": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "fftlb_poll": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), vp]),
        "fftlb_match_energy": (ctypes.c_int, [vp, ctypes.c_double, vp]),
        "fftlb_get_state": (ctypes.c_int, [vp, vp, vp]),
        "fftlb_set_state": (ctypes.c_int, [vp, vp, vp]),
        "fftlb_derivative": (ctypes.c_int, [vp, vp, vp, i32, vp]),
        "fftlb_derivative_static": (ctypes.c_int, [cfgp, vp, vp, i32, vp]),
        "fftlb_run_stage": (ctypes.c_int, [vp, i32, i32, vp]),
        "fftlb_destroy": (ctypes.c_int, [vp]),
        "fftlb_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "fftlb_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def library():
    return _lib


def header_functions(paths=None):
    """Names of the functions declared in the library's headers (include/*.h)."""
    import glob
    names = set()
    for path in paths or sorted(glob.glob(os.path.join(os.path.dirname(HEADER_PATH), "*.h"))):
        txt = open(path).read()
        names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fftlb_\w+)\s*\(", txt, re.M))
    return sorted(names)


def _check(rc: int, what: str):
    if rc != FFTLB_OK:
        raise FFTLBError(rc, what)


def workspace_bytes(nx: int, ny: int, params: Params | None = None) -> int:
    cfg = (params or Params()).config(nx, ny)
    out = ctypes.c_size_t()
    _check(_lib.fftlb_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)), "fftlb_workspace_bytes")
    return out.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _field(x, ny, nx, device):
    t = torch.as_tensor(x, dtype=torch.float32, device=device)
    if t.shape != (ny, nx):
        raise ValueError(f"field shape {tuple(t.shape)} != {(ny, nx)}")
    return t.contiguous()


class Solver:
    """One FFT-LB simulation on one GPU.

    rho0, ux0, uy0, T0: [ny, nx] arrays or tensors (copied to the device as float32).
    The distribution starts at the local equilibrium f^eq(rho0, u0, T0).
    """

    def __init__(self, rho0, ux0, uy0, T0, params: Params | None = None, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the FFT-LB solver runs only through its HIP library")
        self.params = params or Params()
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        rho0 = torch.as_tensor(rho0)
        self.ny, self.nx = int(rho0.shape[0]), int(rho0.shape[1])
        self.cfg = self.params.config(self.nx, self.ny)
        with torch.cuda.device(self.device):
            nbytes = workspace_bytes(self.nx, self.ny, self.params)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            fields = [_field(a, self.ny, self.nx, self.device) for a in (rho0, ux0, uy0, T0)]
            h = ctypes.c_void_p()
            rc = _lib.fftlb_init(ctypes.byref(self.cfg), _ptr(self.workspace), nbytes, *(_ptr(f) for f in fields),
                                 _stream(self.device), ctypes.byref(h))
            _check(rc, "fftlb_init")
        self._h = h
        self._owned = True

    @classmethod
    def _view(cls, handle, nx, ny, params, device, owner):
        """A Solver over a handle owned by a Batch (closing it does not destroy the handle)."""
        v = cls.__new__(cls)
        v.params, v.device, v.nx, v.ny = params, device, nx, ny
        v.cfg = params.config(nx, ny)
        v._h, v._owned, v._owner = handle, False, owner
        return v

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("solver is closed")
        return self._h

    def step(self, nsteps: int = 1):
        with torch.cuda.device(self.device):
            _check(_lib.fftlb_step(self.handle, int(nsteps), _stream(self.device)), "fftlb_step")

    def moments(self, globals_: bool = True):
        """Returns (rho, ux, uy, T) float32 device tensors and a dict of FP64 globals (None
        without globals_).  The globals come from fftlb_poll, which synchronises and returns
        FFTLB_EUNSTABLE for a non-finite state (raised here as FFTLBError)."""
        with torch.cuda.device(self.device):
            outs = [torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device) for _ in range(4)]
            _check(_lib.fftlb_moments(self.handle, *(_ptr(o) for o in outs), None, _stream(self.device)),
                   "fftlb_moments")
            glob = self.poll() if globals_ else None
        return outs, glob

    def poll(self):
        """FP64 globals of the current state as a dict (fftlb_poll: synchronising; raises
        FFTLBError with code FFTLB_EUNSTABLE if the state holds non-finite values)."""
        g = (ctypes.c_double * NGLOBALS)()
        with torch.cuda.device(self.device):
            _check(_lib.fftlb_poll(self.handle, g, _stream(self.device)), "fftlb_poll")
        return dict(zip(GLOBAL_NAMES, g[:]))

    def globals_tensor(self, out):
        """Enqueue the FP64 globals into a device float64[8] tensor (no host sync)."""
        with torch.cuda.device(self.device):
            _check(_lib.fftlb_moments(self.handle, None, None, None, None, _ptr(out), _stream(self.device)),
                   "fftlb_moments")

    def match_energy(self, energy: float):
        """fftlb_match_energy: shift T uniformly so that the state's total energy (Eq. (17))
        equals `energy`, and restart from the local equilibrium."""
        with torch.cuda.device(self.device):
            _check(_lib.fftlb_match_energy(self.handle, float(energy), _stream(self.device)), "fftlb_match_energy")

    def run_stage(self, stage: int, reps: int = 1):
        """Enqueue `reps` launches of one kernel of the step (see fftlb_run_stage)."""
        with torch.cuda.device(self.device):
            _check(_lib.fftlb_run_stage(self.handle, int(stage), int(reps), _stream(self.device)), "fftlb_run_stage")

    def get_state(self):
        with torch.cuda.device(self.device):
            f = torch.empty((Q, self.ny, self.nx), dtype=torch.float32, device=self.device)
            _check(_lib.fftlb_get_state(self.handle, _ptr(f), _stream(self.device)), "fftlb_get_state")
        return f

    def set_state(self, f):
        with torch.cuda.device(self.device):
            t = torch.as_tensor(f, dtype=torch.float32, device=self.device).contiguous()
            if t.shape != (Q, self.ny, self.nx):
                raise ValueError("state shape must be [33, ny, nx]")
            _check(_lib.fftlb_set_state(self.handle, _ptr(t), _stream(self.device)), "fftlb_set_state")
            torch.cuda.current_stream(self.device).synchronize()

    def derivative(self, g, op: int):
        with torch.cuda.device(self.device):
            t = _field(g, self.ny, self.nx, self.device)
            out = torch.empty_like(t)
            _check(_lib.fftlb_derivative(self.handle, _ptr(t), _ptr(out), int(op), _stream(self.device)),
                   "fftlb_derivative")
        return out

    @property
    def plan(self):
        p = Plan()
        _check(_lib.fftlb_get_plan(self.handle, ctypes.byref(p)), "fftlb_get_plan")
        return p.as_tuple()

    def set_plan(self, conv_cols: int, multi_cols: int, conv_radix: int, multi_radix: int):
        p = Plan(int(conv_cols), int(multi_cols), int(conv_radix), int(multi_radix))
        _check(_lib.fftlb_set_plan(self.handle, ctypes.byref(p)), "fftlb_set_plan")

    def autotune(self, reps: int = 10, cache_path: str | None = None):
        """Time the column plans of this grid size and keep the fastest (fftlb_autotune)."""
        p = Plan()
        with torch.cuda.device(self.device):
            _check(_lib.fftlb_autotune(self.handle, int(reps), cache_path.encode() if cache_path else None,
                                       _stream(self.device), ctypes.byref(p)), "fftlb_autotune")
        return p.as_tuple()

    def close(self):
        if self._h is not None:
            if self._owned:
                _lib.fftlb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Independent FFT-LB instances of any mix of grid sizes advanced together
    (fftlb_batch_*): one captured graph of `poll_every` steps of every running instance,
    with on-device retirement of converged instances.

    fields: a sequence of (rho0, ux0, uy0, T0) tuples of [ny, nx] arrays; params: one
    Params for all instances or a sequence of them."""

    def __init__(self, fields, params=None, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the FFT-LB solver runs only through its HIP library")
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        n = len(fields)
        plist = list(params) if isinstance(params, (list, tuple)) else [params or Params()] * n
        if len(plist) != n:
            raise ValueError("one Params per instance")
        self.n = n
        self.params = plist
        self.shapes = []
        cfgs = (Config * n)()
        with torch.cuda.device(self.device):
            tensors = []
            for i, fl in enumerate(fields):
                rho0 = torch.as_tensor(fl[0])
                ny, nx = int(rho0.shape[0]), int(rho0.shape[1])
                self.shapes.append((ny, nx))
                cfgs[i] = plist[i].config(nx, ny)
                tensors.append([_field(a, ny, nx, self.device) for a in fl])
            nbytes = ctypes.c_size_t()
            _check(_lib.fftlb_batch_workspace_bytes(n, cfgs, ctypes.byref(nbytes)), "fftlb_batch_workspace_bytes")
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            arrs = [(ctypes.c_void_p * n)(*[t[k].data_ptr() for t in tensors]) for k in range(4)]
            b = ctypes.c_void_p()
            rc = _lib.fftlb_batch_create(n, cfgs, _ptr(self.workspace), nbytes.value, *arrs, _stream(self.device),
                                         ctypes.byref(b))
            _check(rc, "fftlb_batch_create")
        self._b = b

    @property
    def handle(self):
        if self._b is None:
            raise RuntimeError("batch is closed")
        return self._b

    def autotune(self, reps: int = 10, cache_path: str | None = None):
        with torch.cuda.device(self.device):
            _check(_lib.fftlb_batch_autotune(self.handle, int(reps), cache_path.encode() if cache_path else None,
                                             _stream(self.device)), "fftlb_batch_autotune")

    def run(self, tol: float, consecutive: int = 3, poll_every: int = 100, max_steps: int = 10**6,
            allow_unstable: bool = False) -> int:
        """fftlb_batch_run.  It returns FFTLB_EUNSTABLE when an instance has retired on a
        non-finite value: raised as FFTLBError unless allow_unstable, in which case the code
        is returned (the other instances were advanced; status() tells which retired)."""
        with torch.cuda.device(self.device):
            rc = _lib.fftlb_batch_run(self.handle, float(tol), int(consecutive), int(poll_every), int(max_steps),
                                      _stream(self.device))
        if not (allow_unstable and rc == FFTLB_EUNSTABLE):
            _check(rc, "fftlb_batch_run")
        return rc

    def status(self):
        """dict of numpy arrays: steps, steps_to_tol (-1 unless converged), residual, state."""
        import numpy as np
        n = self.n
        steps = (ctypes.c_int64 * n)()
        stt = (ctypes.c_int64 * n)()
        res = (ctypes.c_double * n)()
        st = (ctypes.c_int32 * n)()
        with torch.cuda.device(self.device):
            _check(_lib.fftlb_batch_status(self.handle, steps, stt, res, st), "fftlb_batch_status")
        return {"steps": np.array(steps[:]), "steps_to_tol": np.array(stt[:]), "residual": np.array(res[:]),
                "state": np.array(st[:])}

    def instance(self, i: int) -> Solver:
        h = ctypes.c_void_p()
        _check(_lib.fftlb_batch_instance(self.handle, int(i), ctypes.byref(h)), "fftlb_batch_instance")
        ny, nx = self.shapes[i]
        return Solver._view(h, nx, ny, self.params[i], self.device, self)

    def close(self):
        if self._b is not None:
            _lib.fftlb_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def svups(nx: int, ny: int, steps: int, seconds: float) -> float:
    """Site-velocity updates per second: 33 nx ny steps / seconds."""
    return Q * nx * ny * steps / seconds if seconds > 0 else math.nan
