"""Python binding of the warm-start network of libfftlb.so (ctypes; include/fftlb_cnn.h).
Argument marshalling only: the forward and backward passes, Adam and the warm-start
transform run in the library's HIP kernels."""
from __future__ import annotations

import ctypes

import torch

from . import fftlb as _F

PARAMS = 38466


def _load():
    lib = _F.library()
    vp, i32, sz, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_float
    sig = {
        "fftlb_cnn_workspace_bytes": [i32, i32, i32, ctypes.POINTER(sz)],
        "fftlb_cnn_create": [i32, i32, i32, vp, sz, vp, vp, ctypes.POINTER(vp)],
        "fftlb_cnn_forward": [vp, vp, vp, i32, vp],
        "fftlb_cnn_gradient": [vp, vp, vp, i32, vp, vp, vp],
        "fftlb_cnn_adam_step": [vp, f32, vp],
        "fftlb_cnn_get_params": [vp, vp, vp],
        "fftlb_cnn_set_params": [vp, vp, vp],
        "fftlb_cnn_read_buffer": [vp, i32, i32, vp, sz, vp],
        "fftlb_cnn_warm_start": [vp, vp, vp, f32, f32, f32, f32, vp, vp, vp],
        "fftlb_cnn_project": [vp, vp, vp, f32, f32, f32, vp, vp, vp],
        "fftlb_cnn_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = args
    return lib


_lib = _load()


def library():
    return _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Network:
    """The warm-start network on one GPU, for inputs of h x w and batches of <= max_batch."""

    def __init__(self, h: int, w: int, max_batch: int, params, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the network runs only through its HIP library")
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.h, self.w, self.max_batch = int(h), int(w), int(max_batch)
        with torch.cuda.device(self.device):
            nb = ctypes.c_size_t()
            _F._check(_lib.fftlb_cnn_workspace_bytes(self.h, self.w, self.max_batch, ctypes.byref(nb)),
                      "fftlb_cnn_workspace_bytes")
            self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
            p = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
            if p.numel() != PARAMS:
                raise ValueError(f"expected {PARAMS} parameters")
            c = ctypes.c_void_p()
            _F._check(_lib.fftlb_cnn_create(self.h, self.w, self.max_batch, _ptr(self.workspace), nb.value, _ptr(p),
                                            _stream(self.device), ctypes.byref(c)), "fftlb_cnn_create")
            torch.cuda.current_stream(self.device).synchronize()
        self._c = c

    @property
    def handle(self):
        if self._c is None:
            raise RuntimeError("network is closed")
        return self._c

    def _x(self, x, ch):
        t = torch.as_tensor(x, dtype=torch.float32).to(self.device).contiguous()
        if t.dim() != 4 or t.shape[1:] != (ch, self.h, self.w) or not 1 <= t.shape[0] <= self.max_batch:
            raise ValueError(f"expected [n, {ch}, {self.h}, {self.w}] with n <= {self.max_batch}")
        return t

    def forward(self, x):
        x = self._x(x, 3)
        with torch.cuda.device(self.device):
            y = torch.empty((x.shape[0], 2, self.h, self.w), dtype=torch.float32, device=self.device)
            _F._check(_lib.fftlb_cnn_forward(self.handle, _ptr(x), _ptr(y), x.shape[0], _stream(self.device)),
                      "fftlb_cnn_forward")
        return y

    def gradient(self, x, target):
        """(loss, gradient) of the mean squared error; the gradient is kept for adam_step."""
        x, t = self._x(x, 3), self._x(target, 2)
        with torch.cuda.device(self.device):
            g = torch.empty(PARAMS, dtype=torch.float32, device=self.device)
            L = torch.empty(1, dtype=torch.float64, device=self.device)
            _F._check(_lib.fftlb_cnn_gradient(self.handle, _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(L),
                                              _stream(self.device)), "fftlb_cnn_gradient")
        return L, g

    def train_step(self, x, target, lr: float):
        L, _ = self.gradient(x, target)
        with torch.cuda.device(self.device):
            _F._check(_lib.fftlb_cnn_adam_step(self.handle, float(lr), _stream(self.device)), "fftlb_cnn_adam_step")
        return L

    @property
    def params(self):
        with torch.cuda.device(self.device):
            p = torch.empty(PARAMS, dtype=torch.float32, device=self.device)
            _F._check(_lib.fftlb_cnn_get_params(self.handle, _ptr(p), _stream(self.device)), "fftlb_cnn_get_params")
        return p

    def set_params(self, params):
        p = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        with torch.cuda.device(self.device):
            _F._check(_lib.fftlb_cnn_set_params(self.handle, _ptr(p), _stream(self.device)), "fftlb_cnn_set_params")
            torch.cuda.current_stream(self.device).synchronize()

    def buffer(self, layer: int, kind: int, n: int, shape):
        """A copy of an internal buffer (see fftlb_cnn_read_buffer) as an [n, *shape] tensor."""
        out = torch.empty((n,) + tuple(shape), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            _F._check(_lib.fftlb_cnn_read_buffer(self.handle, int(layer), int(kind), _ptr(out), out.numel(),
                                                 _stream(self.device)), "fftlb_cnn_read_buffer")
        return out

    def warm_start(self, rho0, T0, T_target: float, rho_c: float, T_c: float, rho_max: float):
        """Predicted (rho, T) [h, w] device tensors for one run."""
        r0 = torch.as_tensor(rho0, dtype=torch.float32).to(self.device).contiguous()
        t0 = torch.as_tensor(T0, dtype=torch.float32).to(self.device).contiguous()
        if r0.shape != (self.h, self.w) or t0.shape != (self.h, self.w):
            raise ValueError("fields must be [h, w]")
        with torch.cuda.device(self.device):
            rho = torch.empty_like(r0)
            T = torch.empty_like(t0)
            _F._check(_lib.fftlb_cnn_warm_start(self.handle, _ptr(r0), _ptr(t0), float(T_target), float(rho_c),
                                                float(T_c), float(rho_max), _ptr(rho), _ptr(T),
                                                _stream(self.device)), "fftlb_cnn_warm_start")
        return rho, T

    def project(self, pred, rho0, rho_c: float, T_c: float, rho_max: float):
        """fftlb_cnn_project: the warm-start transform of a prediction pred [2, h, w]
        (normalised rho, T) into (rho, T) [h, w] device tensors."""
        p = torch.as_tensor(pred, dtype=torch.float32).to(self.device).contiguous()
        r0 = torch.as_tensor(rho0, dtype=torch.float32).to(self.device).contiguous()
        if p.shape != (2, self.h, self.w) or r0.shape != (self.h, self.w):
            raise ValueError("pred must be [2, h, w] and rho0 [h, w]")
        with torch.cuda.device(self.device):
            rho = torch.empty_like(r0)
            T = torch.empty_like(r0)
            _F._check(_lib.fftlb_cnn_project(self.handle, _ptr(p), _ptr(r0), float(rho_c), float(T_c), float(rho_max),
                                             _ptr(rho), _ptr(T), _stream(self.device)), "fftlb_cnn_project")
        return rho, T

    def close(self):
        if self._c is not None:
            _lib.fftlb_cnn_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
