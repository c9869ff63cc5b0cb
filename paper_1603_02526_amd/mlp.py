"""ctypes binding of the warm-start MLP (``admm_mlp_*`` in include/admm.h).
Device arrays are torch tensors (float32, contiguous); the arithmetic runs
in the HIP library's matrix-core kernels."""
from __future__ import annotations

import ctypes

import numpy as np

from .admm import check, lib, _stream

VP = ctypes.c_void_p
FP = ctypes.POINTER(ctypes.c_float)
_done = False


def _setup():
    global _done
    L = lib()
    if _done:
        return L
    st = ctypes.c_int
    L.admm_mlp_create.restype = st
    L.admm_mlp_create.argtypes = [ctypes.c_int32] * 5 + [ctypes.POINTER(VP)]
    L.admm_mlp_n_params.restype = ctypes.c_int64
    L.admm_mlp_n_params.argtypes = [VP]
    L.admm_mlp_set_params.restype = st
    L.admm_mlp_set_params.argtypes = [VP, FP]
    L.admm_mlp_get_params.restype = st
    L.admm_mlp_get_params.argtypes = [VP, FP]
    L.admm_mlp_forward.restype = st
    L.admm_mlp_forward.argtypes = [VP, VP, ctypes.c_int32, VP, VP]
    L.admm_mlp_grads.restype = st
    L.admm_mlp_grads.argtypes = [VP, VP, VP, ctypes.c_int32, VP, VP, VP]
    L.admm_mlp_train_step.restype = st
    L.admm_mlp_train_step.argtypes = [VP, VP, VP, ctypes.c_int32, ctypes.c_float, VP, VP]
    L.admm_mlp_fit_output_scaling.restype = st
    L.admm_mlp_fit_output_scaling.argtypes = [VP, VP, ctypes.c_int64, ctypes.c_float, VP]
    L.admm_mlp_fit_output_scaling_noalloc.restype = st
    L.admm_mlp_fit_output_scaling_noalloc.argtypes = [VP, VP, ctypes.c_int64, ctypes.c_float, VP]
    L.admm_mlp_set_output_scaling.restype = st
    L.admm_mlp_set_output_scaling.argtypes = [VP, FP, FP]
    L.admm_mlp_get_output_scaling.restype = st
    L.admm_mlp_get_output_scaling.argtypes = [VP, FP, FP]
    L.admm_mlp_destroy.restype = st
    L.admm_mlp_destroy.argtypes = [VP]
    _done = True
    return L


def _p(t):
    if t is None:
        return None
    assert t.is_contiguous() and str(t.dtype) == "torch.float32"
    return t.data_ptr()


class MLP:
    """n_in -> hidden -> hidden -> n_out ReLU network on one GPU."""

    def __init__(self, n_in: int, hidden: int, n_out: int, max_batch: int, device: int = 0):
        L = _setup()
        h = VP()
        check(L.admm_mlp_create(n_in, hidden, n_out, max_batch, device, ctypes.byref(h)))
        self._h = h
        self.n_in, self.hidden, self.n_out, self.max_batch = n_in, hidden, n_out, max_batch
        self.n_params = int(L.admm_mlp_n_params(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().admm_mlp_destroy(h)
            except Exception:
                pass
            self._h = None

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.n_params
        check(_setup().admm_mlp_set_params(self._h, a.ctypes.data_as(FP)))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n_params, np.float32)
        check(_setup().admm_mlp_get_params(self._h, a.ctypes.data_as(FP)))
        return a

    def fit_output_scaling(self, targets, sd_min: float = 1e-6, stream=None):
        check(_setup().admm_mlp_fit_output_scaling(self._h, _p(targets), int(targets.shape[0]),
                                                   float(sd_min), _stream(stream)))

    def fit_output_scaling_noalloc(self, targets, sd_min: float = 1e-6, stream=None):
        """As fit_output_scaling, in the library's fixed device workspace
        (no allocation, asynchronous)."""
        check(_setup().admm_mlp_fit_output_scaling_noalloc(
            self._h, _p(targets), int(targets.shape[0]), float(sd_min), _stream(stream)))

    def set_output_scaling(self, mean, sd):
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(sd, dtype=np.float32)
        check(_setup().admm_mlp_set_output_scaling(self._h, m.ctypes.data_as(FP),
                                                   s.ctypes.data_as(FP)))

    def get_output_scaling(self):
        m = np.zeros(self.n_out, np.float32)
        s = np.zeros(self.n_out, np.float32)
        check(_setup().admm_mlp_get_output_scaling(self._h, m.ctypes.data_as(FP),
                                                   s.ctypes.data_as(FP)))
        return m, s

    def forward(self, x, y, stream=None):
        check(_setup().admm_mlp_forward(self._h, _p(x), int(x.shape[0]), _p(y), _stream(stream)))

    def grads(self, x, target, grads=None, loss=None, stream=None):
        check(_setup().admm_mlp_grads(self._h, _p(x), _p(target), int(x.shape[0]), _p(grads),
                                      _p(loss), _stream(stream)))

    def train_step(self, x, target, lr, loss=None, stream=None):
        check(_setup().admm_mlp_train_step(self._h, _p(x), _p(target), int(x.shape[0]),
                                           float(lr), _p(loss), _stream(stream)))


def init_params(n_in: int, hidden: int, n_out: int, seed: int,
                out_scale: float = 0.1) -> np.ndarray:
    """He-uniform weights (the output layer scaled by out_scale so that the
    untrained network predicts values near zero), zero biases.  numpy,
    seeded: the random numbers are drawn here and passed to the library."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (fan_in, fan_out) in enumerate(((n_in, hidden), (hidden, hidden), (hidden, n_out))):
        lim = np.sqrt(6.0 / fan_in) * (out_scale if li == 2 else 1.0)
        parts.append(rng.uniform(-lim, lim, size=(fan_out, fan_in)))
        parts.append(np.zeros(fan_out))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)
