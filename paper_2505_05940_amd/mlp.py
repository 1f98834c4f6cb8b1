"""ctypes binding of the proposal network kernels (include/mlp.h):
argument marshalling only."""
from __future__ import annotations

import ctypes as C

import numpy as np

from .modal import ModalError, _stream_handle
from .modal import lib as _lib

_fp = C.POINTER(C.c_float)
vp = C.c_void_p
_lib.mlp_init.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(C.c_int32), C.c_int32, vp]
_lib.mlp_n_params.argtypes = [vp, C.POINTER(C.c_int64)]
_lib.mlp_set_params.argtypes = [vp, _fp, vp]
_lib.mlp_get.argtypes = [vp, C.c_int32, _fp, vp]
_lib.mlp_forward.argtypes = [vp, _fp, C.c_int32, _fp, vp]
_lib.mlp_backward.argtypes = [vp, _fp, vp]
_lib.mlp_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32, vp]
_lib.mlp_train_step.argtypes = [vp, _fp, _fp, vp, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float,
                                C.c_int32, _fp, vp]
_lib.mlp_train_epoch.argtypes = [vp, _fp, _fp, vp, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float,
                                 C.c_float, _fp, vp]
_lib.mlp_destroy.argtypes = [vp]
_lib.mlp_destroy.restype = None
_lib.mlp_last_error.restype = C.c_char_p
for _f in ("mlp_init", "mlp_n_params", "mlp_set_params", "mlp_get", "mlp_forward",
           "mlp_backward", "mlp_adam_step", "mlp_train_step", "mlp_train_epoch"):
    getattr(_lib, _f).restype = C.c_int


def _check(code):
    if code != 0:
        raise ModalError(code, _lib.mlp_last_error().decode())


def _ptr(t):
    return C.cast(C.c_void_p(t.data_ptr()), _fp)


class MLP:
    """dims[0] -> ... -> dims[-1], ReLU hidden layers, linear output."""

    def __init__(self, dims, max_batch, stream=None):
        self.dims = list(dims)
        self._stream = stream
        self._ctx = vp()
        d = (C.c_int32 * len(dims))(*dims)
        _check(_lib.mlp_init(C.byref(self._ctx), len(dims) - 1, d, max_batch, _stream_handle(stream)))
        n = C.c_int64()
        _check(_lib.mlp_n_params(self._ctx, C.byref(n)))
        self.n_params = n.value
        self.t = 0

    def init_params(self, seed=0):
        """He-normal weights, zero biases (seeded)."""
        rng = np.random.default_rng(seed)
        parts = []
        for i, j in zip(self.dims[:-1], self.dims[1:]):
            parts += [rng.normal(size=i * j) * np.sqrt(2.0 / i), np.zeros(j)]
        self.set_params(np.concatenate(parts))

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.n_params
        _check(_lib.mlp_set_params(self._ctx, a.ctypes.data_as(_fp), _stream_handle(self._stream)))
        self.t = 0

    def params(self):
        a = np.empty(self.n_params, np.float32)
        _check(_lib.mlp_get(self._ctx, 0, a.ctypes.data_as(_fp), _stream_handle(self._stream)))
        return a

    def grads(self):
        a = np.empty(self.n_params, np.float32)
        _check(_lib.mlp_get(self._ctx, 1, a.ctypes.data_as(_fp), _stream_handle(self._stream)))
        return a

    def forward(self, x):
        import torch
        x = x.contiguous().float()
        y = torch.empty((x.shape[0], self.dims[-1]), device=x.device)
        _check(_lib.mlp_forward(self._ctx, _ptr(x), x.shape[0], _ptr(y), _stream_handle(self._stream)))
        return y

    def backward(self, dy):
        dy = dy.contiguous().float()
        _check(_lib.mlp_backward(self._ctx, _ptr(dy), _stream_handle(self._stream)))

    def adam_step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        _check(_lib.mlp_adam_step(self._ctx, lr, b1, b2, eps, self.t, _stream_handle(self._stream)))

    def train_step(self, X, Z, idx, lr, loss_acc=None, b1=0.9, b2=0.999, eps=1e-8):
        """``mlp_train_step``: MSE step on rows idx (int64 CUDA tensor) of
        X and Z (float32 CUDA, contiguous); adds the loss to loss_acc (a
        float32 CUDA scalar) if given."""
        import torch
        assert X.is_contiguous() and Z.is_contiguous() and idx.is_contiguous()
        assert X.dtype == torch.float32 and Z.dtype == torch.float32 and idx.dtype == torch.int64
        assert X.shape[1] == self.dims[0] and Z.shape[1] == self.dims[-1]
        self.t += 1
        acc = _ptr(loss_acc) if loss_acc is not None else None
        _check(_lib.mlp_train_step(self._ctx, _ptr(X), _ptr(Z), C.c_void_p(idx.data_ptr()), idx.shape[0], lr,
                                   b1, b2, eps, self.t, acc, _stream_handle(self._stream)))

    def train_epoch(self, X, Z, order, batch, lr, loss_acc=None, b1=0.9, b2=0.999, eps=1e-8):
        """``mlp_train_epoch``: len(order) // batch MSE steps on consecutive
        slices of order (int64 CUDA tensor, refilled in place between
        epochs so that the recorded epoch is replayed)."""
        import torch
        assert X.is_contiguous() and Z.is_contiguous() and order.is_contiguous()
        assert X.dtype == torch.float32 and Z.dtype == torch.float32 and order.dtype == torch.int64
        assert X.shape[1] == self.dims[0] and Z.shape[1] == self.dims[-1]
        steps = order.shape[0] // batch
        acc = _ptr(loss_acc) if loss_acc is not None else None
        _check(_lib.mlp_train_epoch(self._ctx, _ptr(X), _ptr(Z), C.c_void_p(order.data_ptr()), steps, batch, lr,
                                    b1, b2, eps, acc, _stream_handle(self._stream)))
        self.t += steps

    def close(self):
        if self._ctx:
            _lib.mlp_destroy(self._ctx)
            self._ctx = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
