"""Python binding of the learned-guess network (the C ABI in include/kvnn.h).

Argument marshalling only: the forward and backward passes, the loss and
the optimizer run in the library's HIP kernels.  Tensors are torch float32
CUDA (ROCm) tensors [batch][4][r][r][r]; work is enqueued on the torch stream
current when the network is created.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import kv

KVNN_OK, KVNN_EINVAL, KVNN_ENOMEM, KVNN_EDEVICE = range(4)

# every extern "C" symbol declared in include/kvnn.h
ABI_SYMBOLS = ("kvnn_create", "kvnn_destroy", "kvnn_num_params", "kvnn_get_params", "kvnn_set_params",
               "kvnn_make_inputs", "kvnn_forward", "kvnn_predict", "kvnn_backward", "kvnn_train_step",
               "kvnn_last_error")


class KVNNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kvnn error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("res", ctypes.c_int), ("batch_max", ctypes.c_int),
                ("xc", ctypes.POINTER(ctypes.c_double)), ("yc", ctypes.POINTER(ctypes.c_double)),
                ("zc", ctypes.POINTER(ctypes.c_double)), ("lgr_lo", ctypes.c_double),
                ("lgr_hi", ctypes.c_double), ("seed", ctypes.c_uint64)]


_bound = False


def load():
    global _bound
    lib = kv.load()
    if _bound:
        return lib
    P = ctypes.c_void_p
    lib.kvnn_create.argtypes = [ctypes.POINTER(_Params), P, ctypes.POINTER(P)]
    lib.kvnn_destroy.argtypes = [P]
    lib.kvnn_num_params.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.kvnn_get_params.argtypes = [P, P]
    lib.kvnn_set_params.argtypes = [P, P]
    lib.kvnn_make_inputs.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.c_int, P]
    lib.kvnn_forward.argtypes = [P, P, ctypes.c_int, P]
    lib.kvnn_predict.argtypes = [P, ctypes.c_double, P]
    lib.kvnn_backward.argtypes = [P, P, P, ctypes.c_int, P]
    lib.kvnn_train_step.argtypes = [P, P, P, ctypes.c_int, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]
    lib.kvnn_last_error.argtypes = [P]
    lib.kvnn_last_error.restype = ctypes.c_char_p
    for name in ABI_SYMBOLS:
        if name != "kvnn_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _bound = True
    return lib


def _fptr(t, n):
    return kv._fptr(t, n)


class Net:
    """The U-Net of include/kvnn.h on r^3 cell centres (xc, yc, zc)."""

    def __init__(self, centres, lgr_range, batch_max=4, seed=3, stream=None):
        import torch
        self._lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the network runs on gfx950 only")
        self._cen = [np.ascontiguousarray(np.asarray(c, dtype=np.float64)) for c in centres]
        r = len(self._cen[0])
        if any(len(c) != r for c in self._cen):
            raise ValueError("the network grid is cubic: equal centre counts")
        self.res, self.batch_max = r, int(batch_max)
        self.lgr_range = (float(lgr_range[0]), float(lgr_range[1]))
        p = _Params(r, self.batch_max, *(c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for c in self._cen),
                    self.lgr_range[0], self.lgr_range[1], int(seed))
        s = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self._lib.kvnn_create(ctypes.byref(p), ctypes.c_void_p(s.cuda_stream), ctypes.byref(h))
        if rc != KVNN_OK:
            raise KVNNError(rc, "kvnn_create failed")
        self._h = h
        cnt = ctypes.c_int64()
        self._check(self._lib.kvnn_num_params(self._h, ctypes.byref(cnt)))
        self.num_params = int(cnt.value)

    @property
    def centres(self):
        return self._cen

    def _check(self, rc):
        if rc != KVNN_OK:
            raise KVNNError(rc, self._lib.kvnn_last_error(self._h).decode())

    def _len(self, batch):
        return batch * 4 * self.res ** 3

    def close(self):
        if getattr(self, "_h", None):
            self._lib.kvnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(self.num_params, dtype=np.float32)
        self._check(self._lib.kvnn_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, w):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
        if w.size != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters")
        self._check(self._lib.kvnn_set_params(self._h, w.ctypes.data_as(ctypes.c_void_p)))

    def make_inputs(self, grs, out):
        g = np.ascontiguousarray(np.asarray(grs, dtype=np.float64).reshape(-1))
        self._check(self._lib.kvnn_make_inputs(self._h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               len(g), _fptr(out, self._len(len(g)))))

    def forward(self, inp, batch, out):
        self._check(self._lib.kvnn_forward(self._h, _fptr(inp, self._len(batch)), int(batch),
                                           _fptr(out, self._len(batch))))

    def predict(self, Gr, out):
        self._check(self._lib.kvnn_predict(self._h, float(Gr), _fptr(out, self._len(1))))

    def backward(self, inp, gout, batch):
        g = np.empty(self.num_params, dtype=np.float32)
        self._check(self._lib.kvnn_backward(self._h, _fptr(inp, self._len(batch)), _fptr(gout, self._len(batch)),
                                            int(batch), g.ctypes.data_as(ctypes.c_void_p)))
        return g

    def train_step(self, inp, target, batch, lr):
        loss = ctypes.c_float()
        self._check(self._lib.kvnn_train_step(self._h, _fptr(inp, self._len(batch)),
                                              _fptr(target, self._len(batch)), int(batch), float(lr),
                                              ctypes.byref(loss)))
        return float(loss.value)
