"""Python side of the surrogate-MLP oracle -- TEST INFRASTRUCTURE ONLY.

Drives ``o_mlp_*`` in liboracle.so (see oracle_mlp.c for the definition of
the network, loss and rounding points).  Only tests and the benchmark's CPU
leg use it.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Sequence

import numpy as np

from . import oracle as _o

_dp = C.POINTER(C.c_double)


class OMlp(C.Structure):
    _fields_ = [("dims", C.c_int32 * 6), ("W", _dp * 5), ("b", _dp * 5)]


def _lib():
    L = _o.lib()
    if not getattr(L, "_mlp_declared", False):
        L.o_bf16_round.argtypes = [C.c_double]
        L.o_bf16_round.restype = C.c_double
        L.o_mlp_forward.argtypes = [C.POINTER(OMlp), _dp, C.c_int, C.c_int, _dp, _dp]
        L.o_mlp_backward.argtypes = [C.POINTER(OMlp), _dp, _dp, C.c_int, C.c_double, C.c_int,
                                     C.POINTER(_dp), C.POINTER(_dp)]
        L.o_mlp_backward.restype = C.c_double
        L.o_mlp_loss.argtypes = [C.POINTER(OMlp), _dp, _dp, C.c_int, C.c_double, C.c_int]
        L.o_mlp_loss.restype = C.c_double
        L.o_adam.argtypes = [_dp, _dp, _dp, _dp, C.c_int64, C.c_double, C.c_double, C.c_double,
                             C.c_double, C.c_int64]
        L._mlp_declared = True
    return L


def bf16_round_f32(a: np.ndarray) -> np.ndarray:
    """float32 -> nearest BF16 value (ties to even), returned as float32."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r << 16).astype(np.uint32).view(np.float32)


class OracleMLP:
    def __init__(self, W: Sequence[np.ndarray], b: Sequence[np.ndarray]):
        self.W = [np.ascontiguousarray(w, np.float64) for w in W]
        self.b = [np.ascontiguousarray(v, np.float64) for v in b]
        self.dims = [self.W[0].shape[1]] + [w.shape[0] for w in self.W]
        assert len(self.W) == 5 and self.dims[-1] == 1
        self.net = OMlp()
        self.net.dims[:] = self.dims
        for l in range(5):
            self.net.W[l] = self.W[l].ctypes.data_as(_dp)
            self.net.b[l] = self.b[l].ctypes.data_as(_dp)

    def forward(self, x: np.ndarray, round_bf16: bool = True) -> np.ndarray:
        x = np.ascontiguousarray(x, np.float64)
        z = np.zeros(x.shape[0])
        _lib().o_mlp_forward(C.byref(self.net), x.ctypes.data_as(_dp), x.shape[0],
                             int(round_bf16), z.ctypes.data_as(_dp), C.cast(None, _dp))
        return z

    def loss(self, x, y, pos_weight=1.0, round_bf16=True) -> float:
        x = np.ascontiguousarray(x, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        return _lib().o_mlp_loss(C.byref(self.net), x.ctypes.data_as(_dp), y.ctypes.data_as(_dp),
                                 x.shape[0], pos_weight, int(round_bf16))

    def backward(self, x, y, pos_weight=1.0, round_bf16=True):
        x = np.ascontiguousarray(x, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        dW = [np.zeros_like(w) for w in self.W]
        db = [np.zeros_like(v) for v in self.b]
        pw = (_dp * 5)(*[a.ctypes.data_as(_dp) for a in dW])
        pb = (_dp * 5)(*[a.ctypes.data_as(_dp) for a in db])
        loss = _lib().o_mlp_backward(C.byref(self.net), x.ctypes.data_as(_dp),
                                     y.ctypes.data_as(_dp), x.shape[0], pos_weight,
                                     int(round_bf16), pw, pb)
        return loss, dW, db


def adam(w, m, v, g, lr, beta1, beta2, eps, t):
    w, m, v = (np.ascontiguousarray(a, np.float64) for a in (w, m, v))
    g = np.ascontiguousarray(g, np.float64)
    _lib().o_adam(w.ctypes.data_as(_dp), m.ctypes.data_as(_dp), v.ctypes.data_as(_dp),
                  g.ctypes.data_as(_dp), w.size, lr, beta1, beta2, eps, t)
    return w, m, v
