"""ctypes wrapper of the oracle's FMA-chain matrix product (test infrastructure only).

See oracle/csrc/fma_chain.c: each output is a chain of correctly rounded
fused multiply-adds over the inner index in ascending order, starting at 0.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .build_oracle import LIB, build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        lib = ctypes.CDLL(str(LIB))
        for name, ct in (("f64", ctypes.c_double), ("f32", ctypes.c_float)):
            fn = getattr(lib, f"oracle_fma_matmul_batched_{name}")
            p = ctypes.POINTER(ct)
            fn.argtypes = [p, p, p] + [ctypes.c_int64] * 4
            fn.restype = None
        _lib = lib
    return _lib


def fma_matmul(a: np.ndarray, b: np.ndarray, prec: str) -> np.ndarray:
    """a[..., m, k] @ b[..., k, n] with one FMA chain per output, in prec."""
    dt = np.float64 if prec == "f64" else np.float32
    ct = ctypes.c_double if prec == "f64" else ctypes.c_float
    a = np.ascontiguousarray(a, dtype=dt)
    b = np.ascontiguousarray(b, dtype=dt)
    if a.shape[:-2] != b.shape[:-2] or a.shape[-1] != b.shape[-2]:
        raise ValueError(f"shape mismatch {a.shape} @ {b.shape}")
    batch = a.shape[:-2]
    m, k = a.shape[-2:]
    n = b.shape[-1]
    nb = int(np.prod(batch)) if batch else 1
    c = np.empty(batch + (m, n), dtype=dt)
    fn = getattr(_load(), f"oracle_fma_matmul_batched_{prec}")
    P = ctypes.POINTER(ct)
    fn(a.ctypes.data_as(P), b.ctypes.data_as(P), c.ctypes.data_as(P), nb, m, k, n)
    return c
