"""Single-threaded CPU NTT Toeplitz extractor (``cpu_ntt.c``): a timing baseline
for the benchmark — a plain CPU implementation of the convolution route over the
64-bit prime of the single large-transform configuration. Not the oracle (which
is the schoolbook definition) and not part of the GPU library; built with gcc
on first use."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcpuntt.so")
_SRC = os.path.join(_HERE, "cpu_ntt.c")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.cpu_ntt_toeplitz.argtypes = [u64p, ctypes.c_uint64, u64p, ctypes.c_uint64, ctypes.c_int, u64p]
        lib.cpu_ntt_toeplitz.restype = ctypes.c_int
        _lib = lib
    return _lib


def _arr(words, nbits):
    w = np.zeros(((int(nbits) + 63) >> 6) + 1, np.uint64)
    src = np.asarray(words, np.uint64)[: (int(nbits) + 63) >> 6]
    w[: src.size] = src
    r = int(nbits) & 63
    if r:
        w[(int(nbits) >> 6)] &= np.uint64((1 << r) - 1)
    return w


def toeplitz(x, y, n: int, m: int, seed_order: str = "paper") -> np.ndarray:
    """Packed z (ceil(m/64) words) of the Toeplitz extractor, 1 <= m <= n."""
    n, m = int(n), int(m)
    xx, yy = _arr(x, n), _arr(y, n + m - 1)
    z = np.zeros(((m + 63) >> 6) + 1, np.uint64)
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))  # noqa: E731
    if _load().cpu_ntt_toeplitz(p(xx), n, p(yy), m, int(seed_order == "linear"), p(z)) != 0:
        raise MemoryError("cpu_ntt_toeplitz: out of memory")
    return z[: (m + 63) >> 6]
