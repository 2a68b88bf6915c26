"""Python access to the binary128 reference oracle (``lbessel_oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
the benchmark may use this module; the GPU library never does.  It shares
nothing with the GPU path except the seeded input arrays handed to both.

Every function returns the reference value as a ``(hi, lo)`` pair of float64
arrays whose sum carries the binary128 result to ~2^-106 relative.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbessel_oracle.c")
_LIB = os.path.join(_HERE, "liblbessel_oracle.so")

_lib = None


def compile_oracle(src: str, out: str) -> str:
    """gcc -O2 with OpenMP and libquadmath: src (C) -> out (.so)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unknown-pragmas", src, "-o", tmp, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle; returns the .so path."""
    if force or not os.path.exists(_LIB):
        compile_oracle(_SRC, _LIB)
    return _LIB


def open_library(path: str):
    """ctypes handle of an oracle build at `path` with argument types set."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("lbo_log_iv", "lbo_log_kv", "lbo_dlog_iv", "lbo_dlog_kv"):
        fn = getattr(lib, name)
        fn.argtypes = [dp, dp, dp, dp, ctypes.c_int64]
        fn.restype = None
    lib.lbo_vmf_log_norm.argtypes = [dp, ctypes.c_double, dp, dp, ctypes.c_int64]
    lib.lbo_vmf_log_norm.restype = None
    lib.lbo_max_threads.restype = ctypes.c_int
    lib.lbo_set_threads.argtypes = [ctypes.c_int]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = open_library(_LIB)
    return _lib


class Oracle:
    """The same functions as this module, bound to the build at `path`."""

    def __init__(self, path: str):
        self._lib = open_library(path)

    def _map2(self, name, v, x):
        return _map2(name, v, x, self._lib)

    def log_iv(self, v, x):
        return self._map2("lbo_log_iv", v, x)

    def log_kv(self, v, x):
        return self._map2("lbo_log_kv", v, x)

    def dlog_iv(self, v, x):
        return self._map2("lbo_dlog_iv", v, x)

    def dlog_kv(self, v, x):
        return self._map2("lbo_dlog_kv", v, x)

    def vmf_log_norm(self, kappa, p):
        return vmf_log_norm(kappa, p, self._lib)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _map2(name: str, v, x, lib=None):
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    v, x = np.broadcast_arrays(v, x)
    v = np.ascontiguousarray(v).ravel()
    x = np.ascontiguousarray(x).ravel()
    hi = np.empty_like(v)
    lo = np.empty_like(v)
    getattr(lib or _load(), name)(_ptr(v), _ptr(x), _ptr(hi), _ptr(lo), v.size)
    return hi, lo


def log_iv(v, x):
    """log I_v(x) by the defining power series (binary128)."""
    return _map2("lbo_log_iv", v, x)


def log_kv(v, x):
    """log K_v(x) by trapezoid quadrature of int_0^inf e^{-x cosh t} cosh(vt) dt."""
    return _map2("lbo_log_kv", v, x)


def dlog_iv(v, x):
    """d/dx log I_v(x) from the term-by-term differentiated series."""
    return _map2("lbo_dlog_iv", v, x)


def dlog_kv(v, x):
    """d/dx log K_v(x) by differentiating under the integral sign."""
    return _map2("lbo_dlog_kv", v, x)


def vmf_log_norm(kappa, p: float, lib=None):
    """log C_p(kappa) of the von Mises-Fisher density."""
    k = np.ascontiguousarray(kappa, dtype=np.float64).ravel()
    hi = np.empty_like(k)
    lo = np.empty_like(k)
    (lib or _load()).lbo_vmf_log_norm(_ptr(k), float(p), _ptr(hi), _ptr(lo), k.size)
    return hi, lo


def max_threads() -> int:
    return int(_load().lbo_max_threads())


def set_threads(n: int) -> None:
    _load().lbo_set_threads(int(n))
