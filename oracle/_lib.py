"""Loader for the C part of the oracle (``hsad_oracle.c``).

Test infrastructure only: the product path never imports this package.  The shared
object is compiled with the system C compiler, without fast-math, into this directory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsad_oracle.c")
_SO = os.path.join(_HERE, "libhsad_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE semantics: no fast-math)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


_d = ctypes.POINTER(ctypes.c_double)
_f = ctypes.POINTER(ctypes.c_float)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_SO)
            L.orc_dwt_out_len.restype = ctypes.c_int64
            L.orc_dwt_out_len.argtypes = [ctypes.c_int64, ctypes.c_int]
            L.orc_dwt_level.restype = None
            L.orc_dwt_level.argtypes = [_d, ctypes.c_int64, _d, ctypes.c_int, _d, _d]
            L.orc_dwt_approx.restype = ctypes.c_int64
            L.orc_dwt_approx.argtypes = [_f, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _d,
                                         ctypes.c_int, _d]
            L.orc_dwt_full_len.restype = ctypes.c_int64
            L.orc_dwt_full_len.argtypes = [ctypes.c_int64, ctypes.c_int]
            L.orc_dwt_full_cube.restype = ctypes.c_int64
            L.orc_dwt_full_cube.argtypes = [_f, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _d,
                                            ctypes.c_int, _d]
            L.orc_idwt_full_cube.restype = ctypes.c_int
            L.orc_idwt_full_cube.argtypes = [_f, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _d,
                                             ctypes.c_int, _d]
            L.orc_global_rx.restype = None
            L.orc_global_rx.argtypes = [_d, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, _i64,
                                        ctypes.c_int64, _d, _d, _d]
            L.orc_dwt_full.restype = ctypes.c_int
            L.orc_dwt_full.argtypes = [_d, ctypes.c_int64, ctypes.c_int, _d, ctypes.c_int, _d]
            L.orc_idwt_full.restype = ctypes.c_int
            L.orc_idwt_full.argtypes = [_d, ctypes.c_int64, ctypes.c_int, _d, ctypes.c_int, _d]
            L.orc_window_stats.restype = None
            L.orc_window_stats.argtypes = [_d, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                           ctypes.c_int64, _d, _d, _d, _d, _i64]
            L.orc_loading.restype = ctypes.c_double
            L.orc_loading.argtypes = [_d, ctypes.c_int64, ctypes.c_double]
            L.orc_cholesky.restype = ctypes.c_int
            L.orc_cholesky.argtypes = [_d, ctypes.c_int64]
            L.orc_lrx_dwrx.restype = None
            L.orc_lrx_dwrx.argtypes = [_d, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_double, _i64,
                                       ctypes.c_int64, _d, _d]
            L.orc_round_samples.restype = None
            L.orc_round_samples.argtypes = [_d, ctypes.c_int64, ctypes.c_int, _d]
            L.orc_lrx_dwrx_rounded.restype = None
            L.orc_lrx_dwrx_rounded.argtypes = [_d, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                               ctypes.c_int, ctypes.c_int, ctypes.c_double, _i64,
                                               ctypes.c_int64, _d, _d, ctypes.c_int]
            L.orc_jacobi_eig.restype = ctypes.c_int
            L.orc_jacobi_eig.argtypes = [ctypes.c_int64, _d, _d, _d, ctypes.c_double,
                                         ctypes.c_int]
            L.orc_dwest.restype = None
            L.orc_dwest.argtypes = [_d, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int, ctypes.c_int, _i64, ctypes.c_int64, _d, _d,
                                    _i32]
            L.orc_set_threads.restype = None
            L.orc_set_threads.argtypes = [ctypes.c_int]
            L.orc_max_threads.restype = ctypes.c_int
            L.orc_max_threads.argtypes = []
            _lib = L
    return _lib


def ptr(a: np.ndarray | None, ctype):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ctype))
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def set_threads(n: int | None) -> int:
    """OpenMP thread count for subsequent oracle calls; returns the count in effect."""
    L = lib()
    if n is not None:
        L.orc_set_threads(int(n))
    return int(L.orc_max_threads())
