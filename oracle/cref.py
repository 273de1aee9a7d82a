"""Build and load the plain C + OpenMP twin of the oracle (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
use this module. ``build()`` compiles ``jacobi_ref.c`` with gcc into
``libjacobi_ref.so`` beside it; ``load()`` returns the ctypes handle, building
first when the library is missing.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "jacobi_ref.c")
LIB = os.path.join(_HERE, "libjacobi_ref.so")

_lib = None


def build() -> str:
    """Compile the C twin (gcc, -O2, OpenMP, no fused multiply-add)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    vp = ctypes.c_void_p
    lib.oracle_jacobi5_f64.argtypes = [vp, vp, vp, i64, i64, i32, ctypes.c_double, i32]
    lib.oracle_jacobi5_f64.restype = ctypes.c_int
    lib.oracle_jacobi5_f32.argtypes = [vp, vp, vp, i64, i64, i32, ctypes.c_float, i32]
    lib.oracle_jacobi5_f32.restype = ctypes.c_int
    lib.oracle_threads.argtypes = [i32]
    lib.oracle_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def jacobi5(u0: np.ndarray, T: int, c: float = 0.25, nthreads: int = 0) -> np.ndarray:
    """The C twin of ``oracle.jacobi.jacobi5`` (FP64 or FP32 by u0's dtype)."""
    lib = load()
    u0 = np.ascontiguousarray(u0)
    if u0.dtype == np.float64:
        fn = lib.oracle_jacobi5_f64
    elif u0.dtype == np.float32:
        fn = lib.oracle_jacobi5_f32
    else:
        raise TypeError("u0 must be float32 or float64")
    out = np.empty_like(u0)
    work = np.empty_like(u0)
    H, W = u0.shape
    rc = fn(u0.ctypes.data, out.ctypes.data, work.ctypes.data, H, W, T, c, nthreads)
    if rc != 0:
        raise ValueError("invalid arguments to the C oracle")
    return out


def threads(nthreads: int = 0) -> int:
    """Threads the C twin runs on after requesting `nthreads` (0 = OpenMP default)."""
    return int(load().oracle_threads(nthreads))
