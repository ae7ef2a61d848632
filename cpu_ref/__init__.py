"""CPU FMM reference (3D Laplace single layer), the host-core baseline that
bench.py times beside the GPU path: the same method and tolerance in plain
C++ with OpenMP (fmm3d_laplace.cpp).  It builds its tree and lists through the
library's host planning entry points (cfmm_htree_*), so it needs libcfmm.so;
it runs no GPU code."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_SO = os.path.join(_HERE, "libcpufmm.so")
_SRC = os.path.join(_HERE, "fmm3d_laplace.cpp")
_LIBDIR = os.path.join(_ROOT, "paper_2509_05458_amd")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O3", "-mavx2", "-mfma", "-fcx-limited-range", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
                               "-o", tmp, _SRC, f"-L{_LIBDIR}", "-lcfmm", "-Wl,-rpath,$ORIGIN/../paper_2509_05458_amd"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.cpu_fmm3d_laplace.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                          dp, ctypes.c_int, dp]
        lib.cpu_fmm3d_laplace.restype = ctypes.c_int
        _lib = lib
    return _lib


def fmm3d_laplace(points, sigma, tol, leaf_size=256, sep=2, nthreads=0):
    """u_i = sum_{j != i} sigma_j / (4 pi r_ij) by the CPU FMM; returns (u, (plan_s, eval_s))."""
    lib = _load()
    pts = np.ascontiguousarray(points, dtype=np.complex128)
    sig = np.ascontiguousarray(sigma, dtype=np.complex128)
    u = np.empty(pts.shape[0], dtype=np.complex128)
    tm = np.zeros(2)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.cpu_fmm3d_laplace(pts.shape[0], pts.ctypes.data_as(dp), sig.ctypes.data_as(dp), float(tol),
                               int(leaf_size), int(sep), u.ctypes.data_as(dp), int(nthreads),
                               tm.ctypes.data_as(dp))
    if rc != 0:
        raise RuntimeError(f"cpu_fmm3d_laplace failed ({rc})")
    return u, (float(tm[0]), float(tm[1]))
