"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct CPU implementation of what the complex-
coordinate FMM computes, used to check the HIP library:

* ``direct``   : FP64 direct sum u_i = sum_j G(x_i, y_j) sigma_j with the
                 principal complexified distance (oracle.c);
* ``layer3``   : the 3D layer potentials with charges and dipoles (single
                 and double layer) and their gradients at the targets;
* ``tree``     : the adaptive tree on the real parts and Lists 1-4 (tree.py),
                 the integer result the library's tree must reproduce bit for bit.

Only tests/, ``__graft_entry__.smoke()`` and bench.py's ``cpu_baseline`` leg
may import this package.  It shares no code with the library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

LAPLACE = 0
HELMHOLTZ = 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-std=c11", "-o", tmp, _SRC, "-lm"])
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
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_direct.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int64, dp, ctypes.c_int64, dp, dp, lp,
                                      dp, ctypes.c_int]
        lib.oracle_direct.restype = ctypes.c_int
        lib.oracle_hankel0.argtypes = [ctypes.c_int64, dp, dp]
        lib.oracle_hankel0.restype = None
        lib.oracle_green.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int64, dp, dp]
        lib.oracle_green.restype = None
        lib.oracle_layer3.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, ctypes.c_int64, dp,
                                      dp, dp, lp, dp, dp, ctypes.c_int]
        lib.oracle_layer3.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def kernel_code(kernel: str) -> int:
    return {"laplace": LAPLACE, "helmholtz": HELMHOLTZ}[kernel]


def direct(dim: int, kernel: str, kappa: float, trg: np.ndarray, src: np.ndarray,
           sigma: np.ndarray, self_idx: np.ndarray | None = None,
           nthreads: int = 0) -> np.ndarray:
    """u_i = sum_j G(trg_i, src_j) sigma_j, skipping j == self_idx[i]."""
    lib = _load()
    trg = np.ascontiguousarray(trg, dtype=np.complex128).reshape(-1, dim)
    src = np.ascontiguousarray(src, dtype=np.complex128).reshape(-1, dim)
    sig = np.ascontiguousarray(sigma, dtype=np.complex128).reshape(-1)
    assert sig.shape[0] == src.shape[0]
    out = np.empty(trg.shape[0], dtype=np.complex128)
    sp = None
    if self_idx is not None:
        si = np.ascontiguousarray(self_idx, dtype=np.int64).reshape(-1)
        assert si.shape[0] == trg.shape[0]
        sp = si.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = lib.oracle_direct(dim, kernel_code(kernel), float(kappa), trg.shape[0], _dptr(trg),
                           src.shape[0], _dptr(src), _dptr(sig), sp, _dptr(out), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_direct: invalid arguments")
    return out


def layer3(kernel: str, kappa: float, trg: np.ndarray, src: np.ndarray, charge=None, dipole=None,
           self_idx=None, nthreads: int = 0):
    """3D layer potentials (oracle.c, oracle_layer3): with dipole vectors
    v_j = tau_j nu_j,  u_i = sum_j G sigma_j + v_j . grad_y G,  g_i = grad_x u_i.
    Returns (u [n_trg], g [n_trg, 3])."""
    lib = _load()
    trg = np.ascontiguousarray(trg, dtype=np.complex128).reshape(-1, 3)
    src = np.ascontiguousarray(src, dtype=np.complex128).reshape(-1, 3)
    ns = src.shape[0]
    q = None if charge is None else np.ascontiguousarray(charge, dtype=np.complex128).reshape(ns)
    v = None if dipole is None else np.ascontiguousarray(dipole, dtype=np.complex128).reshape(ns, 3)
    u = np.empty(trg.shape[0], dtype=np.complex128)
    g = np.empty((trg.shape[0], 3), dtype=np.complex128)
    sp = None
    if self_idx is not None:
        si = np.ascontiguousarray(self_idx, dtype=np.int64).reshape(-1)
        sp = si.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = lib.oracle_layer3(kernel_code(kernel), float(kappa), trg.shape[0], _dptr(trg), ns, _dptr(src),
                           None if q is None else _dptr(q), None if v is None else _dptr(v), sp,
                           _dptr(u), _dptr(g), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_layer3: invalid arguments")
    return u, g


def layer3_self(kernel, kappa, pts, charge=None, dipole=None, targets=None, nthreads=0):
    """layer3 with targets = sources (self term left out), optionally at `targets`."""
    pts = np.ascontiguousarray(pts, dtype=np.complex128)
    if targets is None:
        targets = np.arange(pts.shape[0], dtype=np.int64)
    targets = np.asarray(targets, dtype=np.int64)
    return layer3(kernel, kappa, pts[targets], pts, charge, dipole, targets, nthreads)


def direct_self(dim, kernel, kappa, pts, sigma, targets=None, nthreads=0):
    """Targets = sources (self term excluded); optionally only at indices `targets`."""
    pts = np.ascontiguousarray(pts, dtype=np.complex128)
    if targets is None:
        targets = np.arange(pts.shape[0], dtype=np.int64)
    targets = np.asarray(targets, dtype=np.int64)
    return direct(dim, kernel, kappa, pts[targets], pts, sigma, targets, nthreads)


def hankel0(z) -> np.ndarray:
    """The oracle's own H0^(1)(z), elementwise."""
    lib = _load()
    z = np.ascontiguousarray(z, dtype=np.complex128).reshape(-1)
    out = np.empty_like(z)
    lib.oracle_hankel0(z.shape[0], _dptr(z), _dptr(out))
    return out


def green(dim: int, kernel: str, kappa: float, s) -> np.ndarray:
    """G as a function of the squared complex distance s, elementwise."""
    lib = _load()
    s = np.ascontiguousarray(s, dtype=np.complex128).reshape(-1)
    out = np.empty_like(s)
    lib.oracle_green(dim, kernel_code(kernel), float(kappa), s.shape[0], _dptr(s), _dptr(out))
    return out


def rel_l2(u, u0) -> float:
    """||u - u0||_2 / ||u0||_2, the gate metric."""
    u = np.asarray(u)
    u0 = np.asarray(u0)
    return float(np.linalg.norm(u - u0) / np.linalg.norm(u0))


def rel_paper(u, u0, sigma) -> float:
    """||u - u0|| / (||u0|| + ||sigma||), the error measure of the timing tests (Sec. 7.1)."""
    return float(np.linalg.norm(np.asarray(u) - np.asarray(u0)) /
                 (np.linalg.norm(u0) + np.linalg.norm(sigma)))
