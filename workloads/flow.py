"""ctypes binding of the FP64 flow solve in ``flow.c`` (input generation only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flow.c")
_LIB = os.path.join(_HERE, "_flow.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile flow.c with gcc into workloads/_flow.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        lib.flow_solve.argtypes = [i, i, i, d, d, d, p, d, d, d, p, d, i, i, p, p, p, p,
                                   ctypes.POINTER(d), ctypes.POINTER(i)]
        lib.flow_solve.restype = i
        _lib = lib
    return _lib


def solve(K: np.ndarray, dx: float, dy: float, dz: float, h_west: float, h_east: float,
          recharge: float = 0.0, source: np.ndarray | None = None, rtol: float = 1e-12,
          max_iter: int = 200000, nthreads: int = 0):
    """Solve for heads and face flows.

    Returns (head[nz,ny,nx], qx[nz,ny,nx+1], qy[nz,ny+1,nx], qz[nz+1,ny,nx], relres, iters).
    """
    lib = _load()
    K = np.ascontiguousarray(K, dtype=np.float64)
    nz, ny, nx = K.shape
    head = np.empty((nz, ny, nx))
    qx = np.empty((nz, ny, nx + 1))
    qy = np.empty((nz, ny + 1, nx))
    qz = np.empty((nz + 1, ny, nx))
    src = None
    if source is not None:
        src = np.ascontiguousarray(source, dtype=np.float64)
        assert src.shape == K.shape
    rel = ctypes.c_double(0.0)
    its = ctypes.c_int(0)
    rc = lib.flow_solve(nx, ny, nz, dx, dy, dz, K.ctypes.data, h_west, h_east, recharge,
                        None if src is None else src.ctypes.data, rtol, max_iter, nthreads,
                        head.ctypes.data, qx.ctypes.data, qy.ctypes.data, qz.ctypes.data,
                        ctypes.byref(rel), ctypes.byref(its))
    if rc < 0:
        raise ValueError("flow_solve: bad input")
    if rc > 0:
        raise RuntimeError("flow_solve did not converge: relres %.3e after %d iterations"
                           % (rel.value, its.value))
    return head, qx, qy, qz, rel.value, its.value


def cell_balance(qx, qy, qz, source=None):
    """Per-cell net inflow (in - out + source), m^3/d, and the per-cell gross flow sum."""
    net = (qx[:, :, :-1] - qx[:, :, 1:]) + (qy[:, :-1, :] - qy[:, 1:, :]) + (qz[:-1] - qz[1:])
    if source is not None:
        net = net + source
    gross = (np.abs(qx[:, :, :-1]) + np.abs(qx[:, :, 1:]) + np.abs(qy[:, :-1, :]) +
             np.abs(qy[:, 1:, :]) + np.abs(qz[:-1]) + np.abs(qz[1:]))
    return net, gross
