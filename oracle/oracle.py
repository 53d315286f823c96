"""ORACLE -- test infrastructure, not part of the product.

ctypes front end of the plain FP64 CPU tracker in ``pt_oracle.c``.  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It shares nothing with the HIP library; inputs come from the
seeded generators in ``workloads``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pt_oracle.c")
_LIB = os.path.join(_HERE, "_pt_oracle.so")
_lib = None

STATUS = {0: "ACTIVE", 1: "BOUNDARY", 2: "SINK", 3: "MAX_TIME", 4: "STEP_CAP", 5: "STRANDED",
          6: "INVALID_START", 7: "INACTIVE_NEIGHBOR"}
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast math)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + CFLAGS + ["-o", tmp, src, "-lquadmath", "-lm"])
        os.replace(tmp, out)
    return out


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("qx", ctypes.c_void_p), ("qy", ctypes.c_void_p), ("qz", ctypes.c_void_p),
                ("porosity", ctypes.c_void_p), ("porosity_scalar", ctypes.c_double),
                ("flags", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("t_max", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("stop_at_sink", ctypes.c_int32),
                ("snap_times", ctypes.c_void_p), ("n_snap", ctypes.c_int32),
                ("snap_xyz", ctypes.c_void_p), ("out_xyz", ctypes.c_void_p),
                ("path_cap", ctypes.c_int32), ("path_cell", ctypes.c_void_p),
                ("path_face", ctypes.c_void_p), ("path_t", ctypes.c_void_p),
                ("path_xyz", ctypes.c_void_p), ("n_threads", ctypes.c_int32)]


class _Quad(ctypes.Structure):
    _fields_ = [("ncell", ctypes.c_int32), ("box", ctypes.c_void_p), ("sub_off", ctypes.c_void_p),
                ("sub_nb", ctypes.c_void_p), ("sub_q", ctypes.c_void_p), ("sub_lo", ctypes.c_void_p),
                ("sub_hi", ctypes.c_void_p), ("porosity", ctypes.c_void_p),
                ("porosity_scalar", ctypes.c_double), ("flags", ctypes.c_void_p)]


def load(path: str = _LIB):
    """Load (building if absent) an oracle shared library; returns the ctypes handle."""
    global _lib
    if path == _LIB and _lib is not None:
        return _lib
    if not os.path.exists(path):
        build(force=False, out=path)
    lib = ctypes.CDLL(path)
    p = ctypes.c_void_p
    lib.oracle_track.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Opts), ctypes.c_int64,
                                 p, p, p, p, p, p, p, p]
    lib.oracle_track.restype = ctypes.c_int
    lib.oracle_track_transient.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int32, p, ctypes.POINTER(_Opts),
                                           ctypes.c_int64, p, p, p, p, p, p, p, p]
    lib.oracle_track_transient.restype = ctypes.c_int
    lib.oracle_track_quad.argtypes = [ctypes.POINTER(_Quad), ctypes.POINTER(_Opts), ctypes.c_int64,
                                      p, p, p, p, p, p, p, p]
    lib.oracle_track_quad.restype = ctypes.c_int
    if path == _LIB:
        _lib = lib
    return lib


@dataclasses.dataclass
class Result:
    cell: np.ndarray
    xi: np.ndarray
    eta: np.ndarray
    zeta: np.ndarray
    t: np.ndarray
    status: np.ndarray
    ncross: np.ndarray
    path_hash: np.ndarray
    out_xyz: np.ndarray
    snap_xyz: np.ndarray | None = None
    path_cell: np.ndarray | None = None
    path_face: np.ndarray | None = None
    path_t: np.ndarray | None = None
    path_xyz: np.ndarray | None = None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def track(grid, particles, *, direction: int = 1, t_max: float = math.inf,
          max_steps: int = 1 << 20, stop_at_sink: int = 1, snap_times=None, snap_init=None,
          threads: int = 0, path_cap: int = 0, lib=None) -> Result:
    """Track a copy of ``particles`` through ``grid``; returns the final state and outputs.

    ``threads`` OpenMP threads over the particle loop (0: all available cores, at most 16).

    ``snap_init`` (optional [n, n_snap, 3]) is the snapshot buffer before the call,
    which matters only for resumed particles.
    """
    return _run([grid], None, particles, direction=direction, t_max=t_max, max_steps=max_steps,
                stop_at_sink=stop_at_sink, snap_times=snap_times, snap_init=snap_init, threads=threads,
                path_cap=path_cap, lib=lib)


def track_transient(grids, step_end, particles, **kw) -> Result:
    """Transient flow: grids[s] holds the face flows of time step s up to step_end[s]
    (strictly increasing; the last may be inf).  Same keywords as track (forward only)."""
    se = _c(step_end, np.float64)
    assert len(grids) == se.shape[0] >= 1
    return _run(list(grids), se, particles, **kw)


def track_quad(qgrid, particles, **kw) -> Result:
    """Track through a quadtree grid (workloads.quadtree.QuadGrid); same keywords as track."""
    return _run([qgrid], None, particles, quad=True, **kw)


def _run(grid_list, step_end, particles, *, direction: int = 1, t_max: float = math.inf,
         max_steps: int = 1 << 20, stop_at_sink: int = 1, snap_times=None, snap_init=None,
         threads: int = 0, path_cap: int = 0, lib=None, quad: bool = False) -> Result:
    lib = lib or load()
    if threads <= 0:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
    keep = []
    cgs = (_Grid * len(grid_list))()
    cq = None
    if quad:
        g = grid_list[0]
        arrs = [_c(g.box, np.float64), _c(g.sub_off, np.int32), _c(g.sub_nb, np.int32), _c(g.sub_q, np.float64),
                _c(g.sub_lo, np.float64), _c(g.sub_hi, np.float64),
                None if g.porosity is None else _c(g.porosity, np.float64), _c(g.flags, np.int32)]
        keep += arrs
        ptrs = [None if a is None else a.ctypes.data for a in arrs]
        cq = _Quad(g.ncell, *ptrs[:7], g.porosity_scalar, ptrs[7])
        grid_list = []
    for q, g in enumerate(grid_list):
        qx, qy, qz = _c(g.qx, np.float64), _c(g.qy, np.float64), _c(g.qz, np.float64)
        flags = _c(g.flags, np.int32)
        por = None if g.porosity is None else _c(g.porosity, np.float64)
        keep += [qx, qy, qz, flags, por]
        cgs[q] = _Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.x0, g.y0, g.z0, qx.ctypes.data, qy.ctypes.data,
                       qz.ctypes.data, None if por is None else por.ctypes.data, g.porosity_scalar,
                       flags.ctypes.data)
    n = particles.n
    st = [_c(particles.cell, np.int32).copy(), _c(particles.xi, np.float64).copy(),
          _c(particles.eta, np.float64).copy(), _c(particles.zeta, np.float64).copy(),
          _c(particles.t, np.float64).copy(), _c(particles.status, np.int32).copy(),
          _c(particles.ncross, np.int32).copy(), _c(particles.path_hash, np.uint64).copy()]
    out_xyz = np.empty((n, 3))
    snaps = None
    sn = None
    n_snap = 0
    if snap_times is not None:
        sn = _c(snap_times, np.float64)
        n_snap = sn.shape[0]
        snaps = np.full((n, n_snap, 3), np.nan) if snap_init is None else _c(snap_init, np.float64).copy()
    pc = pf = pt = px = None
    if path_cap > 0:
        pc = np.full((n, path_cap), -1, np.int32)
        pf = np.full((n, path_cap), -1, np.int32)
        pt = np.full((n, path_cap), np.nan)
        px = np.full((n, path_cap, 3), np.nan)
    o = _Opts(direction, t_max, max_steps, stop_at_sink, None if sn is None else sn.ctypes.data,
              n_snap, None if snaps is None else snaps.ctypes.data, out_xyz.ctypes.data, path_cap,
              None if pc is None else pc.ctypes.data, None if pf is None else pf.ctypes.data,
              None if pt is None else pt.ctypes.data, None if px is None else px.ctypes.data,
              threads)
    if cq is not None:
        rc = lib.oracle_track_quad(ctypes.byref(cq), ctypes.byref(o), n, *(a.ctypes.data for a in st))
    elif step_end is None:
        rc = lib.oracle_track(ctypes.byref(cgs[0]), ctypes.byref(o), n, *(a.ctypes.data for a in st))
    else:
        rc = lib.oracle_track_transient(cgs, len(grid_list), step_end.ctypes.data, ctypes.byref(o), n,
                                        *(a.ctypes.data for a in st))
    if rc != 0:
        raise ValueError("the oracle rejected its arguments")
    return Result(*st, out_xyz, snaps, pc, pf, pt, px)


def track_groups(grids, particles, group_offsets, group_grid, **kw) -> Result:
    """Several particle groups, group g tracked through grids[group_grid[g]]."""
    parts = []
    for g in range(len(group_grid)):
        lo, hi = int(group_offsets[g]), int(group_offsets[g + 1])
        parts.append(track(grids[int(group_grid[g])], particles.subset(slice(lo, hi)), **kw))
    fields = [f.name for f in dataclasses.fields(Result)]
    vals = []
    for f in fields:
        xs = [getattr(r, f) for r in parts]
        vals.append(None if xs[0] is None else np.concatenate(xs))
    return Result(*vals)
