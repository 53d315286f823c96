"""Python binding of libpt (the C ABI in include/pt.h): argument marshalling only.

Every tracking step runs in the HIP kernels of libpt.so; this module converts
arguments and owns nothing but torch tensors for device memory.  It raises
ImportError when libpt.so has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import dataclasses
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch  # loads the HIP runtime that libpt shares with torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpt.so")

PT_OK = 0
ERR_NAMES = {-1: "PT_ERR_INVALID_ARG", -2: "PT_ERR_BAD_HANDLE", -3: "PT_ERR_OOM", -4: "PT_ERR_NO_DEVICE",
             -5: "PT_ERR_DEVICE", -6: "PT_ERR_UNBALANCED", -7: "PT_ERR_UNSUPPORTED"}
STATUS_NAMES = ["ACTIVE", "BOUNDARY", "SINK", "MAX_TIME", "STEP_CAP", "STRANDED", "INVALID_START",
                "INACTIVE_NEIGHBOR"]
PT_MEM_HOST, PT_MEM_DEVICE = 0, 1
PT_ENDPOINT, PT_TIMESERIES, PT_PATHLINE = 0, 1, 2
PT_FP64, PT_MIXED = 0, 1
PT_SCHED_AUTO, PT_SCHED_STATIC, PT_SCHED_PERSISTENT = 0, 1, 2
PT_LAYOUT_AUTO, PT_LAYOUT_FACES, PT_LAYOUT_CELL = 0, 1, 2
PT_SORT_AUTO, PT_SORT_NONE, PT_SORT_CELL = 0, 1, 2
FNV_OFFSET = 0xCBF29CE484222325

_p = ctypes.c_void_p


class pt_grid_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("qx", _p), ("qy", _p), ("qz", _p), ("porosity", _p),
                ("porosity_scalar", ctypes.c_double), ("flags", _p), ("mem", ctypes.c_int32),
                ("balance_tol", ctypes.c_double)]


class pt_quad_desc(ctypes.Structure):
    _fields_ = [("ncell", ctypes.c_int32), ("nsub", ctypes.c_int32), ("box", _p), ("sub_off", _p),
                ("sub_nb", _p), ("sub_q", _p), ("sub_lo", _p), ("sub_hi", _p), ("porosity", _p),
                ("porosity_scalar", ctypes.c_double), ("flags", _p), ("mem", ctypes.c_int32),
                ("balance_tol", ctypes.c_double)]


class pt_particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cell", _p), ("xi", _p), ("eta", _p), ("zeta", _p), ("t", _p),
                ("status", _p), ("ncross", _p), ("path_hash", _p), ("n_groups", ctypes.c_int32),
                ("group_offsets", _p), ("group_grid", _p)]


class pt_track_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("precision", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("direction", ctypes.c_int32),
                ("stop_at_sink", ctypes.c_int32), ("t_max", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("snap_times", _p), ("n_snap", ctypes.c_int32),
                ("snap_xyz", _p), ("out_xyz", _p), ("use_graph", ctypes.c_int32),
                ("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("refill", ctypes.c_int32), ("steps_per_refill", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("sort", ctypes.c_int32),
                ("path_offsets", _p), ("path_count_only", ctypes.c_int32), ("path_cap", ctypes.c_int64),
                ("path_records", _p), ("n_tsteps", ctypes.c_int32), ("tstep_end", _p)]


class pt_path_record(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double),
                ("cell", ctypes.c_int32), ("face", ctypes.c_int32)]


# host view of pt_path_record arrays
PATH_RECORD_DTYPE = np.dtype([("t", "<f8"), ("x", "<f8"), ("y", "<f8"), ("z", "<f8"), ("cell", "<i4"),
                              ("face", "<i4")])


class pt_summary(ctypes.Structure):
    _fields_ = [("crossings", ctypes.c_int64), ("n_tracked", ctypes.c_int64),
                ("status_count", ctypes.c_int64 * 8), ("kernel_ms", ctypes.c_double),
                ("schedule", ctypes.c_int32), ("layout", ctypes.c_int32), ("block", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("cr_ambiguous", ctypes.c_int64),
                ("path_records", ctypes.c_int64), ("path_dropped", ctypes.c_int64),
                ("recheck_tracks", ctypes.c_int64), ("track_ms", ctypes.c_double)]


EXPORTS = ["pt_load_grid", "pt_load_quad_grid", "pt_track", "pt_track_noalloc", "pt_results", "pt_release",
           "pt_shutdown", "pt_last_error", "pt_default_opts", "pt_version"]
# pt_track_noalloc: its counts array (int64 words) and their meaning
PT_NOALLOC_SCRATCH_BYTES = 32 << 20
PT_COUNTS_WORDS = 16
PT_COUNT_CROSSINGS, PT_COUNT_TRACKED, PT_COUNT_STATUS = 0, 1, 2
PT_COUNT_CR_AMBIGUOUS, PT_COUNT_PATH_RECORDS, PT_COUNT_PATH_DROPPED = 10, 11, 12
PT_COUNT_RECHECK_TRACKS = 13

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpt.so (built by ``python -m paper_2302_13590_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libpt.so is not built (%s); run: python -m paper_2302_13590_amd.build" % path)
    lib = ctypes.CDLL(path)
    lib.pt_load_grid.argtypes = [ctypes.POINTER(pt_grid_desc), _p, ctypes.POINTER(_p)]
    lib.pt_load_grid.restype = ctypes.c_int
    lib.pt_load_quad_grid.argtypes = [ctypes.POINTER(pt_quad_desc), _p, ctypes.POINTER(_p)]
    lib.pt_load_quad_grid.restype = ctypes.c_int
    lib.pt_track.argtypes = [ctypes.POINTER(_p), ctypes.c_int32, ctypes.POINTER(pt_particles),
                             ctypes.POINTER(pt_track_opts), _p, ctypes.POINTER(_p)]
    lib.pt_track.restype = ctypes.c_int
    lib.pt_track_noalloc.argtypes = [ctypes.POINTER(_p), ctypes.c_int32, ctypes.POINTER(pt_particles),
                                     ctypes.POINTER(pt_track_opts), _p, _p]
    lib.pt_track_noalloc.restype = ctypes.c_int
    lib.pt_results.argtypes = [_p, ctypes.POINTER(pt_summary)]
    lib.pt_results.restype = ctypes.c_int
    lib.pt_release.argtypes = [_p]
    lib.pt_release.restype = ctypes.c_int
    lib.pt_last_error.argtypes = []
    lib.pt_last_error.restype = ctypes.c_char_p
    lib.pt_default_opts.argtypes = [ctypes.POINTER(pt_track_opts)]
    lib.pt_default_opts.restype = None
    lib.pt_version.argtypes = []
    lib.pt_version.restype = ctypes.c_int
    lib.pt_shutdown.argtypes = []
    lib.pt_shutdown.restype = ctypes.c_int
    _lib = lib
    # every graph, event and buffer of the library is released before interpreter and HIP
    # runtime teardown (atexit handlers run before the C++ static destructors at exit)
    atexit.register(pt_shutdown)
    return lib


class PtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (ERR_NAMES.get(code, str(code)), msg))
        self.code = code


def _check(rc: int):
    if rc != PT_OK:
        raise PtError(rc, pt_last_error())


def pt_last_error() -> str:
    return load_library().pt_last_error().decode()


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# --------------------------------------------------------------------------------------------- grid

class Grid:
    """Handle of a flow field loaded with pt_load_grid."""

    def __init__(self, handle: int, nx: int, ny: int, nz: int):
        self.handle = handle
        self.shape = (nz, ny, nx)

    def release(self):
        if self.handle:
            pt_release(self.handle)
            self.handle = None


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.data_ptr()
    return a.ctypes.data


def pt_load_grid(grid, stream=None, balance_tol: float = -1.0) -> Grid:
    """Load a grid (an object with nx, ny, nz, dx.., x0.., qx, qy, qz, flags, porosity,
    porosity_scalar; numpy arrays -> host copy, CUDA tensors -> device copy)."""
    lib = load_library()
    arrs = [grid.qx, grid.qy, grid.qz, grid.porosity, grid.flags]
    dev = any(isinstance(a, torch.Tensor) and a.is_cuda for a in arrs if a is not None)
    keep = []

    def conv(a, dtype):
        if a is None:
            return None
        if isinstance(a, torch.Tensor):
            a = a.contiguous()
        else:
            a = np.ascontiguousarray(a, dtype=dtype)
        keep.append(a)
        return _ptr(a)

    d = pt_grid_desc(grid.nx, grid.ny, grid.nz, grid.dx, grid.dy, grid.dz, grid.x0, grid.y0, grid.z0,
                     conv(grid.qx, np.float64), conv(grid.qy, np.float64), conv(grid.qz, np.float64),
                     conv(grid.porosity, np.float64), grid.porosity_scalar, conv(grid.flags, np.int32),
                     PT_MEM_DEVICE if dev else PT_MEM_HOST, balance_tol)
    out = _p()
    _check(lib.pt_load_grid(ctypes.byref(d), _stream_ptr(stream), ctypes.byref(out)))
    return Grid(out.value, grid.nx, grid.ny, grid.nz)


def pt_load_quad_grid(q, stream=None, balance_tol: float = -1.0) -> Grid:
    """Load a quadtree grid (an object with ncell, box, sub_off, sub_nb, sub_q, sub_lo, sub_hi,
    flags, porosity, porosity_scalar as numpy arrays, e.g. workloads.quadtree.QuadGrid)."""
    lib = load_library()
    keep = []

    def conv(a, dtype):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        keep.append(a)
        return a.ctypes.data

    d = pt_quad_desc(q.ncell, int(q.sub_nb.shape[0]), conv(q.box, np.float64), conv(q.sub_off, np.int32),
                     conv(q.sub_nb, np.int32), conv(q.sub_q, np.float64), conv(q.sub_lo, np.float64),
                     conv(q.sub_hi, np.float64), conv(q.porosity, np.float64), q.porosity_scalar,
                     conv(q.flags, np.int32), PT_MEM_HOST, balance_tol)
    out = _p()
    _check(lib.pt_load_quad_grid(ctypes.byref(d), _stream_ptr(stream), ctypes.byref(out)))
    return Grid(out.value, q.ncell, 1, 1)


def load_any_grid(g, stream=None, balance_tol: float = -1.0) -> Grid:
    """pt_load_quad_grid for quadtree grids (objects with sub_off), pt_load_grid otherwise."""
    if hasattr(g, "sub_off"):
        return pt_load_quad_grid(g, stream, balance_tol)
    return pt_load_grid(g, stream, balance_tol)


def pt_shutdown() -> None:
    """Release every grid, run and cached resource of the library (see pt.h); earlier handles
    become invalid.  Registered with atexit when the library is loaded."""
    if _lib is None:
        return
    _check(_lib.pt_shutdown())


def pt_release(handle) -> None:
    if isinstance(handle, (Grid, Run)):
        h = handle.handle
        handle.handle = None
    else:
        h = handle
    _check(load_library().pt_release(h))


# --------------------------------------------------------------------------------------------- particles

@dataclasses.dataclass
class DeviceParticles:
    """Particle state as device tensors (the caller-owned in/out arrays of pt_particles)."""
    cell: torch.Tensor
    xi: torch.Tensor
    eta: torch.Tensor
    zeta: torch.Tensor
    t: torch.Tensor
    status: torch.Tensor
    ncross: torch.Tensor
    path_hash: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.cell.shape[0])

    @staticmethod
    def from_numpy(p, device="cuda") -> "DeviceParticles":
        def T(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(device)
        return DeviceParticles(T(p.cell, np.int32), T(p.xi, np.float64), T(p.eta, np.float64),
                               T(p.zeta, np.float64), T(p.t, np.float64), T(p.status, np.int32),
                               T(p.ncross, np.int32), T(np.asarray(p.path_hash, np.uint64), np.int64))

    def copy_(self, other: "DeviceParticles") -> "DeviceParticles":
        for f in dataclasses.fields(self):
            getattr(self, f.name).copy_(getattr(other, f.name), non_blocking=True)
        return self

    def clone(self) -> "DeviceParticles":
        return DeviceParticles(*(getattr(self, f.name).clone() for f in dataclasses.fields(self)))

    def to_numpy(self) -> dict:
        out = {f.name: getattr(self, f.name).cpu().numpy() for f in dataclasses.fields(self)}
        out["path_hash"] = out["path_hash"].view(np.uint64)
        return out


class Run:
    def __init__(self, handle: int, keep):
        self.handle = handle
        self._keep = keep   # host arrays referenced by the call

    def release(self):
        if self.handle:
            pt_release(self.handle)
            self.handle = None


def pt_default_opts() -> pt_track_opts:
    o = pt_track_opts()
    load_library().pt_default_opts(ctypes.byref(o))
    return o


def make_opts(mode=PT_ENDPOINT, precision=PT_FP64, schedule=PT_SCHED_AUTO, layout=PT_LAYOUT_AUTO,
              direction=1, stop_at_sink=1, t_max=math.inf, max_steps=1 << 20, snap_times=None,
              snap_xyz=None, out_xyz=None, use_graph=0, block=0, blocks_per_cu=0, refill=0,
              steps_per_refill=0, chunk=0, sort=0, path_offsets=None, path_count_only=0, path_cap=0,
              path_records=None, tstep_end=None):
    o = pt_default_opts()
    o.mode, o.precision, o.schedule, o.layout = mode, precision, schedule, layout
    o.direction, o.stop_at_sink, o.t_max, o.max_steps = direction, stop_at_sink, t_max, max_steps
    keep = []
    if snap_times is not None:
        st = np.ascontiguousarray(snap_times, dtype=np.float64)
        keep.append(st)
        o.snap_times = st.ctypes.data
        o.n_snap = st.shape[0]
    o.snap_xyz = _ptr(snap_xyz)
    o.out_xyz = _ptr(out_xyz)
    o.use_graph, o.block, o.blocks_per_cu, o.refill, o.steps_per_refill, o.chunk, o.sort = (
        use_graph, block, blocks_per_cu, refill, steps_per_refill, chunk, sort)
    o.path_offsets, o.path_count_only, o.path_cap = _ptr(path_offsets), path_count_only, path_cap
    o.path_records = _ptr(path_records)
    if tstep_end is not None:
        te = np.ascontiguousarray(tstep_end, dtype=np.float64)
        keep.append(te)
        o.n_tsteps = te.shape[0]
        o.tstep_end = te.ctypes.data
    o._keep = keep
    return o


def _particles_arg(grids, particles, group_offsets, group_grid):
    handles = (_p * len(grids))(*[g.handle for g in grids])
    keep = [handles]
    pp = pt_particles()
    pp.n = particles.n
    for name in ("cell", "xi", "eta", "zeta", "t", "status", "ncross", "path_hash"):
        setattr(pp, name, getattr(particles, name).data_ptr())
    if group_offsets is not None:
        go = np.ascontiguousarray(group_offsets, dtype=np.int64)
        gg = np.ascontiguousarray(group_grid, dtype=np.int32)
        keep += [go, gg]
        pp.n_groups = gg.shape[0]
        pp.group_offsets = go.ctypes.data
        pp.group_grid = gg.ctypes.data
    return handles, pp, keep


def pt_track(grids: Sequence[Grid], particles: DeviceParticles, opts: pt_track_opts, stream=None,
             group_offsets=None, group_grid=None) -> Run:
    """Enqueue tracking; returns a Run (call pt_results, then pt_release)."""
    lib = load_library()
    handles, pp, keep = _particles_arg(grids, particles, group_offsets, group_grid)
    keep.append(opts)
    out = _p()
    _check(lib.pt_track(handles, len(grids), ctypes.byref(pp), ctypes.byref(opts), _stream_ptr(stream),
                        ctypes.byref(out)))
    return Run(out.value, keep)


def pt_track_noalloc(grids: Sequence[Grid], particles: DeviceParticles, opts: pt_track_opts,
                     counts: torch.Tensor, stream=None, group_offsets=None, group_grid=None) -> None:
    """Enqueue tracking with the library's per-device scratch (nothing is allocated); the run's
    counts go to `counts`, a device int64 tensor of PT_COUNTS_WORDS, once the stream reaches them."""
    assert counts.dtype == torch.int64 and counts.numel() >= PT_COUNTS_WORDS and counts.is_contiguous()
    lib = load_library()
    handles, pp, keep = _particles_arg(grids, particles, group_offsets, group_grid)
    _check(lib.pt_track_noalloc(handles, len(grids), ctypes.byref(pp), ctypes.byref(opts), _stream_ptr(stream),
                                counts.data_ptr()))


def counts_summary(counts) -> dict:
    """The fields of a pt_track_noalloc counts array (host copy) as in pt_results' summary."""
    c = [int(v) for v in (counts.cpu().tolist() if isinstance(counts, torch.Tensor) else counts)]
    return dict(crossings=c[PT_COUNT_CROSSINGS], n_tracked=c[PT_COUNT_TRACKED],
                status_count=c[PT_COUNT_STATUS:PT_COUNT_STATUS + 8], cr_ambiguous=c[PT_COUNT_CR_AMBIGUOUS],
                path_records=c[PT_COUNT_PATH_RECORDS], path_dropped=c[PT_COUNT_PATH_DROPPED],
                recheck_tracks=c[PT_COUNT_RECHECK_TRACKS])


def pt_results(run: Run) -> dict:
    s = pt_summary()
    _check(load_library().pt_results(run.handle, ctypes.byref(s)))
    return dict(crossings=s.crossings, n_tracked=s.n_tracked, status_count=list(s.status_count),
                kernel_ms=s.kernel_ms, schedule=s.schedule, layout=s.layout, block=s.block, grid=s.grid,
                cr_ambiguous=s.cr_ambiguous, path_records=s.path_records, path_dropped=s.path_dropped,
                recheck_tracks=s.recheck_tracks, track_ms=s.track_ms)


# --------------------------------------------------------------------------------------------- helper

def track(grids, particles: DeviceParticles, stream=None, group_offsets=None, group_grid=None,
          **opt) -> dict:
    """pt_track + pt_results + pt_release in one call; returns the summary."""
    o = make_opts(**opt)
    run = pt_track(grids, particles, o, stream=stream, group_offsets=group_offsets, group_grid=group_grid)
    try:
        return pt_results(run)
    finally:
        run.release()


def path_record_buffer(m: int, device="cuda") -> torch.Tensor:
    """Device storage for m pt_path_record (40 bytes each) as a float64 [m, 5] tensor."""
    return torch.empty((m, 5), dtype=torch.float64, device=device)


@dataclasses.dataclass
class Pathlines:
    """Pathline records in CSR form: those of particle p are rows offsets[p]:offsets[p+1] of
    `records` (pt_path_record: t, x, y, z, then cell and face as two int32 in column 4)."""
    offsets: torch.Tensor   # int64 [n+1]
    records: torch.Tensor   # float64 [m, 5]

    @property
    def t(self) -> torch.Tensor:
        return self.records[:, 0]

    @property
    def xyz(self) -> torch.Tensor:
        return self.records[:, 1:4]

    @property
    def cell(self) -> torch.Tensor:
        return self.records.view(torch.int32)[:, 8]

    @property
    def face(self) -> torch.Tensor:
        return self.records.view(torch.int32)[:, 9]

    def to_numpy(self):
        """(offsets, structured array of PATH_RECORD_DTYPE) on the host."""
        rec = np.ascontiguousarray(self.records.cpu().numpy()).view(PATH_RECORD_DTYPE).reshape(-1)
        return self.offsets.cpu().numpy(), rec


def track_pathlines(grids, particles: DeviceParticles, stream=None, group_offsets=None, group_grid=None,
                    **opt):
    """Pathline run: the count pass (offsets), a record buffer of the reported size, the record pass.

    Returns (summary of the record pass, Pathlines).  Both passes run in the library; this
    helper only allocates the output tensors between them."""
    dev = particles.cell.device
    offsets = torch.empty(particles.n + 1, dtype=torch.int64, device=dev)
    kw = dict(opt, mode=PT_PATHLINE, path_offsets=offsets)
    s0 = track(grids, particles, stream=stream, group_offsets=group_offsets, group_grid=group_grid,
               path_count_only=1, **kw)
    m = s0["path_records"]
    out = Pathlines(offsets, path_record_buffer(m, dev))
    s = track(grids, particles, stream=stream, group_offsets=group_offsets, group_grid=group_grid,
              path_count_only=0, path_cap=m, path_records=out.records, **kw)
    return s, out
