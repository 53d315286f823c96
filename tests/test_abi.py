"""The C ABI on the CPU: library load, exported symbols, struct layouts, argument validation.

No compute call is made: every call here fails validation (or finds no device) before any
device work.
"""
import ctypes
import math
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2302_13590_amd import pt
from workloads import configs as C

from . import helpers as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pt.h")


def _gpu():
    import torch
    return torch.cuda.is_available()


@pytest.fixture(scope="module")
def lib():
    return pt.load_library()


def test_exports_every_declared_function(lib):
    src = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(pt_\w+)\s*\(", src, re.M))
    assert declared >= {"pt_load_grid", "pt_track", "pt_results", "pt_release", "pt_last_error"}
    out = subprocess.run(["nm", "-D", "--defined-only", pt.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (pt_\w+)$", out, re.M))
    assert declared <= exported, declared - exported
    for name in declared:
        assert hasattr(lib, name)
    assert set(pt.EXPORTS) == declared


def test_struct_layouts_match_binding():
    d = tempfile.mkdtemp(prefix="abi_")
    exe = os.path.join(d, "probe")
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", exe,
                           os.path.join(ROOT, "tests", "native", "abi_probe.c")])
    lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    c = {}
    for ln in lines:
        if ln:
            k, v = ln.split()
            c[k] = int(v)
    for T in (pt.pt_grid_desc, pt.pt_quad_desc, pt.pt_particles, pt.pt_track_opts, pt.pt_summary,
              pt.pt_path_record):
        assert ctypes.sizeof(T) == c[T.__name__ + ".sizeof"], T.__name__
        for name, _ in T._fields_:
            assert getattr(T, name).offset == c["%s.%s" % (T.__name__, name)], (T.__name__, name)


def test_path_record_host_dtype_matches_struct():
    assert pt.PATH_RECORD_DTYPE.itemsize == ctypes.sizeof(pt.pt_path_record) == 40
    for name, _ in pt.pt_path_record._fields_:
        assert pt.PATH_RECORD_DTYPE.fields[name][1] == getattr(pt.pt_path_record, name).offset, name


def test_version_and_defaults(lib):
    assert lib.pt_version() == 104
    o = pt.pt_default_opts()
    assert (o.mode, o.precision, o.schedule, o.layout) == (0, 0, 0, 0)
    assert o.direction == 1 and o.stop_at_sink == 1 and math.isinf(o.t_max) and o.max_steps == 1 << 20
    assert not o.path_offsets and o.path_count_only == 0 and o.path_cap == 0
    assert o.n_tsteps == 0 and not o.tstep_end


def _desc(g, **kw):
    keep = [np.ascontiguousarray(a) for a in (g.qx, g.qy, g.qz, g.flags)]
    d = pt.pt_grid_desc(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.x0, g.y0, g.z0, keep[0].ctypes.data,
                        keep[1].ctypes.data, keep[2].ctypes.data, None, g.porosity_scalar,
                        keep[3].ctypes.data, pt.PT_MEM_HOST, -1.0)
    for k, v in kw.items():
        setattr(d, k, v)
    return d, keep


def _load(lib, d):
    out = ctypes.c_void_p()
    rc = lib.pt_load_grid(ctypes.byref(d) if d is not None else None, None, ctypes.byref(out))
    return rc, out


def test_load_grid_validation(lib):
    g = C.c1().grids[0]
    assert lib.pt_load_grid(None, None, None) == -1
    assert pt.pt_last_error() != ""
    for kw in (dict(nx=0), dict(ny=-1), dict(dx=0.0), dict(dz=float("nan")), dict(x0=float("inf")),
               dict(qx=None), dict(mem=7), dict(porosity_scalar=0.0), dict(balance_tol=float("nan"))):
        d, keep = _desc(g, **kw)
        rc, _ = _load(lib, d)
        assert rc == -1, kw
    d, keep = _desc(g, nx=1 << 16, ny=1 << 16, nz=1)
    assert _load(lib, d)[0] == -7                     # more than 2^31 cells: unsupported


def test_load_grid_data_validation(lib):
    g = H.box_grid(3, 2, 2)
    g.qx[:] = 1.0
    bad = H.box_grid(3, 2, 2)
    bad.qx[0, 0, 1] = np.nan
    d, keep = _desc(bad)
    assert _load(lib, d)[0] == -1 and "not finite" in pt.pt_last_error()
    fl = H.box_grid(3, 2, 2, flags=np.full((2, 2, 3), 5, np.int32))
    d, keep = _desc(fl)
    assert _load(lib, d)[0] == -1 and "unknown bits" in pt.pt_last_error()
    unb = H.box_grid(3, 2, 2)
    unb.qx[0, 0, 1] = 2.0
    d, keep = _desc(unb, balance_tol=1e-6)
    assert _load(lib, d)[0] == -6
    if not _gpu():
        d, keep = _desc(g, balance_tol=1e-12)        # valid and balanced: needs a device
        assert _load(lib, d)[0] == -4


def test_quad_grid_validation(lib):
    """pt_load_quad_grid checks the description on the host before any device work."""
    from workloads import quadtree as QT
    g = C.random_grid(8, 8, 2, 1.0, 2.0, 5)
    q = QT.from_structured(g, QT.block_sizes(8, 8, [(2, 2)], r1=1.0, r2=3.0))
    keep = {}

    def desc(**kw):
        arrs = dict(box=q.box, sub_off=q.sub_off, sub_nb=q.sub_nb, sub_q=q.sub_q, sub_lo=q.sub_lo,
                    sub_hi=q.sub_hi, flags=q.flags)
        arrs.update({k: v for k, v in kw.items() if k in arrs})
        dt = dict(sub_off=np.int32, sub_nb=np.int32, flags=np.int32)
        for k, v in arrs.items():
            keep[k] = np.ascontiguousarray(v, dtype=dt.get(k, np.float64))
        d = pt.pt_quad_desc(kw.get("ncell", q.ncell), kw.get("nsub", q.nsub), *(keep[k].ctypes.data for k in
                            ("box", "sub_off", "sub_nb", "sub_q", "sub_lo", "sub_hi")), None,
                            kw.get("porosity_scalar", 0.3), keep["flags"].ctypes.data, kw.get("mem", pt.PT_MEM_HOST),
                            -1.0)
        return d

    def load(d):
        out = ctypes.c_void_p()
        return lib.pt_load_quad_grid(ctypes.byref(d), None, ctypes.byref(out))

    assert lib.pt_load_quad_grid(None, None, None) == -1
    off_bad = q.sub_off.copy()
    off_bad[3] = off_bad[5] + 1                      # decreasing
    nb_bad = q.sub_nb.copy()
    nb_bad[3] = q.ncell
    lo_bad = q.sub_lo.copy()
    lo_bad[0, 0] = 1.5                               # outside [0, 1]
    box_bad = q.box.copy()
    box_bad[1, 3] = 0.0
    for name, d in (("ncell", desc(ncell=0)), ("nsub", desc(nsub=-1)), ("sub_off", desc(sub_off=off_bad)),
                    ("sub_nb", desc(sub_nb=nb_bad)), ("sub_lo", desc(sub_lo=lo_bad)), ("box", desc(box=box_bad)),
                    ("porosity", desc(porosity_scalar=0.0))):
        assert load(d) == -1, name
    assert load(desc(mem=pt.PT_MEM_DEVICE)) == -7
    many = q.sub_off.copy()
    many[1:] += 40                                   # face 0 of cell 0 would hold 40 subfaces
    assert load(desc(sub_off=many, nsub=q.nsub + 40)) in (-1, -7)
    rc = load(desc())
    assert rc in (0, -4, -5), rc                     # valid: no device here, or loaded


def test_track_validation_without_grid(lib):
    out = ctypes.c_void_p()
    o = pt.pt_default_opts()
    p = pt.pt_particles()
    assert lib.pt_track(None, 1, ctypes.byref(p), ctypes.byref(o), None, ctypes.byref(out)) == -1
    bogus = (ctypes.c_void_p * 1)(0x1234)
    assert lib.pt_track(bogus, 1, ctypes.byref(p), ctypes.byref(o), None, ctypes.byref(out)) == -2
    assert lib.pt_track(bogus, 0, ctypes.byref(p), ctypes.byref(o), None, ctypes.byref(out)) == -1
    assert lib.pt_track(bogus, 1, ctypes.byref(p), ctypes.byref(o), None, None) == -1


def test_release_and_results_handles(lib):
    assert lib.pt_release(None) == 0
    assert lib.pt_release(ctypes.c_void_p(0xDEAD)) == -2
    s = pt.pt_summary()
    assert lib.pt_results(ctypes.c_void_p(0xBEEF), ctypes.byref(s)) == -2
    assert "live" in pt.pt_last_error()


def test_missing_library_fails_loudly(tmp_path):
    saved = pt._lib
    pt._lib = None
    try:
        with pytest.raises(ImportError):
            pt.load_library(str(tmp_path / "absent.so"))
    finally:
        pt._lib = saved


def test_shutdown_with_nothing_live(lib):
    """pt_shutdown holds no device requirement when the library owns nothing: it returns PT_OK
    and may be called repeatedly (it also runs at interpreter exit)."""
    assert lib.pt_shutdown() == pt.PT_OK
    assert lib.pt_shutdown() == pt.PT_OK
    assert lib.pt_release(None) == pt.PT_OK
