"""The C ABI on the GPU: device-resident grids, error paths after load, graph replays."""
import ctypes
import math

import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs as C

from . import helpers as H
from .gpu_util import compare, gpu_track, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    return require_gpu()


def _dev_grid(g):
    import torch
    import copy
    d = copy.copy(g)
    d.qx = torch.from_numpy(np.ascontiguousarray(g.qx)).cuda()
    d.qy = torch.from_numpy(np.ascontiguousarray(g.qy)).cuda()
    d.qz = torch.from_numpy(np.ascontiguousarray(g.qz)).cuda()
    d.flags = torch.from_numpy(np.ascontiguousarray(g.flags)).cuda()
    if g.porosity is not None:
        d.porosity = torch.from_numpy(np.ascontiguousarray(g.porosity)).cuda()
    return d


def test_device_resident_grid_matches_oracle(pt):
    g = C.random_grid(14, 11, 4, 1.0, 3.0, 61, wells=((6, 5, -30.0),), recharge=1e-3, porosity_field=True)
    p = C.release(np.random.Generator(np.random.PCG64(6)), 3333, g.nx, g.ny, g.nz)
    r = O.track(g, p)
    out = gpu_track([_dev_grid(g)], p)
    compare(out, r, label="device grid", spacing=(g.dx, g.dy, g.dz))


def test_device_grid_validation(pt):
    g = H.box_grid(4, 3, 2)
    g.qx[:] = 1.0
    bad = H.box_grid(4, 3, 2)
    bad.qy[1, 2, 3] = np.inf
    with pytest.raises(pt.PtError) as e:
        pt.pt_load_grid(_dev_grid(bad))
    assert e.value.code == -1
    unb = H.box_grid(4, 3, 2)
    unb.qz[1, 1, 1] = 3.0
    with pytest.raises(pt.PtError) as e:
        pt.pt_load_grid(_dev_grid(unb), balance_tol=1e-9)
    assert e.value.code == -6
    h = pt.pt_load_grid(_dev_grid(g), balance_tol=1e-12)
    h.release()


def test_track_option_errors(pt):
    import torch
    g = C.c1().grids[0]
    h = pt.pt_load_grid(g)
    dp = pt.DeviceParticles.from_numpy(C.c1(n=100).particles)
    sx = torch.empty((100, 3, 3), dtype=torch.float64, device="cuda")
    cases = [(dict(precision=1, layout=1), -7), (dict(block=100), -1), (dict(block=512), -7),
             (dict(direction=0), -1), (dict(t_max=math.nan), -1), (dict(max_steps=0), -1),
             (dict(refill=65), -1), (dict(chunk=-1), -1), (dict(stop_at_sink=2), -1),
             (dict(mode=1, snap_times=np.array([1.0, 0.5, 2.0]), snap_xyz=sx), -1),
             (dict(mode=1, snap_times=np.array([1.0, np.inf, 2.0]), snap_xyz=sx), -1),
             (dict(mode=1), -1)]
    for kw, code in cases:
        with pytest.raises(pt.PtError) as e:
            pt.track([h], dp, **kw)
        assert e.value.code == code, (kw, e.value)
    with pytest.raises(pt.PtError) as e:                     # groups must cover the particles
        pt.track([h, h], dp, group_offsets=[0, 50, 99], group_grid=[0, 1])
    assert e.value.code == -1
    with pytest.raises(pt.PtError) as e:
        pt.track([h], dp, group_offsets=[0, 100], group_grid=[1])
    assert e.value.code == -1
    with pytest.raises(pt.PtError) as e:                     # several grids need groups
        pt.track([h, h], dp)
    assert e.value.code == -1
    h.release()


def test_run_handles(pt):
    g = C.c1().grids[0]
    h = pt.pt_load_grid(g)
    dp = pt.DeviceParticles.from_numpy(C.c1(n=500).particles)
    run = pt.pt_track([h], dp, pt.make_opts())
    s1 = pt.pt_results(run)
    s2 = pt.pt_results(run)
    assert s1 == s2 and s1["crossings"] == 500 * 40
    raw = run.handle
    run.release()
    assert pt.load_library().pt_release(ctypes.c_void_p(raw)) == -2
    raw_grid = h.handle
    h.release()
    assert pt.load_library().pt_release(ctypes.c_void_p(raw_grid)) == -2


def test_graph_replays_match_eager(pt):
    """A cached graph replayed several times, with eager work and synchronisation between."""
    import torch
    g = C.random_grid(30, 20, 5, 2.0, 4.0, 71)
    w = C.release(np.random.Generator(np.random.PCG64(8)), 20000, g.nx, g.ny, g.nz)
    h = pt.pt_load_grid(g)
    pristine = pt.DeviceParticles.from_numpy(w)
    work = pristine.clone()
    oxyz = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
    eager = None
    for sched in (1, 2):
        for rep in range(4):
            work.copy_(pristine)
            s = pt.track([h], work, schedule=sched, use_graph=0 if rep == 0 else 1, out_xyz=oxyz)
            torch.cuda.synchronize()
            noise = torch.randn(1 << 20, device="cuda").sum()      # unrelated eager work between replays
            torch.cuda.synchronize()
            res = work.to_numpy()
            res["out_xyz"] = oxyz.cpu().numpy()
            if eager is None:
                eager = (res, s["crossings"], s["status_count"])
                continue
            assert s["crossings"] == eager[1] and s["status_count"] == eager[2], (sched, rep)
            for k in ("cell", "status", "ncross", "path_hash", "xi", "eta", "zeta", "t", "out_xyz"):
                assert np.array_equal(res[k], eager[0][k], equal_nan=True), (sched, rep, k)
    del noise
    h.release()


def test_shutdown_releases_everything_and_library_restarts(pt):
    """pt_shutdown releases live grids, live runs and the pooled runs (with their graphs); every
    earlier handle is then invalid, and the library works again afterwards."""
    lib = pt.load_library()
    g = C.c1().grids[0]
    h = pt.pt_load_grid(g)
    dp = pt.DeviceParticles.from_numpy(C.c1(n=300).particles)
    pooled = pt.pt_track([h], dp, pt.make_opts(use_graph=1))
    pt.pt_results(pooled)
    pooled.release()                                          # goes to the pool, graph cached
    live = pt.pt_track([h], dp.clone(), pt.make_opts())       # never released by the caller
    raw_grid, raw_run = h.handle, live.handle
    assert lib.pt_shutdown() == pt.PT_OK
    assert lib.pt_release(ctypes.c_void_p(raw_run)) == -2
    assert lib.pt_release(ctypes.c_void_p(raw_grid)) == -2
    h.handle = None
    live.handle = None
    p = C.c1(n=300).particles
    r = O.track(g, p)
    out = gpu_track([g], p, use_graph=1)
    compare(out, r, label="after shutdown", spacing=(10.0, 10.0, 10.0))


def test_kernel_time_events(pt):
    """track_ms times the tracking kernel alone: positive, inside the whole call's kernel_ms, in
    graph and eager launches; a call without particles (no tracking kernel) reports ~0 (its two
    events are recorded back to back), also on a pooled run whose events an earlier call recorded."""
    import torch
    g = C.random_grid(30, 20, 5, 1.0, 4.0, 72)
    h = pt.pt_load_grid(g)
    w = C.release(np.random.Generator(np.random.PCG64(9)), 50000, g.nx, g.ny, g.nz)
    empty = C.release(np.random.Generator(np.random.PCG64(9)), 0, g.nx, g.ny, g.nz)
    for graph in (0, 1):
        for rep in range(3):
            s = pt.track([h], pt.DeviceParticles.from_numpy(w), use_graph=graph, sort=pt.PT_SORT_CELL)
            assert s["crossings"] > 0
            assert 0.0 < s["track_ms"] <= s["kernel_ms"], (graph, rep, s["track_ms"], s["kernel_ms"])
            e = pt.track([h], pt.DeviceParticles.from_numpy(empty), use_graph=graph)
            assert e["crossings"] == 0 and 0.0 <= e["track_ms"] < 0.05, (graph, rep, e)
    torch.cuda.synchronize()
    h.release()
