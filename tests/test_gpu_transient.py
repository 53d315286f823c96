"""Transient flow (one field per time step, switched at each step end), FP64 parity with the
oracle through the C ABI: every output bitwise identical, in every kernel form, with staged
releases, weak sinks, time limits, snapshots across step ends and pathlines."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs as C

from . import helpers as H
from . import oracle_pins as PINS
from .gpu_util import bench_opts, compare, gpu_track, require_gpu, sample_indices, tracked_counts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pt():
    return require_gpu()


def _fields():
    """Four time steps on one geometry: different K realisations, a well that switches on
    (a sink from the second step on) and off, and changing recharge."""
    wells = [(), ((8, 8, -60.0),), ((8, 8, -90.0), (17, 5, -30.0)), ()]
    return [C.random_grid(24, 17, 5, 1.5, 3.0, 400 + s, wells=wells[s], recharge=1e-3 * (s + 1))
            for s in range(4)]


ENDS = np.array([35.0, 80.0, 160.0, math.inf])


def _staged(n, g, seed):
    p = C.release(np.random.Generator(np.random.PCG64(seed)), n, g.nx, g.ny, g.nz)
    p.t[:] = 20.0 * (np.arange(n) % 10)          # 10 release stages every 20 d
    p.t[::97] = ENDS[1]                           # some released exactly at a step end
    return p


@pytest.mark.parametrize("sched", [1, 2])
@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("stop_at_sink", [1, 0])
def test_transient_small(pt, sched, layout, stop_at_sink):
    grids = _fields()
    p = _staged(3001, grids[0], 11)
    for t_max in (math.inf, 120.0):
        r = O.track_transient(grids, ENDS, p, stop_at_sink=stop_at_sink, t_max=t_max)
        out = gpu_track(grids, p, tstep_end=ENDS, schedule=sched, layout=layout, stop_at_sink=stop_at_sink,
                        t_max=t_max)
        compare(out, r, label="transient sched %d layout %d sink %d t_max %s" % (sched, layout, stop_at_sink, t_max),
                spacing=(10.0, 10.0, 2.0))
        tracked, counts = tracked_counts(p.status, r.status)
        assert out["summary"]["status_count"] == counts.tolist()


@pytest.mark.parametrize("sched", [1, 2])
def test_transient_timeseries_and_sort(pt, sched):
    grids = _fields()
    p = _staged(2500, grids[0], 12)
    snaps = np.concatenate([np.linspace(0.0, 200.0, 41), ENDS[:3], [400.0, 1000.0]])
    snaps.sort()
    r = O.track_transient(grids, ENDS, p, snap_times=snaps, t_max=900.0)
    for sort in (1, 2):
        out = gpu_track(grids, p, tstep_end=ENDS, snap_times=snaps, t_max=900.0, schedule=sched, sort=sort)
        compare(out, r, label="transient timeseries sched %d sort %d" % (sched, sort), spacing=(10.0, 10.0, 2.0))


def test_transient_channel_closed_form_cases(pt):
    """The oracle pins' channel (piecewise-constant velocity, a stagnant step, sink and
    inactive cells switched on at a step end) on the GPU."""
    x0 = np.array([3.0, 57.5, 120.0, 260.0, 399.0, 212.5, 33.0, 205.0, 155.0, 25.0])
    t0 = np.array([0.0, 0.0, 130.0, 160.0, 190.0, 150.0, 100.0, 0.0, 0.0, 0.0])
    i0 = np.floor(x0 / 10.0).astype(int)
    p = H.particles(i0, x0 / 10.0 - i0, 0.5, 0.5, t0)
    ends = np.array(PINS._TS_END)
    for kw in (dict(), dict(sink_cell=30), dict(inactive_cell=12)):
        grids = PINS._ts_grids(**kw)
        for t_max in (math.inf, 170.0, 150.0):
            for sink in (1, 0):
                r = O.track_transient(grids, ends, p, t_max=t_max, stop_at_sink=sink)
                for sched in (1, 2):
                    out = gpu_track(grids, p, tstep_end=ends, t_max=t_max, stop_at_sink=sink, schedule=sched)
                    compare(out, r, label="channel %s t_max %s sink %d sched %d" % (kw, t_max, sink, sched),
                            spacing=(10.0, 10.0, 10.0))


def test_transient_pathlines(pt):
    from .test_gpu_pathline import compare_paths
    grids = _fields()
    p = _staged(1500, grids[0], 13)
    cap = 4096
    r = O.track_transient(grids, ENDS, p, path_cap=cap)
    cnt = r.ncross.astype(np.int64) - p.ncross.astype(np.int64)
    assert cnt.max() <= cap
    keep = np.arange(cap)[None, :] < cnt[:, None]
    flat = dict(cell=r.path_cell[keep], face=r.path_face[keep], t=r.path_t[keep], xyz=r.path_xyz[keep])
    offs = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    handles = [pt.pt_load_grid(g) for g in grids]
    try:
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        s, pl = pt.track_pathlines(handles, dp, tstep_end=ENDS)
        paths = dict(offsets=pl.offsets.cpu().numpy(), cell=pl.cell.cpu().numpy(), face=pl.face.cpu().numpy(),
                     t=pl.t.cpu().numpy(), xyz=pl.xyz.cpu().numpy())
        compare_paths(paths, offs, flat, "transient pathlines")
    finally:
        for h in handles:
            h.release()


def test_transient_resume(pt):
    """Stopping at a time limit inside a step and resuming gives the single run's result."""
    grids = _fields()
    p = _staged(1200, grids[0], 14)
    one = gpu_track(grids, p, tstep_end=ENDS)
    handles = [pt.pt_load_grid(g) for g in grids]
    try:
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        for t_max in (50.0, 80.0, 300.0, math.inf):
            pt.track(handles, dp, tstep_end=ENDS, t_max=t_max)
        out = dp.to_numpy()
    finally:
        for h in handles:
            h.release()
    for k in ("status", "cell", "ncross", "path_hash"):
        assert np.array_equal(out[k], one[k]), k
    # splitting a step at t_max changes the rounding of the split steps only
    assert np.allclose(out["t"], one["t"], rtol=1e-11, atol=0.0)


def test_transient_option_errors(pt):
    grids = _fields()
    g_other = C.random_grid(20, 17, 5, 1.0, 3.0, 9)
    p = _staged(64, grids[0], 15)
    handles = [pt.pt_load_grid(g) for g in grids]
    other = pt.pt_load_grid(g_other)
    try:
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        cases = [
            (handles[:3], dict(tstep_end=ENDS)),                                   # one grid per step
            (handles, dict(tstep_end=np.array([35.0, 80.0, 80.0, math.inf]))),     # not increasing
            (handles, dict(tstep_end=np.array([35.0, np.nan, 160.0, math.inf]))),  # NaN
            (handles[:3] + [other], dict(tstep_end=ENDS)),                         # other geometry
        ]
        for hs, kw in cases:
            with pytest.raises(pt.PtError) as e:
                pt.track(hs, dp, **kw)
            assert e.value.code == -1, kw
        with pytest.raises(pt.PtError) as e:
            pt.track(handles, dp, tstep_end=ENDS, direction=-1)
        assert e.value.code == -7
        offs = np.array([0, 32, 64], np.int64)
        with pytest.raises(pt.PtError) as e:
            pt.track(handles[:2], dp, tstep_end=ENDS[:2], group_offsets=offs, group_grid=np.array([0, 1], np.int32))
        assert e.value.code == -7
    finally:
        for h in handles:
            h.release()
        other.release()


def test_c6_full_sampled(pt):
    w = C.c6()
    p = w.particles
    out = gpu_track(w.grids, p, tstep_end=w.tstep_end, stop_at_sink=w.stop_at_sink, **bench_opts("C6"))
    s = out["summary"]
    assert s["crossings"] == int(out["ncross"].astype(np.int64).sum())
    idx = sample_indices(p.n, 100_000, seed=61)
    r = O.track_transient(w.grids, w.tstep_end, p.subset(idx), stop_at_sink=w.stop_at_sink)
    compare(out, r, idx=idx, label="C6", spacing=(10.0, 10.0, 2.0))
    print("C6 crossings %d statuses %s kernel ms %.3f" % (s["crossings"], s["status_count"], s["kernel_ms"]))
