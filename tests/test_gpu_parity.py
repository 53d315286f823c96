"""FP64 parity of the HIP path with the oracle, element by element, through the C ABI.

Small seeded grids (several tiles, ragged particle counts) in every kernel form:
static and persistent scheduling, face-array and packed-record layouts, forward and
backward tracking, endpoint and timeseries modes, single and batched grids.
"""
import math
import zlib

import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs as C

from . import helpers as H
from .gpu_util import compare, gpu_track, require_gpu, sample_indices, tracked_counts

pytestmark = pytest.mark.gpu

SCHEDS = [("static", 1), ("persistent", 2)]
LAYOUTS = [("faces", 1), ("cell", 2)]


@pytest.fixture(scope="module")
def pt():
    return require_gpu()


def _small_cases():
    return {
        "lognormal_wells": C.random_grid(24, 17, 5, 1.5, 3.0, 101, wells=((8, 8, -60.0), (17, 5, -40.0)),
                                         recharge=2e-3, origin=(250.0, -40.0, 7.5)),
        "porosity_field": C.random_grid(19, 23, 3, 2.5, 4.0, 202, dx=5.0, dy=8.0, dz=1.0,
                                        porosity_field=True),
        "c1": C.c1().grids[0],
    }


CASES = _small_cases()


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("sched", SCHEDS, ids=lambda s: s[0])
@pytest.mark.parametrize("layout", LAYOUTS, ids=lambda s: s[0])
@pytest.mark.parametrize("direction", [1, -1])
def test_small_grids(pt, case, sched, layout, direction):
    g = CASES[case]
    rng = np.random.Generator(np.random.PCG64(zlib.crc32(case.encode()) % 1000 + 3))
    p = C.release(rng, 4999, g.nx, g.ny, g.nz)
    r = O.track(g, p, direction=direction)
    out = gpu_track([g], p, schedule=sched[1], layout=layout[1], direction=direction)
    compare(out, r, label="%s %s %s dir%d" % (case, sched[0], layout[0], direction),
            spacing=(g.dx, g.dy, g.dz))
    tracked, counts = tracked_counts(p.status, r.status)
    s = out["summary"]
    assert s["crossings"] == int(r.ncross.sum())
    assert s["status_count"] == counts.tolist()
    assert s["n_tracked"] == int(tracked.sum())


@pytest.mark.parametrize("sched", SCHEDS, ids=lambda s: s[0])
@pytest.mark.parametrize("layout", LAYOUTS, ids=lambda s: s[0])
def test_timeseries_small(pt, sched, layout):
    g = CASES["lognormal_wells"]
    rng = np.random.Generator(np.random.PCG64(17))
    p = C.release(rng, 3001, g.nx, g.ny, g.nz)
    p.t[:] = rng.choice([0.0, 3.0, 50.0], size=p.n)      # staged releases
    snaps = np.concatenate([[0.0, 0.5], np.logspace(0, 3.5, 37), [5000.0, 5000.0]])
    for t_max in (math.inf, 700.0):
        r = O.track(g, p, snap_times=snaps, t_max=t_max)
        out = gpu_track([g], p, snap_times=snaps, t_max=t_max, schedule=sched[1], layout=layout[1])
        compare(out, r, label="ts t_max=%s" % t_max, spacing=(g.dx, g.dy, g.dz))


def test_batched_groups(pt):
    grids = [C.random_grid(12, 9, 4, s2, 2.0, 300 + r, wells=((5, 4, -30.0),) if r == 1 else (),
                           recharge=1e-3 * r) for r, s2 in enumerate((0.5, 1.5, 3.0))]
    sizes = [700, 0, 1, 1233, 64, 0, 999]
    gg = np.array([2, 0, 1, 1, 0, 2, 1], np.int32)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    parts = []
    for q, m in enumerate(sizes):
        g = grids[gg[q]]
        parts.append(C.release(np.random.Generator(np.random.PCG64(50 + q)), m, g.nx, g.ny, g.nz))
    p = C.concat(parts)
    r = O.track_groups(grids, p, offs, gg)
    for sched in (1, 2):
        for sort in (1, 2):
            out = gpu_track(grids, p, group_offsets=offs, group_grid=gg, schedule=sched, sort=sort)
            compare(out, r, label="batched sched %d sort %d" % (sched, sort), spacing=(10.0, 10.0, 2.0))
    snaps = np.logspace(-1, 3, 20)
    r = O.track_groups(grids, p, offs, gg, snap_times=snaps, t_max=300.0)
    for kw in (dict(), dict(schedule=1, layout=2), dict(schedule=1, layout=2, sort=2, block=128),
               dict(schedule=2, layout=2)):
        out = gpu_track(grids, p, group_offsets=offs, group_grid=gg, snap_times=snaps, t_max=300.0, **kw)
        compare(out, r, label="batched timeseries %s" % kw, spacing=(10.0, 10.0, 2.0))


def test_edge_cases(pt):
    g = CASES["lognormal_wells"]
    ncell = g.nx * g.ny * g.nz
    # every kind of bad or terminal start, and skipped statuses
    p = H.particles([0, -5, ncell, 3, 4, 5, 6, 8 * g.nx + 8, 7, 9],
                    [0.5, 0.5, 0.5, np.nan, 1.5, 0.2, 1.0, 0.4, 0.3, 0.6],
                    [0.5, 0.5, 0.5, 0.5, 0.5, -0.1, 0.0, 0.4, 0.3, 0.6], 0.5,
                    [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, np.inf, 0.0])
    p.status[9] = 1                 # already at a boundary: untouched
    for sched in (1, 2):
        r = O.track(g, p)
        out = gpu_track([g], p, schedule=sched)
        compare(out, r, label="edge sched %d" % sched, spacing=(10.0, 10.0, 2.0))
    # caps and limits
    rng = np.random.Generator(np.random.PCG64(8))
    q = C.release(rng, 777, g.nx, g.ny, g.nz)
    for kw in (dict(max_steps=1), dict(max_steps=7), dict(t_max=0.0), dict(t_max=12.5),
               dict(stop_at_sink=0)):
        r = O.track(g, q, **kw)
        for sched in (1, 2):
            out = gpu_track([g], q, schedule=sched, **kw)
            compare(out, r, label="edge %s sched %d" % (kw, sched), spacing=(10.0, 10.0, 2.0))


def test_empty_run(pt):
    g = CASES["c1"]
    p = C.release(np.random.Generator(np.random.PCG64(1)), 0, g.nx, g.ny, g.nz)
    out = gpu_track([g], p)
    assert out["summary"]["crossings"] == 0 and out["summary"]["n_tracked"] == 0


def test_resume_matches_single_run(pt):
    g = CASES["lognormal_wells"]
    rng = np.random.Generator(np.random.PCG64(4))
    p = C.release(rng, 2500, g.nx, g.ny, g.nz)
    snaps = np.logspace(0, 3, 25)
    one = gpu_track([g], p, snap_times=snaps, t_max=900.0)
    a = gpu_track([g], p, snap_times=snaps, t_max=60.0)
    mid = H.particles(a["cell"], a["xi"], a["eta"], a["zeta"], a["t"])
    mid.status[:] = a["status"]
    mid.ncross[:] = a["ncross"]
    mid.path_hash[:] = a["path_hash"]
    b = gpu_track([g], mid, snap_times=snaps, snap_init=a["snap_xyz"], t_max=900.0)
    for k in ("status", "cell", "ncross", "path_hash"):
        assert np.array_equal(b[k], one[k]), k
    for k in ("t", "xi", "eta", "zeta"):
        assert np.allclose(b[k], one[k], rtol=1e-12, atol=1e-12), k
    assert np.allclose(b["snap_xyz"], one["snap_xyz"], rtol=1e-12, atol=1e-9, equal_nan=True)
    # and the resumed run equals the oracle's resumed run
    r = O.track(g, mid, snap_times=snaps, snap_init=a["snap_xyz"], t_max=900.0)
    compare(b, r, label="resume", spacing=(10.0, 10.0, 2.0))


def test_schedules_and_shapes_bit_identical(pt):
    g = CASES["porosity_field"]
    rng = np.random.Generator(np.random.PCG64(12))
    p = C.release(rng, 20000, g.nx, g.ny, g.nz)
    ref = gpu_track([g], p, schedule=1, layout=2)
    for kw in (dict(schedule=2), dict(schedule=2, block=64), dict(schedule=2, block=128, refill=1),
               dict(schedule=2, refill=64, steps_per_refill=4), dict(schedule=2, blocks_per_cu=1),
               dict(schedule=2, chunk=1), dict(schedule=2, chunk=1000, refill=16),
               dict(schedule=2, chunk=7, steps_per_refill=3, block=192),
               dict(schedule=2, sort=2), dict(schedule=1, sort=2), dict(schedule=2, sort=2, chunk=1),
               dict(schedule=2, sort=2, use_graph=1),
               dict(schedule=2, use_graph=1), dict(schedule=1, layout=1), dict(schedule=1, block=64)):
        out = gpu_track([g], p, **kw)
        for k in ("status", "cell", "ncross", "path_hash", "xi", "eta", "zeta", "t", "out_xyz"):
            assert np.array_equal(out[k], ref[k], equal_nan=True), (kw, k)


@pytest.mark.parametrize("precision", [0, 1])
def test_deferred_snapshots_match_immediate(pt, precision):
    """The static kernel defers snapshots and evaluates them wave-wide; the persistent kernel and
    the face layout write them at once.  Both forms must give identical snapshots and states in
    either precision, at every block size (the slots are per thread, the flushes per wave), with
    snapshots dense enough that lanes meet a second one while their slot is pending."""
    g = CASES["porosity_field"]
    rng = np.random.Generator(np.random.PCG64(31))
    p = C.release(rng, 5000, g.nx, g.ny, g.nz)
    p.t[:] = rng.choice([0.0, 3.0, 40.0], size=p.n)
    snaps = np.concatenate([np.linspace(0.0, 20.0, 81), np.logspace(1.5, 3.5, 60)])
    snaps.sort()
    kw = dict(snap_times=snaps, t_max=2000.0, precision=precision)
    ref = gpu_track([g], p, schedule=2, layout=2, **kw)
    runs = [dict(schedule=1, layout=2), dict(schedule=1, layout=2, block=64), dict(schedule=1, layout=2, block=192),
            dict(schedule=1, layout=2, sort=2, use_graph=1)]
    if precision == 0:
        runs.append(dict(schedule=1, layout=1))
    for r in runs:
        out = gpu_track([g], p, **r, **kw)
        for k in ("status", "cell", "ncross", "path_hash", "xi", "eta", "zeta", "t", "out_xyz", "snap_xyz"):
            assert np.array_equal(out[k], ref[k], equal_nan=True), (r, k)


def test_sort_on_grid_beyond_histogram():
    """A grid of more cells than the ordering histogram holds (2^24): buckets then cover runs of
    cells.  The order never changes a result: ordered and unordered runs are identical, and
    identical to the oracle on a sample."""
    require_gpu()
    nx, ny, nz = 512, 256, 130                      # 17,039,360 cells > 2^24
    g = H.box_grid(nx, ny, nz, 2.0, 2.0, 1.0, porosity=0.25,
                   qx=np.full((nz, ny, nx + 1), 1.0), qy=np.full((nz, ny + 1, nx), 0.3))
    rng = np.random.Generator(np.random.PCG64(41))
    n = 70_001
    cells = rng.integers(0, nx * ny * nz, size=n)
    p = H.particles(cells, rng.random(n), rng.random(n), rng.random(n))
    ordered = gpu_track([g], p, schedule=1, layout=2, sort=2)
    plain = gpu_track([g], p, schedule=1, layout=2, sort=1)
    for k in ("status", "cell", "ncross", "path_hash", "xi", "eta", "zeta", "t", "out_xyz"):
        assert np.array_equal(ordered[k], plain[k], equal_nan=True), k
    assert (ordered["status"] == 1).all()
    idx = sample_indices(n, 300, seed=42)
    r = O.track(g, p.subset(idx))
    compare(ordered, r, idx=idx, label="large grid", spacing=(2.0, 2.0, 1.0))


def test_deferred_snapshots_many_times(pt):
    """More snapshot times than the block keeps in LDS (read from global memory), in the
    deferred and the immediate form, against the oracle."""
    g = CASES["lognormal_wells"]
    rng = np.random.Generator(np.random.PCG64(33))
    p = C.release(rng, 700, g.nx, g.ny, g.nz)
    snaps = np.linspace(0.0, 400.0, 1500)
    r = O.track(g, p, snap_times=snaps, t_max=400.0)
    for kw in (dict(schedule=1, layout=2), dict(schedule=2, layout=2), dict(schedule=1, layout=2, block=64)):
        out = gpu_track([g], p, snap_times=snaps, t_max=400.0, **kw)
        compare(out, r, label="1500 snapshots %s" % kw, spacing=(10.0, 10.0, 2.0))


def test_ordering_skewed_and_inactive():
    """The two-level ordering sort on skewed inputs: every particle in one cell (one super-bucket
    holds them all), and half of the particles already terminated (they all fall in bucket 0).
    Ordered and unordered runs must be identical: a slot given twice or not at all would leave
    particles untracked or tracked twice."""
    require_gpu()
    g = C.random_grid(40, 30, 6, 1.0, 3.0, 77)
    rng = np.random.Generator(np.random.PCG64(78))
    n = 70_001
    one = H.particles(np.full(n, 17 * 40 + 3), rng.random(n), rng.random(n), rng.random(n))
    half = C.release(rng, n, g.nx, g.ny, g.nz)
    half.status[::2] = 1                                   # already at a boundary: not tracked
    for p in (one, half):
        ordered = gpu_track([g], p, schedule=1, layout=2, sort=2)
        plain = gpu_track([g], p, schedule=1, layout=2, sort=1)
        persistent = gpu_track([g], p, schedule=2, layout=2, sort=2)
        for k in ("status", "cell", "ncross", "path_hash", "xi", "eta", "zeta", "t", "out_xyz"):
            assert np.array_equal(ordered[k], plain[k], equal_nan=True), k
            assert np.array_equal(persistent[k], plain[k], equal_nan=True), k
        assert ordered["summary"]["crossings"] == plain["summary"]["crossings"] > 0
    assert (ordered["status"][::2] == 1).all() and (ordered["status"][1::2] != 0).all()
