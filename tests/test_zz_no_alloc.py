"""pt_track_noalloc (the allocation-free entry point) against pt_track, through the C ABI.

Both run the same kernels; the allocation-free form keeps its counters, tables, ordering buffers
and scan tile sums in the library's per-device scratch array.  Its outputs must be bitwise those
of pt_track on the same inputs, over consecutive calls that reuse the scratch with different
sizes (the second call smaller than the first, so stale contents would show), and sizes beyond
the scratch must be refused before any device work.
"""
import ctypes

import numpy as np
import pytest

from workloads import configs as C

from .gpu_util import require_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
FIELDS = ("cell", "xi", "eta", "zeta", "t", "status", "ncross", "path_hash")


@pytest.fixture(scope="module")
def pt():
    return require_gpu()


@pytest.fixture(scope="module")
def grids(pt):
    gs = [C.random_grid(40, 30, 6, s2, 4.0, 500 + r, wells=((20, 15, -80.0),) if r == 0 else (), recharge=1e-3)
          for r, s2 in enumerate((1.5, 0.7, 3.0))]
    hs = [pt.pt_load_grid(g) for g in gs]
    yield gs, hs
    for h in hs:
        h.release()


def _both(pt, hs, p, group_offsets=None, group_grid=None, snap_times=None, **opt):
    """The same call through pt_track and pt_track_noalloc, on separate copies of the state."""
    n = p.n
    outs = []
    for form in ("track", "noalloc"):
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        oxyz = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
        sx = None
        kw = dict(opt)
        if snap_times is not None:
            sx = torch.full((n, len(snap_times), 3), float("nan"), dtype=torch.float64, device="cuda")
            kw.update(mode=pt.PT_TIMESERIES, snap_times=snap_times, snap_xyz=sx)
        o = pt.make_opts(out_xyz=oxyz, **kw)
        if form == "track":
            run = pt.pt_track(hs, dp, o, group_offsets=group_offsets, group_grid=group_grid)
            s = pt.pt_results(run)
            run.release()
        else:
            counts = torch.full((pt.PT_COUNTS_WORDS,), -7, dtype=torch.int64, device="cuda")
            pt.pt_track_noalloc(hs, dp, o, counts, group_offsets=group_offsets, group_grid=group_grid)
            torch.cuda.synchronize()
            s = pt.counts_summary(counts)
            assert counts.cpu().numpy()[14:].tolist() == [0, 0]
        torch.cuda.synchronize()
        d = dp.to_numpy()
        d["out_xyz"] = oxyz.cpu().numpy()
        d["snap_xyz"] = None if sx is None else sx.cpu().numpy()
        outs.append((d, s))
    (a, sa), (b, sb) = outs
    for k in FIELDS + ("out_xyz",):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    if snap_times is not None:
        assert np.array_equal(a["snap_xyz"], b["snap_xyz"], equal_nan=True)
    for k in ("crossings", "n_tracked", "status_count", "cr_ambiguous", "path_records", "path_dropped",
              "recheck_tracks"):
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    assert sa["crossings"] > 0
    return sa


def test_noalloc_matches_track_two_calls(pt, grids):
    gs, hs = grids
    g = gs[0]
    rng = np.random.Generator(np.random.PCG64(7))
    # first call: large enough to be ordered by starting cell in the scratch (n >= 65536)
    big = C.release(rng, 150_000, g.nx, g.ny, g.nz)
    s1 = _both(pt, hs[:1], big, schedule=pt.PT_SCHED_STATIC)
    # second call, smaller: batched groups over three grids, timeseries, persistent kernel,
    # unordered -- tables in the scratch, stale ordering buffers from the first call
    sizes = [1500, 0, 2501, 999]
    gg = np.array([2, 0, 1, 0], np.int32)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    small = C.concat([C.release(np.random.Generator(np.random.PCG64(30 + q)), m, g.nx, g.ny, g.nz)
                      for q, m in enumerate(sizes)])
    snaps = np.logspace(-1, 3.5, 40)
    s2 = _both(pt, hs, small, group_offsets=offs, group_grid=gg, snap_times=snaps, t_max=2000.0,
               schedule=pt.PT_SCHED_PERSISTENT)
    assert s2["n_tracked"] == small.n < s1["n_tracked"]


def test_noalloc_other_forms(pt, grids):
    gs, hs = grids
    g = gs[1]
    rng = np.random.Generator(np.random.PCG64(8))
    p = C.release(rng, 20_000, g.nx, g.ny, g.nz)
    _both(pt, hs[1:2], p, precision=pt.PT_MIXED, schedule=pt.PT_SCHED_STATIC, sort=pt.PT_SORT_CELL)
    _both(pt, hs[1:2], p, layout=pt.PT_LAYOUT_FACES, schedule=pt.PT_SCHED_PERSISTENT, direction=-1)
    # pathline count pass: offsets scanned with the scratch's tile sums
    offs = []
    for form in ("track", "noalloc"):
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        off = torch.full((p.n + 1,), -1, dtype=torch.int64, device="cuda")
        o = pt.make_opts(mode=pt.PT_PATHLINE, path_offsets=off, path_count_only=1)
        if form == "track":
            s = pt.track(hs[1:2], dp, mode=pt.PT_PATHLINE, path_offsets=off, path_count_only=1)
        else:
            counts = torch.zeros(pt.PT_COUNTS_WORDS, dtype=torch.int64, device="cuda")
            pt.pt_track_noalloc(hs[1:2], dp, o, counts)
            torch.cuda.synchronize()
            s = pt.counts_summary(counts)
        torch.cuda.synchronize()
        offs.append((off.cpu().numpy(), s["path_records"]))
    assert np.array_equal(offs[0][0], offs[1][0]) and offs[0][1] == offs[1][1] == offs[0][0][-1]


def test_noalloc_limits(pt, grids):
    gs, hs = grids
    g = gs[0]
    p = C.release(np.random.Generator(np.random.PCG64(9)), 1000, g.nx, g.ny, g.nz)
    dp = pt.DeviceParticles.from_numpy(p, "cuda")
    counts = torch.zeros(pt.PT_COUNTS_WORDS, dtype=torch.int64, device="cuda")
    # tables beyond 64 KiB: 500 grid views of one grid
    many = [hs[0]] * 500
    offs = np.linspace(0, p.n, 501).astype(np.int64)
    with pytest.raises(pt.PtError) as e:
        pt.pt_track_noalloc(many, dp, pt.make_opts(), counts, group_offsets=offs,
                            group_grid=np.arange(500, dtype=np.int32))
    assert e.value.code == -7
    # ordering beyond the scratch: 3e6 particles need 48 MB of ordering buffers
    n = 3_000_000
    big = pt.DeviceParticles(*(torch.zeros(n, dtype=t, device="cuda") for t in
                               (torch.int32, torch.float64, torch.float64, torch.float64, torch.float64,
                                torch.int32, torch.int32, torch.int64)))
    with pytest.raises(pt.PtError) as e:
        pt.pt_track_noalloc(hs[:1], big, pt.make_opts(sort=pt.PT_SORT_CELL), counts)
    assert e.value.code == -7
    # no counts array
    lib = pt.load_library()
    handles, pp, keep = pt._particles_arg(hs[:1], dp, None, None)
    o = pt.make_opts()
    assert lib.pt_track_noalloc(handles, 1, ctypes.byref(pp), ctypes.byref(o), None, None) == -1
    torch.cuda.synchronize()
    assert counts.cpu().numpy().tolist() == [0] * pt.PT_COUNTS_WORDS     # nothing was launched


def test_noalloc_careful_pass(pt):
    """Inputs that send particles to the careful pass (evaluations within 2^-96 of a rounding
    midpoint): its particle list lives in the scratch too, and the results must still equal
    pt_track's, with the same number of particles re-tracked."""
    from tests import helpers as H
    g = H.box_grid(8, 8, 1, 2.0, 2.0, 1.0, porosity=0.3)
    for i in range(9):
        g.qx[:, :, i] = 0.5 * (1.0 + 0.25 * i)
    for j in range(9):
        g.qy[:, j, :] = 0.5 * (1.0 + 0.25 * j)
    rng = np.random.Generator(np.random.PCG64(92))
    n = 2000
    x = rng.random(n)
    y = np.where(rng.random(n) < 0.5, x, np.clip(x * (1.0 + 10.0 ** rng.uniform(-15, -5, n)), 0, 1))
    i = rng.integers(0, 8, n)
    h = pt.pt_load_grid(g)
    try:
        s = _both(pt, [h], H.particles(i * 8 + i, x, y, 0.5), max_steps=5000)
    finally:
        h.release()
    assert s["recheck_tracks"] > 0 and s["cr_ambiguous"] == 0
