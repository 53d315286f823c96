"""Quadtree (rectangular unstructured) grids, FP64 parity of the HIP path with the oracle
through the C ABI: every output bitwise identical, on unrefined, uniformly flowing and
heterogeneous refined grids, in every output mode, and on a sample of the C7 workload."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs as C
from workloads import quadtree as QT

from . import helpers as H
from .gpu_util import bench_opts, compare, gpu_track, require_gpu, sample_indices, tracked_counts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pt():
    return require_gpu()


def _refined():
    K = np.exp(np.sqrt(1.5) * np.random.Generator(np.random.PCG64(77)).standard_normal((2, 32, 32)))
    src = np.zeros(K.shape)
    src[1, 13, 18] = -2.0
    g = C.make_grid(K, 2.0, 3.0, 1.0, recharge=1e-3, source=src, sink_mask=src < 0)
    return QT.from_structured(g, QT.block_sizes(32, 32, [(18, 13), (5, 25)], r1=3.0, r2=8.0))


def _unrefined():
    g = C.random_grid(9, 7, 3, 1.2, 2.0, 31, dx=4.0, dy=6.0, dz=1.5, wells=((4, 3, -25.0),), recharge=1e-3)
    return QT.from_structured(g, np.ones((g.ny, g.nx), np.int32))


def _uniform():
    g = H.box_grid(16, 16, 1, 1.0, 1.0, 2.0, porosity=0.25)
    g.qx[:] = 0.7 * 0.25 * 2.0
    g.qy[:] = 0.3 * 0.25 * 2.0
    return QT.from_structured(g, QT.block_sizes(16, 16, [(5, 9)], r1=1.5, r2=4.0))


CASES = {"refined": _refined, "unrefined": _unrefined, "uniform": _uniform}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("sched", [1, 2])
@pytest.mark.parametrize("direction", [1, -1])
def test_quad_small(pt, case, sched, direction):
    q = CASES[case]()
    p = QT.release(q, np.random.Generator(np.random.PCG64(len(case) + sched)), 2999)
    for kw in (dict(), dict(t_max=15.0), dict(stop_at_sink=0, max_steps=40)):
        r = O.track_quad(q, p, direction=direction, **kw)
        out = gpu_track([q], p, schedule=sched, direction=direction, **kw)
        compare(out, r, label="quad %s sched %d dir %d %s" % (case, sched, direction, kw), spacing=(1.0, 1.0, 1.0))
        _, counts = tracked_counts(p.status, r.status)
        assert out["summary"]["status_count"] == counts.tolist()


@pytest.mark.parametrize("sched", [1, 2])
def test_quad_timeseries_and_order(pt, sched):
    q = _refined()
    p = QT.release(q, np.random.Generator(np.random.PCG64(5)), 2500)
    p.t[:] = np.random.Generator(np.random.PCG64(6)).choice([0.0, 4.0, 30.0], size=p.n)
    snaps = np.concatenate([[0.0, 1.0], np.logspace(0.5, 3.0, 30)])
    r = O.track_quad(q, p, snap_times=snaps, t_max=600.0)
    for sort in (1, 2):
        out = gpu_track([q], p, snap_times=snaps, t_max=600.0, schedule=sched, sort=sort)
        compare(out, r, label="quad timeseries sched %d sort %d" % (sched, sort), spacing=(1.0, 1.0, 1.0))


def test_quad_pathlines(pt):
    from .test_gpu_pathline import compare_paths, gpu_pathlines
    q = _refined()
    p = QT.release(q, np.random.Generator(np.random.PCG64(8)), 1500)
    cap = 1024
    r = O.track_quad(q, p, path_cap=cap)
    cnt = r.ncross.astype(np.int64) - p.ncross.astype(np.int64)
    assert cnt.max() <= cap
    keep = np.arange(cap)[None, :] < cnt[:, None]
    flat = dict(cell=r.path_cell[keep], face=r.path_face[keep], t=r.path_t[keep], xyz=r.path_xyz[keep])
    offs = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    for sched in (1, 2):
        out, paths = gpu_pathlines(pt, [q], p, schedule=sched)
        compare_paths(paths, offs, flat, "quad pathlines sched %d" % sched)


def test_quad_zero_time_circuit(pt):
    g = H.box_grid(2, 2, 1, 1.0, 1.0, 1.0, porosity=0.5)
    g.qx[0, 0, 1] = 1.0
    g.qy[0, 1, 1] = 1.0
    g.qx[0, 1, 1] = -1.0
    g.qy[0, 1, 0] = -1.0
    q = QT.from_structured(g, np.ones((2, 2), np.int32))
    p = H.particles([0, 0, 2], [1.0, 0.3, 0.0], [1.0, 0.6, 0.0], 0.5)
    snaps = np.array([0.0, 0.5, 3.0, 100.0])
    for kw in (dict(max_steps=100), dict(max_steps=100, snap_times=snaps, t_max=50.0)):
        r = O.track_quad(q, p, **kw)
        assert r.status[0] == 5 and r.ncross[0] == 16
        for sched in (1, 2):
            out = gpu_track([q], p, schedule=sched, **kw)
            compare(out, r, label="circuit %s sched %d" % (sorted(kw), sched), spacing=(1.0, 1.0, 1.0))


def test_quad_option_errors(pt):
    q = _unrefined()
    p = QT.release(q, np.random.Generator(np.random.PCG64(2)), 64)
    h = pt.pt_load_quad_grid(q)
    g2 = pt.pt_load_grid(C.random_grid(9, 7, 3, 1.0, 2.0, 3))
    try:
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        for grids, kw in (([h], dict(precision=pt.PT_MIXED)), ([h], dict(layout=pt.PT_LAYOUT_FACES)),
                          ([h, g2], dict(tstep_end=np.array([5.0, math.inf]))),
                          ([h, h], dict(group_offsets=np.array([0, 32, 64]), group_grid=np.array([0, 1], np.int32)))):
            with pytest.raises(pt.PtError) as e:
                pt.track(grids, dp, **kw)
            assert e.value.code == -7, kw
    finally:
        h.release()
        g2.release()


def test_c7_full_sampled(pt):
    w = QT.c7()
    q = w.grids[0]
    p = w.particles
    out = gpu_track([q], p, **bench_opts("C7"))
    s = out["summary"]
    assert s["crossings"] == int(out["ncross"].astype(np.int64).sum())
    idx = sample_indices(p.n, 100_000, seed=81)
    r = O.track_quad(q, p.subset(idx))
    compare(out, r, idx=idx, label="C7", spacing=(2.5, 2.5, 5.0))
    print("C7 crossings %d statuses %s kernel ms %.3f" % (s["crossings"], s["status_count"], s["kernel_ms"]))
