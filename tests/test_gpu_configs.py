"""Parity at the full workload sizes, in the launch configuration the benchmark times.

The whole workload runs on the GPU; a seeded sample of particles is tracked by the
oracle one by one and compared element by element.  Properties that hold at any
size (counter totals, the status histogram) are checked on every particle.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs as C

from .gpu_util import bench_opts, compare, gpu_track, other_schedule, require_gpu, sample_indices, tracked_counts

pytestmark = pytest.mark.gpu

SP = (10.0, 10.0, 2.0)                                 # cell sizes of C2-C5


@pytest.fixture(scope="module")
def pt():
    return require_gpu()


def _check_invariants(out, p, label):
    """Properties of every particle at any size: local coordinates in [0, 1], times never
    before the release, a BOUNDARY particle on a face of its cell, crossings only added."""
    for name in ("xi", "eta", "zeta"):
        a = out[name]
        assert ((a >= 0.0) & (a <= 1.0)).all(), (label, name)
    tracked = (p.status == 0) | (p.status == 3)
    assert (out["t"][tracked] >= p.t[tracked]).all(), label
    assert (out["ncross"] >= p.ncross).all(), label
    b = out["status"] == 1
    on_face = np.zeros(b.sum(), dtype=bool)
    for name in ("xi", "eta", "zeta"):
        a = out[name][b]
        on_face |= (a == 0.0) | (a == 1.0)
    assert on_face.all(), (label, int((~on_face).sum()))


def _check_counters(out, p):
    tracked, counts = tracked_counts(p.status, out["status"])
    s = out["summary"]
    assert s["crossings"] == int(out["ncross"].astype(np.int64).sum() - p.ncross.astype(np.int64).sum())
    assert s["status_count"] == counts.tolist()
    assert s["n_tracked"] == int(tracked.sum())


def test_c1_full_closed_form(pt):
    w = C.c1()
    p = w.particles
    r = O.track(w.grids[0], p)
    for kw in (dict(schedule=1, layout=1), dict(schedule=1, layout=2), dict(schedule=2, layout=2, use_graph=1)):
        out = gpu_track(w.grids, p, **kw)
        compare(out, r, label="C1 %s" % kw, spacing=(10.0, 10.0, 10.0))
        x0 = (p.cell % 40 + p.xi) * 10.0
        assert np.all(out["ncross"] == 40) and np.all(out["status"] == 1)
        assert np.max(np.abs(out["t"] - 1.2 * (400.0 - x0)) / out["t"]) <= 1e-12


@pytest.mark.parametrize("launch", ["bench", "other"])
def test_c2_full_sampled(pt, launch):
    w = C.c2()
    p = w.particles
    kw = bench_opts("C2")
    if launch == "other":
        kw = other_schedule(kw)
    out = gpu_track(w.grids, p, **kw)
    _check_counters(out, p)
    _check_invariants(out, p, "C2")
    idx = sample_indices(p.n, 4000, seed=21)
    r = O.track(w.grids[0], p.subset(idx))
    compare(out, r, idx=idx, label="C2 %s" % kw, spacing=SP)
    print("C2 %s crossings" % kw, out["summary"]["crossings"], "kernel ms", out["summary"]["kernel_ms"])


def test_c3_full_sampled(pt):
    w = C.c3()
    p = w.particles
    out = gpu_track(w.grids, p, **bench_opts("C3"))
    _check_counters(out, p)
    _check_invariants(out, p, "C3")
    idx = sample_indices(p.n, 3000, seed=31)
    r = O.track(w.grids[0], p.subset(idx))
    compare(out, r, idx=idx, label="C3", spacing=SP)
    sc = out["summary"]["status_count"]
    assert sc[2] > 0 and sc[1] > 0       # wells capture some particles, the rest leave the domain
    print("C3 crossings", out["summary"]["crossings"], "statuses", sc, "ms", out["summary"]["kernel_ms"])


def test_c4_batched_full_sampled(pt):
    w = C.c4()
    p = w.particles
    out = gpu_track(w.grids, p, group_offsets=w.group_offsets, group_grid=w.group_grid, **bench_opts("C4"))
    _check_counters(out, p)
    idx = sample_indices(p.n, 3000, seed=41)
    grp = np.searchsorted(w.group_offsets, idx, side="right") - 1
    sub = p.subset(idx)
    for g in np.unique(w.group_grid[grp]):
        sel = np.nonzero(w.group_grid[grp] == g)[0]
        r = O.track(w.grids[g], sub.subset(sel))
        compare(out, r, idx=idx[sel], label="C4 grid %d" % g, spacing=SP)


def test_c5_timeseries_full_sampled(pt):
    w = C.c5()
    p = w.particles
    out = gpu_track(w.grids, p, snap_times=w.snap_times, t_max=w.t_max, **bench_opts("C5", mode="timeseries"))
    _check_counters(out, p)
    idx = sample_indices(p.n, 2000, seed=51)
    r = O.track(w.grids[0], p.subset(idx), snap_times=w.snap_times, t_max=w.t_max)
    compare(out, r, idx=idx, label="C5", spacing=SP)
    sx = out["snap_xyz"]
    assert sx.shape == (p.n, 100, 3)
    # every particle is defined at its release (t = 0 < 1 d) and NaN after it left the domain
    assert not np.isnan(sx[:, 0, :]).any()


@pytest.mark.parametrize("sigma2,n", [(2.5, 100_000), (5.0, 20_000)])
def test_tc1_shape_sampled(pt, sigma2, n):
    """The scheduling study's workload (first test case's shape): every particle reaches the
    outlet, in both kernels, identical to the oracle on a sample."""
    w = C.tc1(n, sigma2)
    p = w.particles
    idx = sample_indices(p.n, 1500, seed=71)
    r = O.track(w.grids[0], p.subset(idx))
    for sched in (1, 2):
        out = gpu_track(w.grids, p, schedule=sched, layout=2, use_graph=1)
        _check_counters(out, p)
        compare(out, r, idx=idx, label="TC1 s2=%g sched %d" % (sigma2, sched), spacing=(1.0, 1.0, 1.0))
        at_outlet = (out["status"] == 1) & (out["cell"] % 1500 == 1499)
        assert np.mean(at_outlet) > 0.999                       # displaced to the outlet
    print("TC1 s2=%g: crossings %d, per particle mean %.1f max %d" % (
        sigma2, out["summary"]["crossings"], out["ncross"].mean(), out["ncross"].max()))


@pytest.mark.parametrize("cfg", ["C2", "C5"])
def test_mixed_precision_accuracy(pt, cfg):
    """Mixed FP32/FP64 against the FP64 oracle: reported, with loose sanity bounds."""
    w = C.c2() if cfg == "C2" else C.c5()
    p = w.particles
    kw = bench_opts(cfg, "mixed", "timeseries" if w.snap_times is not None else "endpoint")
    if w.snap_times is not None:
        kw.update(snap_times=w.snap_times, t_max=w.t_max)
    out = gpu_track(w.grids, p, **kw)
    _check_counters(out, p)
    idx = sample_indices(p.n, 4000, seed=61)
    r = O.track(w.grids[0], p.subset(idx), snap_times=w.snap_times, t_max=w.t_max)
    same = (out["path_hash"][idx] == r.path_hash) & (out["ncross"][idx] == r.ncross)
    done = r.status == 1
    rel = np.abs(out["t"][idx] - r.t)[done] / r.t[done]
    q = np.quantile(rel, [0.5, 0.99, 1.0])
    print("%s mixed: path agreement %.4f, travel-time rel err p50 %.2e p99 %.2e max %.2e"
          % (cfg, same.mean(), *q))
    assert same.mean() >= 0.5
    assert q[0] <= 1e-4
