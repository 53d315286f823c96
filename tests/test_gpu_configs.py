"""Parity at the full workload sizes, in the launch configuration the benchmark times.

The whole workload runs on the GPU.  C1 and C2 are compared with the oracle particle by
particle in full; for C3-C5 a seeded sample of 100,000 particles is tracked by the oracle and
compared element by element (the paper checks that serial and parallel runs give outputs
"equivalent in value", Methods "Multiprocessing"; here the FP64 outputs are bitwise identical).
Properties that hold at any size (counter totals, the status histogram, local coordinates in
[0, 1], boundary particles on a face) are checked on every particle.

The mixed-precision kernels are compared with the FP64 oracle sample and with the FP64 GPU run
of every particle: path agreement, travel-time error (boundary and sink particles) and, for the
timeseries workload, the position error of every snapshot.  These are reported figures with
loose sanity bounds, not parity.
"""
import functools
import math

import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs as C

from paper_2302_13590_amd import accuracy as ACC

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


SAMPLE = 100_000                                       # oracle sample of C3-C5


@functools.lru_cache(maxsize=1)
def _workload(name):
    return {"C2": C.c2, "C3": C.c3, "C4": C.c4, "C5": C.c5}[name]()


@functools.lru_cache(maxsize=4)
def _oracle_sample(name):
    """The oracle on the seeded sample of a workload (all of C2): (indices, result per grid)."""
    w = _workload(name)
    p = w.particles
    idx = np.arange(p.n) if name == "C2" else sample_indices(p.n, SAMPLE, seed={"C3": 31, "C4": 41, "C5": 51}[name])
    sub = p.subset(idx)
    if w.group_offsets is None:
        return [(idx, O.track(w.grids[0], sub, snap_times=w.snap_times, t_max=w.t_max))]
    grp = np.searchsorted(w.group_offsets, idx, side="right") - 1
    out = []
    for g in np.unique(w.group_grid[grp]):
        sel = np.nonzero(w.group_grid[grp] == g)[0]
        out.append((idx[sel], O.track(w.grids[g], sub.subset(sel))))
    return out


def _run(name, precision="fp64", **extra):
    w = _workload(name)
    mode = "timeseries" if w.snap_times is not None else "endpoint"
    kw = bench_opts(name, precision, mode)
    kw.update(extra)
    if w.snap_times is not None:
        kw.update(snap_times=w.snap_times, t_max=w.t_max)
    return gpu_track(w.grids, w.particles, group_offsets=w.group_offsets, group_grid=w.group_grid, **kw)


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


def test_c2_full_every_particle(pt):
    """C2 in the benchmark's launch: all 1e6 particles bitwise identical to the oracle."""
    w = _workload("C2")
    p = w.particles
    out = _run("C2")
    _check_counters(out, p)
    _check_invariants(out, p, "C2")
    (idx, r), = _oracle_sample("C2")
    compare(out, r, idx=idx, label="C2 full", spacing=SP)
    print("C2: %d particles bitwise identical to the oracle, %d crossings, kernel %.3f ms"
          % (idx.size, out["summary"]["crossings"], out["summary"]["kernel_ms"]))


def test_c2_other_schedule_sampled(pt):
    w = _workload("C2")
    p = w.particles
    kw = other_schedule(bench_opts("C2"))
    out = gpu_track(w.grids, p, **kw)
    _check_counters(out, p)
    idx = sample_indices(p.n, 4000, seed=21)
    r = O.track(w.grids[0], p.subset(idx))
    compare(out, r, idx=idx, label="C2 %s" % kw, spacing=SP)


@pytest.mark.parametrize("name", ["C3", "C4", "C5"])
def test_full_size_sampled(pt, name):
    """C3 (wells, sigma^2 = 4), C4 (batched, 16 realisations) and C5 (timeseries) in the
    benchmark's launch; a 1e5-particle oracle sample bitwise identical."""
    w = _workload(name)
    p = w.particles
    out = _run(name)
    _check_counters(out, p)
    _check_invariants(out, p, name)
    m = 0
    for idx, r in _oracle_sample(name):
        compare(out, r, idx=idx, label="%s sample" % name, spacing=SP)
        m += idx.size
    sc = out["summary"]["status_count"]
    if name == "C3":
        assert sc[2] > 0 and sc[1] > 0       # wells capture some particles, the rest leave the domain
    if name == "C5":
        sx = out["snap_xyz"]
        assert sx.shape == (p.n, 100, 3)
        # every particle is defined at its release (t = 0 < 1 d)
        assert not np.isnan(sx[:, 0, :]).any()
    print("%s: %d sampled particles bitwise identical, crossings %d, statuses %s, kernel %.3f ms"
          % (name, m, out["summary"]["crossings"], sc, out["summary"]["kernel_ms"]))


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


def _state(d, idx=None):
    sel = (lambda a: a) if idx is None else (lambda a: a[idx])
    return {k: sel(d[k]) for k in ("status", "t", "ncross", "path_hash")}


@pytest.mark.parametrize("name", ["C2", "C3", "C4", "C5"])
def test_mixed_precision_accuracy(pt, name):
    """Mixed FP32/FP64 against the FP64 GPU run (every particle) and the FP64 oracle (sample):
    path agreement, travel-time error, and for C5 the snapshot positions; reported with loose
    sanity bounds."""
    w = _workload(name)
    p = w.particles
    mix = _run(name, "mixed")
    _check_counters(mix, p)
    _check_invariants(mix, p, name + " mixed")
    ref = _run(name)
    vs_fp64 = ACC.path_agreement(_state(mix), _state(ref), p.t)
    o_state = {k: [] for k in ("status", "t", "ncross", "path_hash")}
    ids = []
    snaps_m, snaps_o = [], []
    for idx, r in _oracle_sample(name):
        ids.append(idx)
        for k in o_state:
            o_state[k].append(getattr(r, k))
        if r.snap_xyz is not None:
            snaps_m.append(mix["snap_xyz"][idx])
            snaps_o.append(r.snap_xyz)
    idx = np.concatenate(ids)
    vs_oracle = ACC.path_agreement(_state(mix, idx), {k: np.concatenate(v) for k, v in o_state.items()}, p.t[idx])
    print("%s mixed vs FP64 run: %s" % (name, vs_fp64))
    print("%s mixed vs oracle (%d particles): %s" % (name, idx.size, vs_oracle))
    for acc in (vs_fp64, vs_oracle):
        assert acc["path_agreement"] >= 0.5
        assert acc["travel_time_rel_err"]["p50"] <= 1e-4
    if w.snap_times is not None:
        tr_fp64 = ACC.trajectory_error(mix["snap_xyz"], ref["snap_xyz"])
        tr_oracle = ACC.trajectory_error(np.concatenate(snaps_m), np.concatenate(snaps_o))
        print("%s mixed snapshots vs FP64 run: %s" % (name, tr_fp64))
        print("%s mixed snapshots vs oracle: %s" % (name, tr_oracle))
        for tr in (tr_fp64, tr_oracle):
            assert tr["position_err_m"]["p50"] <= 1.0
            assert tr["nan_pattern_agreement"] >= 0.9
