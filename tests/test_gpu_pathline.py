"""Pathline mode (one record per cell crossing), FP64 parity with the oracle through the C ABI.

The library produces pathlines in two passes (a dry count pass that writes the CSR offsets,
then the record pass); the oracle records the same crossings particle by particle.  Every
record (cell left, face, time, position on the face) must be bitwise identical, the offsets
must be the prefix sum of the oracle's crossing counts, and the final state must equal the
oracle's as in endpoint mode.  Slot ranges outside the record arrays are never written.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs as C

from . import helpers as H
from .gpu_util import bench_opts, compare, require_gpu, sample_indices

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
SP = (10.0, 10.0, 2.0)


@pytest.fixture(scope="module")
def pt():
    return require_gpu()


def oracle_paths(grid, p, **kw):
    """Oracle run with a per-particle record capacity large enough for every particle."""
    cap = 256
    while True:
        r = O.track(grid, p, path_cap=cap, **kw)
        cnt = (r.ncross.astype(np.int64) - p.ncross.astype(np.int64))
        if cnt.size == 0 or cnt.max() <= cap:
            break
        cap = int(cnt.max())
    keep = np.arange(cap)[None, :] < cnt[:, None]
    flat = dict(cell=r.path_cell[keep], face=r.path_face[keep], t=r.path_t[keep], xyz=r.path_xyz[keep])
    offs = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    return r, offs, flat


def gpu_pathlines(pt, grids, p, group_offsets=None, group_grid=None, **opt):
    handles = [pt.load_any_grid(g) for g in grids]
    try:
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        oxyz = torch.full((dp.n, 3), float("nan"), dtype=torch.float64, device="cuda")
        s, pl = pt.track_pathlines(handles, dp, group_offsets=group_offsets, group_grid=group_grid,
                                   out_xyz=oxyz, **opt)
        torch.cuda.synchronize()
        out = dp.to_numpy()
        out["out_xyz"] = oxyz.cpu().numpy()
        out["summary"] = s
        paths = dict(offsets=pl.offsets.cpu().numpy(), cell=pl.cell.cpu().numpy(), face=pl.face.cpu().numpy(),
                     t=pl.t.cpu().numpy(), xyz=pl.xyz.cpu().numpy())
        return out, paths
    finally:
        for h in handles:
            h.release()


def compare_paths(paths, offs, flat, label):
    assert np.array_equal(paths["offsets"], offs), "%s: offsets differ" % label
    for name in ("cell", "face"):
        a, b = paths[name], flat[name]
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, "%s: %s differs in %d records, first %s" % (label, name, bad.size, bad[:5])
    for name in ("t", "xyz"):
        a, b = paths[name], flat[name]
        with np.errstate(invalid="ignore"):
            rel = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
        assert np.all(rel <= 1e-12), "%s: %s max rel diff %.3e" % (label, name, float(np.max(rel)))
        assert np.array_equal(a, b), "%s: %s not bitwise identical" % (label, name)


CASES = {
    "lognormal_wells": lambda: C.random_grid(24, 17, 5, 1.5, 3.0, 101, wells=((8, 8, -60.0), (17, 5, -40.0)),
                                             recharge=2e-3, origin=(250.0, -40.0, 7.5)),
    "porosity_field": lambda: C.random_grid(19, 23, 3, 2.5, 4.0, 202, dx=5.0, dy=8.0, dz=1.0,
                                            porosity_field=True),
    "c1": lambda: C.c1().grids[0],
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("sched", [1, 2])
@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("direction", [1, -1])
def test_pathline_small(pt, case, sched, layout, direction):
    g = CASES[case]()
    rng = np.random.Generator(np.random.PCG64(len(case) * 7 + sched))
    p = C.release(rng, 2999, g.nx, g.ny, g.nz)
    r, offs, flat = oracle_paths(g, p, direction=direction)
    out, paths = gpu_pathlines(pt, [g], p, schedule=sched, layout=layout, direction=direction)
    label = "%s sched %d layout %d dir %d" % (case, sched, layout, direction)
    compare(out, r, label=label, spacing=(g.dx, g.dy, g.dz))
    compare_paths(paths, offs, flat, label)
    s = out["summary"]
    assert s["path_records"] == offs[-1] == s["crossings"] and s["path_dropped"] == 0


def test_pathline_limits_and_edge_starts(pt):
    g = CASES["lognormal_wells"]()
    ncell = g.nx * g.ny * g.nz
    p = H.particles([0, -5, ncell, 3, 4, 5, 6, 8 * g.nx + 8, 7, 9],
                    [0.5, 0.5, 0.5, np.nan, 1.5, 0.2, 1.0, 0.4, 0.3, 0.6],
                    [0.5, 0.5, 0.5, 0.5, 0.5, -0.1, 0.0, 0.4, 0.3, 0.6], 0.5,
                    [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, np.inf, 0.0])
    p.status[9] = 1
    r, offs, flat = oracle_paths(g, p)
    out, paths = gpu_pathlines(pt, [g], p)
    compare(out, r, label="edge starts", spacing=SP)
    compare_paths(paths, offs, flat, "edge starts")
    rng = np.random.Generator(np.random.PCG64(8))
    q = C.release(rng, 777, g.nx, g.ny, g.nz)
    for kw in (dict(max_steps=1), dict(max_steps=7), dict(t_max=0.0), dict(t_max=12.5), dict(stop_at_sink=0)):
        r, offs, flat = oracle_paths(g, q, **kw)
        for sched in (1, 2):
            out, paths = gpu_pathlines(pt, [g], q, schedule=sched, **kw)
            compare(out, r, label="limits %s" % kw, spacing=SP)
            compare_paths(paths, offs, flat, "limits %s sched %d" % (kw, sched))


def test_pathline_resume_concatenates(pt):
    g = CASES["lognormal_wells"]()
    rng = np.random.Generator(np.random.PCG64(4))
    p = C.release(rng, 1500, g.nx, g.ny, g.nz)
    _, offs, flat = oracle_paths(g, p)
    handles = [pt.pt_load_grid(g)]
    try:
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        parts = []
        for t_max in (20.0, 150.0, math.inf):
            s, pl = pt.track_pathlines(handles, dp, t_max=t_max)
            parts.append((pl.offsets.cpu().numpy(), pl.t.cpu().numpy(), pl.cell.cpu().numpy()))
        for q in (0, 17, 1499):
            t = np.concatenate([pt_[o[q]:o[q + 1]] for o, pt_, _ in parts])
            c = np.concatenate([c_[o[q]:o[q + 1]] for o, _, c_ in parts])
            assert np.array_equal(t, flat["t"][offs[q]:offs[q + 1]])
            assert np.array_equal(c, flat["cell"][offs[q]:offs[q + 1]])
    finally:
        handles[0].release()


def test_count_pass_is_dry_and_record_pass_bounded(pt):
    g = CASES["porosity_field"]()
    rng = np.random.Generator(np.random.PCG64(12))
    p = C.release(rng, 1234, g.nx, g.ny, g.nz)
    r, offs, flat = oracle_paths(g, p)
    m = int(offs[-1])
    handles = [pt.pt_load_grid(g)]
    try:
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        before = dp.to_numpy()
        oxyz = torch.full((dp.n, 3), 7.0, dtype=torch.float64, device="cuda")
        offsets = torch.full((dp.n + 1,), -99, dtype=torch.int64, device="cuda")
        for sched in (1, 2):
            s = pt.track(handles, dp, mode=pt.PT_PATHLINE, path_offsets=offsets, path_count_only=1,
                         out_xyz=oxyz, schedule=sched)
            after = dp.to_numpy()
            for k in before:
                assert np.array_equal(before[k], after[k]), "count pass wrote %s" % k
            assert torch.all(oxyz == 7.0)
            assert np.array_equal(offsets.cpu().numpy(), offs)
            assert s["path_records"] == m and s["crossings"] == m
        # record pass into arrays that hold half of the records, with a guard zone after them
        cap, guard = m // 2, 4096
        rec = torch.full((cap + guard, 5), -7.0, dtype=torch.float64, device="cuda")
        pl = pt.Pathlines(offsets, rec)
        work = pt.DeviceParticles.from_numpy(p, "cuda")
        s = pt.track(handles, work, mode=pt.PT_PATHLINE, path_offsets=offsets, path_cap=cap, path_records=rec,
                     out_xyz=oxyz)
        assert s["path_dropped"] == m - cap and s["path_records"] == cap
        assert torch.all(rec[cap:] == -7.0)
        assert np.array_equal(pl.cell[:cap].cpu().numpy(), flat["cell"][:cap])
        assert np.array_equal(pl.face[:cap].cpu().numpy(), flat["face"][:cap])
        assert np.array_equal(pl.t[:cap].cpu().numpy(), flat["t"][:cap])
        assert np.array_equal(pl.xyz[:cap].cpu().numpy(), flat["xyz"][:cap])
        compare(dict(work.to_numpy(), out_xyz=oxyz.cpu().numpy(), summary=s), r, label="bounded record pass",
                spacing=(5.0, 8.0, 1.0))
        # offsets that point nowhere: nothing is written, every record is dropped
        bad = torch.full((dp.n + 1,), -5, dtype=torch.int64, device="cuda")
        rec.fill_(-7.0)
        work = pt.DeviceParticles.from_numpy(p, "cuda")
        s = pt.track(handles, work, mode=pt.PT_PATHLINE, path_offsets=bad, path_cap=cap, path_records=rec)
        assert s["path_dropped"] == m and s["path_records"] == 0 and torch.all(rec == -7.0)
        # empty call: only the leading zero
        empty = C.release(rng, 0, g.nx, g.ny, g.nz)
        de = pt.DeviceParticles.from_numpy(empty, "cuda")
        o1 = torch.full((1,), 5, dtype=torch.int64, device="cuda")
        s = pt.track(handles, de, mode=pt.PT_PATHLINE, path_offsets=o1, path_count_only=1)
        assert int(o1.item()) == 0 and s["path_records"] == 0
    finally:
        handles[0].release()


def test_pathline_option_errors(pt):
    g = CASES["c1"]()
    handles = [pt.pt_load_grid(g)]
    try:
        dp = pt.DeviceParticles.from_numpy(C.c1().particles, "cuda")
        offs = torch.zeros(dp.n + 1, dtype=torch.int64, device="cuda")
        for kw in (dict(), dict(path_offsets=offs, path_count_only=2),
                   dict(path_offsets=offs, path_cap=-1), dict(path_offsets=offs, path_cap=10)):
            with pytest.raises(pt.PtError) as e:
                pt.track(handles, dp, mode=pt.PT_PATHLINE, **kw)
            assert e.value.code == -1, kw
    finally:
        handles[0].release()


def test_pathline_batched(pt):
    grids = [C.random_grid(12, 9, 4, s2, 2.0, 300 + r, wells=((5, 4, -30.0),) if r == 1 else (),
                           recharge=1e-3 * r) for r, s2 in enumerate((0.5, 1.5, 3.0))]
    sizes = [700, 0, 1, 1233, 64, 0, 999]
    gg = np.array([2, 0, 1, 1, 0, 2, 1], np.int32)
    go = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    rng = np.random.Generator(np.random.PCG64(77))
    parts = [C.release(rng, s, 12, 9, 4) for s in sizes]
    p = C.concat(parts)
    flats, cnts = [], []
    for q, gi in zip(parts, gg):
        _, offs, flat = oracle_paths(grids[gi], q)
        flats.append(flat)
        cnts.append(np.diff(offs))
    offs = np.concatenate([[0], np.cumsum(np.concatenate(cnts))]).astype(np.int64)
    flat = {k: np.concatenate([f[k] for f in flats]) for k in ("cell", "face", "t", "xyz")}
    for sched in (1, 2):
        out, paths = gpu_pathlines(pt, grids, p, group_offsets=go, group_grid=gg, schedule=sched)
        compare_paths(paths, offs, flat, "batched sched %d" % sched)


def _structure_on_device(pl, grid_shape):
    """Invariants of any pathline, checked on all records on the device: times never decrease
    within a particle, and each record's cell is the neighbour of the previous record's cell
    across that record's face."""
    nx, ny, nz = grid_shape
    starts = torch.zeros(pl.t.shape[0], dtype=torch.bool, device=pl.t.device)
    first = pl.offsets[:-1][pl.offsets[:-1] < pl.offsets[1:]]
    starts[first] = True
    cont = ~starts[1:]
    assert torch.all(pl.t[1:][cont] >= pl.t[:-1][cont])
    f = pl.face[:-1].long()
    step = torch.where(f % 2 == 1, 1, -1)
    stride = torch.tensor([1, nx, nx * ny], device=pl.t.device)[f // 2]
    nxt = pl.cell[:-1].long() + step * stride
    assert torch.all(pl.cell[1:].long()[cont] == nxt[cont])


@pytest.mark.parametrize("precision", [0, 1])
def test_pathline_c2_full_sampled(pt, precision):
    w = C.c2()
    p = w.particles
    handles = [pt.pt_load_grid(g) for g in w.grids]
    try:
        dp = pt.DeviceParticles.from_numpy(p, "cuda")
        # the launch the benchmark's pathline variant times: the tuned FP64 endpoint launch of C2
        kw = dict(bench_opts("C2"), precision=precision)
        s, pl = pt.track_pathlines(handles, dp, **kw)
        m = s["path_records"]
        assert m == s["crossings"] and s["path_dropped"] == 0 and int(pl.offsets[-1]) == m
        _structure_on_device(pl, (100, 100, 10))
        if precision == 0:
            idx = sample_indices(p.n, 1500, seed=23)
            _, offs, flat = oracle_paths(w.grids[0], p.subset(idx))
            o = pl.offsets.cpu().numpy()
            rows = np.concatenate([np.arange(o[q], o[q + 1]) for q in idx])
            sub = dict(offsets=np.concatenate([[0], np.cumsum(o[idx + 1] - o[idx])]).astype(np.int64))
            rows_t = torch.from_numpy(rows).cuda()
            sel = pt.Pathlines(pl.offsets, pl.records[rows_t].contiguous())
            for k in ("cell", "face", "t", "xyz"):
                sub[k] = getattr(sel, k).cpu().numpy()
            compare_paths(sub, offs, flat, "C2 pathline sample")
        print("C2 pathline precision %d records %d kernel ms %.3f" % (precision, m, s["kernel_ms"]))
    finally:
        for h in handles:
            h.release()
