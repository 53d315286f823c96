"""Helpers of the GPU tests: run the HIP path through the C ABI and compare with the oracle."""
from __future__ import annotations

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_13590_amd import pt
    pt.load_library()  # raises ImportError if the library is not built: no fallback
    return pt


def gpu_track(grids_np, particles, *, group_offsets=None, group_grid=None, snap_times=None,
              snap_init=None, out_xyz=True, **opt):
    """Load the grids, copy the particles to the device, track, return numpy outputs + summary."""
    from paper_2302_13590_amd import pt
    dev = "cuda"
    handles = [pt.load_any_grid(g) for g in grids_np]
    try:
        dp = pt.DeviceParticles.from_numpy(particles, dev)
        n = dp.n
        oxyz = torch.full((n, 3), float("nan"), dtype=torch.float64, device=dev) if out_xyz else None
        sx = None
        if snap_times is not None:
            ns = len(snap_times)
            if snap_init is not None:
                sx = torch.from_numpy(np.ascontiguousarray(snap_init)).to(dev)
            else:
                sx = torch.full((n, ns, 3), float("nan"), dtype=torch.float64, device=dev)
            opt["mode"] = pt.PT_TIMESERIES
        summ = pt.track(handles, dp, group_offsets=group_offsets, group_grid=group_grid,
                        snap_times=snap_times, snap_xyz=sx, out_xyz=oxyz, **opt)
        torch.cuda.synchronize()
        out = dp.to_numpy()
        out["out_xyz"] = oxyz.cpu().numpy() if oxyz is not None else None
        out["snap_xyz"] = sx.cpu().numpy() if sx is not None else None
        out["summary"] = summ
        return out
    finally:
        for h in handles:
            h.release()


def compare(g: dict, r, idx=None, rtol: float = 1e-12, label: str = "", spacing=(1.0, 1.0, 1.0),
            exact: bool = True):
    """Element-by-element parity of the GPU outputs g with the oracle result r.

    Cell, status, crossing count and path hash must be identical.  Times agree within
    rtol relative; global positions within rtol relative to the norm of the position
    vector (floor 1); a local coordinate's error is measured in global units (times the
    cell size `spacing`) against the same bound.  idx selects the GPU rows that correspond
    to the oracle rows (sampled comparisons).
    With ``exact`` (the FP64 path, whose every operation including log1p, expm1 and log
    is correctly rounded on both sides) the floating-point outputs must also be bitwise
    identical; the rtol checks run first so that a failure reports its size.
    """
    sel = (lambda a: a) if idx is None else (lambda a: a[idx])
    n = len(r.status)
    bad = {}
    for name, a, b in (("status", sel(g["status"]), r.status), ("cell", sel(g["cell"]), r.cell),
                       ("ncross", sel(g["ncross"]), r.ncross),
                       ("path_hash", sel(g["path_hash"]), r.path_hash)):
        m = a != b
        if m.any():
            bad[name] = np.nonzero(m)[0][:10].tolist()
    assert not bad, "%s: integer mismatch in %d/%d particles: %s" % (
        label, len(set(sum(bad.values(), []))), n, bad)
    pos_scale = np.maximum(np.nan_to_num(np.linalg.norm(r.out_xyz, axis=-1), nan=1.0), 1.0)
    for ax, (name, a, b) in enumerate((("xi", sel(g["xi"]), r.xi), ("eta", sel(g["eta"]), r.eta),
                                       ("zeta", sel(g["zeta"]), r.zeta))):
        with np.errstate(invalid="ignore"):
            d = np.abs(a - b) * spacing[ax]
        ok = (a == b) | (d <= rtol * pos_scale) | (np.isnan(a) & np.isnan(b))
        assert ok.all(), "%s: %s max diff %.3e at %s" % (label, name, np.nanmax(d), np.nonzero(~ok)[0][:5])
    a, b = sel(g["t"]), r.t
    with np.errstate(invalid="ignore"):
        d = np.abs(a - b)
    ok = (a == b) | (d <= rtol * np.maximum(np.abs(b), 1.0)) | (np.isnan(a) & np.isnan(b))
    assert ok.all(), "%s: t max rel diff %.3e" % (label, np.nanmax(d / np.maximum(np.abs(b), 1.0)))
    if g.get("out_xyz") is not None:
        a, b = sel(g["out_xyz"]), r.out_xyz
        close_xyz(a, b, rtol, label + " out_xyz")
    if g.get("snap_xyz") is not None and r.snap_xyz is not None:
        close_xyz(sel(g["snap_xyz"]), r.snap_xyz, rtol, label + " snap_xyz")
    if exact:
        pairs = [("xi", r.xi), ("eta", r.eta), ("zeta", r.zeta), ("t", r.t), ("out_xyz", r.out_xyz)]
        if g.get("snap_xyz") is not None and r.snap_xyz is not None:
            pairs.append(("snap_xyz", r.snap_xyz))
        for name, b in pairs:
            a = sel(g[name])
            same = (a == b) | (np.isnan(a) & np.isnan(b))
            assert same.all(), "%s: %s not bitwise identical in %d entries" % (label, name, int((~same).sum()))
    amb = g.get("summary", {}).get("cr_ambiguous", 0)
    assert amb == 0, "%s: %d undecided correctly rounded evaluations" % (label, amb)


def close_xyz(a, b, rtol, label):
    """Global positions [..., 3]: |a - b| <= rtol * max(|b|, 1), norms taken over the last axis."""
    na, nb = np.isnan(a), np.isnan(b)
    assert (na == nb).all(), "%s: NaN pattern differs in %d entries" % (label, int((na != nb).sum()))
    d = np.linalg.norm(np.where(na, 0.0, a - b), axis=-1)
    scale = np.maximum(np.linalg.norm(np.where(nb, 0.0, b), axis=-1), 1.0)
    assert (d <= rtol * scale).all(), "%s: max rel diff %.3e" % (label, float(np.max(d / scale)))


def sample_indices(n: int, m: int, seed: int = 7) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    if m >= n:
        return np.arange(n)
    return np.sort(rng.choice(n, size=m, replace=False))


def tracked_counts(before_status, after_status):
    tracked = (before_status == 0) | (before_status == 3)
    return tracked, np.bincount(after_status[tracked], minlength=8)


INF = math.inf


def bench_opts(wname, precision="fp64", mode="endpoint"):
    """The launch the benchmark times for a workload: its autotuned parameters (schedule, block,
    order, queue shape) on this device, packed layout, hipGraph; the persistent kernel with its
    defaults where no tuned entry exists."""
    from paper_2302_13590_amd import autotune
    params = autotune.lookup(autotune.key(autotune.device_name(), wname, precision, mode)) or dict(schedule=2)
    return dict(params, layout=2, use_graph=1, precision=0 if precision == "fp64" else 1)


def other_schedule(opts):
    """The other kernel, with its default launch shape."""
    return dict(schedule=1 if opts["schedule"] == 2 else 2, layout=2, use_graph=1, precision=opts["precision"])
