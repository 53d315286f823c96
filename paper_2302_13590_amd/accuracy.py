"""Accuracy of a mixed-precision tracking result against an FP64 one.

The mixed-precision kernels (FP32 in-cell arithmetic; FP64 time, global position and the
near-zero-gradient branch) are not bitwise reproducible against the FP64 path, so their accuracy
is reported: how many cell paths agree exactly, how far the travel times and the timeseries
positions move.  These are plain comparisons of two result sets (no tracking arithmetic), used by
the benchmark and the tests.
"""
from __future__ import annotations

import numpy as np

BOUNDARY, SINK = 1, 2


def _quantiles(v, qs=(0.5, 0.99, 1.0)):
    if v.size == 0:
        return [float("nan")] * len(qs)
    return [float(x) for x in np.quantile(v, qs)]


def path_agreement(mix: dict, ref: dict, t0) -> dict:
    """Cell-path agreement and travel-time error of `mix` against `ref` (final states of the same
    particles: dicts with status, t, ncross, path_hash as numpy arrays; t0 the release times).

    path_agreement: fraction of particles with the same path hash and crossing count.
    travel_time_rel_err: |T_mix - T_ref| / T_ref, T = t - t0, over the particles both runs
    terminated in a boundary face or a sink cell (p50, p99, max)."""
    t0 = np.asarray(t0)
    same = (mix["path_hash"] == ref["path_hash"]) & (mix["ncross"] == ref["ncross"])
    done = np.isin(ref["status"], (BOUNDARY, SINK)) & np.isin(mix["status"], (BOUNDARY, SINK))
    tt = ref["t"][done] - t0[done]
    pos = tt > 0
    rel = np.abs((mix["t"][done] - t0[done])[pos] - tt[pos]) / tt[pos]
    q = _quantiles(rel)
    return {"particles": int(same.size), "path_agreement": round(float(same.mean()), 6) if same.size else None,
            "status_agreement": round(float((mix["status"] == ref["status"]).mean()), 6) if same.size else None,
            "travel_time_rel_err": {"p50": q[0], "p99": q[1], "max": q[2], "particles": int(rel.size)}}


def trajectory_error(snap_mix, snap_ref) -> dict:
    """Timeseries positions of `snap_mix` against `snap_ref` ([n, n_snap, 3], numpy arrays or
    device tensors): |dxyz| (m) over the entries both define (p50, p99, max), and the fraction of
    (particle, time) entries whose definedness (position or NaN) agrees."""
    try:
        import torch
        is_t = isinstance(snap_mix, torch.Tensor)
    except ImportError:  # pragma: no cover
        is_t = False
    if is_t:
        nm = torch.isnan(snap_mix[..., 0])
        nr = torch.isnan(snap_ref[..., 0])
        agree = float((nm == nr).double().mean())
        both = ~nm & ~nr
        d = torch.linalg.vector_norm(snap_mix[both] - snap_ref[both], dim=-1)
        m = int(d.numel())
        if m:
            s, _ = torch.sort(d)
            q = [float(s[min(m - 1, int(round(f * (m - 1))))]) for f in (0.5, 0.99, 1.0)]
        else:
            q = [float("nan")] * 3
    else:
        nm = np.isnan(snap_mix[..., 0])
        nr = np.isnan(snap_ref[..., 0])
        agree = float((nm == nr).mean())
        both = ~nm & ~nr
        d = np.linalg.norm(snap_mix[both] - snap_ref[both], axis=-1)
        m = int(d.size)
        q = _quantiles(d)
    return {"position_err_m": {"p50": q[0], "p99": q[1], "max": q[2], "entries": m},
            "nan_pattern_agreement": round(agree, 6)}
