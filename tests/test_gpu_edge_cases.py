"""FP64 parity with the oracle on the method's per-cell edge cases, through the C ABI.

The semi-analytical step (paper: Introduction; Methods "MODPATH", its stopping conditions) has
cases that random lognormal grids rarely or never reach.  The FP64 kernels choose the exit face
from FP32 estimates and fall back to evaluating all three axes exactly only when an estimate is
unsure or another axis lies within 2^-15 of the candidate; these cases drive that fallback on
purpose:

  * every hand-built single-cell case of the oracle's pins (tests/golden/single_cell.json: exit
    times and positions, uniform, accelerating, decelerating, strong deceleration down to a face
    velocity of 1e-15, tiny gradients 1e-12 and 3e-16, divergent, convergent, stagnant face,
    start on the face), on each axis;
  * the exact corner tie with its zero-time crossing, and multi-axis uniform flow;
  * the stopping conditions and degenerate starts of the pins;
  * exact and near ties (inside the 2^-15 margin) on diagonal flows;
  * velocity fields scaled so that particle velocities leave the FP32 range of the estimate
    (below 2^-100 and above 2^100, and far beyond), and exit times in the FP32 subnormal range,
    where the estimates' rounding can reverse the order of two axes.

Every case runs through the static and persistent kernels in both layouts (face arrays and packed
records), and the single-cell cases also through the batched kernels in one launch; every FP64
output must be bitwise identical to the oracle's.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs as C
from workloads.configs import FLAG_ACTIVE, FLAG_SINK

from . import helpers as H
from .gpu_util import compare, gpu_track, require_gpu, tracked_counts

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "single_cell.json")
FORMS = [dict(schedule=1, layout=1), dict(schedule=1, layout=2), dict(schedule=2, layout=1),
         dict(schedule=2, layout=2, use_graph=1)]


@pytest.fixture(scope="module")
def pt():
    return require_gpu()


def _parity(g, p, label, forms=FORMS, rechecks=None, **kw):
    """Oracle and every kernel form on the same inputs, bitwise; also the counters.  `rechecks`
    collects the particles each run handed to the careful pass."""
    r = O.track(g, p, **kw)
    tracked, counts = tracked_counts(p.status, r.status)
    for f in forms:
        out = gpu_track([g], p, **f, **kw)
        compare(out, r, label="%s %s" % (label, f), spacing=(g.dx, g.dy, g.dz))
        s = out["summary"]
        assert s["crossings"] == int(r.ncross.astype(np.int64).sum() - p.ncross.astype(np.int64).sum()), label
        assert s["status_count"] == counts.tolist(), label
        if rechecks is not None:
            rechecks.append(s["recheck_tracks"])
    return r


def _one_axis_grid(axis, ql, qh, geom, origin=(5.0, -3.0, 11.0)):
    g = H.box_grid(1, 1, 1, geom["dx"], geom["dy"], geom["dz"], origin=origin, porosity=geom["porosity"])
    if axis == 0:
        g.qx[0, 0, 0], g.qx[0, 0, 1] = ql, qh
    elif axis == 1:
        g.qy[0, 0, 0], g.qy[0, 1, 0] = ql, qh
    else:
        g.qz[0, 0, 0], g.qz[1, 0, 0] = ql, qh
    return g


def _golden_cases():
    gold = json.load(open(GOLDEN))
    geom = gold["geometry"]
    out = []
    for kind in ("exit", "position"):
        for case in gold[kind]:
            for axis in range(3):
                loc = [0.5, 0.5, 0.5]
                loc[axis] = case["xi"]
                t_max = case["tau"] if kind == "position" else np.inf
                out.append(("%s/%s/axis%d" % (kind, case["name"], axis),
                            _one_axis_grid(axis, case["q_low"], case["q_high"], geom), loc, t_max))
    return out


def test_golden_single_cell(pt):
    """Every single-cell exit and position case of the oracle's decimal pins, each axis, every
    kernel form; the exit times themselves are pinned to 60-digit closed forms by the oracle's
    tests, so bitwise parity carries the pin to the GPU."""
    for name, g, loc, t_max in _golden_cases():
        _parity(g, H.particles([0], *loc), name, t_max=t_max)


def test_golden_single_cell_batched(pt):
    """All steady single-cell cases as particle groups of one batched launch (one grid each)."""
    cases = [c for c in _golden_cases() if not np.isfinite(c[3])]
    grids = [g for _, g, _, _ in cases]
    p = C.concat([H.particles([0], *loc) for _, _, loc, _ in cases])
    offs = np.arange(len(cases) + 1, dtype=np.int64)
    gg = np.arange(len(cases), dtype=np.int32)
    r = O.track_groups(grids, p, offs, gg)
    for f in (dict(schedule=1), dict(schedule=2), dict(schedule=1, sort=2, use_graph=1)):
        out = gpu_track(grids, p, group_offsets=offs, group_grid=gg, layout=2, **f)
        compare(out, r, label="golden batched %s" % f, spacing=(7.0, 3.0, 2.0))


def test_corner_tie_and_uniform_axes(pt):
    g = H.box_grid(2, 2, 1, 1.0, 1.0, 1.0, porosity=1.0)
    g.qx[:] = 1.0
    g.qy[:] = 1.0
    r = _parity(g, H.particles([0], 0.5, 0.5, 0.5), "corner tie")
    assert r.ncross[0] == 3 and r.t[0] == 1.5 and r.cell[0] == 3          # the zero-time step counts
    dx, dy, dz, n = 4.0, 2.5, 1.25, 0.2
    for q, loc in [((3.0, 2.0, 0.5), (0.1, 0.2, 0.3)), ((-3.0, 2.0, 0.5), (0.9, 0.4, 0.3)),
                   ((1.0, -5.0, 0.1), (0.2, 0.35, 0.75)), ((0.2, 0.3, -4.0), (0.4, 0.6, 0.5))]:
        g = H.box_grid(1, 1, 1, dx, dy, dz, porosity=n)
        g.qx[:], g.qy[:], g.qz[:] = q
        _parity(g, H.particles([0], *loc), "uniform %s" % (q,))


def _line(nx, q=3.0, flags=None):
    g = H.box_grid(nx, 1, 1, 10.0, 10.0, 10.0, porosity=0.3, flags=flags)
    g.qx[:] = q
    return g


def test_stopping_conditions(pt):
    fl = np.full((1, 1, 3), FLAG_ACTIVE, np.int32)
    fl[0, 0, 2] |= FLAG_SINK
    gs = _line(3, flags=fl)
    g2 = _line(3)
    u = 3.0 / (0.3 * 1000.0)
    _parity(gs, H.particles([0, 2], [0.5, 0.3], 0.5, 0.5, [0.0, 7.0]), "sink entry and release")
    _parity(gs, H.particles([0, 2], [0.5, 0.3], 0.5, 0.5), "weak sink", stop_at_sink=0)
    _parity(g2, H.particles([0], 0.5, 0.5, 0.5), "step cap", max_steps=1)
    _parity(g2, H.particles([0], 0.5, 0.5, 0.5), "time limit", t_max=120.0)
    _parity(g2, H.particles([0], 0.5, 0.5, 0.5), "face at t_max", t_max=0.5 / u)
    _parity(g2, H.particles([0], 0.5, 0.5, 0.5, t=300.0), "release after t_max", t_max=200.0)
    _parity(g2, H.particles([-1, 3, 0, 0, 0, 0], [0.5, 0.5, np.nan, 1.5, 0.5, 0.5],
                            [0.5, 0.5, 0.5, 0.5, -0.1, 0.5], 0.5, [0, 0, 0, 0, 0, np.nan]), "invalid starts")
    fl = np.full((1, 1, 3), FLAG_ACTIVE, np.int32)
    fl[0, 0, 1] = 0
    _parity(_line(3, flags=fl), H.particles([1, 0], 0.5, 0.5, 0.5), "inactive neighbour")
    g4 = _line(2, q=0.0)
    _parity(g4, H.particles([1], 0.25, 0.5, 0.75, t=3.0), "no flow")
    _parity(g4, H.particles([1], 0.25, 0.5, 0.75, t=3.0), "no flow, t_max", t_max=10.0)
    _parity(g2, H.particles([0, 0, 2], [1.0, 0.0, 1.0], 0.5, 0.5), "start on a face", max_steps=1)
    _parity(g2, H.particles([1, 2], [0.25, 0.0], 0.5, 0.5), "backward", direction=-1)


def test_ties_inside_the_margin(pt):
    """Diagonal flows: the exit times of x and y tie exactly (equal flows, xi = eta) or differ by
    1e-16 .. 1e-4 relative, inside and just outside the 2^-15 selection margin; the tie-break
    sends the particle through the lower axis first, then a zero-time crossing."""
    rng = np.random.Generator(np.random.PCG64(91))
    n = 3000
    base = rng.uniform(0.02, 0.98, n)
    off = np.where(rng.random(n) < 0.3, 0.0, rng.choice([-1.0, 1.0], n) * 10.0 ** rng.uniform(-16, -3, n))
    eta = np.clip(base + off * base, 0.0, 1.0)
    for d in (0.0, 1e-15, 1e-12, 1e-9, 3e-6, 2.0 ** -15, 1e-4):
        g = H.box_grid(6, 6, 2, 1.0, 1.0, 1.0, porosity=0.5)
        g.qx[:] = 0.7
        g.qy[:] = 0.7 * (1.0 + d)
        g.qz[:] = 1e-3
        g.qz[0] = 0.0
        g.qz[-1] = 0.0
        cells = rng.integers(0, 36, n)
        _parity(g, H.particles(cells, base, eta, rng.random(n)), "ties d=%g" % d)


def test_ties_with_gradients(pt):
    """Accelerating diagonal flow (the same gradient on x and y): ties persist along the path.
    Velocities of a few bits make some log1p and expm1 arguments near 2^-53 .. 2^-50 land within
    2^-100 of a rounding midpoint; the tracking kernels leave those undecided and hand the
    particles to the careful pass, which decides them exactly (27 such evaluations in this
    input): the results must still be bitwise the oracle's, with no undecided evaluation left."""
    rng = np.random.Generator(np.random.PCG64(92))
    g = H.box_grid(8, 8, 1, 2.0, 2.0, 1.0, porosity=0.3)
    for i in range(9):
        g.qx[:, :, i] = 0.5 * (1.0 + 0.25 * i)
    for j in range(9):
        g.qy[:, j, :] = 0.5 * (1.0 + 0.25 * j)
    n = 2000
    x = rng.random(n)
    y = np.where(rng.random(n) < 0.5, x, np.clip(x * (1.0 + 10.0 ** rng.uniform(-15, -5, n)), 0, 1))
    i = rng.integers(0, 8, n)
    cells = i * 8 + i                                  # on the diagonal: both axes see the same flow
    rechecks = []
    _parity(g, H.particles(cells, x, y, 0.5), "gradient ties", rechecks=rechecks, max_steps=5000)
    assert min(rechecks) > 0, rechecks                 # the careful pass ran in every kernel form
    snaps = np.linspace(0.0, 40.0, 33)
    r = O.track(g, H.particles(cells, x, y, 0.5), snap_times=snaps, max_steps=5000)
    for f in FORMS:
        out = gpu_track([g], H.particles(cells, x, y, 0.5), snap_times=snaps, max_steps=5000, **f)
        compare(out, r, label="gradient ties, timeseries %s" % f, spacing=(g.dx, g.dy, g.dz))
        assert out["summary"]["recheck_tracks"] > 0


@pytest.mark.parametrize("scale", [1e-35, 1e-300, 1e33, 1e300])
def test_flows_beyond_the_fp32_range(pt, scale):
    """A lognormal grid with a well and recharge, every face flow scaled: particle velocities
    below 2^-100 (1e-35), near the bottom of FP64 (1e-300), above 2^100 (1e33) and near the top
    of FP64 (1e300) make the FP32 estimates unsure on every axis.  Scaling every flow by the same
    factor keeps the paths, so the crossing counts must also equal the unscaled run's."""
    g = C.random_grid(9, 7, 3, 1.5, 2.0, 55, wells=((4, 3, -30.0),), recharge=2e-3)
    rng = np.random.Generator(np.random.PCG64(56))
    p = C.release(rng, 1500, g.nx, g.ny, g.nz)
    ref = O.track(g, p)
    gs = C.Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.x0, g.y0, g.z0, g.qx * scale, g.qy * scale,
                g.qz * scale, g.flags, None, g.porosity_scalar)
    r = _parity(gs, p, "scaled %g" % scale)
    assert np.all(np.isfinite(r.t))
    assert np.mean(r.path_hash == ref.path_hash) > 0.5       # scaling moves only near-ties
    t_mid = float(np.median(r.t))
    _parity(gs, p, "scaled %g, t_max" % scale, t_max=t_mid)


def test_subnormal_exit_times(pt):
    """Exit times in the FP32 subnormal range: a particle 1.2542e-43 from its exit face on x
    (u = -0.125) and 1.00515e-42 on y (u = -1) leaves through x first (1.00336e-42 against
    1.00515e-42), although FP32 estimates rounded to multiples of 2^-149 order the two the other
    way.  Random variants: distances from 1e-320 to 1e-30 on two axes, velocities of either sign."""
    g = H.box_grid(1, 1, 1, 1.0, 1.0, 1.0, porosity=1.0)
    g.qx[:] = -0.125
    g.qy[:] = -1.0
    r = _parity(g, H.particles([0], 1.2542e-43, 1.00515e-42, 0.5), "subnormal counterexample")
    assert r.status[0] == 1 and r.xi[0] == 0.0 and r.eta[0] > 0.0       # out through the low x face
    rng = np.random.Generator(np.random.PCG64(93))
    n = 4000
    for ux, uy in ((-0.125, -1.0), (-3.0, -2.9999), (-1e-20, -1e-21), (-1e20, -3e19)):
        g = H.box_grid(1, 1, 1, 1.0, 1.0, 1.0, porosity=1.0)
        g.qx[:] = ux
        g.qy[:] = uy
        a = 10.0 ** rng.uniform(-320, -30, n)
        b = a * np.where(rng.random(n) < 0.5, abs(uy / ux), 10.0 ** rng.uniform(-2, 2, n)) * \
            (1.0 + rng.uniform(-1e-3, 1e-3, n))
        _parity(g, H.particles(np.zeros(n, np.int64), a, np.clip(b, 0.0, 1.0), 0.5), "subnormal %g %g" % (ux, uy))
