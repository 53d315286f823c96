"""Pins of the oracle against what the mathematics fixes.

Each ``pin_*`` function takes an oracle library handle and raises AssertionError
if the oracle disagrees with a closed form, an invariant, a special case, or a
brute-force RK4 integration.  ``test_oracle_pins.py`` runs them on the real
oracle; ``test_oracle_mutations.py`` runs them on copies of the oracle with a
planted mistake and requires at least one to fail for every mistake.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from oracle import oracle as O
from workloads import configs as C
from workloads.configs import FLAG_ACTIVE, FLAG_SINK

from . import helpers as H

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BOUNDARY, SINK, MAX_TIME, STEP_CAP, STRANDED, INVALID, INACTIVE_NB = 1, 2, 3, 4, 5, 6, 7


def _one_axis_grid(axis, ql, qh, geom, origin=(5.0, -3.0, 11.0)):
    g = H.box_grid(1, 1, 1, geom["dx"], geom["dy"], geom["dz"], origin=origin,
                   porosity=geom["porosity"])
    if axis == 0:
        g.qx[0, 0, 0], g.qx[0, 0, 1] = ql, qh
    elif axis == 1:
        g.qy[0, 0, 0], g.qy[0, 1, 0] = ql, qh
    else:
        g.qz[0, 0, 0], g.qz[1, 0, 0] = ql, qh
    return g


def _close(a, b, rel, absol=0.0):
    return abs(a - b) <= max(rel * abs(b), absol)


def pin_single_cell_exit(lib):
    """Exit time of one axis equals ln(u_e/u_p)/A (60-digit decimal), on each axis in turn."""
    gold = json.load(open(os.path.join(GOLDEN, "single_cell.json")))
    geom = gold["geometry"]
    d = (geom["dx"], geom["dy"], geom["dz"])
    for case in gold["exit"]:
        for axis in range(3):
            g = _one_axis_grid(axis, case["q_low"], case["q_high"], geom)
            loc = [0.5, 0.5, 0.5]
            loc[axis] = case["xi"]
            r = O.track(g, H.particles([0], *loc), lib=lib)
            name = "%s axis %d" % (case["name"], axis)
            if case["t"] is None:
                assert r.status[0] == STRANDED, name
                assert r.ncross[0] == 0 and r.t[0] == 0.0, name
                assert [r.xi[0], r.eta[0], r.zeta[0]] == loc, name
                continue
            t_exact = float(case["t"])
            assert r.status[0] == BOUNDARY, (name, r.status[0])
            assert r.ncross[0] == 1, name
            assert _close(r.t[0], t_exact, 4e-16, 1e-300), (name, r.t[0], t_exact)
            # the particle sits on the exit face; the other axes did not move
            side = 1.0 if case["q_high"] > 0 and (case["q_low"] + (case["q_high"] - case["q_low"])
                                                  * case["xi"]) > 0 else 0.0
            fin = [r.xi[0], r.eta[0], r.zeta[0]]
            assert fin[axis] == side, (name, fin)
            for b in range(3):
                if b != axis:
                    assert fin[b] == 0.5, name
            org = (g.x0, g.y0, g.z0)
            assert r.out_xyz[0, axis] == org[axis] + side * d[axis], name


def pin_single_cell_position(lib):
    """In-cell position at t_max equals xi + u_p (exp(A tau) - 1)/A (60-digit decimal)."""
    gold = json.load(open(os.path.join(GOLDEN, "single_cell.json")))
    geom = gold["geometry"]
    for case in gold["position"]:
        for axis in range(3):
            g = _one_axis_grid(axis, case["q_low"], case["q_high"], geom)
            loc = [0.5, 0.5, 0.5]
            loc[axis] = case["xi"]
            r = O.track(g, H.particles([0], *loc), t_max=case["tau"], lib=lib)
            name = "%s axis %d" % (case["name"], axis)
            assert r.status[0] in (MAX_TIME, STRANDED), name
            assert r.t[0] == case["tau"], name
            fin = [r.xi[0], r.eta[0], r.zeta[0]]
            assert abs(fin[axis] - float(case["xi_tau"])) <= 4e-16, (name, fin[axis], case["xi_tau"])


def pin_multi_axis_uniform(lib):
    """Uniform flow on all three axes of a non-cubic cell: t = min_a (xi_e - xi_a)/u_a."""
    dx, dy, dz, n = 4.0, 2.5, 1.25, 0.2
    V = (dx * dy) * dz
    cases = [((3.0, 2.0, 0.5), (0.1, 0.2, 0.3)), ((-3.0, 2.0, 0.5), (0.9, 0.4, 0.3)),
             ((1.0, -5.0, 0.1), (0.2, 0.35, 0.75)), ((0.2, 0.3, -4.0), (0.4, 0.6, 0.5))]
    for q, loc in cases:
        g = H.box_grid(1, 1, 1, dx, dy, dz, porosity=n)
        g.qx[:] = q[0]
        g.qy[:] = q[1]
        g.qz[:] = q[2]
        r = O.track(g, H.particles([0], *loc), lib=lib)
        u = [qa / (n * V) for qa in q]
        times = [((1.0 if u[a] > 0 else 0.0) - loc[a]) / u[a] for a in range(3)]
        a_min = int(np.argmin(times))
        t = times[a_min]
        assert r.status[0] == BOUNDARY and _close(r.t[0], t, 2e-15), (q, r.t[0], t)
        fin = [r.xi[0], r.eta[0], r.zeta[0]]
        for a in range(3):
            want = (1.0 if u[a] > 0 else 0.0) if a == a_min else loc[a] + u[a] * t
            assert abs(fin[a] - want) <= 2e-15, (q, a, fin[a], want)


def pin_corner_tie(lib):
    """Exact corner tie: the lower axis crosses first, the other follows with a zero-time step."""
    g = H.box_grid(2, 2, 1, 1.0, 1.0, 1.0, porosity=1.0)
    g.qx[:] = 1.0
    g.qy[:] = 1.0
    r = O.track(g, H.particles([0], 0.5, 0.5, 0.5), path_cap=8, lib=lib)
    assert r.status[0] == BOUNDARY
    assert list(r.path_cell[0, :3]) == [0, 1, 3], r.path_cell[0]
    assert list(r.path_face[0, :3]) == [1, 3, 1], r.path_face[0]
    assert list(r.path_t[0, :3]) == [0.5, 0.5, 1.5]
    assert r.ncross[0] == 3 and r.t[0] == 1.5 and r.cell[0] == 3
    assert (r.xi[0], r.eta[0]) == (1.0, 1.0)
    assert int(r.path_hash[0]) == H.fnv_path([0, 1, 3])


def _line(nx, q=3.0, porosity=0.3, flags=None, dx=10.0):
    g = H.box_grid(nx, 1, 1, dx, 10.0, 10.0, porosity=porosity, flags=flags)
    g.qx[:] = q
    return g


def pin_stops(lib):
    """Stopping conditions and degenerate starts (sink, cap, time limit, invalid, inactive)."""
    fl = np.full((1, 1, 3), FLAG_ACTIVE, np.int32)
    fl[0, 0, 2] |= FLAG_SINK
    g = _line(3, flags=fl)
    u = 3.0 / (0.3 * 1000.0)
    # entry into a sink cell stops there
    r = O.track(g, H.particles([0], 0.5, 0.5, 0.5), lib=lib)
    assert r.status[0] == SINK and r.cell[0] == 2 and r.ncross[0] == 2 and r.xi[0] == 0.0
    assert _close(r.t[0], 1.5 / u, 1e-15)
    # weak-sink pass-through
    r = O.track(g, H.particles([0], 0.5, 0.5, 0.5), stop_at_sink=0, lib=lib)
    assert r.status[0] == BOUNDARY and r.ncross[0] == 3 and _close(r.t[0], 2.5 / u, 1e-15)
    # release inside a sink
    r = O.track(g, H.particles([2], 0.3, 0.5, 0.5, t=7.0), lib=lib)
    assert r.status[0] == SINK and r.ncross[0] == 0 and r.t[0] == 7.0 and r.xi[0] == 0.3
    # step cap
    g2 = _line(3)
    r = O.track(g2, H.particles([0], 0.5, 0.5, 0.5), max_steps=1, lib=lib)
    assert r.status[0] == STEP_CAP and r.ncross[0] == 1 and r.cell[0] == 1 and r.xi[0] == 0.0
    # time limit inside a cell
    r = O.track(g2, H.particles([0], 0.5, 0.5, 0.5), t_max=120.0, lib=lib)
    assert r.status[0] == MAX_TIME and r.cell[0] == 1 and r.t[0] == 120.0
    assert abs(r.xi[0] - (0.5 + u * 120.0 - 1.0)) <= 1e-15
    # a face reached exactly at t_max is crossed (strict comparison)
    r = O.track(g2, H.particles([0], 0.5, 0.5, 0.5), t_max=0.5 / u, lib=lib)
    assert r.ncross[0] == 1 and r.cell[0] == 1 and r.status[0] == MAX_TIME
    # release after t_max: nothing moves
    r = O.track(g2, H.particles([0], 0.5, 0.5, 0.5, t=300.0), t_max=200.0, lib=lib)
    assert r.status[0] == MAX_TIME and r.t[0] == 300.0 and r.ncross[0] == 0
    # invalid starts
    bad = H.particles([-1, 3, 0, 0, 0, 0], [0.5, 0.5, np.nan, 1.5, 0.5, 0.5],
                      [0.5, 0.5, 0.5, 0.5, -0.1, 0.5], 0.5, [0, 0, 0, 0, 0, np.nan])
    r = O.track(g2, bad, lib=lib)
    assert list(r.status) == [INVALID] * 6 and np.isnan(r.out_xyz).all()
    fl = np.full((1, 1, 3), FLAG_ACTIVE, np.int32)
    fl[0, 0, 1] = 0
    g3 = _line(3, flags=fl)
    r = O.track(g3, H.particles([1, 0], 0.5, 0.5, 0.5), lib=lib)
    assert r.status[0] == INVALID
    assert r.status[1] == INACTIVE_NB and r.cell[1] == 0 and r.xi[1] == 1.0 and r.ncross[1] == 1
    # no flow anywhere: stranded, unchanged
    g4 = _line(2, q=0.0)
    r = O.track(g4, H.particles([1], 0.25, 0.5, 0.75, t=3.0), lib=lib)
    assert r.status[0] == STRANDED and r.t[0] == 3.0 and r.xi[0] == 0.25 and r.ncross[0] == 0
    r = O.track(g4, H.particles([1], 0.25, 0.5, 0.75, t=3.0), t_max=10.0, lib=lib)
    assert r.status[0] == STRANDED and r.t[0] == 10.0 and r.xi[0] == 0.25
    # start on the exit face: zero-time crossing
    r = O.track(g2, H.particles([0], 1.0, 0.5, 0.5), max_steps=1, lib=lib)
    assert r.ncross[0] == 1 and r.t[0] == 0.0 and r.cell[0] == 1 and r.xi[0] == 0.0
    # terminated particles are left untouched
    p = H.particles([0], 0.5, 0.5, 0.5)
    p.status[:] = BOUNDARY
    r = O.track(g2, p, lib=lib)
    assert r.status[0] == BOUNDARY and r.t[0] == 0.0 and r.xi[0] == 0.5
    # backward tracking exits through the low face
    r = O.track(g2, H.particles([1], 0.25, 0.5, 0.5), direction=-1, lib=lib)
    assert r.status[0] == BOUNDARY and r.cell[0] == 0 and r.xi[0] == 0.0
    assert _close(r.t[0], 1.25 / u, 1e-15)


def pin_porosity_field(lib):
    """Per-cell porosity: crossing time of a uniform-flow line is sum of n_c V / Q."""
    g = _line(4, q=2.0)
    g.porosity = np.array([[[0.1, 0.2, 0.3, 0.4]]])
    r = O.track(g, H.particles([0], 0.0, 0.5, 0.5), lib=lib)
    V = 1000.0
    want = sum(n * V / 2.0 for n in (0.1, 0.2, 0.3, 0.4))
    assert r.status[0] == BOUNDARY and _close(r.t[0], want, 4e-16), (r.t[0], want)


def _c1_row_cells(cell):
    return [cell + i for i in range(40)]


def pin_c1_closed_form(lib):
    """Homogeneous C1: v = K dh/L / n = 5/6 m/d, t = 1.2 (400 - x0) d, 40 crossings, straight row."""
    w = C.c1()
    p = w.particles
    r = O.track(w.grids[0], p, lib=lib)
    x0 = (p.cell % 40 + p.xi) * 10.0
    assert (r.status == BOUNDARY).all()
    assert (r.ncross == 40).all()
    assert np.max(np.abs(r.t - 1.2 * (400.0 - x0)) / r.t) <= 1e-12
    assert (r.out_xyz[:, 0] == 400.0).all()
    assert (r.eta == p.eta).all() and (r.zeta == p.zeta).all()
    for q in range(0, p.n, 97):
        assert int(r.path_hash[q]) == H.fnv_path(_c1_row_cells(int(p.cell[q])))


def pin_timeseries_c1(lib):
    """C1 positions in time: x(s) = x0 + v s before the exit, undefined (NaN) from the exit on."""
    w = C.c1(n=200)
    p = w.particles
    snaps = np.array([0.0, 10.0, 55.5, 100.0, 250.0, 400.0, 479.0, 481.0])
    r = O.track(w.grids[0], p, snap_times=snaps, lib=lib)
    v = 0.25 / 0.3
    x0 = (p.cell % 40 + p.xi) * 10.0
    y0 = (p.cell // 40 + p.eta) * 10.0
    for q in range(p.n):
        for k, s in enumerate(snaps):
            if s < r.t[q]:
                assert _close(r.snap_xyz[q, k, 0], x0[q] + v * s, 1e-12), (q, k)
                assert r.snap_xyz[q, k, 1] == y0[q]
            else:
                assert np.isnan(r.snap_xyz[q, k]).all(), (q, k)


def _rand_grid(nx=6, ny=5, nz=3, seed=11, sigma2=0.5, wells=((2, 2, -30.0),), recharge=1e-3):
    return C.random_grid(nx, ny, nz, sigma2, 2.0, seed, wells=wells, recharge=recharge)


def pin_outflow_exits(lib):
    """Every crossing leaves through a face whose flow points out of the cell."""
    g = _rand_grid()
    rng = np.random.Generator(np.random.PCG64(5))
    p = C.release(rng, 300, g.nx, g.ny, g.nz)
    r = O.track(g, p, path_cap=256, max_steps=5000, lib=lib)
    assert set(np.unique(r.status)) <= {BOUNDARY, SINK}
    nx, ny = g.nx, g.ny
    for q in range(p.n):
        for s in range(r.ncross[q]):
            c, f = int(r.path_cell[q, s]), int(r.path_face[q, s])
            k, rem = divmod(c, nx * ny)
            j, i = divmod(rem, nx)
            axis, hi = divmod(f, 2)
            if axis == 0:
                qf = g.qx[k, j, i + hi]
            elif axis == 1:
                qf = g.qy[k, j + hi, i]
            else:
                qf = g.qz[k + hi, j, i]
            assert (qf > 0) if hi else (qf < 0), (q, s, c, f, qf)
        assert int(r.path_hash[q]) == H.fnv_path(r.path_cell[q, :r.ncross[q]])
        # crossing times never decrease, and the last one is the final time
        ts = r.path_t[q, :r.ncross[q]]
        if r.ncross[q] > 0:
            assert (np.diff(ts) >= 0).all() and ts[-1] == r.t[q]


def pin_reversibility(lib):
    """Forward for time T, then backward (negated flows) for T, returns to the start."""
    g = _rand_grid(wells=(), recharge=0.0, sigma2=0.5, seed=3)
    rng = np.random.Generator(np.random.PCG64(9))
    p = C.release(rng, 200, g.nx, g.ny, g.nz, i_range=(0, 2))
    T = 4.0
    f = O.track(g, p, t_max=T, path_cap=256, max_steps=5000, lib=lib)
    keep = f.status == MAX_TIME
    assert keep.sum() > 50
    back = H.particles(f.cell, f.xi, f.eta, f.zeta)
    b = O.track(g, back, direction=-1, t_max=T, path_cap=256, max_steps=5000, lib=lib)
    for q in np.nonzero(keep)[0]:
        assert b.status[q] == MAX_TIME and b.cell[q] == p.cell[q], q
        for a, (x1, x0) in enumerate(((b.xi, p.xi), (b.eta, p.eta), (b.zeta, p.zeta))):
            assert abs(x1[q] - x0[q]) <= 1e-9, (q, a, x1[q], x0[q])
        fw = list(f.path_cell[q, :f.ncross[q]]) + [int(f.cell[q])]
        bw = list(b.path_cell[q, :b.ncross[q]]) + [int(b.cell[q])]
        assert bw == fw[::-1], q


def pin_resume(lib):
    """A run stopped at t1 and resumed to t2 follows the single run to t2."""
    g = _rand_grid(seed=21)
    rng = np.random.Generator(np.random.PCG64(2))
    p = C.release(rng, 200, g.nx, g.ny, g.nz)
    snaps = np.array([1.0, 5.0, 20.0, 40.0, 80.0, 160.0])
    one = O.track(g, p, t_max=120.0, snap_times=snaps, lib=lib)
    a = O.track(g, p, t_max=40.0, snap_times=snaps, lib=lib)
    mid = H.particles(a.cell, a.xi, a.eta, a.zeta, a.t)
    mid.status[:] = a.status
    mid.ncross[:] = a.ncross
    mid.path_hash[:] = a.path_hash
    b = O.track(g, mid, t_max=120.0, snap_times=snaps, snap_init=a.snap_xyz, lib=lib)
    assert (b.status == one.status).all() and (b.cell == one.cell).all()
    assert (b.ncross == one.ncross).all() and (b.path_hash == one.path_hash).all()
    for x, y in ((b.t, one.t), (b.xi, one.xi), (b.eta, one.eta), (b.zeta, one.zeta)):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-12)
    assert np.allclose(b.snap_xyz, one.snap_xyz, rtol=1e-12, atol=1e-9, equal_nan=True)


def _rk4_compare(lib, g, n, seed, snaps=()):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = C.release(rng, n, g.nx, g.ny, g.nz)
    r = O.track(g, p, path_cap=512, snap_times=np.array(snaps) if len(snaps) else None, max_steps=5000,
                lib=lib)
    scale = max(g.dx, g.dy, g.dz)
    for q in range(n):
        cr, fin, sn = H.rk4_track(g, int(p.cell[q]), (p.xi[q], p.eta[q], p.zeta[q]),
                                  snap_times=snaps)
        m = int(r.ncross[q])
        assert len(cr) == m, (q, len(cr), m)
        for s in range(m):
            c, a, side, t, xyz = cr[s]
            assert r.path_cell[q, s] == c and r.path_face[q, s] == 2 * a + side, (q, s)
            assert abs(r.path_t[q, s] - t) <= 1e-7 * max(1.0, t), (q, s, r.path_t[q, s], t)
            assert np.max(np.abs(r.path_xyz[q, s] - np.array(xyz))) <= 1e-7 * scale, (q, s)
        for k, s in enumerate(snaps):
            if s in sn:
                assert np.max(np.abs(r.snap_xyz[q, k] - np.array(sn[s]))) <= 1e-7 * scale, (q, k)


def pin_rk4(lib):
    """Brute-force RK4 of the same velocity field gives the same cells, faces, times, positions."""
    _rk4_compare(lib, C.random_grid(8, 4, 3, 0.8, 1.5, 41, dx=10.0, dy=6.0, dz=2.0,
                                    origin=(100.0, -50.0, 3.0)), 16, 1)
    _rk4_compare(lib, C.random_grid(6, 5, 2, 0.5, 2.0, 43, wells=((3, 2, -20.0),), recharge=2e-3,
                                    porosity_field=True), 16, 2, snaps=(3.0, 30.0, 90.0))


def pin_positions_stay_in_cell(lib):
    """Local coordinates stay in [0,1]: crossing points lie on the closed box of the cell left.

    Diagonal uniform flows with equal exit times on two axes make the tie-break advance the
    second axis by exactly the distance to its face, where rounding can overshoot.
    """
    g = H.box_grid(2, 2, 1, 1.0, 1.0, 1.0, porosity=1.0)
    starts = np.linspace(0.01, 0.99, 99)
    for q in (0.1, 0.3, 0.7, 1.9, 3.3):
        g.qx[:] = q
        g.qy[:] = q
        r = O.track(g, H.particles([0] * starts.size, starts, starts, 0.5), path_cap=8, lib=lib)
        for a in (r.xi, r.eta, r.zeta):
            assert ((a >= 0.0) & (a <= 1.0)).all(), q
        for p_ in range(starts.size):
            for s in range(r.ncross[p_]):
                c = int(r.path_cell[p_, s])
                i, j = c % 2, c // 2
                x, y = r.path_xyz[p_, s, 0], r.path_xyz[p_, s, 1]
                assert i <= x <= i + 1 and j <= y <= j + 1, (q, p_, s, x, y)


# ----------------------------------------------------------------------------- transient flow
# A 40-cell channel (cells of 10 m, porosity 0.3, cross-section 100 m^2): a uniform face flow
# q gives the velocity q / 30 m/d everywhere.  Time step s scales every flow by F[s] (the
# third step is stagnant), so a particle's position is piecewise linear in time.
_TS_Q = 30.0
_TS_F = (1.0, 2.0, 0.0, 0.5)
_TS_END = (100.0, 150.0, 180.0, math.inf)


def _ts_grids(sink_cell=None, inactive_cell=None, at_step=1):
    grids = []
    for s, f in enumerate(_TS_F):
        fl = np.full((1, 1, 40), FLAG_ACTIVE, np.int32)
        if s >= at_step and sink_cell is not None:
            fl[0, 0, sink_cell] |= FLAG_SINK
        if s >= at_step and inactive_cell is not None:
            fl[0, 0, inactive_cell] = 0
        grids.append(_line(40, q=_TS_Q * f, flags=fl))
    return grids


def _ts_position(x0, t0, t):
    """Closed form: x at time t of a particle released at x0 at time t0 (no exit)."""
    x, a = x0, t0
    for f, b in zip(_TS_F, _TS_END):
        if b <= a:
            continue
        hi = min(b, t)
        if hi > a:
            x += f * (_TS_Q / 30.0) * (hi - a)
            a = hi
        if a >= t:
            break
    return x


def _ts_exit_time(x0, t0, L=400.0):
    a, dist = t0, L - x0
    for f, b in zip(_TS_F, _TS_END):
        if b <= a:
            continue
        v = f * _TS_Q / 30.0
        if v > 0 and dist <= v * (b - a):
            return a + dist / v
        dist -= v * (b - a) if math.isfinite(b) else dist
        a = b
    return math.inf


def pin_transient_closed_form(lib):
    """Transient flow: piecewise-constant velocity in time, staged releases (one at a step
    end exactly), a stagnant step; exit times, crossings, and positions at a time limit."""
    grids = _ts_grids()
    x0 = np.array([3.0, 57.5, 120.0, 260.0, 399.0, 212.5, 33.0])
    t0 = np.array([0.0, 0.0, 130.0, 160.0, 190.0, 150.0, 100.0])
    i0 = np.floor(x0 / 10.0).astype(int)
    p = H.particles(i0, x0 / 10.0 - i0, 0.5, 0.5, t0)
    r = O.track_transient(grids, _TS_END, p, lib=lib)
    for q in range(p.n):
        want = _ts_exit_time(x0[q], t0[q])
        assert r.status[q] == BOUNDARY and r.ncross[q] == 40 - i0[q], (q, r.status[q], r.ncross[q])
        assert _close(r.t[q], want, 1e-12), (q, r.t[q], want)
    for t_max in (170.0, 150.0, 99.0):
        r = O.track_transient(grids, _TS_END, p, t_max=t_max, lib=lib)
        for q in range(p.n):
            if t0[q] > t_max:
                assert r.status[q] == MAX_TIME and r.t[q] == t0[q], q
                continue
            if _ts_exit_time(x0[q], t0[q]) <= t_max:
                assert r.status[q] == BOUNDARY, (t_max, q)
                continue
            want = _ts_position(x0[q], t0[q], t_max)
            # the step the particle is in when it reaches t_max: no reachable face there
            # (the stagnant step) means STRANDED, as in a steady field
            s_rel = min(k for k, b in enumerate(_TS_END) if t0[q] < b)   # a release at a step end
            s_lim = max(s_rel, min(k for k, b in enumerate(_TS_END) if t_max <= b))   # is in the next
            want_status = STRANDED if _TS_F[s_lim] == 0.0 else MAX_TIME
            assert r.status[q] == want_status and r.t[q] == t_max, (t_max, q, r.status[q])
            assert _close(r.out_xyz[q, 0], want, 1e-12), (t_max, q, r.out_xyz[q, 0], want)


def pin_transient_timeseries(lib):
    """Positions at snapshot times across time-step ends follow the piecewise closed form."""
    grids = _ts_grids()
    snaps = np.array([0.0, 50.0, 100.0, 125.0, 150.0, 165.0, 180.0, 250.0, 300.0])
    p = H.particles([0, 8], [0.3, 0.25], 0.5, 0.5, [0.0, 60.0])
    r = O.track_transient(grids, _TS_END, p, snap_times=snaps, lib=lib)
    for q, (x0, t0) in enumerate(((3.0, 0.0), (82.5, 60.0))):
        for k, s_ in enumerate(snaps):
            if s_ < t0 or s_ >= r.t[q]:
                assert np.isnan(r.snap_xyz[q, k]).all(), (q, k)
            else:
                assert _close(r.snap_xyz[q, k, 0], _ts_position(x0, t0, s_), 1e-12), (q, k)


def pin_transient_switch_rules(lib):
    """At a time-step end the particle keeps its cell and position: a cell that is a sink in
    the next field stops it (stop_at_sink = 1) or not (0); one made inactive stops it.
    Cell 30 (x in [300, 310)) is a sink from the second step (t >= 100) on."""
    p = H.particles([20, 15, 2], 0.5, 0.5, 0.5)        # x0 = 205, 155, 25 m
    r = O.track_transient(_ts_grids(sink_cell=30), _TS_END, p, lib=lib)
    # x = 305 at t = 100: inside cell 30 when it becomes a sink
    assert r.status[0] == SINK and r.t[0] == 100.0 and int(r.cell[0]) == 30, (r.status[0], r.t[0])
    assert _close(r.out_xyz[0, 0], 305.0, 1e-12), r.out_xyz[0]
    # x = 255 at t = 100, then 2 m/d: enters cell 30 at t = 122.5
    assert r.status[1] == SINK and int(r.cell[1]) == 30 and _close(r.t[1], 122.5, 1e-12), (r.status[1], r.t[1])
    # x = 125 at 100, 225 at 150, stagnant to 180, then 0.5 m/d: enters cell 30 at t = 330
    assert r.status[2] == SINK and _close(r.t[2], 330.0, 1e-12), (r.status[2], r.t[2])
    r = O.track_transient(_ts_grids(sink_cell=30), _TS_END, p, stop_at_sink=0, lib=lib)
    assert (r.status == BOUNDARY).all()
    # cell 12 inactive from t = 100: the third particle is inside it then
    r = O.track_transient(_ts_grids(inactive_cell=12), _TS_END, p, lib=lib)
    assert r.status[2] == INACTIVE_NB and r.t[2] == 100.0 and int(r.cell[2]) == 12, (r.status[2], r.t[2])
    assert r.status[0] == BOUNDARY and r.status[1] == BOUNDARY


def pin_transient_identical_fields(lib):
    """Time steps that all hold the same field reproduce the steady run: same cells, path
    hashes, crossings and statuses, times and positions equal to 1e-11."""
    g = _rand_grid(nx=9, ny=7, nz=3, seed=21, sigma2=1.0, wells=((4, 3, -40.0),), recharge=2e-3)
    rng = np.random.Generator(np.random.PCG64(5))
    p = C.release(rng, 300, g.nx, g.ny, g.nz)
    steady = O.track(g, p, max_steps=5000, lib=lib)
    ends = np.array([7.5, 40.0, 41.0, 300.0, math.inf])
    tr = O.track_transient([g] * ends.size, ends, p, max_steps=5000, lib=lib)
    for name in ("status", "cell", "ncross", "path_hash"):
        assert (getattr(tr, name) == getattr(steady, name)).all(), name
    assert np.allclose(tr.t, steady.t, rtol=1e-11, atol=0.0)
    assert np.allclose(tr.out_xyz, steady.out_xyz, rtol=1e-11, atol=1e-11)


# ----------------------------------------------------------------------------- quadtree grids

def _quad(g, size):
    from workloads import quadtree as QT
    return QT.from_structured(g, size)


def pin_quad_unrefined_matches_structured(lib):
    """A quadtree grid without refinement is the structured grid: identical paths, states and
    times (bitwise), global positions to 1e-13 (formed from the cell box instead of i*dx)."""
    g = C.random_grid(9, 7, 3, 1.2, 2.0, 31, dx=4.0, dy=6.0, dz=1.5, wells=((4, 3, -25.0),), recharge=1e-3)
    q = _quad(g, np.ones((g.ny, g.nx), np.int32))
    rng = np.random.Generator(np.random.PCG64(31))
    p = C.release(rng, 400, g.nx, g.ny, g.nz)
    for kw in (dict(), dict(direction=-1), dict(t_max=37.0)):
        a = O.track(g, p, max_steps=5000, lib=lib, **kw)
        b = O.track_quad(q, p, max_steps=5000, lib=lib, **kw)
        for name in ("status", "cell", "ncross", "path_hash", "xi", "eta", "zeta", "t"):
            assert np.array_equal(getattr(a, name), getattr(b, name)), (kw, name)
        assert np.allclose(a.out_xyz, b.out_xyz, rtol=1e-13, atol=1e-13), kw


def _uniform_quad(vx=0.7, vy=0.3):
    """16 x 16 fine cells of 1 m (height 2 m, porosity 0.25) with a uniform velocity (vx, vy),
    merged into blocks of 4 / 2 / 1 cells around the point (5, 9)."""
    from workloads import quadtree as QT
    g = H.box_grid(16, 16, 1, 1.0, 1.0, 2.0, porosity=0.25)
    g.qx[:] = vx * 0.25 * 2.0
    g.qy[:] = vy * 0.25 * 2.0
    return QT.from_structured(g, QT.block_sizes(16, 16, [(5, 9)], r1=1.5, r2=4.0))


def pin_quad_uniform_flow_line(lib):
    """Uniform flow through a refined quadtree: straight-line motion; the exit time, the final
    position and every crossing (time and position) follow the closed form, and each crossing
    lies on the boundary of the cell it leaves."""
    vx, vy = 0.7, 0.3
    q = _uniform_quad(vx, vy)
    from workloads import quadtree as QT
    rng = np.random.Generator(np.random.PCG64(9))
    p = QT.release(q, rng, 300)
    x0 = q.box[p.cell, 0] + p.xi * q.box[p.cell, 3]
    y0 = q.box[p.cell, 1] + p.eta * q.box[p.cell, 4]
    r = O.track_quad(q, p, path_cap=64, lib=lib)
    t_exit = np.minimum((16.0 - x0) / vx, (16.0 - y0) / vy)
    assert (r.status == BOUNDARY).all()
    assert np.allclose(r.t, t_exit, rtol=1e-12, atol=1e-12)
    assert np.allclose(r.out_xyz[:, 0], x0 + vx * r.t, rtol=0, atol=1e-11)
    assert np.allclose(r.out_xyz[:, 1], y0 + vy * r.t, rtol=0, atol=1e-11)
    for k in range(p.n):
        for s_ in range(r.ncross[k]):
            c, tt, xyz = int(r.path_cell[k, s_]), r.path_t[k, s_], r.path_xyz[k, s_]
            assert abs(xyz[0] - (x0[k] + vx * tt)) <= 1e-11 and abs(xyz[1] - (y0[k] + vy * tt)) <= 1e-11, (k, s_)
            b = q.box[c]
            on_x = min(abs(xyz[0] - b[0]), abs(xyz[0] - b[0] - b[3])) <= 1e-12
            on_y = min(abs(xyz[1] - b[1]), abs(xyz[1] - b[1] - b[4])) <= 1e-12
            inside = (b[0] - 1e-12 <= xyz[0] <= b[0] + b[3] + 1e-12) and (b[1] - 1e-12 <= xyz[1] <= b[1] + b[4] + 1e-12)
            assert inside and (on_x or on_y), (k, s_, c, xyz, b)


def pin_quad_paths_connect(lib):
    """On a heterogeneous refined grid with a well: each crossing point lies on a face of the
    cell left and in the closed box of the next cell of the path (neighbour lookup and the
    coordinate mapping agree with the geometry)."""
    from workloads import quadtree as QT
    K = np.exp(np.sqrt(1.5) * np.random.Generator(np.random.PCG64(77)).standard_normal((2, 32, 32)))
    src = np.zeros(K.shape)
    src[1, 13, 18] = -2.0
    sink = src < 0
    g = C.make_grid(K, 2.0, 3.0, 1.0, recharge=1e-3, source=src, sink_mask=sink)
    q = QT.from_structured(g, QT.block_sizes(32, 32, [(18, 13)], r1=3.0, r2=8.0))
    assert q.cells[:, 2].min() == 1 and q.cells[:, 2].max() == 4
    p = QT.release(q, np.random.Generator(np.random.PCG64(78)), 500)
    r = O.track_quad(q, p, path_cap=512, max_steps=512, lib=lib)
    assert (r.ncross < 512).all()
    for k in range(p.n):
        n = int(r.ncross[k])
        cells = list(r.path_cell[k, :n]) + [int(r.cell[k])]
        for s_ in range(n):
            xyz = r.path_xyz[k, s_]
            a, b = q.box[cells[s_]], q.box[cells[s_ + 1]]
            f = int(r.path_face[k, s_])
            ax, side = f // 2, f % 2
            assert abs(xyz[ax] - (a[ax] + side * a[3 + ax])) <= 1e-12 * (1 + abs(xyz[ax])), (k, s_)
            if s_ + 1 < n or r.status[k] != BOUNDARY:
                for m in range(3):
                    assert b[m] - 1e-9 <= xyz[m] <= b[m] + b[3 + m] + 1e-9, (k, s_, m, xyz, b)


def pin_quad_zero_time_circuit(lib):
    """Four cells whose face flows circulate around their shared corner: a particle on the
    corner is handed round with zero-time crossings and is stopped there as stranded after 16;
    particles elsewhere circle the corner with finite times until the step cap."""
    g = H.box_grid(2, 2, 1, 1.0, 1.0, 1.0, porosity=0.5)
    g.qx[0, 0, 1] = 1.0      # (0,0) -> (1,0)
    g.qy[0, 1, 1] = 1.0      # (1,0) -> (1,1)
    g.qx[0, 1, 1] = -1.0     # (1,1) -> (0,1)
    g.qy[0, 1, 0] = -1.0     # (0,1) -> (0,0)
    q = _quad(g, np.ones((2, 2), np.int32))
    p = H.particles([0, 0], [1.0, 0.3], [1.0, 0.6], 0.5)
    r = O.track_quad(q, p, max_steps=100, lib=lib)
    assert r.status[0] == STRANDED and r.ncross[0] == 16 and r.t[0] == 0.0, (r.status[0], r.ncross[0], r.t[0])
    assert np.array_equal(r.out_xyz[0], [1.0, 1.0, 0.5])
    assert r.status[1] == STEP_CAP and r.ncross[1] == 100


QUICK_PINS = [pin_single_cell_exit, pin_single_cell_position, pin_multi_axis_uniform,
              pin_corner_tie, pin_stops, pin_porosity_field, pin_c1_closed_form,
              pin_timeseries_c1, pin_outflow_exits, pin_reversibility, pin_resume,
              pin_positions_stay_in_cell, pin_transient_closed_form, pin_transient_timeseries,
              pin_transient_switch_rules, pin_transient_identical_fields,
              pin_quad_unrefined_matches_structured, pin_quad_uniform_flow_line, pin_quad_paths_connect,
              pin_quad_zero_time_circuit]
ALL_PINS = QUICK_PINS + [pin_rk4]
