"""Grid builders and independent reference computations used by the tests.

Nothing here calls the oracle or the HIP library: these are hand-built inputs
and plain re-derivations (closed forms in high precision, brute-force RK4)
that pin the oracle to the mathematics.
"""
from __future__ import annotations

import decimal
import math

import numpy as np

from workloads.configs import FLAG_ACTIVE, FLAG_SINK, FNV_OFFSET, Grid, Particles

D = decimal.Decimal
decimal.getcontext().prec = 60


def box_grid(nx, ny, nz, dx=10.0, dy=10.0, dz=10.0, origin=(0.0, 0.0, 0.0), porosity=0.3,
             qx=None, qy=None, qz=None, flags=None) -> Grid:
    """Grid with hand-set face flows (default zero) and all cells active."""
    qx = np.zeros((nz, ny, nx + 1)) if qx is None else np.asarray(qx, dtype=np.float64)
    qy = np.zeros((nz, ny + 1, nx)) if qy is None else np.asarray(qy, dtype=np.float64)
    qz = np.zeros((nz + 1, ny, nx)) if qz is None else np.asarray(qz, dtype=np.float64)
    if flags is None:
        flags = np.full((nz, ny, nx), FLAG_ACTIVE, np.int32)
    return Grid(nx, ny, nz, dx, dy, dz, origin[0], origin[1], origin[2], qx, qy, qz,
                np.asarray(flags, np.int32), None, porosity)


def particles(cells, xi, eta, zeta, t=0.0) -> Particles:
    n = len(cells)
    return Particles(np.asarray(cells, np.int32), np.asarray(xi, np.float64) * np.ones(n),
                     np.asarray(eta, np.float64) * np.ones(n), np.asarray(zeta, np.float64) * np.ones(n),
                     np.asarray(t, np.float64) * np.ones(n), np.zeros(n, np.int32),
                     np.zeros(n, np.int32), np.full(n, FNV_OFFSET, np.uint64))


def fnv_path(cells) -> int:
    h = FNV_OFFSET
    for c in cells:
        h = ((h ^ (int(c) & 0xFFFFFFFF)) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def exit_time_decimal(u1: float, u2: float, xi: float):
    """High-precision exit time of one axis: ln(u_e/u_p)/A (or D/u_p when A = 0), None if no exit."""
    a1, a2, x = D(u1), D(u2), D(xi)
    A = a2 - a1
    up = a1 + A * x
    if up > 0:
        ue, xe = a2, D(1)
        if not ue > 0:
            return None
    elif up < 0:
        ue, xe = a1, D(0)
        if not ue < 0:
            return None
    else:
        return None
    if A == 0:
        return float((xe - x) / up)
    return float((ue / up).ln() / A)


def position_decimal(u1: float, u2: float, xi: float, tau: float) -> float:
    """High-precision xi(tau) of the linear-velocity ODE, clamped to [0,1]."""
    a1, a2, x, t = D(u1), D(u2), D(xi), D(tau)
    A = a2 - a1
    up = a1 + A * x
    if A == 0:
        v = x + up * t
    else:
        v = x + up * ((A * t).exp() - 1) / A
    return float(min(max(v, D(0)), D(1)))


# ----------------------------------------------------------------------------- brute force

def _cell_vel(g: Grid, i, j, k, sign=1.0):
    n = g.porosity[k, j, i] if g.porosity is not None else g.porosity_scalar
    V = g.dx * g.dy * g.dz
    u = np.array([[g.qx[k, j, i], g.qx[k, j, i + 1]],
                  [g.qy[k, j, i], g.qy[k, j + 1, i]],
                  [g.qz[k, j, i], g.qz[k + 1, j, i]]]) * sign / (n * V)
    return u


def rk4_track(g: Grid, cell: int, loc, t_max=math.inf, max_cells=200, sign=1.0, rel_step=1e-3,
              snap_times=()):
    """Brute-force RK4 of dxi/dt = u1 + (u2-u1) xi per axis, cell by cell.

    Each cell is integrated with fixed steps of rel_step times the cell's shortest crossing
    time; the face event is located by bisection on the step length.  Returns the list of
    (cell, axis, side, t, xyz) crossings, the final (cell, loc, t, how) and positions at
    snap_times (NaN after the particle has left the domain).
    """
    nx, ny = g.nx, g.ny
    k, rem = divmod(cell, nx * ny)
    j, i = divmod(rem, nx)
    x = np.array(loc, dtype=np.float64)
    t = 0.0
    crossings = []
    snaps = {}
    snap_times = list(snap_times)

    def gxyz(i, j, k, x):
        return (g.x0 + (i + x[0]) * g.dx, g.y0 + (j + x[1]) * g.dy, g.z0 + (k + x[2]) * g.dz)

    if g.flags[k, j, i] & FLAG_SINK:
        return crossings, (int(cell), x, t, "sink"), snaps
    for _ in range(max_cells):
        u = _cell_vel(g, i, j, k, sign)
        A = u[:, 1] - u[:, 0]

        def f(y):
            return u[:, 0] + A * y

        def rk(y, h):
            k1 = f(y)
            k2 = f(y + 0.5 * h * k1)
            k3 = f(y + 0.5 * h * k2)
            k4 = f(y + h * k3)
            return y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

        vmax = np.max(np.abs(u))
        if vmax == 0:
            return crossings, (int((k * ny + j) * nx + i), x, t, "stranded"), snaps
        h = rel_step / vmax
        steps = 0
        while True:
            y = rk(x, h)
            out = (y < 0) | (y > 1)
            # snapshots inside this step
            for s in snap_times:
                if t <= s < t + h and s not in snaps:
                    yy = rk(x, s - t)
                    if not ((yy < 0) | (yy > 1)).any():
                        snaps[s] = gxyz(i, j, k, yy)
            if t + h > t_max and not out.any():
                x = rk(x, t_max - t)
                return crossings, (int((k * ny + j) * nx + i), x, t_max, "max_time"), snaps
            if out.any():
                lo, hi = 0.0, h
                for _b in range(200):
                    mid = 0.5 * (lo + hi)
                    if ((rk(x, mid) < 0) | (rk(x, mid) > 1)).any():
                        hi = mid
                    else:
                        lo = mid
                    if hi - lo <= 1e-15 * max(1.0, t + hi):
                        break
                tc = hi
                yc = rk(x, tc)
                over = np.maximum(yc - 1, -yc)
                a = int(np.argmax(over))
                side = 1 if yc[a] > 0.5 else 0
                for s in snap_times:
                    if t <= s < t + tc and s not in snaps:
                        snaps[s] = gxyz(i, j, k, np.clip(rk(x, s - t), 0, 1))
                t = t + tc
                xc = np.clip(yc, 0.0, 1.0)
                xc[a] = float(side)
                crossings.append((int((k * ny + j) * nx + i), a, side, t, gxyz(i, j, k, xc)))
                ii, jj, kk = i, j, k
                step = 1 if side else -1
                if a == 0:
                    ii += step
                elif a == 1:
                    jj += step
                else:
                    kk += step
                if not (0 <= ii < g.nx and 0 <= jj < g.ny and 0 <= kk < g.nz):
                    return crossings, (int((k * ny + j) * nx + i), xc, t, "boundary"), snaps
                i, j, k = ii, jj, kk
                x = xc
                x[a] = 1.0 - side
                c2 = (k * ny + j) * nx + i
                if g.flags[k, j, i] & FLAG_SINK:
                    return crossings, (int(c2), x, t, "sink"), snaps
                break
            x = y
            t += h
            steps += 1
            if steps > 2_000_000:
                raise RuntimeError("rk4: too many steps in one cell")
    return crossings, (int((k * ny + j) * nx + i), x, t, "cap"), snaps
