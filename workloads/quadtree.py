"""Seeded quadtree (rectangular unstructured) grids with balanced face flows.

The second test case of the paper (Methods "Synthetic test cases") refines a layered
model with a quadtree near its boundary conditions; its model files are not available.
These grids stand in for it: a fine structured grid is solved for face flows (workloads.flow),
and blocks of s x s fine cells (s = 1, 2 or 4, the same in every layer) far from the
refinement points are merged into one cell.  A merged cell's face is the union of fine
faces; consecutive fine faces shared with the same neighbour form one subface whose flow is
their sum, so every cell balances exactly as the fine solution did.

Cell faces are numbered f = 2*axis + side (axis 0 = x, 1 = y, 2 = z; side 1 = high face).
Each face lists its subfaces in order; a subface has a neighbour cell (-1 = domain
boundary), a flow (m^3/d, positive along +axis) and its extent [lo, hi] in the face's two
tangential local coordinates of the cell (x-face: eta, zeta; y-face: xi, zeta; z-face:
xi, eta).

This module generates inputs only; it contains none of the tracking arithmetic.
"""
from __future__ import annotations

import dataclasses
import functools
from typing import Optional

import numpy as np

from . import configs as C
from . import kfield


@dataclasses.dataclass
class QuadGrid:
    ncell: int
    box: np.ndarray          # float64 [ncell, 6]: x_lo, y_lo, z_lo, hx, hy, hz
    sub_off: np.ndarray      # int32 [ncell*6 + 1]: subfaces of face f of cell c are sub_off[6c+f] ..
    sub_nb: np.ndarray       # int32 [nsub] neighbour cell, -1 = boundary
    sub_q: np.ndarray        # float64 [nsub] flow through the subface, + = +axis
    sub_lo: np.ndarray       # float64 [nsub, 2] extent in the face's tangential local coordinates
    sub_hi: np.ndarray       # float64 [nsub, 2]
    flags: np.ndarray        # int32 [ncell]
    porosity: Optional[np.ndarray] = None
    porosity_scalar: float = C.POROSITY
    meta: dict = dataclasses.field(default_factory=dict)
    # fine-grid description (for generating particles and for tests)
    fine: Optional[C.Grid] = None
    owner: Optional[np.ndarray] = None   # int32 [nz, ny_f, nx_f] cell of each fine cell
    cells: Optional[np.ndarray] = None   # int32 [ncell, 4]: i0, j0, s, k in fine units

    @property
    def nsub(self) -> int:
        return int(self.sub_nb.shape[0])


def block_sizes(nx: int, ny: int, points, r1: float, r2: float) -> np.ndarray:
    """Size (1, 2 or 4 fine cells) of the block holding each fine column: 4 x 4 super-blocks
    whose centre is farther than r2 (fine cells) from every point stay whole; otherwise their
    2 x 2 quarters stay whole if farther than r1, else split into single cells."""
    assert nx % 4 == 0 and ny % 4 == 0
    size = np.zeros((ny, nx), np.int32)
    pts = np.asarray(points, np.float64).reshape(-1, 2)

    def far(ci, cj, r):
        if pts.size == 0:
            return True
        return bool(np.min(np.hypot(pts[:, 0] - ci, pts[:, 1] - cj)) > r)

    for J in range(0, ny, 4):
        for I in range(0, nx, 4):
            if far(I + 2.0, J + 2.0, r2):
                size[J:J + 4, I:I + 4] = 4
                continue
            for dj in (0, 2):
                for di in (0, 2):
                    s = 2 if far(I + di + 1.0, J + dj + 1.0, r1) else 1
                    size[J + dj:J + dj + 2, I + di:I + di + 2] = s
    return size


def from_structured(g: C.Grid, size: np.ndarray, meta=None) -> QuadGrid:
    """Merge the fine cells of g into blocks of the given size (same in every layer)."""
    nz, ny, nx = g.nz, g.ny, g.nx
    cells = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                s = int(size[j, i])
                if i % s == 0 and j % s == 0 and size[j - j % s, i - i % s] == s:
                    cells.append((i, j, s, k))
    cells = np.array(cells, np.int32)
    ncell = cells.shape[0]
    owner = np.full((nz, ny, nx), -1, np.int32)
    for c, (i0, j0, s, k) in enumerate(cells):
        owner[k, j0:j0 + s, i0:i0 + s] = c
    assert (owner >= 0).all()
    hx, hy, hz = g.dx, g.dy, g.dz
    box = np.empty((ncell, 6))
    box[:, 0] = g.x0 + cells[:, 0] * hx
    box[:, 1] = g.y0 + cells[:, 1] * hy
    box[:, 2] = g.z0 + cells[:, 3] * hz
    box[:, 3] = cells[:, 2] * hx
    box[:, 4] = cells[:, 2] * hy
    box[:, 5] = hz
    off = [0]
    nb_l, q_l, lo_l, hi_l = [], [], [], []

    def emit(runs):
        for nb, q, lo, hi in runs:
            nb_l.append(nb)
            q_l.append(q)
            lo_l.append(lo)
            hi_l.append(hi)
        off.append(len(nb_l))

    for c, (i0, j0, s, k) in enumerate(cells):
        for f in range(6):
            axis, side = f // 2, f % 2
            runs = []
            if axis < 2:
                # the s fine faces along the tangential in-plane axis, grouped by neighbour
                for t in range(s):
                    if axis == 0:
                        ii = i0 + (s if side else 0)
                        j = j0 + t
                        q = float(g.qx[k, j, ii])
                        nbi = ii if side else ii - 1
                        nb = int(owner[k, j, nbi]) if 0 <= nbi < nx else -1
                    else:
                        jj = j0 + (s if side else 0)
                        i = i0 + t
                        q = float(g.qy[k, jj, i])
                        nbj = jj if side else jj - 1
                        nb = int(owner[k, nbj, i]) if 0 <= nbj < ny else -1
                    lo, hi = t / s, (t + 1) / s
                    if runs and runs[-1][0] == nb:
                        runs[-1][1] += q
                        runs[-1][3] = [hi, 1.0]
                    else:
                        runs.append([nb, q, [lo, 0.0], [hi, 1.0]])
            else:
                kk = k + (1 if side else 0)
                nbk = kk if side else kk - 1
                q = 0.0
                for j in range(j0, j0 + s):
                    for i in range(i0, i0 + s):
                        q += float(g.qz[kk, j, i])
                if 0 <= nbk < nz:
                    nbs = set(int(v) for v in owner[nbk, j0:j0 + s, i0:i0 + s].ravel())
                    assert len(nbs) == 1, "layers must share the refinement"
                    nb = nbs.pop()
                else:
                    nb = -1
                runs.append([nb, q, [0.0, 0.0], [1.0, 1.0]])
            emit(runs)
    flags = np.empty(ncell, np.int32)
    for c, (i0, j0, s, k) in enumerate(cells):
        flags[c] = int(np.bitwise_or.reduce(g.flags[k, j0:j0 + s, i0:i0 + s].ravel()))
    return QuadGrid(ncell, box, np.array(off, np.int32), np.array(nb_l, np.int32), np.array(q_l),
                    np.array(lo_l, np.float64).reshape(-1, 2), np.array(hi_l, np.float64).reshape(-1, 2),
                    flags, None, g.porosity_scalar, dict(meta or {}), g, owner, cells)


def release(q: QuadGrid, rng: np.random.Generator, n: int, region=None, layer=None) -> C.Particles:
    """Particles uniform over fine cells (optionally those with i in region[0]..region[1] and in
    one layer), local coordinates in the owning cell."""
    g = q.fine
    nz, ny, nx = g.nz, g.ny, g.nx
    ilo, ihi = (0, nx) if region is None else region
    i = rng.integers(ilo, ihi, size=n)
    j = rng.integers(0, ny, size=n)
    k = rng.integers(0, nz, size=n) if layer is None else np.full(n, layer)
    u = rng.random((3, n))
    c = q.owner[k, j, i]
    i0, j0, s = q.cells[c, 0], q.cells[c, 1], q.cells[c, 2]
    xi = (i - i0 + u[0]) / s
    eta = (j - j0 + u[1]) / s
    return C.Particles(c.astype(np.int32), np.ascontiguousarray(xi), np.ascontiguousarray(eta),
                       np.ascontiguousarray(u[2]), np.zeros(n), np.zeros(n, np.int32),
                       np.zeros(n, np.int32), np.full(n, C.FNV_OFFSET, dtype=np.uint64))


# ----------------------------------------------------------------------------- C7

C7_WELLS = ((80, 150, 0, 300.0), (170, 90, 2, 300.0))   # fine (i, j), layer, rate m^3/d


@functools.lru_cache(maxsize=2)
def c7_grid() -> QuadGrid:
    """Layered aquifer (top aquifer, aquitard, bottom aquifer) on 256 x 256 fine cells of
    2.5 m, refined around one well in each aquifer: 4 x 4 blocks far away, 2 x 2 closer,
    single cells near the wells."""
    shape = (3, 256, 256)
    y = kfield.lognormal_k(shape, 1.0, 1.0, 12.0, 1000 * 7)
    K = np.empty(shape)
    K[0] = 20.0 * y[0]
    K[1] = 0.05 * y[1]
    K[2] = 10.0 * y[2]
    source = np.zeros(shape)
    sink = np.zeros(shape, dtype=bool)
    for (i, j, k, rate) in C7_WELLS:
        source[k, j, i] = -rate
        sink[k, j, i] = True
    g = C.make_grid(K, 2.5, 2.5, 5.0, recharge=2e-4, source=source, sink_mask=sink,
                    meta=dict(name="C7 fine"))
    size = block_sizes(256, 256, [(w[0], w[1]) for w in C7_WELLS], r1=10.0, r2=28.0)
    return from_structured(g, size, meta=dict(name="C7"))


def c7(n: int = 1_000_000) -> C.Workload:
    q = c7_grid()
    rng = np.random.Generator(np.random.PCG64(2000 * 7))
    p = release(q, rng, n, layer=0)
    return C.Workload("C7", [q], p)
