"""Seeded synthetic workloads: grids with face flows, and released particles.

The paper's test cases (section "Synthetic test cases", Tables 1 and 2) need a
sequential-Gaussian realisation and MODFLOW-6 models that are not available,
so these seeded inputs stand in for them.  They borrow the construction of the
first test case: a lognormal K built from a standardised Gaussian field with
an exponential covariance, a west-to-east head gradient, and particles
released near the west inlet.

  C1  40x40x1 cells of 10 m, homogeneous K = 10 m/d, porosity 0.3, heads 10 m
      (west) / 0 m (east); 1,000 particles in the first column.
  C2  100x100x10 cells of 10x10x2 m, lognormal K (geometric mean 10 m/d,
      sigma^2 = 1, correlation length 5 cells); 1e6 particles in i < 10.
  C3  200x200x20 cells of 10x10x2 m, sigma^2 = 4, correlation length 8 cells,
      two pumping-well columns of 500 m^3/d each (sink cells), recharge
      1e-4 m/d; 1e7 particles uniform over the domain.
  C4  16 realisations of C2's grid with sigma^2 ~ U[0.5, 4]; 64 particle groups
      with log-uniform sizes in [1e3, 2e6], group g on realisation g mod 16.
  C5  200x200x20, sigma^2 = 2, correlation length 8; 1e6 particles in i < 5;
      positions at 100 log-spaced times from 1 d to 1e5 d.
  C6  transient flow on C2's grid: 12 time steps (an initial steady period, ten
      transient steps, a final steady period, as in the second test case) in
      which a pumping-well column switches on, ramps up and off again; 1e6
      particles in i < 10 released in 10 stages every 20 d; weak sinks (the
      well cells) pass particles through.
  TC1 the first test case's shape (Table 1): a two-dimensional aquifer of
      1500x300 cells of 1 m, K = exp(sigma Y) with one standardised field Y
      (correlation length 10 m) for every sigma^2 in [0.1, 5], heads 1510 m
      (inlet) and 10 m (outlet), so a unit mean gradient; particles on the
      line x = 10 m, uniform along y; endpoint runs to the outlet.

Seeds: K field 1000*cfg + realisation, particles 2000*cfg (+ group), numpy
PCG64.  Particles are placed by drawing a cell uniformly in the release region
and local coordinates uniformly in [0,1)^3.

This module generates inputs only; it contains none of the tracking arithmetic.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import Optional

import numpy as np

from . import flow, kfield

FLAG_ACTIVE = 1
FLAG_SINK = 2
FNV_OFFSET = 0xCBF29CE484222325

POROSITY = 0.3
H_WEST = 10.0
H_EAST = 0.0


@dataclasses.dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    x0: float
    y0: float
    z0: float
    qx: np.ndarray          # [nz, ny, nx+1] m^3/d, + = +i
    qy: np.ndarray          # [nz, ny+1, nx]
    qz: np.ndarray          # [nz+1, ny, nx]
    flags: np.ndarray       # [nz, ny, nx] int32, bit0 active, bit1 sink
    porosity: Optional[np.ndarray] = None   # [nz, ny, nx] or None -> porosity_scalar
    porosity_scalar: float = POROSITY
    source: Optional[np.ndarray] = None     # well terms used by the flow solve (for balance checks)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Particles:
    cell: np.ndarray        # int32 linear cell id (k*ny + j)*nx + i
    xi: np.ndarray          # float64 local coordinates in [0,1]
    eta: np.ndarray
    zeta: np.ndarray
    t: np.ndarray           # float64 release time
    status: np.ndarray      # int32, 0 = ACTIVE (to be tracked)
    ncross: np.ndarray      # int32
    path_hash: np.ndarray   # uint64

    @property
    def n(self) -> int:
        return int(self.cell.shape[0])

    def copy(self) -> "Particles":
        return Particles(*(a.copy() for a in dataclasses.astuple(self)))

    def subset(self, idx) -> "Particles":
        return Particles(*(np.ascontiguousarray(a[idx]) for a in dataclasses.astuple(self)))


@dataclasses.dataclass
class Workload:
    name: str
    grids: list             # list[Grid]
    particles: Particles
    mode: str = "endpoint"  # or "timeseries"
    t_max: float = math.inf
    snap_times: Optional[np.ndarray] = None
    group_offsets: Optional[np.ndarray] = None   # int64 [n_groups+1]
    group_grid: Optional[np.ndarray] = None      # int32 [n_groups]
    tstep_end: Optional[np.ndarray] = None       # transient flow: grids[s] holds until tstep_end[s]
    stop_at_sink: int = 1


def make_grid(K: np.ndarray, dx: float, dy: float, dz: float, recharge: float = 0.0,
              source: Optional[np.ndarray] = None, sink_mask: Optional[np.ndarray] = None,
              origin=(0.0, 0.0, 0.0), porosity: float = POROSITY, meta=None,
              h_west: float = H_WEST, h_east: float = H_EAST) -> Grid:
    nz, ny, nx = K.shape
    _, qx, qy, qz, rel, its = flow.solve(K, dx, dy, dz, h_west, h_east, recharge, source)
    flags = np.full((nz, ny, nx), FLAG_ACTIVE, dtype=np.int32)
    if sink_mask is not None:
        flags[sink_mask] |= FLAG_SINK
    m = dict(meta or {})
    m.update(solver_relres=rel, solver_iters=its)
    return Grid(nx, ny, nz, dx, dy, dz, origin[0], origin[1], origin[2], qx, qy, qz, flags,
                None, porosity, source, m)


def release(rng: np.random.Generator, n: int, nx: int, ny: int, nz: int,
            i_range=None, t0: float = 0.0) -> Particles:
    """Uniform release: cell uniform over i in i_range (default all), all j and k; xi,eta,zeta ~ U[0,1)."""
    ilo, ihi = (0, nx) if i_range is None else i_range
    i = rng.integers(ilo, ihi, size=n)
    j = rng.integers(0, ny, size=n)
    k = rng.integers(0, nz, size=n)
    loc = rng.random((3, n))
    cell = ((k * ny + j) * nx + i).astype(np.int32)
    return Particles(cell, np.ascontiguousarray(loc[0]), np.ascontiguousarray(loc[1]),
                     np.ascontiguousarray(loc[2]), np.full(n, t0), np.zeros(n, np.int32),
                     np.zeros(n, np.int32), np.full(n, FNV_OFFSET, dtype=np.uint64))


def concat(parts) -> Particles:
    fields = list(zip(*(dataclasses.astuple(p) for p in parts)))
    return Particles(*(np.ascontiguousarray(np.concatenate(f)) for f in fields))


# ----------------------------------------------------------------------------- configs

def c1(n: int = 1000) -> Workload:
    K = np.full((1, 40, 40), 10.0)
    g = make_grid(K, 10.0, 10.0, 10.0, meta=dict(name="C1"))
    rng = np.random.Generator(np.random.PCG64(2000 * 1))
    p = release(rng, n, 40, 40, 1, i_range=(0, 1))
    return Workload("C1", [g], p)


@functools.lru_cache(maxsize=32)
def c2_grid(realization: int = 0, sigma2: float = 1.0, cfg: int = 2) -> Grid:
    K = kfield.lognormal_k((10, 100, 100), 10.0, sigma2, 5.0, 1000 * cfg + realization)
    return make_grid(K, 10.0, 10.0, 2.0, meta=dict(name="C%d/r%d" % (cfg, realization), sigma2=sigma2))


def c2(n: int = 1_000_000) -> Workload:
    g = c2_grid()
    rng = np.random.Generator(np.random.PCG64(2000 * 2))
    p = release(rng, n, 100, 100, 10, i_range=(0, 10))
    return Workload("C2", [g], p)


WELLS_C3 = ((66, 100), (133, 100))   # (i, j) columns, all layers


@functools.lru_cache(maxsize=32)
def c3_grid() -> Grid:
    shape = (20, 200, 200)
    K = kfield.lognormal_k(shape, 10.0, 4.0, 8.0, 1000 * 3)
    source = np.zeros(shape)
    sink = np.zeros(shape, dtype=bool)
    for (i, j) in WELLS_C3:
        source[:, j, i] = -500.0 / shape[0]
        sink[:, j, i] = True
    return make_grid(K, 10.0, 10.0, 2.0, recharge=1e-4, source=source, sink_mask=sink,
                     meta=dict(name="C3", sigma2=4.0))


def c3(n: int = 10_000_000) -> Workload:
    g = c3_grid()
    rng = np.random.Generator(np.random.PCG64(2000 * 3))
    p = release(rng, n, 200, 200, 20)
    return Workload("C3", [g], p)


def c4_sigma2(n_real: int = 16) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(1000 * 4 + 999))
    return rng.uniform(0.5, 4.0, size=n_real)


def c4_group_sizes(n_groups: int = 64) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(2000 * 4))
    return np.round(np.exp(rng.uniform(math.log(1e3), math.log(2e6), size=n_groups))).astype(np.int64)


def c4(n_real: int = 16, n_groups: int = 64, scale: float = 1.0) -> Workload:
    s2 = c4_sigma2(n_real)
    grids = [c2_grid(r, float(s2[r]), cfg=4) for r in range(n_real)]
    sizes = np.maximum(1, np.round(c4_group_sizes(n_groups) * scale)).astype(np.int64)
    parts = []
    for g in range(n_groups):
        rng = np.random.Generator(np.random.PCG64(2000 * 4 + 1 + g))
        parts.append(release(rng, int(sizes[g]), 100, 100, 10, i_range=(0, 10)))
    offs = np.zeros(n_groups + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    ggrid = (np.arange(n_groups) % n_real).astype(np.int32)
    return Workload("C4", grids, concat(parts), group_offsets=offs, group_grid=ggrid)


def c5_snap_times(n_snap: int = 100) -> np.ndarray:
    k = np.arange(n_snap, dtype=np.float64)
    return 10.0 ** (5.0 * k / (n_snap - 1))


@functools.lru_cache(maxsize=32)
def c5_grid() -> Grid:
    K = kfield.lognormal_k((20, 200, 200), 10.0, 2.0, 8.0, 1000 * 5)
    return make_grid(K, 10.0, 10.0, 2.0, meta=dict(name="C5", sigma2=2.0))


def c5(n: int = 1_000_000) -> Workload:
    g = c5_grid()
    rng = np.random.Generator(np.random.PCG64(2000 * 5))
    p = release(rng, n, 200, 200, 20, i_range=(0, 5))
    return Workload("C5", [g], p, mode="timeseries", t_max=1e5, snap_times=c5_snap_times())


C6_WELL = (50, 50)                                  # (i, j) column, all layers
C6_RATE = (0.0, 250.0, 500.0, 750.0, 1000.0, 1000.0, 750.0, 500.0, 250.0, 0.0, 0.0, 0.0)   # m^3/d
C6_END = (50.0, 100.0, 150.0, 200.0, 300.0, 400.0, 600.0, 800.0, 1200.0, 1600.0, 2400.0, math.inf)


@functools.lru_cache(maxsize=16)
def c6_grid(step: int) -> Grid:
    """C2's K field under the well rate of time step `step` (recharge 1e-4 m/d throughout);
    each step's face flows are the steady solution of its boundary conditions."""
    K = kfield.lognormal_k((10, 100, 100), 10.0, 1.0, 5.0, 1000 * 2)
    rate = C6_RATE[step]
    source = np.zeros(K.shape)
    sink = np.zeros(K.shape, dtype=bool)
    if rate > 0:
        source[:, C6_WELL[1], C6_WELL[0]] = -rate / K.shape[0]
        sink[:, C6_WELL[1], C6_WELL[0]] = True
    return make_grid(K, 10.0, 10.0, 2.0, recharge=1e-4, source=source, sink_mask=sink,
                     meta=dict(name="C6/step%d" % step, rate=rate))


def c6(n: int = 1_000_000) -> Workload:
    grids = [c6_grid(s) for s in range(len(C6_RATE))]
    rng = np.random.Generator(np.random.PCG64(2000 * 6 + 1))
    p = release(rng, n, 100, 100, 10, i_range=(0, 10))
    p.t[:] = 20.0 * (np.arange(n) % 10)                  # 10 release stages every 20 d
    return Workload("C6", grids, p, tstep_end=np.array(C6_END), stop_at_sink=0)


CONFIGS = {"C1": c1, "C2": c2, "C3": c3, "C4": c4, "C5": c5, "C6": c6}


# ----------------------------------------------------------------------------- first test case's shape

TC1_SHAPE = (1, 300, 1500)          # nz, ny, nx; cells of 1 m
TC1_SIGMA2 = (0.1, 1.0, 2.5, 5.0)   # the paper's range of aquifer variances
TC1_NP = (1_000, 10_000, 100_000, 1_000_000, 10_000_000)


@functools.lru_cache(maxsize=1)
def tc1_field() -> np.ndarray:
    """The standardised field Y shared by every variance (seed 1000*6)."""
    rng = np.random.Generator(np.random.PCG64(1000 * 6))
    return kfield.gaussian_field(TC1_SHAPE, 10.0, rng)


@functools.lru_cache(maxsize=8)
def tc1_grid(sigma2: float) -> Grid:
    K = np.exp(np.sqrt(sigma2) * tc1_field())
    return make_grid(K, 1.0, 1.0, 1.0, h_west=1510.0, h_east=10.0,
                     meta=dict(name="TC1/s2=%g" % sigma2, sigma2=sigma2))


def tc1(n: int, sigma2: float) -> Workload:
    """n particles on the line x = 10 m (cell column 10, xi = 0), uniform along y."""
    g = tc1_grid(sigma2)
    rng = np.random.Generator(np.random.PCG64(2000 * 6))
    y = rng.random(n) * g.ny
    j = np.minimum(np.floor(y).astype(np.int64), g.ny - 1)
    cell = (j * g.nx + 10).astype(np.int32)
    p = Particles(cell, np.zeros(n), np.ascontiguousarray(y - j), np.full(n, 0.5), np.zeros(n),
                  np.zeros(n, np.int32), np.zeros(n, np.int32), np.full(n, FNV_OFFSET, dtype=np.uint64))
    return Workload("TC1/s2=%g/n=%d" % (sigma2, n), [g], p)


# ----------------------------------------------------------------------------- small cases

def random_grid(nx: int, ny: int, nz: int, sigma2: float, corr_len: float, seed: int,
                dx: float = 10.0, dy: float = 10.0, dz: float = 2.0, wells=(), recharge: float = 0.0,
                origin=(0.0, 0.0, 0.0), porosity_field: bool = False) -> Grid:
    """Small seeded lognormal grid for tests (optionally wells as sink columns, recharge)."""
    K = kfield.lognormal_k((nz, ny, nx), 10.0, sigma2, corr_len, seed) if sigma2 > 0 else \
        np.full((nz, ny, nx), 10.0)
    source = None
    sink = None
    if wells:
        source = np.zeros((nz, ny, nx))
        sink = np.zeros((nz, ny, nx), dtype=bool)
        for (i, j, q) in wells:
            source[:, j, i] = q / nz
            sink[:, j, i] = True
    g = make_grid(K, dx, dy, dz, recharge=recharge, source=source, sink_mask=sink, origin=origin)
    if porosity_field:
        rng = np.random.Generator(np.random.PCG64(seed + 77))
        g.porosity = rng.uniform(0.2, 0.4, size=(nz, ny, nx))
    return g
