"""The seeded input generators: conductivity moments, flow solve, balance, determinism."""
import numpy as np

from workloads import configs as C
from workloads import flow, kfield


def test_c1_heads_exactly_linear():
    w = C.c1()
    g = w.grids[0]
    # K dh/L * area = 10 * (10/400) * 100 = 25 m^3/d through every x face, nothing across y/z
    assert np.all(g.qx == 25.0)
    assert np.all(g.qy == 0.0) and np.all(g.qz == 0.0)
    assert w.particles.n == 1000 and np.all(w.particles.cell % 40 == 0)


def test_lognormal_moments_and_determinism():
    K1 = kfield.lognormal_k((10, 40, 40), 10.0, 2.0, 5.0, 123)
    K2 = kfield.lognormal_k((10, 40, 40), 10.0, 2.0, 5.0, 123)
    assert np.array_equal(K1, K2)
    y = np.log(K1 / 10.0)
    assert abs(y.mean()) < 1e-12 and abs(y.var() - 2.0) < 1e-9
    # positive short-range correlation along each axis
    for ax in range(3):
        a = np.moveaxis(y, ax, 0)
        r = np.corrcoef(a[:-1].ravel(), a[1:].ravel())[0, 1]
        assert r > 0.5, (ax, r)


def test_flow_balance_and_residual():
    g = C.random_grid(30, 20, 5, 2.0, 4.0, 77, wells=((10, 10, -40.0),), recharge=1e-3)
    assert g.meta["solver_relres"] <= 1e-12
    net, gross = flow.cell_balance(g.qx, g.qy, g.qz, g.source)
    assert np.max(np.abs(net)) <= 1e-9 * np.max(gross)
    # outflow at the east face, recharge in at the top, nothing through north/south/bottom
    assert np.all(g.qy[:, 0, :] == 0) and np.all(g.qy[:, -1, :] == 0) and np.all(g.qz[-1] == 0)
    assert np.all(g.qz[0] > 0)


def test_flow_thread_count_independent():
    K = kfield.lognormal_k((4, 12, 16), 10.0, 1.0, 3.0, 5)
    a = flow.solve(K, 10.0, 10.0, 2.0, 10.0, 0.0, nthreads=1)
    b = flow.solve(K, 10.0, 10.0, 2.0, 10.0, 0.0, nthreads=3)
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)


def test_c4_groups():
    sizes = C.c4_group_sizes()
    assert sizes.shape == (64,) and sizes.min() >= 1000 and sizes.max() <= 2_000_000
    s2 = C.c4_sigma2()
    assert s2.shape == (16,) and s2.min() >= 0.5 and s2.max() <= 4.0


def test_snapshot_times():
    t = C.c5_snap_times()
    assert t.shape == (100,) and t[0] == 1.0 and abs(t[-1] - 1e5) < 1e-9 and np.all(np.diff(t) > 0)
