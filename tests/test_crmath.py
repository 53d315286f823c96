"""The library's correctly rounded log1p / expm1 / log (host build of pt_crmath.h).

Every result must equal the quad-precision (113-bit, libquadmath) value rounded once to
double, which is the correctly rounded result whenever the quad value is not within
2^-112 of a rounding boundary.  The quick and accurate phases must also stay within the
error bounds their rounding tests assume (2^-68 and 2^-96 relative).
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FN = {"log1p": 0, "expm1": 1, "log": 2}


@pytest.fixture(scope="module")
def libs():
    d = tempfile.mkdtemp(prefix="crmath_")
    shim = os.path.join(d, "shim.so")
    quad = os.path.join(d, "quad.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-o", shim, os.path.join(HERE, "native", "crmath_shim.cpp")])
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", quad,
                           os.path.join(HERE, "native", "quad_ref.c"), "-lquadmath", "-lm"])
    S, Q = ctypes.CDLL(shim), ctypes.CDLL(quad)
    p, i, l = ctypes.c_void_p, ctypes.c_int, ctypes.c_long
    S.ptcr_eval.restype = ctypes.c_uint
    S.ptcr_eval.argtypes = [i, p, p, l]
    S.ptcr_phases.argtypes = [i, p, p, p, p, p, l]
    Q.quad_eval.argtypes = [i, p, p, p, l]
    Q.quad_relerr.argtypes = [i, p, p, p, p, l]
    return S, Q


def _eval(libs, fn, x):
    S, Q = libs
    x = np.ascontiguousarray(x, dtype=np.float64)
    y, r, m = np.empty_like(x), np.empty_like(x), np.empty_like(x)
    amb = S.ptcr_eval(FN[fn], x.ctypes.data, y.ctypes.data, x.size)
    Q.quad_eval(FN[fn], x.ctypes.data, r.ctypes.data, m.ctypes.data, x.size)
    return y, r, m, amb


def _inputs(fn, rng, n):
    if fn == "log1p":
        return np.concatenate([rng.uniform(-1, 1, n), np.exp(rng.uniform(-60, 60, n)),
                               -np.exp(rng.uniform(-60, 0, n)) * (1 - 2**-52), rng.uniform(-1e-4, 1e-4, n),
                               rng.uniform(-0.5, 3.0, n)])
    if fn == "expm1":
        return np.concatenate([rng.uniform(-40, 710, n), rng.uniform(-1, 1, n), rng.uniform(-1e-3, 1e-3, n),
                               rng.uniform(709, 710, n // 10), rng.uniform(-41, -30, n // 10),
                               rng.uniform(-30, 30, n)])
    return np.concatenate([np.exp(rng.uniform(-740, 709, n)), rng.uniform(0, 0.5, n), rng.uniform(0.5, 2, n)])


@pytest.mark.parametrize("fn", sorted(FN))
def test_correctly_rounded_random(libs, fn):
    rng = np.random.Generator(np.random.PCG64(FN[fn] + 100))
    x = _inputs(fn, rng, 300_000)
    y, r, m, amb = _eval(libs, fn, x)
    bad = ~((y == r) & (np.signbit(y) == np.signbit(r)) | (np.isnan(y) & np.isnan(r)))
    assert not bad.any(), (fn, x[bad][:5], y[bad][:5], r[bad][:5])
    assert amb == 0
    # some inputs lie close enough to a rounding boundary to exercise the accurate phase
    assert np.min(m) < 2.0**-15


@pytest.mark.parametrize("fn", sorted(FN))
def test_special_values(libs, fn):
    tiny = [0.0, -0.0, 5e-324, -5e-324, 2.0**-1022, 2.0**-61, -(2.0**-61), 2.0**-60, 2.0**-59, 1e-300]
    big = [np.inf, -np.inf, np.nan, 1e308, -1e308, 700.0, 709.78, 709.7827128933840, 709.79, 710.0,
           -1.0, -0.5, 0.5, 1.0, 2.0, -40.0, -39.9, -37.4, 0.00270760086, -0.00270760086]
    x = np.array(tiny + big + [1 - 2.0**-53, 1 + 2.0**-52, -1 + 2.0**-53, 0.7071067811865476,
                               1.4142135623730951, 2.0**-26, 3.0, 0.25])
    y, r, m, amb = _eval(libs, fn, x)
    same = ((y == r) & (np.signbit(y) == np.signbit(r))) | (np.isnan(y) & np.isnan(r))
    assert same.all(), (fn, x[~same], y[~same], r[~same])


@pytest.mark.parametrize("fn", sorted(FN))
def test_phase_error_bounds(libs, fn):
    S, Q = libs
    rng = np.random.Generator(np.random.PCG64(FN[fn] + 200))
    x = _inputs(fn, rng, 40_000)
    if fn == "expm1":
        x = x[(np.abs(x) >= 2.0**-60) & (x <= 709.0) & (x >= -40.0)]
    elif fn == "log1p":
        x = x[(np.abs(x) >= 2.0**-60) & (x > -1)]
    x = np.ascontiguousarray(x)
    qh, ql, ah, al, e = (np.empty_like(x) for _ in range(5))
    S.ptcr_phases(FN[fn], x.ctypes.data, qh.ctypes.data, ql.ctypes.data, ah.ctypes.data, al.ctypes.data, x.size)
    Q.quad_relerr(FN[fn], x.ctypes.data, qh.ctypes.data, ql.ctypes.data, e.ctypes.data, x.size)
    assert np.max(e) < 2.0**-68, np.log2(np.max(e))
    Q.quad_relerr(FN[fn], x.ctypes.data, ah.ctypes.data, al.ctypes.data, e.ctypes.data, x.size)
    assert np.max(e) < 2.0**-96, np.log2(np.max(e))


def _decimal_series(fn, x):
    """expm1(x) or log1p(x) for |x| < 2^-40 by its Taylor series in 110-digit decimal."""
    import decimal
    ctx = decimal.Context(prec=110)
    X = decimal.Decimal(x)
    s, t, k = decimal.Decimal(0), X, 1
    while True:
        term = t if fn == "expm1" else ctx.divide(t, k) * (1 if k % 2 else -1)
        if abs(term) < abs(X) * decimal.Decimal(10) ** -105:
            return s
        s = ctx.add(s, term)
        k += 1
        t = ctx.divide(ctx.multiply(t, X), k) if fn == "expm1" else ctx.multiply(t, X)


def _nearest(v):
    import decimal
    import math
    f = float(v)
    with decimal.localcontext(decimal.Context(prec=110)):
        return min((f, float(np.nextafter(f, math.inf)), float(np.nextafter(f, -math.inf))),
                   key=lambda z: abs(decimal.Decimal(z) - v))


@pytest.mark.parametrize("fn", ["expm1", "log1p"])
def test_small_arguments_near_midpoints(libs, fn):
    """Arguments 2^-58 .. 2^-42 with regular bit patterns (powers of two, 1.5 and 1.25 times them,
    moved by up to 40 ulps): there the x^2/2 term lies within 2^-100 of half an ulp of x, so the
    rounding is decided by the x^3 term or beyond.  Every result must be the double nearest to
    the 110-digit series value; undecided evaluations are allowed only where that value lies
    within 2^-140 of a rounding midpoint (relative), and even then the result must be right."""
    import decimal
    rng = np.random.Generator(np.random.PCG64(FN[fn] + 300))
    xs = []
    for e in range(-58, -41):
        for base in (2.0 ** e, 1.5 * 2.0 ** e, 1.25 * 2.0 ** e):
            for k in range(40):
                xs += [base * (1 - k * 2.0 ** -52), base * (1 + k * 2.0 ** -52)]
        xs += list(2.0 ** e * rng.uniform(1, 2, 50))
    x = np.array(xs + [-v for v in xs])
    S, _ = libs
    y = np.empty_like(x)
    amb = S.ptcr_eval(FN[fn], x.ctypes.data, y.ctypes.data, x.size)
    want = np.empty_like(x)
    close = 0
    with decimal.localcontext(decimal.Context(prec=110)):
        for i, v in enumerate(x):
            ex = _decimal_series(fn, float(v))
            want[i] = _nearest(ex)
            d = decimal.Decimal(want[i])
            for nb in (np.nextafter(want[i], np.inf), np.nextafter(want[i], -np.inf)):
                mid = (d + decimal.Decimal(float(nb))) / 2
                if abs(ex - mid) < abs(ex) * decimal.Decimal(2) ** -140:
                    close += 1
    assert np.array_equal(y, want), (fn, x[y != want][:5])
    assert amb <= close, (fn, amb, close)
