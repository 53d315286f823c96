"""Error bounds of the FP32 exit-time and advance formulas of the tracking kernels, emulated on the host.

The FP64 kernel picks the exit face from FP32 estimates of the three axes' exit times and evaluates only
the candidate's correctly rounded time when every other axis is more than 2^-15 (relative) behind it.
That choice is the exact one only if every estimate is within half that margin of the true time; the
kernel's comments claim 1.5e-6.  These tests emulate the estimate operation by operation in float32 --
log1p(x)/x in Goldberg's form log(u)/(u - 1), u = fl(1 + x), the ratio u_e/u_p for x <= -1/2 -- with
the hardware reciprocal and base-2 logarithm replaced by correctly rounded ones perturbed by up to
2 ulp (the worst case measured for v_rcp_f32 and v_log_f32 on gfx950), and compare with the exit time
ln(u_e/u_p)/A of the analytic solution (the definition in the paper's semi-analytical method), evaluated
in float64.

The mixed kernel's advance uses expm1(y)/y = (v - 1)/log(v), v = fl(e^y) (Kahan) for |y| < 1/8 and
(v - 1)/y beyond; its accuracy is only reported, but the formula is checked here against expm1(y)/y.
"""
import numpy as np

F = np.float32
ULP2 = 2.0 ** -23          # 2 ulp of a float32 value, relative
BOUND = 1.5e-6              # claimed relative error of the FP32 estimate
MARGIN = 2.0 ** -15         # selection margin of the FP64 kernel


def _perturb(v, rng):
    """Correctly rounded float32 values moved by up to 2 ulp (relative), then rounded again."""
    return (v.astype(np.float64) * (1.0 + rng.uniform(-ULP2, ULP2, v.shape))).astype(F)


def _rcp(v, rng):
    return _perturb((F(1.0) / v).astype(F), rng)


def _log2(v, rng):
    return _perturb(np.log2(v).astype(F), rng)


def estimate(D, up, A, ue, rng, with_unsure=False):
    """The FP64 kernel's FP32 exit-time estimate, step by step in float32; with ``with_unsure``
    also the kernel's flag for estimates it cannot bound (operands or result outside
    [2^-100, 2^100], a zero distance), which sends the selection to the exact evaluation."""
    with np.errstate(divide="ignore", invalid="ignore", over="ignore", under="ignore"):
        upf = up.astype(F)
        Df = D.astype(F)
        rup = _rcp(upf, rng)
        rf = (Df * rup).astype(F)
        xf = (A.astype(F) * rf).astype(F)
        u = (F(1.0) + xf).astype(F)
        ratio = ~(xf > F(-0.5))
        uef = ue.astype(F)
        q = np.where(ratio, (uef * rup).astype(F), u)
        den = np.where(ratio, xf, (u - F(1.0)).astype(F))
        lg = (_log2(q, rng) * F(0.693147181)).astype(F)
        ph = np.where(u == F(1.0), F(1.0), (lg * _rcp(den, rng)).astype(F))
        E = (rf * ph).astype(F)
    if not with_unsure:
        return E
    lo, hi = F(2.0 ** -100), F(2.0 ** 100)
    # the kernel's form: one minimum over the operands (fminf, like np.fmin, ignores a NaN), then
    # NaN-safe range tests of |u_p| and of the estimate
    m = np.fmin(np.fmin(np.abs(Df), np.abs(upf)), np.fmin(q, np.where(ratio, np.abs(uef), F(1.0))))
    unsure = ~(m >= lo) | ~(np.abs(upf) <= hi) | ~((E >= lo) & (E <= F(2.0 ** 120)))
    # the same set as testing every operand on its own: a NaN q comes only with a zero distance or
    # a |u_p| outside [2^-100, 2^100], which the minimum or the |u_p| test catch
    each = ~(q >= lo) | ~(np.abs(Df) >= lo) | (ratio & ~(np.abs(uef) >= lo))
    each |= ~((np.abs(upf) >= lo) & (np.abs(upf) <= hi)) | ~((E >= lo) & (E <= F(2.0 ** 120)))
    assert np.array_equal(unsure, each)
    return E, unsure


def exact_exit(u1, u2, xi):
    """Exit time to the face the velocity points at, float64 (feasible axes only)."""
    A = u2 - u1
    up = u1 + A * xi
    xe = np.where(up > 0, 1.0, 0.0)
    ue = np.where(up > 0, u2, u1)
    D = xe - xi
    x = A * D / up
    with np.errstate(divide="ignore", invalid="ignore"):
        ph = np.where(np.abs(x) < 1e-8, 1.0 - x / 2.0, np.log1p(x) / x)
    return A, up, ue, D, x, (D / up) * ph


def _axes(rng, n):
    """Face velocities and positions spanning the regimes of the workloads: gradients from none to
    strong deceleration (u_e/u_p down to 1e-6) and acceleration (u_e/u_p up to 1e6), magnitudes
    over twelve decades, positions anywhere in the cell and on its faces."""
    mag = 10.0 ** rng.uniform(-6, 6, n)
    u1 = mag * rng.uniform(0.1, 1.0, n)
    ratio = 10.0 ** rng.uniform(-6, 6, n)
    u2 = u1 * ratio
    u2 = np.where(rng.random(n) < 0.05, u1, u2)                    # uniform flow along the axis
    u2 = np.where(rng.random(n) < 0.05, u1 * (1 + 1e-7 * rng.standard_normal(n)), u2)   # x -> 0
    xi = rng.random(n)
    xi = np.where(rng.random(n) < 0.02, 0.0, xi)
    sgn = np.where(rng.random(n) < 0.5, 1.0, -1.0)                 # flow in -axis direction too
    return sgn * u1, sgn * u2, xi


def test_exit_estimate_within_claimed_bound():
    rng = np.random.default_rng(20230227)
    worst = 0.0
    for _ in range(8):
        u1, u2, xi = _axes(rng, 250_000)
        A, up, ue, D, x, t = exact_exit(u1, u2, xi)
        ok = (ue * up > 0) & (D != 0)                              # feasible, not already on the face
        E = estimate(D[ok], up[ok], A[ok], ue[ok], rng).astype(np.float64)
        rel = np.abs(E / t[ok] - 1.0)
        assert np.all(np.isfinite(rel))
        worst = max(worst, float(rel.max()))
    assert worst < BOUND, worst
    # two estimates' errors and the FP32 rounding of the limit E_w (1 + 2^-15) stay inside the margin
    assert 2 * BOUND + 2.0 ** -24 < MARGIN


def test_exit_estimate_regimes_separately():
    """The three branches of the formula: tiny x (u == 1), Goldberg's quotient, the direct ratio."""
    rng = np.random.default_rng(7)
    n = 100_000
    up = 10.0 ** rng.uniform(-3, 3, n)
    D = rng.uniform(1e-6, 1.0, n)
    for x in (rng.uniform(-1e-9, 1e-9, n),                  # u rounds to 1
              rng.uniform(-1e-3, 1e-3, n),                  # small x, Goldberg's form
              rng.uniform(-0.4999, 50.0, n),                # moderate to strong acceleration
              -1.0 + 10.0 ** rng.uniform(-6, np.log10(0.5), n)):   # x <= -1/2: ratio form
        A = x * up / D
        ue = up * (1.0 + x)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(np.abs(x) < 1e-12, D / up, np.log1p(x) / A)
        E = estimate(D, up, A, ue, rng).astype(np.float64)
        assert np.abs(E / t - 1.0).max() < BOUND


def _kahan_psi(y, rng):
    """The mixed kernel's expm1(y)/y for 2^-10 <= |y|, in float32 with perturbed exp2/log2/rcp."""
    yf = y.astype(F)
    v = _perturb(np.exp2((yf * F(1.44269504)).astype(F)).astype(F), rng)
    small = np.abs(yf) < F(0.125)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        den = np.where(small, (_log2(v, rng) * F(0.693147181)).astype(F), yf)
        return ((v - F(1.0)).astype(F) * _rcp(den, rng)).astype(F)


def test_kahan_expm1_over_y():
    rng = np.random.default_rng(11)
    n = 200_000
    y = np.concatenate([rng.uniform(2.0 ** -10, 0.125, n), -rng.uniform(2.0 ** -10, 0.125, n),
                        rng.uniform(0.125, 30.0, n), -rng.uniform(0.125, 60.0, n)])
    y = y.astype(F).astype(np.float64)          # the kernel's argument is a float32
    ps = _kahan_psi(y, rng).astype(np.float64)
    ref = np.expm1(y) / y
    rel = np.abs(ps / ref - 1.0)
    # a few ulp of float32 away from y = 0, where (v - 1)/y alone would lose ~|y|^-1 ulp
    assert rel.max() < 2e-6, rel.max()
    naive = ((np.exp2((y.astype(F) * F(1.44269504)).astype(F)).astype(F) - F(1.0)).astype(F)
             / y.astype(F)).astype(np.float64)
    tiny = np.abs(y) < 2.0 ** -8
    assert np.abs(naive[tiny] / ref[tiny] - 1.0).max() > 10 * rel[tiny].max()   # the form matters there


def _select(E, unsure_axes):
    """The kernel's candidate choice from three estimates (strict <, lowest axis on ties) and
    whether it falls back to the exact three-axis evaluation."""
    w, Ew = -1, np.float32(np.inf)
    for a in range(3):
        if E[a] < Ew:
            w, Ew = a, E[a]
    lim = np.float32(Ew * np.float32(1.0 + MARGIN))
    near = any(a != w and E[a] <= lim for a in range(3))
    return w, bool(near or any(unsure_axes))


def test_subnormal_estimates_fall_back_to_exact():
    """Exit times in the FP32 subnormal range: the estimates' rounding (2^-149 absolute) can
    reverse the order of two axes, so the kernel must not trust them.  A particle 1.2542e-43
    from its exit face on axis 0 (u = -0.125) and 1.00515e-42 on axis 1 (u = -1): the exact
    times are 1.00336e-42 and 1.00515e-42 (axis 0 first), the FP32 estimates order them the
    other way and no axis lies within the 2^-15 margin of the candidate -- only the unsure
    flag keeps the choice exact."""
    rng = np.random.default_rng(3)
    xi = np.array([1.2542e-43, 1.00515e-42, 0.5])
    u = np.array([-0.125, -1.0, 0.0])
    t = np.array([xi[0] / 0.125, xi[1] / 1.0, np.inf])
    assert t[0] < t[1]
    D = -xi[:2]
    E, uns = estimate(D, u[:2], np.zeros(2), u[:2], rng, with_unsure=True)
    E = np.array([E[0], E[1], np.float32(np.inf)])
    w_old, fallback_old = _select(E, [False, False, False])
    assert w_old == 1 and not fallback_old          # the unguarded rule would take axis 1
    w, fallback = _select(E, list(uns) + [False])
    assert fallback                                 # the guarded rule evaluates every axis exactly


def test_estimate_bounded_whenever_trusted():
    """Over distances down to the FP64 subnormal range and velocities over +-120 decades, every
    estimate the kernel trusts (unsure not raised) is within the claimed bound; every other one
    is decided by the exact evaluation."""
    rng = np.random.default_rng(99)
    worst, trusted, total = 0.0, 0, 0
    for _ in range(6):
        n = 200_000
        mag = 10.0 ** rng.uniform(-40, 40, n)
        u1 = mag * rng.uniform(0.1, 1.0, n) * np.where(rng.random(n) < 0.5, 1.0, -1.0)
        u2 = u1 * 10.0 ** rng.uniform(-6, 6, n)
        xi = np.where(rng.random(n) < 0.5, rng.random(n), 10.0 ** rng.uniform(-320, 0, n))
        xi = np.where(rng.random(n) < 0.5, xi, 1.0 - xi)
        A, up, ue, D, x, t = exact_exit(u1, u2, xi)
        ok = (ue * up > 0) & np.isfinite(t) & (t > 0)
        E, uns = estimate(D[ok], up[ok], A[ok], ue[ok], rng, with_unsure=True)
        keep = ~uns
        rel = np.abs(E[keep].astype(np.float64) / t[ok][keep] - 1.0)
        trusted += int(keep.sum())
        total += int(ok.sum())
        if rel.size:
            worst = max(worst, float(rel.max()))
    assert trusted > total // 4 and trusted < total     # both outcomes occur in this range
    assert worst < BOUND, worst


def test_unsure_on_degenerate_operands():
    """Operands that make the FP32 estimate NaN or meaningless (a zero distance, a particle
    velocity that rounds to zero, FP32 subnormal or beyond the FP32 range, gradients and face
    velocities beyond the FP32 range) always raise the flag; the kernel's single-minimum form of
    the range test flags exactly what testing every operand on its own flags (estimate() checks
    that equality on every call)."""
    rng = np.random.default_rng(5)
    cases = [  # D, u_p, A, u_e
        (0.0, 1.0, 1e39, 2.0),          # zero distance, gradient beyond FP32: A * 0 = inf * 0
        (0.0, 1e-50, 0.0, 1e-50),       # zero distance, u_p rounds to zero: 0 * inf
        (0.5, 1e-50, 1.0, 1.0),         # u_p below the FP32 range
        (0.5, 1e-41, 1.0, 1.0),         # u_p FP32-subnormal
        (0.5, 1e39, -1e39, 1e39),       # u_p beyond the FP32 range
        (0.5, 1e20, -4e39, -1e39),      # gradient beyond FP32, strong deceleration
        (1e-44, 1.0, 1.0, 2.0),         # distance FP32-subnormal
        (0.5, -1.0, 1e38, -1e-45),      # ratio form with u_e below the FP32 range
    ]
    D, up, A, ue = (np.array(c, dtype=np.float64) for c in zip(*cases))
    E, uns = estimate(D, up, A, ue, rng, with_unsure=True)
    assert uns.all(), (E, uns)
