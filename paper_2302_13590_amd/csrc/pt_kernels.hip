// Tracking kernels for gfx950 (CDNA4, wave64).
//
// The hot path of semi-analytical particle tracking (the paper: Introduction;
// Methods, "MODPATH" and "Multiprocessing"): every particle is displaced cell
// by cell, one analytic step per cell up to the earliest reachable face, and
// is handed to the neighbour across that face until a stopping condition
// (boundary face, maximum time, sink cell) holds.  Particles are independent,
// so the kernels are data parallel over particles:
//
//   * static:     one thread per particle for its whole track (the analogue of
//                 the paper's static scheduling, Methods "Multiprocessing"); the
//                 work is ordered by starting cell and dealt to the dies in chunks,
//                 and in timeseries runs a wave evaluates the snapshots its lanes
//                 meet together, once enough are pending;
//   * persistent: resident waves pull particle indices from a device work
//                 queue; lanes whose particle stopped are refilled at wave level
//                 (ballot + mbcnt prefix count, one atomic per wave), so slow
//                 particles do not idle a whole wave -- the device form of the
//                 paper's dynamic scheduling (Methods "Multiprocessing",
//                 Results "Thread scheduling").
//
// Per step (one cell crossing): gather the cell's six face velocities and its
// flag word (one 64-byte record, or the face arrays), compute each axis' exit
// time from the linear-velocity solution, take the earliest (ties to the lowest
// axis), apply the time limit, advance the other axes analytically, and
// transfer to the neighbour.  Compiled with -ffp-contract=off: no FMA
// contraction, so the FP64 path rounds exactly as written.
//
// Template arguments of both kernels: precision (FP64 / mixed), layout (face
// arrays, packed structured records, quadtree records), output (endpoint,
// timeseries positions, pathline records: the paper's three simulation types,
// Methods "MODPATH") and whether a lane reads its grid from a table (batched
// particle groups, or transient flow, where the table holds one field per time
// step and the lane's index is its current step).
#include <math.h>

#include <type_traits>

#include "pt_crmath.h"
#include "pt_internal.h"

namespace pt {
namespace {

constexpr unsigned long long kFnvPrime = 0x100000001b3ull;
constexpr int kBlock = 256;

enum : int32_t {
    ST_ACTIVE = 0,
    ST_BOUNDARY = 1,
    ST_SINK = 2,
    ST_MAX_TIME = 3,
    ST_STEP_CAP = 4,
    ST_STRANDED = 5,
    ST_INVALID = 6,
    ST_INACTIVE_NB = 7,
    ST_SKIP = -1,  // not tracked by this call (already terminated)
};

__device__ __forceinline__ double dinf() { return __builtin_huge_val(); }

// ---------------------------------------------------------------------------------------------
// One axis, FP64.  u1/u2: velocities at the low/high face (1/d), xi: local coordinate.
// Exit time to the face the velocity points at; +inf when that face is never reached
// (zero particle velocity, or a face velocity of zero or opposite sign).  The exit time
// ln(u_e/u_p)/A is evaluated as (D/u_p) * log1p(x)/x with x = A D/u_p, which stays exact
// as A -> 0; for x < -1/2 (strong deceleration) the ratio u_e/u_p is formed directly.
// log1p, log and expm1 are correctly rounded (pt_crmath.h), so every FP64 operation of a
// step has one defined result.  `amb` counts roundings the accurate phase could not decide.
template <int CR>
__device__ __forceinline__ double exit_time64(double u1, double u2, double xi, double& xe,
                                              unsigned& amb) {
    const double A = u2 - u1;
    const double up = u1 + A * xi;
    double ue;
    if (up > 0.0) {
        xe = 1.0;
        ue = u2;
        if (!(ue > 0.0)) return dinf();
    } else if (up < 0.0) {
        xe = 0.0;
        ue = u1;
        if (!(ue < 0.0)) return dinf();
    } else {
        return dinf();
    }
    const double D = xe - xi;
    const double r = D / up;
    const double x = A * r;
    double dt = r;
    if (x != 0.0) {
        // One logarithm site for both forms, so a wave whose lanes take different forms
        // runs the correctly rounded logarithm once: log(u_e/u_p) when x < -1/2, then
        // dt = log / A; otherwise log1p(x) = log(1 + x) with 1 + x as a double-double,
        // then dt = r * (log1p / x).
        const bool ratio = x < -0.5;
        double L, yh, yl;
        bool done;
        if (ratio) {
            yh = ue / up;
            yl = 0.0;
            done = ptcr::log_special(yh, &L);
        } else {
            const ptcr::dd y = ptcr::two_sum(1.0, x);
            yh = y.h;
            yl = y.l;
            done = ptcr::log1p_special(x, &L);
        }
        if (!done) L = ptcr::log_dd_cr<CR>(yh, yl, &amb);
        const double q = L / (ratio ? A : x);
        dt = ratio ? q : r * q;
    }
    if (dt < 0.0) dt = 0.0;
    return dt;
}

// Position along one axis after tau: xi + u_p tau expm1(A tau)/(A tau), clamped to [0,1];
// A = u2 - u1 and u_p = u1 + A xi as the exit selection already formed them.
template <int CR>
__device__ __forceinline__ double adv64_au(double A, double up, double xi, double tau, unsigned& amb) {
    if (up == 0.0) return xi;
    const double y = A * tau;
    const double psi = (y == 0.0) ? 1.0 : ptcr::expm1_cr<CR>(y, &amb) / y;
    double xn = xi + (up * tau) * psi;
    xn = (xn < 0.0) ? 0.0 : xn;
    xn = (xn > 1.0) ? 1.0 : xn;
    return xn;
}

template <int CR>
__device__ __forceinline__ double adv64(double u1, double u2, double xi, double tau, unsigned& amb) {
    const double A = u2 - u1;
    const double up = u1 + A * xi;
    return adv64_au<CR>(A, up, xi, tau, amb);
}

// Earliest exit over the three axes, FP64, with the same result as evaluating exit_time64 on
// every axis and keeping the strictly smallest (ties to the lowest axis).  A cheap FP32
// estimate E of each axis' time is formed first (relative error below 1.5e-6); when one axis
// is ahead of every other by more than 2^-15 relative, only its correctly rounded time is
// evaluated -- the others cannot be smaller.  Otherwise (near ties, estimates out of the FP32
// range) every axis is evaluated exactly.  The estimates and the limit stay in FP32: the limit's
// own rounding (2^-24) is far inside the margin left by two estimates' errors.
constexpr double kFilterMargin = 0x1p-15;

// FP32 estimate of (D/u_p) log1p(x)/x, x = A D/u_p, from the hardware reciprocal and base-2
// logarithm (within 2 ulp each, relative, over the whole normal range: checked exhaustively on
// gfx950).  log1p(x)/x is taken as log(u)/(u - 1) with u = fl(1 + x) (Goldberg's form: u - 1 is
// exact for x > -1/2, and the quotient stays accurate however small x is), one formula for all
// lanes; for x <= -1/2 the ratio u_e/u_p is formed directly.  Error: ~7 ulp in x, propagated
// with a factor below 1, ~10 ulp in the quotient, ~6 ulp in D/u_p: below 1.5e-6 relative, a
// tenth of what the selection margin allows.  The bound needs normal FP32 operands and results:
// `unsure` is raised when u_p, the distance D, the ratio numerator u_e or the estimate itself
// leaves [2^-100, 2^100] (or the estimate is not finite).  A subnormal distance or estimate
// carries an absolute rounding of 2^-149, i.e. any relative error, and a zero distance (a
// particle already on the face, a zero-time crossing) is decided exactly as well.
__device__ __forceinline__ float exit_estimate(double D, double up, double A, double ue, bool& unsure) {
    const float upf = (float)up;
    const float Df = (float)D;
    const float rup = __builtin_amdgcn_rcpf(upf);
    const float rf = Df * rup;
    const float xf = (float)A * rf;
    const float u = 1.0f + xf;
    const bool ratio = !(xf > -0.5f);
    const float uef = (float)ue;
    const float q = ratio ? uef * rup : u;   // u_e/u_p
    const float den = ratio ? xf : u - 1.0f;
    const float ph = (u == 1.0f) ? 1.0f   // |x| < 2^-24: log1p(x)/x = 1 - x/2 + ...
                                 : (__builtin_amdgcn_logf(q) * 0.693147181f) * __builtin_amdgcn_rcpf(den);
    const float E = rf * ph;
    // one range test for the operands (none can be NaN here: a NaN q needs a zero distance, which
    // the test catches), NaN-safe comparisons for the estimate
    const float lo = fminf(fminf(fabsf(Df), fabsf(upf)), fminf(q, ratio ? fabsf(uef) : 1.0f));
    unsure = unsure || !(lo >= 0x1p-100f) || !(fabsf(upf) <= 0x1p100f) || !(E >= 0x1p-100f && E <= 0x1p120f);
    return E;
}

template <int CR>
__device__ __forceinline__ void select_exit64(const double (&u1)[3], const double (&u2)[3],
                                              const double (&xi)[3], double& dt, int32_t& axis,
                                              double& xe, unsigned& amb, double (&Ao)[3],
                                              double (&upo)[3]) {
    float E[3];
    bool unsure = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double A = u2[a] - u1[a];
        const double up = u1[a] + A * xi[a];
        Ao[a] = A;
        upo[a] = up;
        double ue, e;
        bool feasible;
        if (up > 0.0) {
            e = 1.0;
            ue = u2[a];
            feasible = ue > 0.0;
        } else if (up < 0.0) {
            e = 0.0;
            ue = u1[a];
            feasible = ue < 0.0;
        } else {
            e = 0.0;
            ue = 0.0;
            feasible = false;
        }
        float est = __builtin_inff();
        if (feasible) est = exit_estimate(e - xi[a], up, A, ue, unsure);
        E[a] = est;
    }
    // candidate axis, then its inputs by selects (constant indices only: the arrays stay in
    // registers)
    int32_t w = -1;
    float Ew = __builtin_inff();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool lt = E[a] < Ew;
        Ew = lt ? E[a] : Ew;
        w = lt ? a : w;
    }
    const double w1 = (w == 0) ? u1[0] : ((w == 1) ? u1[1] : u1[2]);
    const double w2 = (w == 0) ? u2[0] : ((w == 1) ? u2[1] : u2[2]);
    const double wx = (w == 0) ? xi[0] : ((w == 1) ? xi[1] : xi[2]);
    const float lim = Ew * (1.0f + (float)kFilterMargin);   // exact: 1 + 2^-15 is a float
#pragma unroll
    for (int a = 0; a < 3; ++a) unsure = unsure || (a != w && E[a] <= lim);
    if (!unsure) {
        if (w >= 0) {
            dt = exit_time64<CR>(w1, w2, wx, xe, amb);
            axis = w;
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double e = 0.0;
        const double ta = exit_time64<CR>(u1[a], u2[a], xi[a], e, amb);
        if (ta < dt) {
            dt = ta;
            axis = a;
            xe = e;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// One axis, mixed precision: FP32 velocities, local coordinate and in-cell arithmetic, with
// the hardware reciprocal, base-2 logarithm and exponential (within 2 ulp each, relative);
// FP64 for time and for the near-zero-gradient branch (|x| < 2^-10 or |A tau| < 2^-10), where
// short series are evaluated in double.  Beyond it one branch-free formula serves every lane:
// log1p(x)/x = log(u)/(u - 1) with u = fl(1 + x) (Goldberg), and expm1(y)/y = (v - 1)/log(v)
// with v = fl(e^y) (Kahan: the logarithm of the rounded exponential compensates its rounding).
constexpr float kNearZero = 0x1p-10f;
constexpr float kLn2f = 0.693147181f;
constexpr float kLog2ef = 1.44269504f;

// Local coordinates of the mixed kernels: FP32, or FP64 (kMixedCoord64) -- then the distance to
// the face is formed in FP64 before it is rounded to FP32, and advances are added in FP64.
constexpr bool kMixedCoord64 = false;
using MixCoord = std::conditional_t<kMixedCoord64, double, float>;

__device__ __forceinline__ double exit_time_mix(float u1, float u2, MixCoord xc, float& xe, unsigned& amb) {
    (void)amb;
    const float xi = (float)xc;
    const float A = u2 - u1;
    const float up = fmaf(A, xi, u1);
    const bool pos = up > 0.0f;
    xe = pos ? 1.0f : 0.0f;
    const float ue = pos ? u2 : u1;
    if (!((pos && ue > 0.0f) | (up < 0.0f && ue < 0.0f))) return dinf();
    const float D = (float)((MixCoord)xe - xc);
    const float rup = __builtin_amdgcn_rcpf(up);
    const float r = D * rup;
    const float x = A * r;
    if (fabsf(x) < kNearZero) {
        // D/u_p from the FP32 quotient and its residual D - u_p r (exact in FP64: u_p r is a
        // 48-bit product), corrected once with the FP32 reciprocal: relative error ~2^-46.
        // log1p(x)/x = 1 - x/2 + x^2/3 - x^3/4 + x^4/5 - ..., truncation below 2^-52 here
        const double rd0 = (double)r;
        const double rd = fma((double)rup, fma(-(double)up, rd0, (double)D), rd0);
        const double xd = (double)A * rd;
        const double ph = fma(xd, fma(xd, fma(xd, fma(xd, 0.2, -0.25), 1.0 / 3.0), -0.5), 1.0);
        return rd * ph;
    }
    // u - 1 is exact for x > -1/2 and not zero here; for x <= -1/2 the ratio q = u_e/u_p is formed
    // directly and divided by x
    const float u = 1.0f + x;
    const bool ratio = !(x > -0.5f);
    const float q = ratio ? ue * rup : u;
    const float den = ratio ? x : u - 1.0f;
    const float ph = (__builtin_amdgcn_logf(q) * kLn2f) * __builtin_amdgcn_rcpf(den);
    float dt = r * ph;
    if (dt < 0.0f) dt = 0.0f;
    return (double)dt;
}

__device__ __forceinline__ MixCoord adv_mix_au(float A, float up, MixCoord xi, double tau) {
    if (up == 0.0f) return xi;
    const float tf = (float)tau;
    const float y = A * tf;
    MixCoord xn;
    if (fabsf(y) < kNearZero) {
        // expm1(y)/y = 1 + y/2 + y^2/6 + y^3/24 + y^4/120 + ..., truncation below 2^-59 here
        const double yd = (double)A * tau;
        const double psi = fma(yd, fma(yd, fma(yd, fma(yd, 1.0 / 120.0, 1.0 / 24.0), 1.0 / 6.0), 0.5), 1.0);
        xn = (MixCoord)fma((double)up * tau, psi, (double)xi);
    } else {
        // v - 1 is exact for |y| < 1/8 (Sterbenz) and not zero here; beyond, (v - 1)/y
        const float v = __builtin_amdgcn_exp2f(y * kLog2ef);
        const float den = (fabsf(y) < 0.125f) ? __builtin_amdgcn_logf(v) * kLn2f : y;
        const float ps = (v - 1.0f) * __builtin_amdgcn_rcpf(den);
        if constexpr (kMixedCoord64) xn = xi + (double)((up * tf) * ps);
        else xn = fmaf(up * tf, ps, xi);
    }
    xn = (xn < (MixCoord)0) ? (MixCoord)0 : xn;
    xn = (xn > (MixCoord)1) ? (MixCoord)1 : xn;
    return xn;
}

__device__ __forceinline__ MixCoord adv_mix(float u1, float u2, MixCoord xi, double tau, unsigned& amb) {
    (void)amb;
    const float A = u2 - u1;
    return adv_mix_au(A, fmaf(A, (float)xi, u1), xi, tau);
}

// ---------------------------------------------------------------------------------------------
template <int PREC> struct Real;
template <> struct Real<P64> { using T = double; };
template <> struct Real<PMIX> { using T = float; };
// Type of the local coordinates of a lane.
template <int PREC> struct Coord;
template <> struct Coord<P64> { using T = double; };
template <> struct Coord<PMIX> { using T = MixCoord; };

template <int PREC, int CR>
__device__ __forceinline__ double exit_time(typename Real<PREC>::T u1, typename Real<PREC>::T u2,
                                            typename Coord<PREC>::T xi, typename Real<PREC>::T& xe,
                                            unsigned& amb) {
    if constexpr (PREC == P64) return exit_time64<CR>(u1, u2, xi, xe, amb);
    else return exit_time_mix(u1, u2, xi, xe, amb);
}

template <int PREC, int CR>
__device__ __forceinline__ typename Coord<PREC>::T adv(typename Real<PREC>::T u1,
                                                       typename Real<PREC>::T u2,
                                                       typename Coord<PREC>::T xi, double tau,
                                                       unsigned& amb) {
    if constexpr (PREC == P64) return adv64<CR>(u1, u2, xi, tau, amb);
    else return adv_mix(u1, u2, xi, tau, amb);
}

// Lane state of one particle.
template <int PREC>
struct Lane {
    using R = typename Real<PREC>::T;
    int64_t pid;        // particle index, -1 when the lane is idle
    int32_t c, i, j, k; // cell
    int32_t g;          // grid index (batched runs)
    int32_t ncross;
    int32_t ks;         // next snapshot index
    unsigned amb;       // undecided roundings of the correctly rounded functions
    unsigned drop;      // pathline records that had no slot
    unsigned drop0;     // pathline: `drop` when this particle began
    unsigned long long hash;
    double t;
    double s_next;      // time of snapshot ks (+inf past the last)
    typename Coord<PREC>::T x[3];   // local coordinates
    R v1[3], v2[3];     // packed layout: the current cell's face velocities (low, high face)
    int32_t fl;         // packed layout: the current cell's flag word
    int32_t nc0;        // pathline: crossings before this call
    int32_t zrun;       // quadtree: zero-time crossings in a row
    int64_t pq, pend;   // pathline record pass: next slot, end of the particle's slots
};

template <bool BATCHED>
__device__ __forceinline__ const GridDev& grid_of(const TrackParams& P, int32_t g) {
    if constexpr (BATCHED) return P.grids[g];
    else return P.g0;
}

// Layouts whose cells are packed records (structured records, quadtree records).
template <int LAYOUT> constexpr bool kPacked = (LAYOUT == L_CELL || LAYOUT == L_QUAD);

// Whether a lane keeps its cell's (i, j, k) up to date at every crossing: the face layout needs
// them for its face indices, timeseries and pathline outputs for their positions.  Endpoint runs
// on packed structured records only need them at the end, formed from the cell id there.
template <int LAYOUT, int OUT> constexpr bool kTrackIJK = !(LAYOUT == L_CELL && OUT == O_END);

// (i, j, k) of structured cell c.
__device__ __forceinline__ void cell_ijk(const GridDev& G, int32_t c, int32_t& i, int32_t& j, int32_t& k) {
    const int32_t plane = G.nx * G.ny;
    k = c / plane;
    const int32_t rem = c - k * plane;
    j = rem / G.nx;
    i = rem - j * G.nx;
}

// Gather one packed cell record: face velocities (with the direction sign) and the flag word.
template <int PREC>
__device__ __forceinline__ void load_rec(const GridDev& G, int32_t c, double sign,
                                         typename Real<PREC>::T (&u1)[3],
                                         typename Real<PREC>::T (&u2)[3], int32_t& fl) {
    if constexpr (PREC == P64) {
        const double2* r = reinterpret_cast<const double2*>(G.rec64 + c);
        const double2 a = r[0], b = r[1], d = r[2];
        fl = G.rec64[c].flags;
        u1[0] = a.x; u2[0] = a.y;
        u1[1] = b.x; u2[1] = b.y;
        u1[2] = d.x; u2[2] = d.y;
        if (sign != 1.0) {   // backward tracking (uniform across the launch)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                u1[q] = sign * u1[q];
                u2[q] = sign * u2[q];
            }
        }
    } else {
        const float4* r = reinterpret_cast<const float4*>(G.rec32 + c);
        const float4 a = r[0];
        const float4 b = r[1];
        fl = __float_as_int(b.z);
        u1[0] = a.x; u2[0] = a.y;
        u1[1] = a.z; u2[1] = a.w;
        u1[2] = b.x; u2[2] = b.y;
        if (sign != 1.0) {   // backward tracking (uniform across the launch)
            const float fs = (float)sign;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                u1[q] = fs * u1[q];
                u2[q] = fs * u2[q];
            }
        }
    }
}

// Gather one cell: face velocities (with the direction sign) and the flag word.
template <int PREC, int LAYOUT>
__device__ __forceinline__ void load_cell(const GridDev& G, const Lane<PREC>& L, double sign,
                                          typename Real<PREC>::T (&u1)[3],
                                          typename Real<PREC>::T (&u2)[3], int32_t& fl) {
    if constexpr (kPacked<LAYOUT>) {
        if constexpr (PREC == P64) {
            const double2* r = reinterpret_cast<const double2*>(G.rec64 + L.c);
            const double2 a = r[0], b = r[1], d = r[2];
            fl = G.rec64[L.c].flags;
            u1[0] = sign * a.x; u2[0] = sign * a.y;
            u1[1] = sign * b.x; u2[1] = sign * b.y;
            u1[2] = sign * d.x; u2[2] = sign * d.y;
        } else {
            const float4* r = reinterpret_cast<const float4*>(G.rec32 + L.c);
            const float4 a = r[0];
            const float4 b = r[1];
            const float fs = (float)sign;
            fl = __float_as_int(b.z);
            u1[0] = fs * a.x; u2[0] = fs * a.y;
            u1[1] = fs * a.z; u2[1] = fs * a.w;
            u1[2] = fs * b.x; u2[2] = fs * b.y;
        }
    } else {
        static_assert(PREC == P64, "the faces layout is FP64 only");
        const int64_t nx = G.nx, ny = G.ny;
        const int64_t fx = ((int64_t)L.k * ny + L.j) * (nx + 1) + L.i;
        const int64_t fy = ((int64_t)L.k * (ny + 1) + L.j) * nx + L.i;
        const int64_t fz = ((int64_t)L.k * ny + L.j) * nx + L.i;
        const double n_c = G.por ? G.por[L.c] : G.por_scalar;
        const double d = n_c * G.V;
        u1[0] = (sign * G.qx[fx]) / d;
        u2[0] = (sign * G.qx[fx + 1]) / d;
        u1[1] = (sign * G.qy[fy]) / d;
        u2[1] = (sign * G.qy[fy + nx]) / d;
        u1[2] = (sign * G.qz[fz]) / d;
        u2[2] = (sign * G.qz[fz + nx * ny]) / d;
        fl = G.flags[L.c];
    }
}

__device__ __forceinline__ void put_nan3(double* p) {
    const double q = __builtin_nan("");
    p[0] = q;
    p[1] = q;
    p[2] = q;
}

// Global position of local coordinates (a, b, d) in cell (i, j, k).
__device__ __forceinline__ void global_xyz(const GridDev& G, int32_t i, int32_t j, int32_t k, double a,
                                           double b, double d, double* out) {
    out[0] = G.x0 + ((double)i + a) * G.dx;
    out[1] = G.y0 + ((double)j + b) * G.dy;
    out[2] = G.z0 + ((double)k + d) * G.dz;
}

// Global position of local coordinates (a, b, d) in cell c: from (i, j, k) on a structured
// grid, from the cell's box on a quadtree grid.
template <int LAYOUT>
__device__ __forceinline__ void cell_xyz(const GridDev& G, int32_t c, int32_t i, int32_t j, int32_t k, double a,
                                         double b, double d, double* out) {
    if constexpr (LAYOUT == L_QUAD) {
        const QuadBox& B = G.qbox[c];
        out[0] = B.lo[0] + a * B.h[0];
        out[1] = B.lo[1] + b * B.h[1];
        out[2] = B.lo[2] + d * B.h[2];
    } else {
        (void)c;
        global_xyz(G, i, j, k, a, b, d, out);
    }
}

// Position at snapshot time s of a particle whose step started at time t in cell c (i, j, k)
// with local coordinates x: tau = s - t on every axis.
template <int PREC, int LAYOUT, int CR>
__device__ __forceinline__ void eval_snap(const GridDev& G, const typename Real<PREC>::T (&u1)[3],
                                          const typename Real<PREC>::T (&u2)[3],
                                          const typename Coord<PREC>::T (&x)[3], double t, int32_t c,
                                          int32_t i, int32_t j, int32_t k, double s, double* out,
                                          unsigned& amb) {
    const double tau = s - t;
    const double a = (double)adv<PREC, CR>(u1[0], u2[0], x[0], tau, amb);
    const double b = (double)adv<PREC, CR>(u1[1], u2[1], x[1], tau, amb);
    const double d = (double)adv<PREC, CR>(u1[2], u2[2], x[2], tau, amb);
    cell_xyz<LAYOUT>(G, c, i, j, k, a, b, d, out);
}

// Snapshot ks of a particle whose step started at (t, x) in cell c.
template <int PREC, int LAYOUT, int CR>
__device__ __forceinline__ void snap_at(const GridDev& G, const TrackParams& P,
                                        const typename Real<PREC>::T (&u1)[3],
                                        const typename Real<PREC>::T (&u2)[3],
                                        const typename Coord<PREC>::T (&x)[3], double t, int32_t c, int32_t i,
                                        int32_t j, int32_t k, int64_t pid, int32_t ks, double s, unsigned& amb) {
    eval_snap<PREC, LAYOUT, CR>(G, u1, u2, x, t, c, i, j, k, s, P.snap_xyz + (pid * P.n_snap + ks) * 3, amb);
}

// Positions at the snapshot times s with s < to (or s <= to when closed), evaluated from the
// state at the start of the step with tau = s - t.
template <int PREC, int LAYOUT, int CR>
__device__ __forceinline__ void write_snaps(Lane<PREC>& L, const GridDev& G,
                                            const typename Real<PREC>::T (&u1)[3],
                                            const typename Real<PREC>::T (&u2)[3],
                                            const TrackParams& P, const double* snap, double to,
                                            bool closed) {
    while (L.ks < P.n_snap) {
        const double s = L.s_next;
        if (closed ? !(s <= to) : !(s < to)) break;
        snap_at<PREC, LAYOUT, CR>(G, P, u1, u2, L.x, L.t, L.c, L.i, L.j, L.k, L.pid, L.ks, s, L.amb);
        ++L.ks;
        L.s_next = (L.ks < P.n_snap) ? snap[L.ks] : dinf();
    }
}

// Deferred snapshots (static kernel, timeseries, packed layouts).  In a wave, only the few lanes
// whose step holds a snapshot time would run the snapshot arithmetic at that step, while the
// others wait.  Instead a lane records its step-start state and snapshot range in its LDS slot;
// once kSnapFlush lanes of the wave have a pending slot (or no lane is left tracking), the wave
// evaluates all pending snapshots together, each lane taking one (slot, snapshot) pair.  Each
// snapshot is the same function of the same state, so the results do not change.
constexpr int kSnapFlush = 32;

// Ordering of the LDS slots between the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The snapshots of a step ending at `to` (open interval): into the lane's slot when it is free,
// else evaluated at once.
template <int PREC, int LAYOUT, int CR>
__device__ __forceinline__ void queue_snaps(Lane<PREC>& L, const GridDev& G,
                                            const typename Real<PREC>::T (&u1)[3],
                                            const typename Real<PREC>::T (&u2)[3], const TrackParams& P,
                                            const double* snap, double to,
                                            SnapJob<typename Real<PREC>::T>* job) {
    const int32_t ks0 = L.ks;
    while (L.ks < P.n_snap && L.s_next < to) {
        ++L.ks;
        L.s_next = (L.ks < P.n_snap) ? snap[L.ks] : dinf();
    }
    const int32_t cnt = L.ks - ks0;
    if (cnt == 0) return;
    if (job->cnt == 0) {
        job->x[0] = L.x[0];
        job->x[1] = L.x[1];
        job->x[2] = L.x[2];
        job->t = L.t;
        job->c = L.c;
        job->i = L.i;
        job->j = L.j;
        job->k = L.k;
        job->g = L.g;
        job->pid = (int32_t)L.pid;
        job->ks0 = ks0;
        job->cnt = cnt;
    } else {
        for (int32_t q = ks0; q < L.ks; ++q)
            snap_at<PREC, LAYOUT, CR>(G, P, u1, u2, L.x, L.t, L.c, L.i, L.j, L.k, L.pid, q, snap[q], L.amb);
    }
}

// All lanes of the wave: evaluate every pending snapshot of the wave's 64 slots W and free them.
template <int PREC, int LAYOUT, bool BATCHED, int CR>
__device__ __forceinline__ void flush_snaps(SnapJob<typename Real<PREC>::T>* W, const TrackParams& P,
                                            const double* snap) {
    using R = typename Real<PREC>::T;
    const int lane = (int)(threadIdx.x & 63u);
    const int cnt = W[lane].cnt;
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    W[lane].start = incl - cnt;
    wave_sync();
    for (int q = lane; q < total; q += 64) {
        // the slot holding pair q: the last one whose first pair is at most q (it has cnt > 0)
        int lo = 0, hi = 64;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (W[mid].start <= q) lo = mid;
            else hi = mid;
        }
        const SnapJob<R>& J = W[lo];
        const GridDev& G = grid_of<BATCHED>(P, J.g);
        R u1[3], u2[3];
        typename Coord<PREC>::T x[3];
        int32_t fl;
        load_rec<PREC>(G, J.c, P.sign, u1, u2, fl);
        x[0] = J.x[0];
        x[1] = J.x[1];
        x[2] = J.x[2];
        const int32_t ks = J.ks0 + (q - J.start);
        unsigned a = 0u;
        snap_at<PREC, LAYOUT, CR>(G, P, u1, u2, x, J.t, J.c, J.i, J.j, J.k, (int64_t)J.pid, ks, snap[ks], a);
        if (a) W[lo].amb = a;   // the slot's owner hands its particle to the careful pass
    }
    wave_sync();
    W[lane].cnt = 0;
    wave_sync();
}

template <int PREC>
__device__ __forceinline__ void nan_rest(Lane<PREC>& L, const TrackParams& P) {
    double* row = P.snap_xyz + L.pid * (int64_t)P.n_snap * 3;
    for (int32_t q = L.ks; q < P.n_snap; ++q) put_nan3(row + 3 * (int64_t)q);
    L.ks = P.n_snap;
}

// Pathline record staging.  A lane's records form one contiguous stream (40 bytes each), but
// the lanes of a wave write to as many streams, so written one by one they leave partial 64-byte
// segments that the L2 evicts before the next record completes them (measured on C2: 1.8x the
// record bytes written to HBM plus reads for the partial segments).  Staged in the lane's LDS
// slot, the stream is written in whole 64-byte segments; only the segments at the ends of the
// stream, which it shares with its neighbours, are written in 8-byte words.
__device__ __forceinline__ PathStage* path_stage_slot() {
    extern __shared__ __align__(16) double dyn_lds[];
    return reinterpret_cast<PathStage*>(dyn_lds) + threadIdx.x;
}

__device__ __forceinline__ void stage_record(const TrackParams& P, int64_t q, double t, double x,
                                             double y, double z, int32_t cell, int32_t face) {
    PathStage* S = path_stage_slot();
    const int64_t B = 40 * q;                       // byte offset of the record in the stream
    const int64_t wb = B & ~(int64_t)63;            // its segment
    const int o = (int)((B - wb) >> 3);             // in doubles: 0 .. 7
    S->buf[o] = t;
    S->buf[o + 1] = x;
    S->buf[o + 2] = y;
    S->buf[o + 3] = z;
    S->buf[o + 4] = __longlong_as_double((long long)(((uint64_t)(uint32_t)face << 32) | (uint32_t)cell));
    if (o + 5 >= 8) {
        // the segment is complete: write it (from the particle's first byte if it starts there)
        double* dst = reinterpret_cast<double*>(reinterpret_cast<char*>(P.path_rec) + wb);
        const int64_t B0 = 40 * S->q0;
        if (B0 <= wb) {
            const double2* src = reinterpret_cast<const double2*>(S->buf);
            double2* d2 = reinterpret_cast<double2*>(dst);
            d2[0] = src[0];
            d2[1] = src[1];
            d2[2] = src[2];
            d2[3] = src[3];
        } else {
            for (int k = (int)((B0 - wb) >> 3); k < 8; ++k) dst[k] = S->buf[k];
        }
        for (int k = 8; k < o + 5; ++k) S->buf[k - 8] = S->buf[k];
    }
}

// Write what is left of the staged stream [q0, qend) (its last, partial segment).
__device__ __forceinline__ void flush_records(const TrackParams& P, int64_t qend) {
    PathStage* S = path_stage_slot();
    const int64_t N = 40 * qend, B0 = 40 * S->q0;
    if (N <= B0) return;
    const int64_t wb = N & ~(int64_t)63;
    const int hi = (int)((N - wb) >> 3);
    const int lo = (B0 > wb) ? (int)((B0 - wb) >> 3) : 0;
    double* dst = reinterpret_cast<double*>(reinterpret_cast<char*>(P.path_rec) + wb);
    for (int k = lo; k < hi; ++k) dst[k] = S->buf[k];
}

// Group of particle `pid` (largest g with group_offsets[g] <= pid, empty groups skipped).
__device__ __forceinline__ int32_t find_group(const TrackParams& P, int64_t pid) {
    int32_t lo = 0, hi = P.n_groups;  // invariant: offsets[lo] <= pid < offsets[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (P.group_offsets[mid] <= pid) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Time step of a particle at time t (transient flow): the first step whose end is after t.
__device__ __forceinline__ int32_t step_of(const TrackParams& P, double t) {
    int32_t s = 0;
    while (s < P.n_tsteps - 1 && !(t < P.tstep_end[s])) ++s;
    return s;
}

// Release checks (S0).  Returns 0 when the particle is to be tracked, ST_SKIP when it is
// not tracked by this call, or a final status.
template <int PREC, int LAYOUT, int OUT, bool BATCHED>
__device__ int32_t begin(Lane<PREC>& L, const TrackParams& P, const double* snap) {
    const int64_t p = L.pid;
    const int32_t st = P.status[p];
    L.g = 0;
    if constexpr (BATCHED) {
        if (P.n_tsteps) L.g = step_of(P, P.t[p]);   // transient: the grid is the time step's
        else L.g = P.group_grid[find_group(P, p)];
    }
    const GridDev& G = grid_of<BATCHED>(P, L.g);
    const int64_t ncell = (int64_t)G.nx * G.ny * G.nz;
    const int32_t c = P.cell[p];
    if (st != ST_ACTIVE && st != ST_MAX_TIME) {
        if constexpr (OUT == O_PATH) {
            if (P.path_count) {
                P.path_off[p + 1] = 0;   // dry run: nothing else is written
                return ST_SKIP;
            }
        }
        if (P.out_xyz) {
            double* o = P.out_xyz + 3 * p;
            if (st == ST_INVALID || c < 0 || c >= ncell) {
                put_nan3(o);
            } else {
                const int32_t plane = G.nx * G.ny;
                const int32_t k = c / plane, rem = c - k * plane;
                const int32_t j = rem / G.nx, i = rem - j * G.nx;
                cell_xyz<LAYOUT>(G, c, i, j, k, P.xi[p], P.eta[p], P.zeta[p], o);
            }
        }
        return ST_SKIP;
    }
    const bool fresh = (st == ST_ACTIVE);
    const double a = P.xi[p], b = P.eta[p], d = P.zeta[p], t = P.t[p];
    bool bad = (c < 0 || (int64_t)c >= ncell);
    int32_t own = 0;
    if (!bad) {
        if constexpr (kPacked<LAYOUT>) {
            own = (PREC == P64) ? G.rec64[c].flags : G.rec32[c].flags;
        } else {
            own = G.flags[c];
        }
        bad = !(own & CF_ACTIVE);
    }
    if (!(a >= 0.0 && a <= 1.0) || !(b >= 0.0 && b <= 1.0) || !(d >= 0.0 && d <= 1.0)) bad = true;
    if (!(t == t) || __builtin_isinf(t)) bad = true;
    if (bad) {
        if constexpr (OUT == O_SERIES) {
            L.ks = 0;
            nan_rest(L, P);
        }
        return ST_INVALID;
    }
    if constexpr (kPacked<LAYOUT>) load_rec<PREC>(G, c, P.sign, L.v1, L.v2, L.fl);
    L.c = c;
    L.zrun = 0;
    if constexpr (kTrackIJK<LAYOUT, OUT>) cell_ijk(G, c, L.i, L.j, L.k);
    L.x[0] = (typename Coord<PREC>::T)a;
    L.x[1] = (typename Coord<PREC>::T)b;
    L.x[2] = (typename Coord<PREC>::T)d;
    L.t = t;
    L.ncross = P.ncross[p];
    L.hash = P.hash[p];
    if constexpr (OUT == O_PATH) {
        L.nc0 = L.ncross;
        L.drop0 = L.drop;
        if (!P.path_count) {
            L.pq = P.path_off[p];
            const int64_t e = P.path_off[p + 1];
            L.pend = (e < P.path_cap) ? e : P.path_cap;
            if (P.path_stage) path_stage_slot()->q0 = L.pq;
        }
    }
    if constexpr (OUT == O_SERIES) {
        double* row = P.snap_xyz + p * (int64_t)P.n_snap * 3;
        int32_t q = 0;
        while (q < P.n_snap && snap[q] < t) {
            if (fresh) put_nan3(row + 3 * (int64_t)q);
            ++q;
        }
        L.ks = q;
        L.s_next = (q < P.n_snap) ? snap[q] : dinf();
    }
    if ((own & CF_SINK) && P.stop_at_sink) return ST_SINK;
    if (t > P.t_max) return ST_MAX_TIME;
    if constexpr (BATCHED) {
        if (P.n_tsteps && t > P.tstep_end[P.n_tsteps - 1]) return ST_MAX_TIME;
    }
    return 0;
}

// Write the final state of a tracked particle.
template <int PREC, int LAYOUT, int OUT, bool BATCHED>
__device__ void finish(Lane<PREC>& L, int32_t st, const TrackParams& P, unsigned int* s_hist) {
    const int64_t p = L.pid;
    atomicAdd(&s_hist[st], 1u);
    if constexpr (OUT == O_PATH) {
        if (P.path_count) {   // dry run: the crossing count is the only output
            P.path_off[p + 1] = (st == ST_INVALID) ? 0 : (int64_t)(L.ncross - L.nc0);
            return;
        }
        if (P.path_stage && st != ST_INVALID) flush_records(P, (L.pq < L.pend) ? L.pq : L.pend);
    }
    P.status[p] = st;
    if (st == ST_INVALID) {
        if (P.out_xyz) put_nan3(P.out_xyz + 3 * p);
        return;
    }
    P.cell[p] = L.c;
    P.xi[p] = (double)L.x[0];
    P.eta[p] = (double)L.x[1];
    P.zeta[p] = (double)L.x[2];
    P.t[p] = L.t;
    P.ncross[p] = L.ncross;
    P.hash[p] = L.hash;
    if (P.out_xyz) {
        const GridDev& G = grid_of<BATCHED>(P, L.g);
        if constexpr (!kTrackIJK<LAYOUT, OUT>) cell_ijk(G, L.c, L.i, L.j, L.k);
        cell_xyz<LAYOUT>(G, L.c, L.i, L.j, L.k, (double)L.x[0], (double)L.x[1], (double)L.x[2], P.out_xyz + 3 * p);
    }
    if constexpr (OUT == O_SERIES) nan_rest(L, P);
}

// Quadtree transfer (after the crossing through face f of axis `axis`): the subface holding
// the exit point (the first in order on an edge between two) gives the neighbour; in it, a
// face coordinate carries over when both cells span the same range on that axis and is
// mapped through the global coordinate otherwise.  A particle handed round a point in
// kQuadZeroRun zero-time crossings in a row (face velocities of split faces are averages,
// so they can circulate there) stops as stranded.
constexpr int kQuadZeroRun = 16;

template <int PREC, int OUT>
__device__ int32_t quad_transfer(Lane<PREC>& L, const GridDev& G, const TrackParams& P, const double* snap,
                                 int32_t axis, int32_t f, double xe, double dt) {
    const QuadRec& R = reinterpret_cast<const QuadRec*>(G.rec64)[L.c];
    const uint32_t counts = R.counts;
    int32_t q0 = R.sub_base;
    for (int32_t g = 0; g < f; ++g) q0 += (int32_t)((counts >> (5 * g)) & 31u);
    const int32_t q1 = q0 + (int32_t)((counts >> (5 * f)) & 31u);
    const int ta1 = (axis == 0) ? 1 : 0;
    const int ta2 = (axis == 2) ? 1 : 2;
    const double t1 = (ta1 == 0) ? (double)L.x[0] : (double)L.x[1];
    const double t2 = (ta2 == 1) ? (double)L.x[1] : (double)L.x[2];
    // the last subface is taken when no earlier one holds the point, so it is never tested (a
    // face with one subface reads no extent)
    int32_t hit = q1 - 1;
    for (int32_t q = q0; q < q1 - 1; ++q) {
        const double4 r = G.sub_rect[q];
        if (r.x <= t1 && t1 <= r.z && r.y <= t2 && t2 <= r.w) {
            hit = q;
            break;
        }
    }
    const int32_t nb = (q1 > q0) ? G.sub_nb[hit] : -1;
    if (nb < 0) return ST_BOUNDARY;
    // the neighbour's record, gathered at once (its flags decide the transfer; the velocities
    // of the cell left are not read again)
    load_rec<PREC>(G, nb, P.sign, L.v1, L.v2, L.fl);
    const int32_t nfl = L.fl;
    if (!(nfl & CF_ACTIVE)) return ST_INACTIVE_NB;
    const QuadBox& B = G.qbox[L.c];
    const QuadBox& N = G.qbox[nb];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a == axis) continue;
        if (N.lo[a] == B.lo[a] && N.h[a] == B.h[a]) continue;   // same span: unchanged
        const double x = B.lo[a] + (double)L.x[a] * B.h[a];
        double l = (x - N.lo[a]) / N.h[a];
        l = (l < 0.0) ? 0.0 : l;
        l = (l > 1.0) ? 1.0 : l;
        L.x[a] = l;
    }
    // constant indices only: the lane state stays in registers
    L.x[0] = (axis == 0) ? 1.0 - xe : L.x[0];
    L.x[1] = (axis == 1) ? 1.0 - xe : L.x[1];
    L.x[2] = (axis == 2) ? 1.0 - xe : L.x[2];
    L.c = nb;
    if ((nfl & CF_SINK) && P.stop_at_sink) return ST_SINK;
    if ((int64_t)L.ncross >= P.max_steps) return ST_STEP_CAP;
    if (dt == 0.0) {
        if (++L.zrun >= kQuadZeroRun) {
            if constexpr (OUT == O_SERIES) {
                // stranded on the circuit: the position holds up to t_max
                double* row = P.snap_xyz + L.pid * (int64_t)P.n_snap * 3;
                while (L.ks < P.n_snap && snap[L.ks] <= P.t_max) {
                    cell_xyz<L_QUAD>(G, L.c, 0, 0, 0, (double)L.x[0], (double)L.x[1], (double)L.x[2],
                                     row + 3 * (int64_t)L.ks);
                    ++L.ks;
                }
            }
            return ST_STRANDED;
        }
    } else {
        L.zrun = 0;
    }
    return 0;
}

// End of a time step (transient flow): the particle continues in the next step's field from the
// same cell and position; it stops there if the cell is inactive, or a sink with stop_at_sink.
template <int PREC, int LAYOUT, bool BATCHED>
__device__ __forceinline__ int32_t step_switch(Lane<PREC>& L, const TrackParams& P) {
    L.g += 1;
    const GridDev& G2 = grid_of<BATCHED>(P, L.g);
    int32_t own;
    if constexpr (kPacked<LAYOUT>) {
        load_rec<PREC>(G2, L.c, P.sign, L.v1, L.v2, L.fl);
        own = L.fl;
    } else {
        own = G2.flags[L.c];
    }
    if (!(own & CF_ACTIVE)) return ST_INACTIVE_NB;
    if ((own & CF_SINK) && P.stop_at_sink) return ST_SINK;
    return 0;
}

// One cell crossing (S1-S7).  Returns 0 to continue, or the final status.  `job`: the lane's
// slot for deferred snapshots, or null to write them at once.
template <int PREC, int LAYOUT, int OUT, bool BATCHED, int CR>
__device__ __forceinline__ int32_t track_step(Lane<PREC>& L, const TrackParams& P, const double* snap,
                                              unsigned long long& crossings,
                                              SnapJob<typename Real<PREC>::T>* job = nullptr) {
    using R = typename Real<PREC>::T;
    const GridDev& G = grid_of<BATCHED>(P, L.g);
    R u1[3], u2[3];
    int32_t fl;
    if constexpr (kPacked<LAYOUT>) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u1[a] = L.v1[a];
            u2[a] = L.v2[a];
        }
        fl = L.fl;
    } else {
        load_cell<PREC, LAYOUT>(G, L, P.sign, u1, u2, fl);
    }

    // earliest reachable face; exact ties go to the lowest axis
    double dt = dinf();
    int32_t axis = -1;
    R xe = 0;
    double Aa[3], upa[3];   // FP64: gradient and particle velocity of each axis at the step start
    if constexpr (PREC == P64) {
        select_exit64<CR>(u1, u2, L.x, dt, axis, xe, L.amb, Aa, upa);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R e = 0;
            const double ta = exit_time<PREC, CR>(u1[a], u2[a], L.x[a], e, L.amb);
            if (ta < dt) {
                dt = ta;
                axis = a;
                xe = e;
            }
        }
    }

    // time limit: t_max, or the end of the current time step when that comes first (transient
    // flow); a face reached exactly at the limit is crossed
    double lim = P.t_max;
    bool next_step = false;
    if constexpr (BATCHED) {
        if (P.n_tsteps) {
            const double e = P.tstep_end[L.g];
            if (e < lim) {
                lim = e;
                next_step = L.g + 1 < P.n_tsteps;
            }
        }
    }
    if (axis < 0 && __builtin_isinf(lim)) {
        if constexpr (OUT == O_SERIES) write_snaps<PREC, LAYOUT, CR>(L, G, u1, u2, P, snap, dinf(), true);
        return ST_STRANDED;
    }
    const double t_exit = L.t + dt;
    // The limit comes first: every axis moves analytically to it and no face is crossed.  The
    // two axes other than the exit axis (axis 0 when no face is reachable) move by the same
    // code as in a crossing step, so lanes of a wave that stop at a limit (or at the end of a
    // time step) and lanes that cross a face diverge only in the exit axis' own advance.
    const bool at_lim = t_exit > lim;
    const double tau = at_lim ? lim - L.t : dt;

    const int32_t hi = (xe == (R)1) ? 1 : 0;
    const int32_t f = 2 * axis + hi;
    const int32_t step = hi ? 1 : -1;

    if constexpr (OUT == O_SERIES) {
        if (at_lim) write_snaps<PREC, LAYOUT, CR>(L, G, u1, u2, P, snap, lim, true);
        else if (job) queue_snaps<PREC, LAYOUT, CR>(L, G, u1, u2, P, snap, t_exit, job);
        else write_snaps<PREC, LAYOUT, CR>(L, G, u1, u2, P, snap, t_exit, false);
    }
    {
        const int ae = axis < 0 ? 0 : axis;
        const int a1 = (ae == 0) ? 1 : 0;
        const int a2 = (ae == 2) ? 1 : 2;
        const typename Coord<PREC>::T xa = (a1 == 0) ? L.x[0] : L.x[1];
        const typename Coord<PREC>::T xb = (a2 == 1) ? L.x[1] : L.x[2];
        typename Coord<PREC>::T na, nb, ne = xe;
        if constexpr (PREC == P64) {
            const double Ax = (a1 == 0) ? Aa[0] : Aa[1], ux = (a1 == 0) ? upa[0] : upa[1];
            const double Ay = (a2 == 1) ? Aa[1] : Aa[2], uy = (a2 == 1) ? upa[1] : upa[2];
            na = adv64_au<CR>(Ax, ux, xa, tau, L.amb);
            nb = adv64_au<CR>(Ay, uy, xb, tau, L.amb);
            if (at_lim) {
                const double Ae = (ae == 0) ? Aa[0] : ((ae == 1) ? Aa[1] : Aa[2]);
                const double ue = (ae == 0) ? upa[0] : ((ae == 1) ? upa[1] : upa[2]);
                const double xc = (ae == 0) ? L.x[0] : ((ae == 1) ? L.x[1] : L.x[2]);
                ne = adv64_au<CR>(Ae, ue, xc, tau, L.amb);
            }
        } else {
            // the gradient and particle velocity as the exit times formed them
            const float A0 = u2[0] - u1[0], A1 = u2[1] - u1[1], A2 = u2[2] - u1[2];
            const float p0 = fmaf(A0, (float)L.x[0], u1[0]), p1 = fmaf(A1, (float)L.x[1], u1[1]),
                        p2 = fmaf(A2, (float)L.x[2], u1[2]);
            na = adv_mix_au((a1 == 0) ? A0 : A1, (a1 == 0) ? p0 : p1, xa, tau);
            nb = adv_mix_au((a2 == 1) ? A1 : A2, (a2 == 1) ? p1 : p2, xb, tau);
            if (at_lim) {
                // the same gradient and velocity, formed again from the face velocities
                const typename Coord<PREC>::T xc = (ae == 0) ? L.x[0] : ((ae == 1) ? L.x[1] : L.x[2]);
                ne = adv_mix((ae == 0) ? u1[0] : ((ae == 1) ? u1[1] : u1[2]),
                             (ae == 0) ? u2[0] : ((ae == 1) ? u2[1] : u2[2]), xc, tau, L.amb);
            }
        }
        L.x[0] = (ae == 0) ? ne : na;
        L.x[1] = (ae == 1) ? ne : ((a1 == 1) ? na : nb);
        L.x[2] = (ae == 2) ? ne : nb;
    }
    if (at_lim) {
        L.t = lim;
        if constexpr (BATCHED) {
            if (next_step) return step_switch<PREC, LAYOUT, BATCHED>(L, P);
        }
        return axis < 0 ? ST_STRANDED : ST_MAX_TIME;
    }

    L.t = t_exit;
    L.ncross += 1;
    crossings += 1;
    L.hash = (L.hash ^ (unsigned long long)(uint32_t)L.c) * kFnvPrime;
    if constexpr (OUT == O_PATH) {
        // pathline record: the cell left, the face, the time and the position on the face
        if (!P.path_count) {
            const int64_t q = L.pq++;
            if (q >= 0 && q < L.pend) {
                // one 40-byte record: a particle's records form one contiguous stream
                double xyz[3];
                cell_xyz<LAYOUT>(G, L.c, L.i, L.j, L.k, (double)L.x[0], (double)L.x[1], (double)L.x[2], xyz);
                if (P.path_stage) {
                    stage_record(P, q, L.t, xyz[0], xyz[1], xyz[2], L.c, f);
                } else {
                    PathRec r;
                    r.t = L.t;
                    r.x = xyz[0];
                    r.y = xyz[1];
                    r.z = xyz[2];
                    r.cell = L.c;
                    r.face = f;
                    P.path_rec[q] = r;
                }
            } else {
                L.drop += 1u;
            }
        }
    }

    if constexpr (LAYOUT == L_QUAD) return quad_transfer<PREC, OUT>(L, G, P, snap, axis, f, xe, dt);

    // transfer to the neighbour across the exit face
    int32_t nfl_sink;
    if constexpr (LAYOUT == L_CELL) {
        if ((fl >> (NB_OUT + f)) & 1) return ST_BOUNDARY;
        if ((fl >> (NB_INACTIVE + f)) & 1) return ST_INACTIVE_NB;
        nfl_sink = (fl >> (NB_SINK + f)) & 1;
    } else {
        const int32_t ii = L.i + (axis == 0 ? step : 0);
        const int32_t jj = L.j + (axis == 1 ? step : 0);
        const int32_t kk = L.k + (axis == 2 ? step : 0);
        if (ii < 0 || ii >= G.nx || jj < 0 || jj >= G.ny || kk < 0 || kk >= G.nz) return ST_BOUNDARY;
        const int32_t nfl = G.flags[(kk * G.ny + jj) * G.nx + ii];
        if (!(nfl & CF_ACTIVE)) return ST_INACTIVE_NB;
        nfl_sink = (nfl & CF_SINK) ? 1 : 0;
    }
    // cell id stride of the axis, selected from uniform values (no per-lane multiply)
    const int32_t stride = (axis == 0) ? 1 : ((axis == 1) ? G.nx : G.plane);
    L.c += hi ? stride : -stride;
    if constexpr (kTrackIJK<LAYOUT, OUT>) {
        L.i += (axis == 0) ? step : 0;
        L.j += (axis == 1) ? step : 0;
        L.k += (axis == 2) ? step : 0;
    }
    L.x[0] = (axis == 0) ? (R)1 - xe : L.x[0];
    L.x[1] = (axis == 1) ? (R)1 - xe : L.x[1];
    L.x[2] = (axis == 2) ? (R)1 - xe : L.x[2];
    if (nfl_sink && P.stop_at_sink) return ST_SINK;
    if ((int64_t)L.ncross >= P.max_steps) return ST_STEP_CAP;
    // the particle continues: gather the new cell's record
    if constexpr (kPacked<LAYOUT>) load_rec<PREC>(G, L.c, P.sign, L.v1, L.v2, L.fl);
    return 0;
}

// Block-level setup shared by both kernels: LDS tables, snapshot times and counters.
struct BlockCounters {
    unsigned int hist[8];
    unsigned long long cross;
    unsigned int amb;
    unsigned int drop;
};

template <bool TS> struct BlockShared;
template <> struct BlockShared<false> : BlockCounters {};
template <> struct BlockShared<true> : BlockCounters {
    double snap[kMaxSnapLds];
};

template <int PREC, bool TS>
__device__ __forceinline__ const double* block_setup(BlockShared<TS>& S, const TrackParams& P) {
    if (threadIdx.x < 8) S.hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        S.cross = 0ull;
        S.amb = 0u;
        S.drop = 0u;
    }
    if constexpr (PREC == P64) ptcr::lds_tables_init();   // the FP32 path has no table lookups
    const double* snap = P.snap_times;
    if constexpr (TS) {
        if (P.n_snap <= kMaxSnapLds) {
            for (int q = threadIdx.x; q < P.n_snap; q += blockDim.x) S.snap[q] = P.snap_times[q];
            snap = S.snap;
        }
    }
    __syncthreads();
    return snap;
}

__device__ __forceinline__ void block_flush(BlockCounters& S, const TrackParams& P,
                                            unsigned long long crossings, unsigned amb,
                                            unsigned drop) {
    // wave-level reduction of the crossing count, one LDS atomic per wave
    for (int off = 32; off > 0; off >>= 1) crossings += __shfl_down(crossings, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&S.cross, crossings);
    if (amb) atomicAdd(&S.amb, amb);
    if (drop) atomicAdd(&S.drop, drop);
    __syncthreads();
    if (threadIdx.x == 0 && S.amb) atomicAdd(&P.counters->cr_ambiguous, (unsigned long long)S.amb);
    if (threadIdx.x == 0 && S.drop) atomicAdd(&P.counters->path_dropped, (unsigned long long)S.drop);
    if (threadIdx.x < 8 && S.hist[threadIdx.x])
        atomicAdd(&P.counters->status[threadIdx.x], (unsigned long long)S.hist[threadIdx.x]);
    if (threadIdx.x == 0 && S.cross) atomicAdd(&P.counters->crossings, S.cross);
}

// At the end of a particle in the fast FP64 kernels: if one of its correctly rounded evaluations
// was left undecided (L.amb != 0; a value within 2^-96 of a rounding midpoint, which the fast
// kernels do not settle -- that would take registers their loop does not have), hand it to the
// careful pass instead of finishing it.  Its input state in memory is untouched, so the careful
// kernel tracks it again from there; this call's crossings of it are taken back and nothing of it
// is written back.  Returns false (finish it) when there is no free entry; the undecided
// evaluations are then counted as such.
template <int PREC, int OUT>
__device__ __forceinline__ bool hand_off(Lane<PREC>& L, const TrackParams& P, unsigned long long& crossings) {
    const unsigned long long q = atomicAdd(&P.counters->recheck_tracks, 1ull);
    const unsigned amb = L.amb;
    L.amb = 0u;
    if (q < (unsigned long long)P.recheck_cap) {
        P.recheck_pid[q] = (int32_t)L.pid;
        crossings -= (unsigned long long)(L.ncross - P.ncross[L.pid]);
        if constexpr (OUT == O_PATH) L.drop = L.drop0;
        return true;
    }
    atomicAdd(&P.counters->cr_ambiguous, (unsigned long long)amb);
    return false;
}

// Finish a particle of the fast kernels (st > 0), or hand it to the careful pass.
template <int PREC, int LAYOUT, int OUT, bool BATCHED>
__device__ __forceinline__ void finish_fast(Lane<PREC>& L, int32_t st, const TrackParams& P, unsigned int* s_hist,
                                            unsigned long long& crossings) {
    if constexpr (PREC == P64) {
        if (L.amb && hand_off<PREC, OUT>(L, P, crossings)) return;
    }
    finish<PREC, LAYOUT, OUT, BATCHED>(L, st, P, s_hist);
}

// ---------------------------------------------------------------------------------------------
// Waves per SIMD the register allocator is asked to fit.  FP64: four (128 VGPRs, a constant of
// the rare accurate phase in scratch) instead of three at 136 VGPRs -- the fourth wave hides
// more of the dependent FP64 latency and the record gathers (C2 -9%, C3 -10%); five (96 VGPRs)
// spill live loop values and are slower.  Mixed: eight for endpoint runs (C3 -5%), six for
// timeseries and pathlines (C5 -4%; eight spills there).
// Rounding mode of the fast kernels: undecided evaluations go to the careful pass.
constexpr int kFastCr = ptcr::CR_FLAG;

template <int PREC, int OUT>
constexpr int kWavesStatic = PREC == P64 ? 4 : (OUT == O_END ? 8 : 6);
// Persistent kernel: FP64 three (168 VGPRs instead of ~175, a few bytes of rarely used values in
// scratch: C3 -20%, C2 -13%; four spill 110-230 bytes per lane and are slower); mixed six for
// endpoint runs (C4 -7%), four otherwise.
template <int PREC, int OUT>
constexpr int kWavesPersistent = PREC == P64 ? 3 : (OUT == O_END ? 6 : 4);

template <int PREC, int LAYOUT, int OUT, bool BATCHED>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWavesStatic<PREC, OUT>)))
k_track_static(TrackParams P) {
    __shared__ BlockShared<OUT == O_SERIES> S;
    const double* snap = block_setup<PREC, OUT == O_SERIES>(S, P);
    unsigned long long crossings = 0;
    Lane<PREC> L;
    L.amb = 0u;
    L.drop = 0u;
    // Block b runs on die b mod 8.  The slots are dealt to the dies in chunks of kDieChunk
    // consecutive blocks, round robin: a die's concurrent blocks hold neighbouring particles
    // (they share record lines in its L2), and every die sweeps the whole ordered work, so no die
    // is left with a heavier part of it (gridDim.x is a multiple of 8 * kDieChunk).
    const int64_t die = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
    const int64_t blk = ((j / kDieChunk) * kXcd + die) * kDieChunk + j % kDieChunk;
    const int64_t slot = blk * blockDim.x + threadIdx.x;
    if constexpr (OUT == O_SERIES && kPacked<LAYOUT>) {
        // timeseries: the wave steps its lanes together so that it can evaluate the deferred
        // snapshots of all of them at once
        using J = SnapJob<typename Real<PREC>::T>;
        extern __shared__ __align__(16) double dyn_lds[];   // blockDim.x slots
        J* jobs = reinterpret_cast<J*>(dyn_lds);
        J* W = jobs + (threadIdx.x & ~63u);
        jobs[threadIdx.x].cnt = 0;
        jobs[threadIdx.x].amb = 0u;
        wave_sync();
        int32_t st = ST_SKIP;
        if (slot < P.n) {
            L.pid = P.order ? (int64_t)P.order[slot] : slot;
            st = begin<PREC, LAYOUT, OUT, BATCHED>(L, P, snap);
        }
        for (;;) {
            if (st == 0) st = track_step<PREC, LAYOUT, OUT, BATCHED, kFastCr>(L, P, snap, crossings, &jobs[threadIdx.x]);
            wave_sync();
            const unsigned long long pend = __ballot(jobs[threadIdx.x].cnt > 0);
            const unsigned long long live = __ballot(st == 0);
            if (pend != 0ull && (__popcll(pend) >= kSnapFlush || live == 0ull))
                flush_snaps<PREC, LAYOUT, BATCHED, kFastCr>(W, P, snap);
            if (live == 0ull) break;
        }
        L.amb |= jobs[threadIdx.x].amb;   // undecided snapshots evaluated for this lane by the wave
        if (st > 0) finish_fast<PREC, LAYOUT, OUT, BATCHED>(L, st, P, S.hist, crossings);
    } else {
        if (slot < P.n) {
            L.pid = P.order ? (int64_t)P.order[slot] : slot;
            int32_t st = begin<PREC, LAYOUT, OUT, BATCHED>(L, P, snap);
            while (st == 0) st = track_step<PREC, LAYOUT, OUT, BATCHED, kFastCr>(L, P, snap, crossings);
            if (st > 0) finish_fast<PREC, LAYOUT, OUT, BATCHED>(L, st, P, S.hist, crossings);
        }
    }
    block_flush(S, P, crossings, L.amb, L.drop);
}

// Lane 0's value of a 64-bit quantity as a wave-uniform (scalar) value.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

template <int PREC, int LAYOUT, int OUT, bool BATCHED>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWavesPersistent<PREC, OUT>)))
k_track_persistent(TrackParams P) {
    __shared__ BlockShared<OUT == O_SERIES> S;
    const double* snap = block_setup<PREC, OUT == O_SERIES>(S, P);
    unsigned long long crossings = 0;
    const unsigned long long n = (unsigned long long)P.n;
    const int refill = P.refill;
    const int steps = P.steps_per_refill;
    const unsigned long long chunk = (unsigned long long)P.chunk;
    // Wave-uniform state: the wave's current chunk [cnext, cend) of queue slots, claimed with one
    // atomic; idle lanes are refilled from it at every refill point.
    unsigned long long cnext = 0, cend = 0;
    bool exhausted = false;  // every die's segment is empty
    // The slots are split into kXcd segments; a wave first drains its own die's segment
    // (L2 locality), then the following ones.
    const unsigned long long seg = (n + kXcd - 1) / kXcd;
    const int die = blockIdx.x % kXcd;
    int tried = 0;           // segments found empty so far (wave-uniform)
    Lane<PREC> L;
    L.amb = 0u;
    L.drop = 0u;
    L.pid = -1;
    for (;;) {
        const unsigned long long idle = __ballot(L.pid < 0);
        const int nidle = __popcll(idle);
        const unsigned long long avail = cend - cnext;
        if (nidle > 0 && (nidle >= refill || nidle == 64) && (avail > 0 || !exhausted)) {
            unsigned long long nbase = 0, nlen = 0;
            while (avail < (unsigned long long)nidle && !exhausted && nlen == 0) {
                const int sg = (die + tried) % kXcd;
                const unsigned long long lo = (unsigned long long)sg * seg;
                const unsigned long long hi = (lo + seg < n) ? lo + seg : n;
                // one claim covers every idle lane: at least a chunk, more when more lanes are idle
                // (a wave's first fill takes 64 consecutive slots, as in the static kernel)
                const unsigned long long want = (unsigned long long)nidle - avail;
                const unsigned long long amount = want > chunk ? want : chunk;
                unsigned long long base = 0;
                if ((threadIdx.x & 63) == 0) base = atomicAdd(&P.counters->queue[sg], amount);
                base = lo + uniform_u64(base);   // lane 0's claim, kept in scalar registers
                if (base < hi) {
                    nbase = base;
                    nlen = (hi - base < amount) ? hi - base : amount;
                }
                if (base + amount >= hi) {
                    ++tried;
                    if (tried == kXcd) exhausted = true;
                }
            }
            if (L.pid < 0) {
                const unsigned long long rank =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                long long slot = -1;
                if (rank < avail) slot = (long long)(cnext + rank);
                else if (rank - avail < nlen) slot = (long long)(nbase + (rank - avail));
                if (slot >= 0) {
                    L.pid = P.order ? (int64_t)P.order[slot] : slot;
                    const int32_t st = begin<PREC, LAYOUT, OUT, BATCHED>(L, P, snap);
                    if (st != 0) {
                        if (st > 0) finish<PREC, LAYOUT, OUT, BATCHED>(L, st, P, S.hist);
                        L.pid = -1;
                    }
                }
            }
            if (avail >= (unsigned long long)nidle) {
                cnext += (unsigned long long)nidle;
            } else {
                const unsigned long long used = (unsigned long long)nidle - avail;
                cnext = nbase + (used < nlen ? used : nlen);
                cend = nbase + nlen;
            }
        }
        if (__ballot(L.pid >= 0) == 0ull) {
            if (exhausted && cnext >= cend) break;
            continue;
        }
        for (int s = 0; s < steps; ++s) {
            if (L.pid >= 0) {
                const int32_t st = track_step<PREC, LAYOUT, OUT, BATCHED, kFastCr>(L, P, snap, crossings);
                if (st != 0) {
                    finish_fast<PREC, LAYOUT, OUT, BATCHED>(L, st, P, S.hist, crossings);
                    L.pid = -1;
                }
            }
        }
    }
    block_flush(S, P, crossings, L.amb, L.drop);
}

// Careful pass, FP64: the particles the tracking kernel handed over are tracked again from their
// input state with every correctly rounded evaluation decided exactly (CR_EXACT), one thread per
// particle, snapshots and pathline records written again in full.  The list is usually empty; the
// grid is fixed and strides over it.
template <int LAYOUT, int OUT, bool BATCHED>
__global__ void __launch_bounds__(kBlock) k_track_careful(TrackParams P) {
    __shared__ BlockShared<OUT == O_SERIES> S;
    const unsigned long long cnt = P.counters->recheck_tracks;
    const int64_t n = (int64_t)(cnt < (unsigned long long)P.recheck_cap ? cnt : (unsigned long long)P.recheck_cap);
    if (n == 0) return;   // uniform across the grid: no barrier below is skipped by part of a block
    const double* snap = block_setup<P64, OUT == O_SERIES>(S, P);
    unsigned long long crossings = 0;
    Lane<P64> L;
    L.amb = 0u;
    L.drop = 0u;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        L.pid = P.recheck_pid[q];
        int32_t st = begin<P64, LAYOUT, OUT, BATCHED>(L, P, snap);
        while (st == 0) st = track_step<P64, LAYOUT, OUT, BATCHED, ptcr::CR_EXACT>(L, P, snap, crossings);
        if (st > 0) finish<P64, LAYOUT, OUT, BATCHED>(L, st, P, S.hist);
    }
    block_flush(S, P, crossings, L.amb, L.drop);
}

// Allocation-free entry point: write the argument's bytes to dst.
__global__ void __launch_bounds__(256) k_fill(FillArgs A) {
    for (uint32_t q = threadIdx.x; q < A.nbytes; q += blockDim.x) A.dst[q] = A.bytes[q];
}

// Allocation-free entry point: the run's counters as the caller's counts (the fields of
// pt_summary that the device computes, in the order PT_COUNT_* of pt.h).
__global__ void k_counts(CountsParams C) {
    if (threadIdx.x != 0) return;
    const Counters& c = *C.c;
    int64_t tracked = 0;
    for (int q = 0; q < 8; ++q) {
        C.out[2 + q] = (int64_t)c.status[q];
        tracked += (int64_t)c.status[q];
    }
    C.out[0] = (int64_t)c.crossings;
    C.out[1] = tracked;
    C.out[10] = (int64_t)c.cr_ambiguous;
    C.out[11] = C.path_pass == 1 ? (int64_t)c.crossings
                                 : (C.path_pass == 2 ? (int64_t)c.crossings - (int64_t)c.path_dropped : 0);
    C.out[12] = C.path_pass == 2 ? (int64_t)c.path_dropped : 0;
    C.out[13] = (int64_t)c.recheck_tracks;
    C.out[14] = 0;
    C.out[15] = 0;
}

__global__ void k_reset(Counters* c) {
    unsigned long long* w = reinterpret_cast<unsigned long long*>(c);
    const int n = sizeof(Counters) / sizeof(unsigned long long);
    if ((int)threadIdx.x < n) w[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------------------------------------
// Block-wide inclusive scan of one value per thread (Hillis-Steele in LDS).
__device__ __forceinline__ int64_t block_scan(int64_t* part, int64_t x) {
    part[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        const int64_t a = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += a;
        __syncthreads();
    }
    return part[threadIdx.x];
}

// Spatial ordering: the particles sorted by their starting cell (bucket), in two levels with LDS
// counters only -- returning atomics on a global histogram run at the L2 atomic units' ~25 G/s
// on random buckets, which made a one-level counting sort of 1.8e7 particles take 1 ms.  Ranks
// inside a bucket come from LDS atomics, so the order inside a bucket is arbitrary.  The order
// only changes which lanes and dies process which particles, never a result.

// The group of particle p: the last group whose first particle is at or before p, searched in
// [lo, n_groups).
__device__ __forceinline__ int32_t group_at(const int64_t* offsets, int32_t lo, int32_t n_groups, int64_t p) {
    int32_t hi = n_groups;   // invariant: offsets[lo] <= p < offsets[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (offsets[mid] <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Bucket of particle p.  Called with the lanes of a wave on consecutive particles (the first
// active lane on the lowest): the group of that lane is searched once with wave-uniform values,
// and only lanes past the end of its group search on their own.
__device__ __forceinline__ uint32_t sort_bucket(const SortParams& S, int64_t p) {
    int64_t key = 0;
    if (S.n_groups > 0) {
        const int64_t p0 = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)p >> 32)) << 32) |
                                     __builtin_amdgcn_readfirstlane((uint32_t)p));
        const int32_t g0 = group_at(S.group_offsets, 0, S.n_groups, p0);
        const int64_t end0 = (g0 + 1 < S.n_groups) ? S.group_offsets[g0 + 1] : INT64_MAX;
        const int32_t g = (p < end0) ? g0 : group_at(S.group_offsets, g0 + 1, S.n_groups, p);
        key = S.grid_base[S.group_grid[g]];
    }
    const int32_t c = S.cell[p];
    const int32_t st = S.status[p];
    if (c < 0 || (st != ST_ACTIVE && st != ST_MAX_TIME)) return 0u;
    key += c;
    const int64_t b = key >> S.shift;
    return (uint32_t)(b < S.nbuckets ? b : S.nbuckets - 1);
}

// Level 1: each tile of kSortTile particles keeps its particles' buckets and counts them per
// super-bucket; the counts go to cnt[super][tile].
__global__ void __launch_bounds__(256) k_sort_tiles(SortParams S) {
    __shared__ unsigned c[kMaxSuper];
    for (int q = threadIdx.x; q < S.nsuper; q += 256) c[q] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int q = threadIdx.x; q < kSortTile; q += 256) {
        const int64_t p = base + q;
        if (p < S.n) {
            const uint32_t b = sort_bucket(S, p);
            S.bucket[p] = b;
            atomicAdd(&c[b / (uint32_t)S.fine], 1u);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < S.nsuper; q += 256) S.cnt[(int64_t)q * S.ptiles + blockIdx.x] = c[q];
}

// Exclusive prefix sum of the tile counts (super-bucket-major) in three passes: within each tile
// of kScanTile entries (tile totals to S.part), over the tile totals (one workgroup), then each
// tile adds the total of the tiles before it.  Counts and sums stay below n < 2^31.
__global__ void __launch_bounds__(kScanBlock) k_sort_scan_tiles(SortParams S) {
    __shared__ int64_t part[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    unsigned v[kScanPer];
    int64_t sum = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = (base + q < S.ncnt) ? S.cnt[base + q] : 0u;
        sum += v[q];
    }
    const int64_t incl = block_scan(part, sum);
    int64_t run = incl - sum;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        if (base + q < S.ncnt) S.cnt[base + q] = (unsigned)run;
        run += v[q];
    }
    if (threadIdx.x == kScanBlock - 1) S.part[blockIdx.x] = (unsigned)incl;
}

__global__ void __launch_bounds__(kScanBlock) k_sort_scan_partials(SortParams S) {
    __shared__ int64_t part[kScanBlock];
    const int per = (S.ntiles + kScanBlock - 1) / kScanBlock;
    const int lo = (int)threadIdx.x * per;
    const int hi = (lo + per < S.ntiles) ? lo + per : S.ntiles;
    int64_t sum = 0;
    for (int q = lo; q < hi; ++q) sum += S.part[q];
    int64_t run = block_scan(part, sum) - sum;
    for (int q = lo; q < hi; ++q) {
        const unsigned h = S.part[q];
        S.part[q] = (unsigned)run;
        run += h;
    }
}

__global__ void __launch_bounds__(kScanBlock) k_sort_scan_add(SortParams S) {
    const unsigned add = S.part[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int64_t q = threadIdx.x; q < kScanTile; q += kScanBlock)
        if (base + q < S.ncnt) S.cnt[base + q] += add;
}

// Level 1, placement: each tile writes its particles (index and bucket) from the first slot of
// its share of each super-bucket on, ranked by LDS atomics.
__global__ void __launch_bounds__(256) k_sort_spread(SortParams S) {
    __shared__ unsigned at[kMaxSuper];
    for (int q = threadIdx.x; q < S.nsuper; q += 256) at[q] = S.cnt[(int64_t)q * S.ptiles + blockIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int q = threadIdx.x; q < kSortTile; q += 256) {
        const int64_t p = base + q;
        if (p < S.n) {
            const uint32_t b = S.bucket[p];
            const unsigned k = atomicAdd(&at[b / (uint32_t)S.fine], 1u);
            S.sidx[k] = (int32_t)p;
            S.sbucket[k] = b;
        }
    }
}

// Level 2: one block per super-bucket orders its range [lo, hi) by bucket: an LDS histogram of
// its `fine` buckets, the histogram's exclusive prefix sum, then LDS-atomic ranks.
__global__ void __launch_bounds__(kFineBlock) k_sort_fine(SortParams S) {
    __shared__ unsigned h[kFineMax];
    __shared__ int64_t part[kFineBlock];
    const int s = blockIdx.x;
    const int64_t lo = S.cnt[(int64_t)s * S.ptiles];
    const int64_t hi = (s + 1 < S.nsuper) ? (int64_t)S.cnt[(int64_t)(s + 1) * S.ptiles] : S.n;
    const uint32_t b0 = (uint32_t)s * (uint32_t)S.fine;
    for (int q = threadIdx.x; q < S.fine; q += kFineBlock) h[q] = 0u;
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += kFineBlock) atomicAdd(&h[S.sbucket[i] - b0], 1u);
    __syncthreads();
    // exclusive prefix sum of h[0, fine): each thread a run of consecutive buckets
    const int per = (S.fine + kFineBlock - 1) / kFineBlock;
    const int q0 = (int)threadIdx.x * per;
    const int q1 = (q0 + per < S.fine) ? q0 + per : S.fine;
    int64_t sum = 0;
    for (int q = q0; q < q1; ++q) sum += h[q];
    int64_t run = block_scan(part, sum) - sum;
    for (int q = q0; q < q1; ++q) {
        const unsigned v = h[q];
        h[q] = (unsigned)run;
        run += v;
    }
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += kFineBlock) {
        const unsigned r = atomicAdd(&h[S.sbucket[i] - b0], 1u);
        S.order[lo + r] = S.sidx[i];
    }
}

// ---------------------------------------------------------------------------------------------
// Pathline offsets: inclusive prefix sum, in place, of the per-particle crossing counts written
// by the count pass (v = path_offsets + 1), and path_offsets[0] = 0.


// Tile b (kScanTile elements): scan within the tile, tile total to part[b].
__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(ScanParams S) {
    __shared__ int64_t part[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int64_t v[kScanPer];
    int64_t sum = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = (base + q < S.n) ? S.v[base + q] : 0;
        sum += v[q];
    }
    const int64_t incl = block_scan(part, sum);
    int64_t run = incl - sum;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        run += v[q];
        if (base + q < S.n) S.v[base + q] = run;
    }
    if (threadIdx.x == kScanBlock - 1) S.part[blockIdx.x] = incl;
}

// One workgroup: exclusive scan of the tile totals; writes the leading zero.
__global__ void __launch_bounds__(kScanBlock) k_scan_partials(ScanParams S) {
    __shared__ int64_t part[kScanBlock];
    const int64_t per = (S.ntiles + kScanBlock - 1) / kScanBlock;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = (lo + per < S.ntiles) ? lo + per : S.ntiles;
    int64_t sum = 0;
    for (int64_t q = lo; q < hi; ++q) sum += S.part[q];
    int64_t run = block_scan(part, sum) - sum;
    for (int64_t q = lo; q < hi; ++q) {
        const int64_t h = S.part[q];
        S.part[q] = run;
        run += h;
    }
    if (threadIdx.x == 0 && S.head) *S.head = 0;
}

// Tile b adds the total of the tiles before it.
__global__ void __launch_bounds__(kScanBlock) k_scan_add(ScanParams S) {
    const int64_t add = S.part[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int64_t q = threadIdx.x; q < kScanTile; q += kScanBlock)
        if (base + q < S.n) S.v[base + q] += add;
}

// Quadtree grid load: each face's total flow (its subfaces summed in order), the velocities
// u = Q / (n V), the own flags, the first subface and the per-face subface counts.
__global__ void __launch_bounds__(256) k_build_quad(BuildQuadParams B) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B.ncell) return;
    const QuadBox& X = B.box[c];
    const double V = (X.h[0] * X.h[1]) * X.h[2];
    const double n_c = B.por ? B.por[c] : B.por_scalar;
    const int32_t own = B.flags ? B.flags[c] : CF_ACTIVE;
    double Q[6];
    bool finite = true;
    uint32_t counts = 0u;
    for (int f = 0; f < 6; ++f) {
        const int32_t a = B.sub_off[6 * c + f], b = B.sub_off[6 * c + f + 1];
        double q = 0.0;
        for (int32_t s = a; s < b; ++s) {
            finite = finite && __builtin_isfinite(B.sub_q[s]);
            q += B.sub_q[s];
        }
        Q[f] = q;
        counts |= (uint32_t)(b - a) << (5 * f);
    }
    if (!finite) atomicOr(&B.err[0], 1);
    if (!(n_c > 0.0) || !__builtin_isfinite(n_c)) atomicOr(&B.err[1], 1);
    if (own & ~(CF_ACTIVE | CF_SINK)) atomicOr(&B.err[2], 1);
    if (B.balance_tol >= 0.0 && (own & CF_ACTIVE) && !(own & CF_SINK) && finite) {
        const double net = (Q[0] - Q[1]) + (Q[2] - Q[3]) + (Q[4] - Q[5]);
        double gross = 0.0;
        for (int32_t s = B.sub_off[6 * c]; s < B.sub_off[6 * c + 6]; ++s) gross += fabs(B.sub_q[s]);
        if (fabs(net) > B.balance_tol * gross) atomicOr(&B.err[3], 1);
    }
    const double d = n_c * V;
    QuadRec r;
    for (int f = 0; f < 6; ++f) r.u[f] = Q[f] / d;
    r.flags = own & (CF_ACTIVE | CF_SINK);
    r.sub_base = B.sub_off[6 * c];
    r.counts = counts;
    r.pad0 = 0;
    B.rec[c] = r;
}

// Grid load: validate the field and build both packed records of every cell.
__global__ void __launch_bounds__(256) k_build(BuildParams B) {
    const GridDev& G = B.g;
    const int64_t ncell = (int64_t)G.nx * G.ny * G.nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int64_t nx = G.nx, ny = G.ny, nz = G.nz;
    const int64_t plane = nx * ny;
    const int64_t k = c / plane, rem = c - k * plane;
    const int64_t j = rem / nx, i = rem - j * nx;
    const int64_t fx = (k * ny + j) * (nx + 1) + i;
    const int64_t fy = (k * (ny + 1) + j) * nx + i;
    const int64_t fz = (k * ny + j) * nx + i;
    const double q[6] = {G.qx[fx], G.qx[fx + 1], G.qy[fy], G.qy[fy + nx], G.qz[fz], G.qz[fz + plane]};
    const double n_c = G.por ? G.por[c] : G.por_scalar;
    const int32_t own = G.flags ? G.flags[c] : CF_ACTIVE;
    bool finite = true;
    for (int f = 0; f < 6; ++f) finite = finite && __builtin_isfinite(q[f]);
    if (!finite) atomicOr(&B.err[0], 1);
    if (!(n_c > 0.0) || !__builtin_isfinite(n_c)) atomicOr(&B.err[1], 1);
    if (own & ~(CF_ACTIVE | CF_SINK)) atomicOr(&B.err[2], 1);
    if (B.balance_tol >= 0.0 && (own & CF_ACTIVE) && !(own & CF_SINK) && finite) {
        const double net = (q[0] - q[1]) + (q[2] - q[3]) + (q[4] - q[5]);
        const double gross = fabs(q[0]) + fabs(q[1]) + fabs(q[2]) + fabs(q[3]) + fabs(q[4]) + fabs(q[5]);
        if (fabs(net) > B.balance_tol * gross) atomicOr(&B.err[3], 1);
    }
    const double d = n_c * G.V;
    int32_t word = own & (CF_ACTIVE | CF_SINK);
    const int64_t ncoord[3] = {i, j, k};
    const int64_t ndim[3] = {nx, ny, nz};
    const int64_t nstride[3] = {1, nx, plane};
    for (int f = 0; f < 6; ++f) {
        const int a = f >> 1;
        const int64_t s = (f & 1) ? 1 : -1;
        const int64_t cc = ncoord[a] + s;
        if (cc < 0 || cc >= ndim[a]) {
            word |= 1 << (NB_OUT + f);
        } else {
            const int32_t nf = G.flags ? G.flags[c + s * nstride[a]] : CF_ACTIVE;
            if (!(nf & CF_ACTIVE)) word |= 1 << (NB_INACTIVE + f);
            if (nf & CF_SINK) word |= 1 << (NB_SINK + f);
        }
    }
    CellRec64 r64;
    CellRec32 r32;
    for (int f = 0; f < 6; ++f) {
        const double u = q[f] / d;
        r64.u[f] = u;
        r32.u[f] = (float)u;
    }
    r64.flags = word;
    r64.pad0 = 0;
    r64.pad1 = 0.0;
    r32.flags = word;
    r32.pad0 = 0;
    B.rec64[c] = r64;
    B.rec32[c] = r32;
}

template <int PREC, int LAYOUT, int OUT, bool BATCHED>
const void* pick_sched(int sched) {
    if (sched == S_STATIC) return reinterpret_cast<const void*>(&k_track_static<PREC, LAYOUT, OUT, BATCHED>);
    return reinterpret_cast<const void*>(&k_track_persistent<PREC, LAYOUT, OUT, BATCHED>);
}

template <int PREC, int LAYOUT, int OUT>
const void* pick_batched(const KernelKey& k) {
    return k.batched ? pick_sched<PREC, LAYOUT, OUT, true>(k.sched) : pick_sched<PREC, LAYOUT, OUT, false>(k.sched);
}

template <int PREC, int LAYOUT>
const void* pick_out(const KernelKey& k) {
    if (k.out == O_SERIES) return pick_batched<PREC, LAYOUT, O_SERIES>(k);
    if (k.out == O_PATH) return pick_batched<PREC, LAYOUT, O_PATH>(k);
    return pick_batched<PREC, LAYOUT, O_END>(k);
}

}  // namespace

const void* track_kernel(const KernelKey& k) {
    if (k.layout == L_QUAD) {   // FP64, single grid
        if (k.out == O_SERIES) return pick_sched<P64, L_QUAD, O_SERIES, false>(k.sched);
        if (k.out == O_PATH) return pick_sched<P64, L_QUAD, O_PATH, false>(k.sched);
        return pick_sched<P64, L_QUAD, O_END, false>(k.sched);
    }
    if (k.precision == PMIX) return pick_out<PMIX, L_CELL>(k);
    if (k.layout == L_FACES) return pick_out<P64, L_FACES>(k);
    return pick_out<P64, L_CELL>(k);
}

template <int LAYOUT, int OUT>
const void* pick_careful(const KernelKey& k) {
    return k.batched ? reinterpret_cast<const void*>(&k_track_careful<LAYOUT, OUT, true>)
                     : reinterpret_cast<const void*>(&k_track_careful<LAYOUT, OUT, false>);
}

template <int LAYOUT>
const void* pick_careful_out(const KernelKey& k) {
    if (k.out == O_SERIES) return pick_careful<LAYOUT, O_SERIES>(k);
    if (k.out == O_PATH) return pick_careful<LAYOUT, O_PATH>(k);
    return pick_careful<LAYOUT, O_END>(k);
}

const void* careful_kernel(const KernelKey& k) {
    if (k.layout == L_QUAD) {   // single grid
        if (k.out == O_SERIES) return reinterpret_cast<const void*>(&k_track_careful<L_QUAD, O_SERIES, false>);
        if (k.out == O_PATH) return reinterpret_cast<const void*>(&k_track_careful<L_QUAD, O_PATH, false>);
        return reinterpret_cast<const void*>(&k_track_careful<L_QUAD, O_END, false>);
    }
    if (k.layout == L_FACES) return pick_careful_out<L_FACES>(k);
    return pick_careful_out<L_CELL>(k);
}

const void* reset_kernel() { return reinterpret_cast<const void*>(&k_reset); }
const void* fill_kernel() { return reinterpret_cast<const void*>(&k_fill); }
const void* counts_kernel() { return reinterpret_cast<const void*>(&k_counts); }
const void* sort_tiles_kernel() { return reinterpret_cast<const void*>(&k_sort_tiles); }
const void* sort_scan_tiles_kernel() { return reinterpret_cast<const void*>(&k_sort_scan_tiles); }
const void* sort_scan_partials_kernel() { return reinterpret_cast<const void*>(&k_sort_scan_partials); }
const void* sort_scan_add_kernel() { return reinterpret_cast<const void*>(&k_sort_scan_add); }
const void* sort_spread_kernel() { return reinterpret_cast<const void*>(&k_sort_spread); }
const void* sort_fine_kernel() { return reinterpret_cast<const void*>(&k_sort_fine); }
const void* scan_tiles_kernel() { return reinterpret_cast<const void*>(&k_scan_tiles); }
const void* scan_partials_kernel() { return reinterpret_cast<const void*>(&k_scan_partials); }
const void* scan_add_kernel() { return reinterpret_cast<const void*>(&k_scan_add); }
const void* build_kernel() { return reinterpret_cast<const void*>(&k_build); }
const void* build_quad_kernel() { return reinterpret_cast<const void*>(&k_build_quad); }

}  // namespace pt
