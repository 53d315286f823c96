// Correctly rounded FP64 log1p, expm1 and log for the FP64 tracking path.
//
// Each function returns the double nearest to the exact function value.  A
// quick phase evaluates the function as a double-double with a relative error
// below 2^-68 and applies a rounding test (Ziv's strategy): if every real number
// within that error of the double-double rounds to the same double, that double
// is the correctly rounded result.  Otherwise an accurate phase (error below
// 2^-96) is evaluated and tested again; if that test fails too (an input closer
// to a rounding boundary than 2^-96 relative), the nearest double of the
// accurate value is returned and `ambiguous` is raised.
//
// Reductions:
//   log(y),  y = 2^k m, m in [sqrt(1/2), sqrt(2)]:  c = RN(256/j), j = round(256 m),
//            r = m c - 1 (|r| < 2^-8.4, formed exactly with FMA products),
//            log y = k ln2 - ln c + log1p(r), log1p(r) by its Taylor series.
//   log1p(x) = log(y) with y = 1 + x carried exactly as a double-double.
//   expm1(x), x = (128 k + j) ln2/128 + r (|r| <= ln2/256):
//            expm1 x = (2^k 2^(j/128) - 1) + 2^k 2^(j/128) (e^r - 1),
//            e^r - 1 by its Taylor series.
// Constants come from pt_crtables.h (double-double, generated in decimal).
//
// Written for both the device (HIP) and a host build used by the CPU tests.
#pragma once

#include <math.h>
#include <stdint.h>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define PT_CR_HD __host__ __device__ inline
#define PT_CR_COLD __host__ __device__ inline
#define PT_CR_TABLE static constexpr
#else
#define PT_CR_HD static inline
#define PT_CR_COLD static inline
#define PT_CR_TABLE static constexpr
#endif

#include "pt_crtables.h"

namespace ptcr {

// Table access.  In device code the tables of the quick phase live in LDS (copied once
// per workgroup by lds_tables_init): an LDS read is short and is counted apart from
// global memory loads, so the tables never make a wave wait for an outstanding gather.
#if defined(__HIP_DEVICE_COMPILE__)
__shared__ double lds_log_c[PT_CR_LOG_J1 - PT_CR_LOG_J0 + 1];
__shared__ double lds_log_l[PT_CR_LOG_J1 - PT_CR_LOG_J0 + 1][2];
__shared__ double lds_exp_t[128][2];
#define PT_CR_LOGC(i) (::ptcr::lds_log_c[(i)])
#define PT_CR_LOGL(i, h) (::ptcr::lds_log_l[(i)][(h)])
#define PT_CR_EXPT(i, h) (::ptcr::lds_exp_t[(i)][(h)])
#else
#define PT_CR_LOGC(i) (PT_CR_LOG_C[(i)])
#define PT_CR_LOGL(i, h) (PT_CR_LOG_L[(i)][(h)])
#define PT_CR_EXPT(i, h) (PT_CR_EXP_T[(i)][(h)])
#endif

#ifdef __HIPCC__
// Copy the quick-phase tables into this workgroup's LDS; the caller synchronises the
// workgroup before the first evaluation.
__device__ inline void lds_tables_init() {
#if defined(__HIP_DEVICE_COMPILE__)
    const int n = PT_CR_LOG_J1 - PT_CR_LOG_J0 + 1;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        lds_log_c[q] = PT_CR_LOG_C[q];
        lds_log_l[q][0] = PT_CR_LOG_L[q][0];
        lds_log_l[q][1] = PT_CR_LOG_L[q][1];
    }
    for (int q = threadIdx.x; q < 128; q += blockDim.x) {
        lds_exp_t[q][0] = PT_CR_EXP_T[q][0];
        lds_exp_t[q][1] = PT_CR_EXP_T[q][1];
    }
#endif
}
#endif

struct dd {
    double h, l;
};

PT_CR_HD dd two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

// requires |a| >= |b| or a == 0
PT_CR_HD dd fast_two_sum(double a, double b) {
    const double s = a + b;
    const double e = b - (s - a);
    return {s, e};
}

PT_CR_HD dd two_prod(double a, double b) {
    const double p = a * b;
    return {p, fma(a, b, -p)};
}

PT_CR_HD dd dd_add(dd x, dd y) {
    const dd s = two_sum(x.h, y.h);
    const dd t = two_sum(x.l, y.l);
    const dd v = fast_two_sum(s.h, s.l + t.h);
    return fast_two_sum(v.h, t.l + v.l);
}

// x + y when |x.h| >= |y.h| (or x.h == 0) and no cancellation beyond a factor of a few can occur:
// the two high parts are summed exactly by the ordered error-free sum, the low parts plainly.
// Every caller meets the ordering: in log_sum |ln c_j| >= ln(256/255) > |log1p(r)| (|r| < 2^-8.4)
// or c_j = 1, and |k ln 2| >= ln 2 > |ln m| (m in [sqrt(1/2), sqrt(2)]) or k = 0; in expm1_combine
// |2^k T_j q| < 0.502 |2^k T_j - 1|.
PT_CR_HD dd dd_add_fast(dd x, dd y) {
    const dd s = fast_two_sum(x.h, y.h);
    return fast_two_sum(s.h, s.l + (x.l + y.l));
}

PT_CR_HD dd dd_add_d(dd x, double d) {
    const dd s = two_sum(x.h, d);
    return fast_two_sum(s.h, s.l + x.l);
}

PT_CR_HD dd dd_mul(dd x, dd y) {
    dd p = two_prod(x.h, y.h);
    p.l += fma(x.h, y.l, x.l * y.h);
    return fast_two_sum(p.h, p.l);
}

PT_CR_HD dd dd_mul_d(dd x, double d) {
    dd p = two_prod(x.h, d);
    p.l = fma(x.l, d, p.l);
    return fast_two_sum(p.h, p.l);
}

// If every real within eps*|v| of v.h + v.l rounds to the same double, store it and
// return true.
PT_CR_HD bool round_test(dd v, double eps, double* out) {
    const double e = eps * fabs(v.h);
    const double a = v.h + (v.l - e);
    const double b = v.h + (v.l + e);
    if (a == b) {
        *out = a;
        return true;
    }
    return false;
}

constexpr double kEpsQuick = 0x1p-68;
constexpr double kEpsAccurate = 0x1p-96;

// What an evaluation does when the accurate phase cannot decide the rounding either.
//   CR_EXACT: arguments below 2^-40 are decided from exact parts (below); any other such argument
//             (closer than 2^-96 to a midpoint, not expected to occur) is counted in `ambiguous`.
//   CR_FLAG:  every such argument is counted in `ambiguous` and the nearest double of the accurate
//             value is returned -- for code that re-runs the flagged work with CR_EXACT elsewhere
//             (the exact path needs registers that a hot loop does not have).
enum CrMode { CR_EXACT = 0, CR_FLAG = 1 };

// ----------------------------------------------------------------------------------- small arguments
// For 2^-60 <= |x| < 2^-40, expm1(x) = x + x^2/2 + ... and log1p(x) = x - x^2/2 + ... lie within a
// few ulps of x, and for x near 2^-53 .. 2^-50 the x^2/2 term is close to half an ulp of x: the
// value can sit within 2^-100 of a rounding midpoint for structural reasons (x with a regular bit
// pattern, such as values just below a power of two), which the 2^-96 accurate phase cannot
// decide.  When the accurate phase fails on such an argument, the value is summed from exact
// parts instead and the rounding is decided by an exact comparison with the midpoint.

// RN(s + th + tl) for a double s, a tail th with |th| <= |s| whose sum with s is formed exactly,
// and tl, known to within err, far below ulp(s).
PT_CR_HD double round_sum3(double s, double th, double tl, double err, unsigned* ambiguous) {
    const dd w = fast_two_sum(s, th);                     // s + th = w.h + w.l exactly
    // the neighbour of w.h on w.l's side (w.h finite and non-zero here): one step of the
    // magnitude's bit pattern away from or towards zero
    int64_t bits;
    __builtin_memcpy(&bits, &w.h, sizeof bits);
    bits += ((w.l > 0.0) == (w.h > 0.0)) ? 1 : -1;
    double nb;
    __builtin_memcpy(&nb, &bits, sizeof nb);
    const double m = 0.5 * (nb - w.h);                    // the midpoint on w.l's side, signed (exact)
    if (!(fabs(w.l) >= 0.5 * fabs(m))) return w.h;        // tl cannot carry the sum to the midpoint
    const double g = w.l - m;                             // exact (Sterbenz)
    const double d = g + tl;                              // its sign is the side of the midpoint
    if (m > 0.0 ? d > err : d < -err) return nb;
    if (m > 0.0 ? d < -err : d > err) return w.h;
    *ambiguous += 1u;
    return (m > 0.0 ? d >= 0.0 : d <= 0.0) ? nb : w.h;
}

// expm1(x) for 2^-60 <= |x| < 2^-40: x + x^2/2 + x^3/6 + x^4/24, truncation below 2^-166 |x|.
// x^2 = p + pe and x p = q + qe exactly; x^3/6 as a double-double to ~2^-100 of itself.
PT_CR_HD double expm1_small(double x, unsigned* ambiguous) {
    const double p = x * x, pe = fma(x, x, -p);
    const double q = x * p, qe = fma(x, p, -q);
    const double c3 = q / 6.0;
    const double c3l = ((fma(-c3, 6.0, q) + qe) + x * pe) / 6.0;
    const double c4 = (p * p) / 24.0;
    const dd v = two_sum(x, 0.5 * p);                     // x + x^2/2 (high part) exactly
    const dd t = two_sum(v.l, c3);
    const double tl = t.l + ((0.5 * pe + c3l) + c4);
    return round_sum3(v.h, t.h, tl, 0x1p-140 * fabs(x), ambiguous);
}

// log1p(x) for 2^-60 <= |x| < 2^-40: x - x^2/2 + x^3/3 - x^4/4, truncation below 2^-160 |x|.
PT_CR_HD double log1p_small(double x, unsigned* ambiguous) {
    const double p = x * x, pe = fma(x, x, -p);
    const double q = x * p, qe = fma(x, p, -q);
    const double c3 = q / 3.0;
    const double c3l = ((fma(-c3, 3.0, q) + qe) + x * pe) / 3.0;
    const double c4 = -0.25 * (p * p);
    const dd v = two_sum(x, -0.5 * p);
    const dd t = two_sum(v.l, c3);
    const double tl = t.l + ((-0.5 * pe + c3l) + c4);
    return round_sum3(v.h, t.h, tl, 0x1p-140 * fabs(x), ambiguous);
}

// ----------------------------------------------------------------------------------- log

struct LogRed {
    int k;
    int j;
    dd r;
};

// y = yh + yl > 0 (yh normal or subnormal, |yl| <= ulp(yh)).
PT_CR_HD LogRed log_reduce(double yh, double yl) {
    int e;
    double m = frexp(yh, &e);   // m in [1/2, 1)
    m *= 2.0;
    e -= 1;                     // m in [1, 2)
    if (m > PT_CR_SQRT2) {
        m *= 0.5;
        e += 1;
    }
    const double ml = ldexp(yl, -e);
    const int j = (int)rint(m * 256.0);
    const double c = PT_CR_LOGC(j - PT_CR_LOG_J0);
    const dd p = two_prod(m, c);              // exact
    // p.h - 1 is exact; ml*c is below 2^-52 |m c| and joins the low part
    const dd r = fast_two_sum(p.h - 1.0, p.l + ml * c);
    return {e, j, r};
}

// Same reduction with the correction term carried exactly (accurate phase).
PT_CR_HD LogRed log_reduce_accurate(double yh, double yl) {
    int e;
    double m = frexp(yh, &e);
    m *= 2.0;
    e -= 1;
    if (m > PT_CR_SQRT2) {
        m *= 0.5;
        e += 1;
    }
    const double ml = ldexp(yl, -e);
    const int j = (int)rint(m * 256.0);
    const double c = PT_CR_LOGC(j - PT_CR_LOG_J0);
    const dd p = two_prod(m, c);
    dd r = fast_two_sum(p.h - 1.0, p.l);
    r = dd_add(r, two_prod(ml, c));
    return {e, j, r};
}

PT_CR_HD dd log_sum_accurate(const LogRed& R, dd p) {
    const double kd = (double)R.k;
    dd kl = two_prod(kd, PT_CR_LN2_H);
    kl.l = fma(kd, PT_CR_LN2_L, kl.l);
    const dd L = {PT_CR_LOGL(R.j - PT_CR_LOG_J0, 0), PT_CR_LOGL(R.j - PT_CR_LOG_J0, 1)};
    return dd_add(kl, dd_add(L, p));
}

PT_CR_HD dd log_sum(const LogRed& R, dd p) {
    const double kd = (double)R.k;
    dd kl = two_prod(kd, PT_CR_LN2_H);
    kl.l = fma(kd, PT_CR_LN2_L, kl.l);
    const dd L = {PT_CR_LOGL(R.j - PT_CR_LOG_J0, 0), PT_CR_LOGL(R.j - PT_CR_LOG_J0, 1)};
    // |L + p| >= |p|/2 (L = ln(m_j), p = ln(m/m_j), same sign or |p| < |L|/2 within a bin),
    // and k ln2 dominates L + p whenever k != 0
    return dd_add_fast(kl, dd_add_fast(L, p));
}

// log1p(r) for r = x + l (|r| < 2^-8.4, |l| <= ulp(x)/2), as a double-double with relative
// error below 2^-69.5:
//   log1p(r) = x - x^2/2 + x^3 T(x) + l (1 - x + x^2) + O(2^-100 |r|),
//   T = 1/3 - x/4 + ... - x^7/10 (truncation below 2^-83 |r|).
// x^2 = p + pe exactly, x - p/2 is summed exactly; the remaining terms are below
// 2^-18.5 |r| and are evaluated in double.
PT_CR_HD dd log1p_series_quick(dd r) {
    const double x = r.h;
    double T = -0x1.999999999999ap-4;                 // -1/10
    T = fma(x, T, 0x1.c71c71c71c71cp-4);              //  1/9
    T = fma(x, T, -0x1.0000000000000p-3);             // -1/8
    T = fma(x, T, 0x1.2492492492492p-3);              //  1/7
    T = fma(x, T, -0x1.5555555555555p-3);             // -1/6
    T = fma(x, T, 0x1.999999999999ap-3);              //  1/5
    T = fma(x, T, -0x1.0000000000000p-2);             // -1/4
    T = fma(x, T, 0x1.5555555555555p-2);              //  1/3
    const double p = x * x;
    const double pe = fma(x, x, -p);
    const double h = -0.5 * p;                        // exact
    const double lo = fma(r.l, p - x, r.l) + fma(p * x, T, -0.5 * pe);
    const dd s = fast_two_sum(x, h);                  // |h| < |x| 2^-9.4
    return fast_two_sum(s.h, s.l + lo);
}

// log1p(r) for |r| < 2^-8.4 with relative error < 2^-100.
PT_CR_HD dd log1p_series_accurate(dd r) {
    // log1p(r) = r * sum_{k>=1} (-1)^(k+1) r^(k-1) / k, Horner from k = 14
    dd S = {PT_CR_INVK[14][0], PT_CR_INVK[14][1]};
    S.h = -S.h;
    S.l = -S.l;
    for (int k = 13; k >= 1; --k) {
        dd c = {PT_CR_INVK[k][0], PT_CR_INVK[k][1]};
        if (!(k & 1)) {
            c.h = -c.h;
            c.l = -c.l;
        }
        S = dd_add(c, dd_mul(r, S));
    }
    return dd_mul(r, S);
}

// Accurate phase: it runs for about one evaluation in 2^15.  With CR_EXACT, a log1p argument x
// below 2^-40 (y = 1 + x carried as yh + yl) that it cannot decide is decided from exact parts.
template <int M>
PT_CR_COLD double log_accurate(double yh, double yl, unsigned* ambiguous) {
    const LogRed R = log_reduce_accurate(yh, yl);
    const dd a = log_sum_accurate(R, log1p_series_accurate(R.r));
    double out;
    if (round_test(a, kEpsAccurate, &out)) return out;
    if (M == CR_EXACT) {
        const double x = (yh - 1.0) + yl;   // exact when y = 1 + x was formed from a double x this small
        if (fabs(x) < 0x1p-40 && fabs(yh - 1.0) <= 0x1p-39) return log1p_small(x, ambiguous);
    }
    *ambiguous += 1u;
    return a.h + a.l;
}

template <int M = CR_EXACT>
PT_CR_HD double log_dd_cr(double yh, double yl, unsigned* ambiguous) {
    const LogRed R = log_reduce(yh, yl);
    double out;
    const dd q = log_sum(R, log1p_series_quick(R.r));
    if (round_test(q, kEpsQuick, &out)) return out;
    return log_accurate<M>(yh, yl, ambiguous);
}

// Inputs of log1p that need no reduction: stores the result and returns true.
PT_CR_HD bool log1p_special(double x, double* out) {
    if (!(x > -1.0)) {
        *out = (x == -1.0) ? -__builtin_huge_val() : __builtin_nan("");   // x < -1 or NaN
        return true;
    }
    if (fabs(x) < 0x1p-60 || x == __builtin_huge_val()) {
        *out = x;                       // log1p(x) = x (1 - x/2 + ...) rounds to x
        return true;
    }
    return false;
}

// Inputs of log that need no reduction: stores the result and returns true.
PT_CR_HD bool log_special(double x, double* out) {
    if (!(x > 0.0)) {
        *out = (x == 0.0) ? -__builtin_huge_val() : __builtin_nan("");
        return true;
    }
    if (x == __builtin_huge_val() || x == 1.0) {
        *out = (x == 1.0) ? 0.0 : x;
        return true;
    }
    return false;
}

// Correctly rounded log1p(x).
template <int M = CR_EXACT>
PT_CR_HD double log1p_cr(double x, unsigned* ambiguous) {
    double out;
    if (log1p_special(x, &out)) return out;
    const dd y = two_sum(1.0, x);       // 1 + x exactly
    return log_dd_cr<M>(y.h, y.l, ambiguous);
}

// Correctly rounded log(x).
template <int M = CR_EXACT>
PT_CR_HD double log_cr(double x, unsigned* ambiguous) {
    double out;
    if (log_special(x, &out)) return out;
    return log_dd_cr<M>(x, 0.0, ambiguous);
}

// ----------------------------------------------------------------------------------- expm1

struct ExpRed {
    int k;
    int j;
    dd r;
};

PT_CR_HD ExpRed exp_reduce(double x) {
    const double Kd = rint(x * PT_CR_INV_LN2_128);
    const int K = (int)Kd;
    const double r0 = x - Kd * PT_CR_LN2_128_1;   // exact
    dd m = two_prod(Kd, PT_CR_LN2_128_2);
    m.l = fma(Kd, PT_CR_LN2_128_3, m.l);
    const dd h = two_sum(r0, -m.h);
    const dd r = fast_two_sum(h.h, h.l - m.l);
    return {K >> 7, K & 127, r};
}

// e^r - 1 for r = x + l (|r| <= ln2/256, |l| <= ulp(x)/2), as a double-double with relative
// error below 2^-70:
//   e^r - 1 = x + x^2/2 + x^3 U(x) + l (1 + x + x^2/2) + O(2^-100 |r|),
//   U = 1/3! + x/4! + ... + x^5/8! (truncation below 2^-88 |r|).
// x^2 = p + pe exactly, x + p/2 is summed exactly; the remaining terms are below
// 2^-19.6 |r| and are evaluated in double.
PT_CR_HD dd expm1_series_quick(dd r) {
    const double x = r.h;
    double U = 0x1.a01a01a01a01ap-16;              // 1/8!
    U = fma(x, U, 0x1.a01a01a01a01ap-13);          // 1/7!
    U = fma(x, U, 0x1.6c16c16c16c17p-10);          // 1/6!
    U = fma(x, U, 0x1.1111111111111p-7);           // 1/5!
    U = fma(x, U, 0x1.5555555555555p-5);           // 1/4!
    U = fma(x, U, 0x1.5555555555555p-3);           // 1/3!
    const double p = x * x;
    const double pe = fma(x, x, -p);
    const double h = 0.5 * p;                      // exact
    const double lo = fma(r.l, x + h, r.l) + fma(p * x, U, 0.5 * pe);
    const dd s = fast_two_sum(x, h);               // |h| < |x| 2^-9.5
    return fast_two_sum(s.h, s.l + lo);
}

// e^r - 1 for |r| <= ln2/256 with relative error < 2^-100.
PT_CR_HD dd expm1_series_accurate(dd r) {
    dd S = {PT_CR_INVF[15][0], PT_CR_INVF[15][1]};
    for (int k = 14; k >= 1; --k) S = dd_add({PT_CR_INVF[k][0], PT_CR_INVF[k][1]}, dd_mul(r, S));
    return dd_mul(r, S);
}

// (2^k T_j - 1) + 2^k T_j q, scaled by 2^-s (s > 0 only near overflow).  When (k, j) is not
// (0, 0), |x - r| >= ln2/128 and |2^k T_j q| < 0.502 |2^k T_j - 1| (worst at x - r = ln2/128,
// r = -ln2/256), so the sum cancels by about a factor of 2 at most: the quick phase adds
// the low parts plainly (dd_add_fast, error below 2^-100 relative).
//
// Quick phase, -1 <= k <= 52: T.h - one is exact (T.h / one = 2^k T_j lies in [1/2, 2^53): for
// T.h <= 2 one by Sterbenz's lemma, above because one is then a multiple of ulp(T.h) and the
// difference keeps T.h's exponent or one less), so A = (T.h - one) + T.l needs no error-free sum;
// its low part may exceed half an ulp of its high part, which dd_add_fast accepts.
template <bool FAST>
PT_CR_HD dd expm1_combine(const ExpRed& R, dd q, int s) {
    if (R.k == 0 && R.j == 0) return q;
    const int k = R.k - s;
    const dd T = {ldexp(PT_CR_EXPT(R.j, 0), k), ldexp(PT_CR_EXPT(R.j, 1), k)};
    const double one = ldexp(1.0, -s);
    if (FAST) {
        dd A;
        if (R.k >= -1 && R.k <= 52) A = {T.h - one, T.l};
        else A = dd_add_d(T, -one);
        return dd_add_fast(A, dd_mul(T, q));
    }
    const dd A = dd_add_d(T, -one);
    return dd_add(A, dd_mul(T, q));
}

// Accurate phase of expm1 (x in the main range).
template <int M>
PT_CR_COLD double expm1_accurate(double x, unsigned* ambiguous) {
    const ExpRed R = exp_reduce(x);
    const int s = (R.k > 1000) ? 2 : 0;
    const double back = s ? 4.0 : 1.0;
    const dd a = expm1_combine<false>(R, expm1_series_accurate(R.r), s);
    double out;
    if (round_test(a, kEpsAccurate, &out)) return out * back;
    if (M == CR_EXACT && fabs(x) < 0x1p-40) return expm1_small(x, ambiguous);
    *ambiguous += 1u;
    return (a.h + a.l) * back;
}

// Correctly rounded expm1(x).
template <int M = CR_EXACT>
PT_CR_HD double expm1_cr(double x, unsigned* ambiguous) {
    if (!(x == x)) return x;
    if (fabs(x) < 0x1p-60) return x;     // expm1(x) = x (1 + x/2 + ...) rounds to x
    if (x > 710.0) return __builtin_huge_val();
    if (x < -40.0) return -1.0;          // e^x < 2^-57: -1 + e^x rounds to -1
    const ExpRed R = exp_reduce(x);
    const int s = (R.k > 1000) ? 2 : 0;  // keep 2^k finite; the final scaling by 4 is exact
    const double back = s ? 4.0 : 1.0;
    double out;
    const dd q = expm1_combine<true>(R, expm1_series_quick(R.r), s);
    if (round_test(q, kEpsQuick, &out)) return out * back;
    return expm1_accurate<M>(x, ambiguous);
}

}  // namespace ptcr
