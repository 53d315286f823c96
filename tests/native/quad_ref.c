/* Reference values for the CPU tests: log1p / expm1 / log in 113-bit quad precision
 * (libquadmath), rounded once to double.  Also returns the quad value's distance to the
 * nearest rounding boundary of double, in units of the double's ulp. */
#include <quadmath.h>
#include <math.h>

void quad_eval(int fn, const double* x, double* y, double* margin, long n) {
    for (long i = 0; i < n; ++i) {
        __float128 q = (__float128)x[i];
        __float128 v = fn == 0 ? log1pq(q) : fn == 1 ? expm1q(q) : logq(q);
        double d = (double)v;
        y[i] = d;
        if (margin) {
            if (isfinite(d) && d != 0.0) {
                double up = nextafter(d, INFINITY), dn = nextafter(d, -INFINITY);
                __float128 mid_up = ((__float128)d + (__float128)up) / 2;
                __float128 mid_dn = ((__float128)d + (__float128)dn) / 2;
                __float128 a = fabsq(v - mid_up), b = fabsq(v - mid_dn);
                __float128 m = a < b ? a : b;
                margin[i] = (double)(m / ((__float128)up - (__float128)d));
            } else {
                margin[i] = INFINITY;
            }
        }
    }
}

/* Relative error of double-doubles (h + l) against the quad value of fn(x), as double. */
void quad_relerr(int fn, const double* x, const double* h, const double* l, double* err, long n) {
    for (long i = 0; i < n; ++i) {
        __float128 q = (__float128)x[i];
        __float128 v = fn == 0 ? log1pq(q) : fn == 1 ? expm1q(q) : logq(q);
        __float128 s = (__float128)h[i] + (__float128)l[i];
        err[i] = v == 0 ? 0.0 : (double)fabsq((s - v) / v);
    }
}
