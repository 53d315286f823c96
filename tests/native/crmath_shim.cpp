// Host build of the library's correctly rounded log1p / expm1 / log, for the CPU tests.
#include "../../paper_2302_13590_amd/csrc/pt_crmath.h"

extern "C" {
unsigned ptcr_eval(int fn, const double* x, double* y, long n) {
    unsigned amb = 0;
    for (long i = 0; i < n; ++i) {
        if (fn == 0) y[i] = ptcr::log1p_cr(x[i], &amb);
        else if (fn == 1) y[i] = ptcr::expm1_cr(x[i], &amb);
        else y[i] = ptcr::log_cr(x[i], &amb);
    }
    return amb;
}
}

// Quick- and accurate-phase double-doubles (before rounding), to check their error bounds.
extern "C" void ptcr_phases(int fn, const double* x, double* qh, double* ql, double* ah, double* al,
                            long n) {
    for (long i = 0; i < n; ++i) {
        ptcr::dd q, a;
        if (fn == 1) {
            const ptcr::ExpRed R = ptcr::exp_reduce(x[i]);
            q = ptcr::expm1_combine<true>(R, ptcr::expm1_series_quick(R.r), 0);
            a = ptcr::expm1_combine<false>(R, ptcr::expm1_series_accurate(R.r), 0);
        } else {
            const ptcr::dd y = fn == 0 ? ptcr::two_sum(1.0, x[i]) : ptcr::dd{x[i], 0.0};
            const ptcr::LogRed R = ptcr::log_reduce(y.h, y.l);
            q = ptcr::log_sum(R, ptcr::log1p_series_quick(R.r));
            const ptcr::LogRed RA = ptcr::log_reduce_accurate(y.h, y.l);
            a = ptcr::log_sum_accurate(RA, ptcr::log1p_series_accurate(RA.r));
        }
        qh[i] = q.h; ql[i] = q.l; ah[i] = a.h; al[i] = a.l;
    }
}
