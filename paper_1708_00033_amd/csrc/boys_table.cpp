// Host generation of the Boys-function tables used by the device evaluator.
//   F_m(T) = int_0^1 t^{2m} e^{-T t^2} dt
// evaluated in long double from the everywhere-convergent positive series
//   F_m(T) = e^{-T} sum_{k>=0} (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)),
// stored per order L as rows F_{L+j}(T_k)/j!, j = 0..7 (Taylor coefficients),
// the order-L block at position boys_block(L); then e^{-T_k} for every k.
#include <cmath>

#include "hfx_internal.h"

void hfx_boys_table(double* tab) {
    const int mmax = BOYS_NL + BOYS_ROW;
    long double F[BOYS_NL + BOYS_ROW];
    for (int k = 0; k < BOYS_NT; ++k) {
        const long double T = (long double)k * (long double)BOYS_DT;
        const long double eT = expl(-T);
        tab[BOYS_EXP_OFF + k] = (double)eT;
        for (int m = 0; m < mmax; ++m) {
            long double term = 1.0L / (2 * m + 1), sum = term;
            for (int j = 1; j < 4000; ++j) {
                term *= 2.0L * T / (2 * m + 2 * j + 1);
                sum += term;
                if (term < 1e-22L * sum) break;
            }
            F[m] = eT * sum;
        }
        for (int L = 0; L < BOYS_NL; ++L) {
            long double fact = 1.0L;
            for (int j = 0; j < BOYS_ROW; ++j) {
                if (j > 0) fact *= j;
                tab[((size_t)boys_block(L) * BOYS_NT + k) * BOYS_ROW + j] = (double)(F[L + j] / fact);
            }
        }
    }
}
