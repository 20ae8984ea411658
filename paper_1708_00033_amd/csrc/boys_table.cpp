// Host generation of the Boys-function table used by the device evaluator.
//   F_m(T) = int_0^1 t^{2m} e^{-T t^2} dt
// evaluated in long double from the everywhere-convergent positive series
//   F_m(T) = e^{-T} sum_{k>=0} (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)).
#include <cmath>

#include "hfx_internal.h"

void hfx_boys_table(double* tab) {
    for (int k = 0; k < BOYS_NT; ++k) {
        const long double T = (long double)k * (long double)BOYS_DT;
        const long double eT = expl(-T);
        for (int m = 0; m < BOYS_NM; ++m) {
            long double term = 1.0L / (2 * m + 1), sum = term;
            for (int j = 1; j < 4000; ++j) {
                term *= 2.0L * T / (2 * m + 2 * j + 1);
                sum += term;
                if (term < 1e-22L * sum) break;
            }
            tab[k * BOYS_NM + m] = (double)(eT * sum);
        }
    }
}
