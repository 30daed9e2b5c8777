// boys_table.h -- host-side construction of the Boys-function grid used by the
// device Taylor expansion (see boys() in shg_math.h).
//
// table[i * BOYS_STRIDE + n] = F_n(i / BOYS_PER_UNIT), n = 0..BOYS_NTAB-1, where
// F_n(T) = int_0^1 exp(-T t^2) t^(2n) dt (supplement eq. 3). Each grid point is
// evaluated in long double: F_{nmax} from the convergent series
//   F_n(T) = exp(-T) sum_{i>=0} (2T)^i / ((2n+1)(2n+3)...(2n+2i+1)),
// then the lower orders by the downward recurrence F_n = (2T F_{n+1} + e^-T)/(2n+1).
#pragma once
#include <math.h>
#include "shg_math.h"

namespace shg {

inline void build_boys_table(double *table)
{
    const int nmax = BOYS_NTAB - 1;
    for (int i = 0; i < BOYS_NPTS; ++i) {
        long double T = (long double)i / BOYS_PER_UNIT;
        long double term = 1.0L / (2 * nmax + 1), sum = term;
        for (int k = 1; k < 100000; ++k) {
            term *= 2 * T / (long double)(2 * nmax + 2 * k + 1);
            sum += term;
            if (term < 1e-22L * sum) break;
        }
        long double e = expl(-T);
        long double F[BOYS_NTAB];
        F[nmax] = e * sum;
        for (int n = nmax - 1; n >= 0; --n) F[n] = (2 * T * F[n + 1] + e) / (2 * n + 1);
        for (int n = 0; n < BOYS_NTAB; ++n) table[(size_t)i * BOYS_STRIDE + n] = (double)F[n];
    }
}

}  // namespace shg
