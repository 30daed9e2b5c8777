// Host mirror of the engine's arithmetic: CPU entry points used by the tests
// to check shg_math.h against the oracle without a GPU.
#include <stdlib.h>
#include <algorithm>
#include <vector>
#include "shg_hostmirror.h"

extern "C" int shgm_pairs(int32_t nshell, const double *center, const int32_t *l, const int32_t *nprim,
                          const int64_t *prim_off, const double *exps, const double *coefs, int op,
                          double omega, const int32_t *pairs, int64_t n, const int64_t *out_off,
                          double *out, double *dout)
{
    static std::vector<double> tab;
    if (tab.empty()) {
        tab.resize((size_t)BOYS_NPTS * BOYS_STRIDE);
        build_boys_table(tab.data());
    }
    int64_t np = 0;
    for (int i = 0; i < nshell; ++i) np = std::max<int64_t>(np, prim_off[i] + nprim[i]);
    std::vector<double> w(np);
    for (int i = 0; i < nshell; ++i) {
        if (l[i] < 0 || l[i] > 4 || nprim[i] < 1 || nprim[i] > 7) return -1;
        double N = shell_norm(l[i], nprim[i], exps + prim_off[i], coefs + prim_off[i]);
        for (int k = 0; k < nprim[i]; ++k) {
            double a2 = 2 * exps[prim_off[i] + k], p = 1;
            for (int q = 0; q < l[i]; ++q) p *= a2;
            w[prim_off[i] + k] = N * coefs[prim_off[i] + k] / p;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        int a = pairs[2 * i], b = pairs[2 * i + 1];
        double X[3] = {center[3 * a] - center[3 * b], center[3 * a + 1] - center[3 * b + 1],
                       center[3 * a + 2] - center[3 * b + 2]};
        int D = dout ? 1 : 0;
        static const pair_fn *tabs[5] = {hm_table_op0(), hm_table_op1(), hm_table_op2(), hm_table_op3(),
                                         hm_table_op4()};
        pair_fn f = tabs[op][(l[a] * 5 + l[b]) * 2 + D];
        if (!f) return -2;   // class not instantiated in this build
        f(exps + prim_off[a], w.data() + prim_off[a], nprim[a], exps + prim_off[b], w.data() + prim_off[b],
          nprim[b], X, omega, tab.data(), out + out_off[i], dout ? dout + 3 * out_off[i] : nullptr);
    }
    return 0;
}

extern "C" void shgm_boys_table(double *out) { build_boys_table(out); }

extern "C" void shgm_boys(int nmax, double T, double *F)
{
    static std::vector<double> tab;
    if (tab.empty()) {
        tab.resize((size_t)BOYS_NPTS * BOYS_STRIDE);
        build_boys_table(tab.data());
    }
    double f[10];
    boys<0, 9>(T, tab.data(), f);
    for (int i = 0; i <= nmax && i < 10; ++i) F[i] = f[i];
}
