// Host mirror of (a|r_a^{2n}|b): the engine's double-double monopole T^(k) of
// eq. T_rab2_deriv (shg_r2n_math.h), then its block assembly (pair_block_from_O).
#include <algorithm>
#include <utility>
#include <vector>
#include "shg_hostmirror.h"
#include "../../paper_1701_06588_amd/csrc/shg_r2n_math.h"

template <int LA, int LB, bool D, int NR>
static void r2n_pair(const double *ea, const double *wa, int ka, const double *eb, const double *wb, int kb,
                     const double *X, double *out, double *dout)
{
    constexpr int KLO = cmax(LA, LB), KHI = LA + LB + (D ? 1 : 0), NK = KHI - KLO + 1;
    const double R2 = fma(X[0], X[0], fma(X[1], X[1], X[2] * X[2]));
    dd T[NK];
    for (int k = 0; k < NK; ++k) T[k] = dd{0.0, 0.0};
    for (int ia = 0; ia < ka; ++ia)
        for (int ib = 0; ib < kb; ++ib) r2n_accumulate<LA, NR, KLO, KHI>(ea[ia], eb[ib], R2, wa[ia] * wb[ib], T);
    double O[NK];
    for (int k = 0; k < NK; ++k) O[k] = T[k].hi + T[k].lo;
    pair_block_from_O<LA, LB, D>(O, X, out, dout);
}

typedef void (*r2n_fn)(const double *, const double *, int, const double *, const double *, int, const double *,
                       double *, double *);

template <int... I>
static const r2n_fn *make_table(std::integer_sequence<int, I...>)
{
    // index ((nr * 5 + la) * 5 + lb) * 2 + D
    static const r2n_fn t[] = {&r2n_pair<(I / 2) / 5 % 5, (I / 2) % 5, (I % 2) == 1, I / 50>...};
    return t;
}

extern "C" int shgm_r2n(int32_t nshell, const double *center, const int32_t *l, const int32_t *nprim,
                        const int64_t *prim_off, const double *exps, const double *coefs, int nr,
                        const int32_t *pairs, int64_t n, const int64_t *out_off, double *out, double *dout)
{
    static const r2n_fn *tab = make_table(std::make_integer_sequence<int, 300>{});
    if (nr < 0 || nr > 5) return -1;
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
        tab[((nr * 5 + l[a]) * 5 + l[b]) * 2 + (dout ? 1 : 0)](
            exps + prim_off[a], w.data() + prim_off[a], nprim[a], exps + prim_off[b], w.data() + prim_off[b],
            nprim[b], X, out + out_off[i], dout ? dout + 3 * out_off[i] : nullptr);
    }
    return 0;
}
