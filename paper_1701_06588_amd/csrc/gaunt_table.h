// gaunt_table.h -- host construction of the real Gaunt coefficients used by the
// three-index overlap (Sec. II.D, eq. CG_expansion and the final (a b a~) formula).
//
// With orthonormal real spherical harmonics Y^r_{l,m} (m < 0 sine type, no
// Condon-Shortley phase; Y^r_{l,m} = sqrt((2l+1)/4pi) * A_{l,|m|} R^{c/s}_{l,|m|}(u)
// on the unit sphere, eqs. A and regular_scaled_harmonics_recursion),
//     G^{L,l,lt}_{M,m,mt} = int Y^r_{l,m} Y^r_{lt,mt} Y^r_{L,M} dOmega,
// so that Y^r_{l,m} Y^r_{lt,mt} = sum_{L,M} G Y^r_{L,M}. Evaluated in long
// double by Gauss-Legendre quadrature in cos(theta) times the trapezoidal rule in
// phi, exact for the polynomial degrees involved (<= 2 (l + lt) <= 18).
//
// Sparse layout per (l, lt): for every output pair (m, mt) a list of
// (L, M, G) with |G| > 1e-15.
#pragma once
#include <math.h>
#include <vector>

namespace shg {

struct GauntEntry {
    int L, M;
    double g;
};

// real spherical harmonics Y^r_{l,m}(u), l <= lmax, at one unit vector; index l*l + l + m
inline void real_sph_ld(int lmax, long double x, long double y, long double z, long double *Y)
{
    const long double PI_L = 3.141592653589793238462643383279502884L;
    int n = (lmax + 1) * (lmax + 2) / 2;
    std::vector<long double> Rc(n), Rs(n);
    auto id = [](int l, int m) { return l * (l + 1) / 2 + m; };
    long double r2 = x * x + y * y + z * z;
    Rc[0] = 1;
    Rs[0] = 0;
    for (int l = 0; l < lmax; ++l) {
        Rc[id(l + 1, l + 1)] = -(x * Rc[id(l, l)] - y * Rs[id(l, l)]) / (2 * l + 2);
        Rs[id(l + 1, l + 1)] = -(y * Rc[id(l, l)] + x * Rs[id(l, l)]) / (2 * l + 2);
        for (int m = 0; m <= l; ++m) {
            long double pc = (m <= l - 1) ? Rc[id(l - 1, m)] : 0, ps = (m <= l - 1) ? Rs[id(l - 1, m)] : 0;
            long double den = (long double)(l + m + 1) * (l - m + 1);
            Rc[id(l + 1, m)] = ((2 * l + 1) * z * Rc[id(l, m)] - r2 * pc) / den;
            Rs[id(l + 1, m)] = ((2 * l + 1) * z * Rs[id(l, m)] - r2 * ps) / den;
        }
    }
    for (int l = 0; l <= lmax; ++l)
        for (int m = -l; m <= l; ++m) {
            int mu = m < 0 ? -m : m;
            long double f = 1;
            for (int i = 2; i <= l + mu; ++i) f *= i;
            for (int i = 2; i <= l - mu; ++i) f *= i;
            long double A = ((mu & 1) ? -1 : 1) * sqrtl((mu == 0 ? 1 : 2) * f);
            long double R = m < 0 ? Rs[id(l, mu)] : Rc[id(l, mu)];
            Y[l * l + l + m] = sqrtl((2 * l + 1) / (4 * PI_L)) * A * R;
        }
}

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on the Legendre recurrence)
inline void gauss_legendre_ld(int n, std::vector<long double> &x, std::vector<long double> &w)
{
    const long double PI_L = 3.141592653589793238462643383279502884L;
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        long double t = cosl(PI_L * (i + 0.75L) / (n + 0.5L)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = t;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1);
            long double dt = p1 / dp;
            t -= dt;
            if (fabsl(dt) < 1e-20L) break;
        }
        x[i] = t;
        w[i] = 2 / ((1 - t * t) * dp * dp);
    }
}

// table[(l * (ltmax+1) + lt)][ (m+l) * (2lt+1) + (mt+lt) ] -> entries
struct GauntTable {
    int lmax = 0, ltmax = 0;
    std::vector<std::vector<std::vector<GauntEntry>>> t;
    const std::vector<GauntEntry> &at(int l, int lt, int m, int mt) const
    {
        return t[l * (ltmax + 1) + lt][(m + l) * (2 * lt + 1) + (mt + lt)];
    }
};

inline GauntTable build_gaunt_table(int lmax, int ltmax)
{
    const long double PI_L = 3.141592653589793238462643383279502884L;
    int Lmax = lmax + ltmax;
    int nt = Lmax + 2, np = 2 * Lmax + 4;
    std::vector<long double> ct, wt;
    gauss_legendre_ld(nt, ct, wt);
    int ny = (Lmax + 1) * (Lmax + 1);
    std::vector<long double> Y((size_t)nt * np * ny), W((size_t)nt * np);
    for (int i = 0; i < nt; ++i)
        for (int j = 0; j < np; ++j) {
            long double ph = 2 * PI_L * j / np, st = sqrtl(1 - ct[i] * ct[i]);
            real_sph_ld(Lmax, st * cosl(ph), st * sinl(ph), ct[i], &Y[((size_t)i * np + j) * ny]);
            W[(size_t)i * np + j] = wt[i] * 2 * PI_L / np;
        }
    GauntTable G;
    G.lmax = lmax;
    G.ltmax = ltmax;
    G.t.resize((size_t)(lmax + 1) * (ltmax + 1));
    for (int l = 0; l <= lmax; ++l)
        for (int lt = 0; lt <= ltmax; ++lt) {
            auto &blk = G.t[l * (ltmax + 1) + lt];
            blk.resize((size_t)(2 * l + 1) * (2 * lt + 1));
            for (int m = -l; m <= l; ++m)
                for (int mt = -lt; mt <= lt; ++mt)
                    for (int L = (l > lt ? l - lt : lt - l); L <= l + lt; L += 2)
                        for (int M = -L; M <= L; ++M) {
                            long double s = 0;
                            for (size_t q = 0; q < (size_t)nt * np; ++q) {
                                const long double *y = &Y[q * ny];
                                s += W[q] * y[l * l + l + m] * y[lt * lt + lt + mt] * y[L * L + L + M];
                            }
                            if (fabsl(s) > 1e-15L)
                                blk[(m + l) * (2 * lt + 1) + (mt + lt)].push_back(GauntEntry{L, M, (double)s});
                        }
        }
    return G;
}

}  // namespace shg
