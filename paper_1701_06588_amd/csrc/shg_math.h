// shg_math.h -- FP64 arithmetic of the SHG integral scheme for one shell pair
// (or triple). Everything here is device code for gfx950; the functions are
// also host-callable so that the unit tests can run the same arithmetic on the
// CPU (SHG_HD expands to __host__ __device__ under hipcc and to nothing under a
// plain C++ compiler).
//
// Method: Golze et al., arXiv:1701.06588.
//   radial   (0_a|O|0_b)^(k), k-th derivative w.r.t. R_ab^2      Table S1
//   contract O^(k)_{la,lb} = sum w_alpha w_beta (0|O|0)^(k)      eq. O_rab2_deriv
//            with w_alpha = N_l c_alpha / (2 alpha)^l             eq. O_rab2, N_l
//   angular  R^{c/s}_{l,m}(X), X = R_a - R_b                       eq. regular_scaled_harmonics_recursion
//            W_{l,m,j,kappa}, Q = W_a W_b^T                         eqs. W_matrix, Q_matrix
//   assemble (a|O|b) = sum_j O^(la+lb-j) Qtilde_j                 eqs. final_r12int_ab, Q_tilde
//   deriv    eq. dev_ab with the lower-l recurrences               eqs. cartesian_dev_x/y/z
//   (a b a~) Gaunt expansion + P^(k), eq. devsra2ms radial          Sec. II.D
#pragma once

#include <stdint.h>
#include <math.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define SHG_HD __host__ __device__
#define SHG_INL __forceinline__
#else
#define SHG_HD
#define SHG_INL inline __attribute__((always_inline))
#endif

namespace shg {

// ---------------------------------------------------------------------------
// compile-time constants
// ---------------------------------------------------------------------------
constexpr double cfact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }
constexpr double cdfact(int n) { double f = 1; for (int i = n; i > 1; i -= 2) f *= i; return f; }  // n!!, (-1)!! = 1
constexpr double csqrt(double x)
{
    if (x <= 0) return 0;
    double g = x > 1 ? x : 1;
    for (int i = 0; i < 200; ++i) g = 0.5 * (g + x / g);
    return g;
}
constexpr double cpow2(int n) { double f = 1; for (int i = 0; i < n; ++i) f *= 2; return f; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cabs(int a) { return a < 0 ? -a : a; }

// A_{l,m} = (-1)^m sqrt((2 - delta_m0)(l+|m|)!(l-|m|)!)   (eq. A; A_{l,-1} = A_{l,1})
constexpr double A_lm(int l, int m)
{
    int mu = cabs(m);
    double s = csqrt((mu == 0 ? 1.0 : 2.0) * cfact(l + mu) * cfact(l - mu));
    return (mu & 1) ? -s : s;
}
// B_{j,kappa} = 1 / ((2 - delta_kappa0)(j+kappa)!(j-kappa)!)   (eq. B)
constexpr double B_jk(int j, int k) { return 1.0 / ((k == 0 ? 1.0 : 2.0) * cfact(j + k) * cfact(j - k)); }

constexpr double PI = 3.141592653589793238462643383279502884;
constexpr double PI_1_5 = 5.568327996831707845284817982118835702;    // pi^(3/2)
constexpr double PI_2_5 = 17.493418327624862846262821679872926940;   // pi^(5/2)
constexpr double PI_3 = 31.006276680299820175476315067101395202;     // pi^3

// ---------------------------------------------------------------------------
// Boys function F_n(T) = int_0^1 exp(-T t^2) t^(2n) dt  (supplement eq. 3)
// T < BOYS_TMAX: 8-term Taylor expansion of F_nhi about the nearest grid point
//   (spacing 1/16, |dT| <= 1/32, dF_n/dT = -F_{n+1}, supplement eq. 4), then
//   the downward recurrence F_n = (2T F_{n+1} + e^-T) / (2n+1);
// T >= BOYS_TMAX: F_0 = sqrt(pi/T)/2 (erf(sqrt T) = 1 to double precision for
//   T >= 36) and the upward recurrence F_{n+1} = ((2n+1) F_n - e^-T) / (2T),
//   stable there because (2n+1)/(2T) < 1.
// ---------------------------------------------------------------------------
constexpr int BOYS_NTAB = 17;          // tabulated orders 0..16
constexpr int BOYS_STRIDE = 17;
constexpr int BOYS_PER_UNIT = 16;      // grid points per unit of T
constexpr double BOYS_TMAX = 36.0;
constexpr int BOYS_NPTS = 36 * 16 + 2;
constexpr int BOYS_TAYLOR = 8;

template <int NLO, int NHI>
SHG_HD SHG_INL void boys(double T, const double *__restrict__ tab, double (&F)[NHI - NLO + 1])
{
    // no implicit multiply-add contraction: every kernel inlining this rounds alike
#pragma clang fp contract(off)
    static_assert(NHI + BOYS_TAYLOR - 1 < BOYS_NTAB, "Boys table too short");
    double e = exp(-T);
    if (T < BOYS_TMAX) {
        int i = (int)(T * BOYS_PER_UNIT + 0.5);
        double d = T - i * (1.0 / BOYS_PER_UNIT);
        const double *row = tab + (size_t)i * BOYS_STRIDE + NHI;
        double acc = row[BOYS_TAYLOR - 1];
#pragma unroll
        for (int k = BOYS_TAYLOR - 2; k >= 0; --k) acc = fma(acc, -d * (1.0 / (k + 1)), row[k]);
        F[NHI - NLO] = acc;
        double tt = 2 * T;
#pragma unroll
        for (int n = NHI - 1; n >= NLO; --n) F[n - NLO] = fma(tt, F[n + 1 - NLO], e) * (1.0 / (2 * n + 1));
    } else {
        double inv2t = 0.5 / T;
        double f = 0.5 * sqrt(PI / T);
        if (NLO == 0) F[0] = f;
#pragma unroll
        for (int n = 0; n < NHI; ++n) {
            f = ((2 * n + 1) * f - e) * inv2t;
            if (n + 1 >= NLO) F[n + 1 - NLO] = f;
        }
    }
}

// ---------------------------------------------------------------------------
// s-s integrals and their R^2 derivatives, Table S1 (k = KLO..KHI)
// ---------------------------------------------------------------------------
enum { OP_OVERLAP = 0, OP_COULOMB = 1, OP_ERF = 2, OP_ERFC = 3, OP_GAUSS = 4 };

template <int OP, int KLO, int KHI>
SHG_HD SHG_INL void radial(double a, double b, double R2, double omega, const double *__restrict__ tab,
                           double (&g)[KHI - KLO + 1])
{
    // no implicit multiply-add contraction: every kernel inlining this rounds alike
#pragma clang fp contract(off)
    constexpr int NK = KHI - KLO + 1;
    double p = a + b, ip = 1.0 / p, rho = a * b * ip, T = rho * R2;
    if (OP == OP_OVERLAP || OP == OP_GAUSS) {
        double pre, fac;
        if (OP == OP_OVERLAP) {
            pre = PI_1_5 * ip * sqrt(ip) * exp(-T);
            fac = -rho;
        } else {
            double q = rho + omega, iq = 1.0 / q, u = ip * iq;
            pre = PI_3 * u * sqrt(u) * exp(-omega * T * iq);
            fac = -omega * rho * iq;
        }
        double f = pre;
#pragma unroll
        for (int k = 0; k < KLO; ++k) f *= fac;
#pragma unroll
        for (int k = 0; k < NK; ++k) { g[k] = f; f *= fac; }
    } else {
        double pre = 2.0 * PI_2_5 / (a * b * sqrt(p));
        double Fc[NK];
        if (OP == OP_COULOMB || OP == OP_ERFC) {
            boys<KLO, KHI>(T, tab, Fc);
            double f = pre;
#pragma unroll
            for (int k = 0; k < KLO; ++k) f *= -rho;
#pragma unroll
            for (int k = 0; k < NK; ++k) { g[k] = f * Fc[k]; f *= -rho; }
        }
        if (OP == OP_ERF || OP == OP_ERFC) {
            double w2 = omega * omega, s = w2 / (w2 + rho);
            double Fe[NK];
            boys<KLO, KHI>(T * s, tab, Fe);
            double fac = -rho * s, f = pre * sqrt(s);
#pragma unroll
            for (int k = 0; k < KLO; ++k) f *= fac;
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                double v = f * Fe[k];
                g[k] = (OP == OP_ERF) ? v : g[k] - v;
                f *= fac;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// regular scaled solid harmonics R^{c/s}_{l,m}(X), 0 <= m <= l <= L
// (eq. regular_scaled_harmonics_recursion; the three-term step is used for
// 0 <= m <= l with R_{l-1,m} = 0 when m > l-1)
// ---------------------------------------------------------------------------
constexpr int ridx(int l, int m) { return l * (l + 1) / 2 + m; }

template <int L>
struct RTab {
    double c[(L + 1) * (L + 2) / 2];
    double s[(L + 1) * (L + 2) / 2];
};

template <int L>
SHG_HD SHG_INL void solid_R(double x, double y, double z, RTab<L> &R)
{
    double r2 = x * x + y * y + z * z;
    R.c[0] = 1.0;
    R.s[0] = 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        double inv = 1.0 / (2 * l + 2);
        R.c[ridx(l + 1, l + 1)] = -(x * R.c[ridx(l, l)] - y * R.s[ridx(l, l)]) * inv;
        R.s[ridx(l + 1, l + 1)] = -(y * R.c[ridx(l, l)] + x * R.s[ridx(l, l)]) * inv;
#pragma unroll
        for (int m = 0; m <= l; ++m) {
            double den = 1.0 / ((l + m + 1) * (l - m + 1));
            double zc = (2 * l + 1) * z * R.c[ridx(l, m)];
            if (m <= l - 1) zc -= r2 * R.c[ridx(l - 1, m)];
            R.c[ridx(l + 1, m)] = zc * den;
            if (m == 0) {
                R.s[ridx(l + 1, 0)] = 0.0;
            } else {
                double zs = (2 * l + 1) * z * R.s[ridx(l, m)];
                if (m <= l - 1) zs -= r2 * R.s[ridx(l - 1, m)];
                R.s[ridx(l + 1, m)] = zs * den;
            }
        }
    }
}

// presence of R^{c/s}_{l,m} (signed m): zero outside |m| <= l; R^s_{l,0} = 0
constexpr bool rc_nz(int l, int m) { return l >= 0 && cabs(m) <= l; }
constexpr bool rs_nz(int l, int m) { return l >= 0 && cabs(m) <= l && m != 0; }

// R^c_{l,-m} = (-1)^m R^c_{l,m},  R^s_{l,-m} = -(-1)^m R^s_{l,m}
template <int L>
SHG_HD SHG_INL double Rc(const RTab<L> &R, int l, int m)
{
    int mu = cabs(m);
    double v = R.c[ridx(l, mu)];
    return (m < 0 && (mu & 1)) ? -v : v;
}
template <int L>
SHG_HD SHG_INL double Rs(const RTab<L> &R, int l, int m)
{
    int mu = cabs(m);
    double v = R.s[ridx(l, mu)];
    return (m < 0 && !(mu & 1)) ? -v : v;
}

// ---------------------------------------------------------------------------
// Real translation matrix W_{l,m,j,kappa} (eq. W_matrix), evaluated with the
// solid harmonics at X = R_a - R_b: Q(R_ab) = W(-R_ab) W^T(-R_ab) (eq. Q_matrix)
// and W(R_ab) takes its harmonics at -R_ab, so the two negations cancel.
// Row t (0 = c, 1 = s), column s (0 = c, 1 = s): W[c][c], W[c][s], W[s][c], W[s][s].
// Absent terms are dropped at compile time (all indices are constants once the
// caller's loops are unrolled).
// ---------------------------------------------------------------------------
constexpr bool w_nz(int l, int m, int j, int k)
{
    return l >= 0 && j <= l && (rc_nz(l - j, m - k) || rc_nz(l - j, m + k));
}

// sum of +-R terms with compile-time presence: s1*R(l,m1) + s2*R(l,m2)
template <int L>
SHG_HD SHG_INL double rc_comb(const RTab<L> &R, int l, int m1, double s1, int m2, double s2)
{
    bool p1 = rc_nz(l, m1), p2 = rc_nz(l, m2);
    if (p1 && p2) return s2 > 0 ? s1 * Rc(R, l, m1) + Rc(R, l, m2) : s1 * Rc(R, l, m1) - Rc(R, l, m2);
    if (p1) return s1 * Rc(R, l, m1);
    if (p2) return s2 * Rc(R, l, m2);
    return 0.0;
}
template <int L>
SHG_HD SHG_INL double rs_comb(const RTab<L> &R, int l, int m1, double s1, int m2, double s2)
{
    bool p1 = rs_nz(l, m1), p2 = rs_nz(l, m2);
    if (p1 && p2) return s2 > 0 ? s1 * Rs(R, l, m1) + Rs(R, l, m2) : s1 * Rs(R, l, m1) - Rs(R, l, m2);
    if (p1) return s1 * Rs(R, l, m1);
    if (p2) return s2 * Rs(R, l, m2);
    return 0.0;
}
// is entry (t, s) of W_{l,m,j,k} structurally non-zero?
constexpr bool wentry_nz(int l, int m, int j, int k, int t, int s)
{
    // column s = 1 (cs, ss) vanishes for kappa = 0; row t = 1 at m = 0 vanishes
    if (s == 1 && k == 0) return false;
    if (t == 1 && m == 0) return false;
    int lj = l - j;
    bool use_c = (t == s);   // cc and ss use R^c, cs and sc use R^s
    return use_c ? (rc_nz(lj, m - k) || rc_nz(lj, m + k)) : (rs_nz(lj, m - k) || rs_nz(lj, m + k));
}

template <int L>
SHG_HD SHG_INL double wentry(const RTab<L> &R, int l, int m, int j, int k, int t, int s)
{
    int lj = l - j;
    double sg = (k & 1) ? -1.0 : 1.0;
    double half = (k == 0) ? 0.5 : 1.0;
    if (t == 0 && s == 0) return half * rc_comb(R, lj, m - k, 1.0, m + k, sg);     // W^cc
    if (t == 0 && s == 1) return rs_comb(R, lj, m - k, -1.0, m + k, sg);           // W^cs
    if (t == 1 && s == 0) return half * rs_comb(R, lj, m - k, 1.0, m + k, sg);     // W^sc
    return rc_comb(R, lj, m - k, 1.0, m + k, -sg);                                 // W^ss
}

// ---------------------------------------------------------------------------
// compile-time loop
// ---------------------------------------------------------------------------
template <int V>
struct IC {
    static constexpr int value = V;
};
template <int B, int E, class F>
SHG_HD SHG_INL void static_for(F &&f)
{
    if constexpr (B < E) {
        f(IC<B>{});
        static_for<B + 1, E>(f);
    }
}

// ---------------------------------------------------------------------------
// Qhat^{ta,tb}_{la,ma,lb,mb,j} = (-1)^lb 2^(la+lb-j) (2j-1)!! sum_kappa B_{j,kappa}
//                                 Q^{ta,tb}_{la,ma,lb,mb,j,kappa}
// i.e. Qtilde of eq. Q_tilde without the factor A_{la,ma} A_{lb,mb}. ma, mb are
// signed (the derivative recurrences reach m = -1), t = 0 cosine, 1 sine.
// ---------------------------------------------------------------------------
constexpr bool qhat_nz(int la, int ma, int ta, int lb, int mb, int tb, int j)
{
    if (la < 0 || lb < 0 || j < 0 || j > cmin(la, lb)) return false;
    if (cabs(ma) > la || cabs(mb) > lb) return false;
    if ((ta == 1 && ma == 0) || (tb == 1 && mb == 0)) return false;
    for (int k = 0; k <= j; ++k)
        for (int s = 0; s < 2; ++s)
            if (wentry_nz(la, ma, j, k, ta, s) && wentry_nz(lb, mb, j, k, tb, s)) return true;
    return false;
}

template <int LA, int MA, int TA, int LB, int MB, int TB, int J, int L>
SHG_HD SHG_INL double qhat(const RTab<L> &R)
{
    constexpr double pref = ((LB & 1) ? -1.0 : 1.0) * cpow2(LA + LB - J) * cdfact(2 * J - 1);
    double acc = 0.0;
    bool first = true;
    static_for<0, J + 1>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        static_for<0, 2>([&](auto SS) {
            constexpr int S = decltype(SS)::value;
            if constexpr (wentry_nz(LA, MA, J, K, TA, S) && wentry_nz(LB, MB, J, K, TB, S)) {
                constexpr double c = pref * B_jk(J, K);
                double t = c * wentry(R, LA, MA, J, K, TA, S) * wentry(R, LB, MB, J, K, TB, S);
                acc = first ? t : acc + t;
                first = false;
            }
        });
    });
    return acc;
}

// adds sgn * Qhat(...) to acc when the term is structurally non-zero
template <int LA, int MA, int TA, int LB, int MB, int TB, int J, int L>
SHG_HD SHG_INL void qhat_acc(const RTab<L> &R, double sgn, double &acc)
{
    if constexpr (qhat_nz(LA, MA, TA, LB, MB, TB, J)) acc = fma(sgn, qhat<LA, MA, TA, LB, MB, TB, J>(R), acc);
}

// ---------------------------------------------------------------------------
// Shell preparation: N_l (eq. N_l) and the folded weights
// w_alpha = N_l c_alpha / (2 alpha)^l (eq. O_rab2).
// ---------------------------------------------------------------------------
// N_l = K_l [ sum pi^(1/2) (2l+2)! c c' / (2^(2l+3) (l+1)! (a+a')^(l+3/2)) ]^(-1/2):
// one term of the sum without the constant factor, and N_l from the summed terms
SHG_HD SHG_INL double shell_norm_term(int l, double ea, double eb, double ca, double cb)
{
    double ab = ea + eb;
    double pw = ab;
    for (int q = 0; q < l; ++q) pw *= ab;
    return ca * cb / (pw * sqrt(ab));
}
SHG_HD SHG_INL double shell_norm_from_sum(int l, double s)
{
    double f2l2 = 1, fl1 = 1, p2 = 1;
    for (int i = 2; i <= 2 * l + 2; ++i) f2l2 *= i;
    for (int i = 2; i <= l + 1; ++i) fl1 *= i;
    for (int i = 0; i < 2 * l + 3; ++i) p2 *= 2;
    s *= sqrt(PI) * f2l2 / (p2 * fl1);
    double Kl = sqrt((2 * l + 1) / (4 * PI));
    return Kl / sqrt(s);
}
SHG_HD SHG_INL double shell_norm(int l, int K, const double *e, const double *c)
{
    double s = 0;
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) s += shell_norm_term(l, e[i], e[j], c[i], c[j]);
    return shell_norm_from_sum(l, s);
}

// ---------------------------------------------------------------------------
// Contraction of the radial terms for one shell pair (eq. O_rab2_deriv):
// O^(k) = sum_{alpha,beta} w_alpha w_beta (0|O|0)^(k), k = KLO..KHI with
// KLO = max(la,lb), KHI = la+lb (+1 with derivatives).
// ---------------------------------------------------------------------------
template <int LA, int LB, bool D>
struct PairK {
    static constexpr int KLO = cmax(LA, LB), KHI = LA + LB + (D ? 1 : 0), NK = KHI - KLO + 1;
};

template <int LA, int LB, int OP, bool D>
SHG_HD SHG_INL void contract_pair(const double *__restrict__ ea, const double *__restrict__ wa, int ka,
                                  const double *__restrict__ eb, const double *__restrict__ wb, int kb,
                                  double R2, double omega, const double *__restrict__ tab,
                                  double (&O)[PairK<LA, LB, D>::NK])
{
    using PK = PairK<LA, LB, D>;
#pragma unroll
    for (int k = 0; k < PK::NK; ++k) O[k] = 0.0;
    for (int i = 0; i < ka; ++i) {
        double a = ea[i], w1 = wa[i];
        for (int j = 0; j < kb; ++j) {
            double g[PK::NK];
            radial<OP, PK::KLO, PK::KHI>(a, eb[j], R2, omega, tab, g);
            double ww = w1 * wb[j];
#pragma unroll
            for (int k = 0; k < PK::NK; ++k) O[k] = fma(ww, g[k], O[k]);
        }
    }
}

// The operator-independent part of one element: per j the Qhat sum of the
// value (q) and the three derivative source sums (tx, ty, tz), and the
// operator-dependent part that combines them with the contracted radial terms.
// pair_elem = elem_terms + elem_apply, in the same floating-point order.
template <int LA, int LB, bool D>
struct ElemTerms {
    static constexpr int JM = cmin(LA, LB);
    double q[JM + 1], tx[JM + 1], ty[JM + 1], tz[JM + 1];
};

template <int LA, int LB, int IA, int IB, bool D, int L>
SHG_HD SHG_INL void elem_terms(const RTab<L> &R, ElemTerms<LA, LB, D> &T)
{
    constexpr int JM = cmin(LA, LB);
    constexpr int MA = IA - LA, MUA = cabs(MA), TA = MA < 0 ? 1 : 0;
    constexpr int MB = IB - LB, MUB = cabs(MB), TB = MB < 0 ? 1 : 0;
    constexpr double SA = TA ? -1.0 : 1.0, SB = TB ? -1.0 : 1.0;
    static_for<0, JM + 1>([&](auto JJ) {
        constexpr int J = decltype(JJ)::value;
        if constexpr (qhat_nz(LA, MUA, TA, LB, MUB, TB, J)) T.q[J] = qhat<LA, MUA, TA, LB, MUB, TB, J>(R);
        if constexpr (D) {
            double tx = 0.0, ty = 0.0, tz = 0.0;
            qhat_acc<LA - 1, MUA + 1, TA, LB, MUB, TB, J>(R, 1.0, tx);
            qhat_acc<LA - 1, MUA - 1, TA, LB, MUB, TB, J>(R, -1.0, tx);
            qhat_acc<LA, MUA, TA, LB - 1, MUB + 1, TB, J>(R, -1.0, tx);
            qhat_acc<LA, MUA, TA, LB - 1, MUB - 1, TB, J>(R, 1.0, tx);
            qhat_acc<LA - 1, MUA + 1, 1 - TA, LB, MUB, TB, J>(R, SA, ty);
            qhat_acc<LA - 1, MUA - 1, 1 - TA, LB, MUB, TB, J>(R, SA, ty);
            qhat_acc<LA, MUA, TA, LB - 1, MUB + 1, 1 - TB, J>(R, -SB, ty);
            qhat_acc<LA, MUA, TA, LB - 1, MUB - 1, 1 - TB, J>(R, -SB, ty);
            qhat_acc<LA - 1, MUA, TA, LB, MUB, TB, J>(R, 2.0, tz);
            qhat_acc<LA, MUA, TA, LB - 1, MUB, TB, J>(R, -2.0, tz);
            T.tx[J] = tx;
            T.ty[J] = ty;
            T.tz[J] = tz;
        }
    });
}

template <int LA, int LB, int IA, int IB, bool D>
SHG_HD SHG_INL void elem_apply(const ElemTerms<LA, LB, D> &T, const double *O, const double X[3], double *res)
{
    using PK = PairK<LA, LB, D>;
    constexpr int JM = cmin(LA, LB);
    constexpr int MA = IA - LA, MUA = cabs(MA), TA = MA < 0 ? 1 : 0;
    constexpr int MB = IB - LB, MUB = cabs(MB), TB = MB < 0 ? 1 : 0;
    constexpr double AA = A_lm(LA, MUA) * A_lm(LB, MUB);
    double v = 0.0, v1 = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
    static_for<0, JM + 1>([&](auto JJ) {
        constexpr int J = decltype(JJ)::value;
        constexpr int K0 = LA + LB - J - PK::KLO;
        if constexpr (qhat_nz(LA, MUA, TA, LB, MUB, TB, J)) {
            v = fma(O[K0], T.q[J], v);
            if constexpr (D) v1 = fma(O[K0 + 1], T.q[J], v1);
        }
        if constexpr (D) {
            dx = fma(O[K0], T.tx[J], dx);
            dy = fma(O[K0], T.ty[J], dy);
            dz = fma(O[K0], T.tz[J], dz);
        }
    });
    res[0] = AA * v;
    if constexpr (D) {
        double t1 = 2.0 * v1;
        res[1] = AA * fma(t1, X[0], dx);
        res[2] = AA * fma(t1, X[1], dy);
        res[3] = AA * fma(t1, X[2], dz);
    }
}

// ---------------------------------------------------------------------------
// One block element (m_a = IA - LA, m_b = IB - LB) of (a|O|b) and, with D, of
// d/dR_a:
//   value  = A_a A_b sum_j O^(la+lb-j) Qhat_j                    eq. final_r12int_ab
//   d/dR_i = A_a A_b [ 2 X_i sum_j O^(la+lb-j+1) Qhat_j
//                      + sum_j O^(la+lb-j) dQhat_j/dR_i ]          eq. dev_ab
// with dQtilde/dR_i from (l-1) terms, eqs. cartesian_dev_x/y/z (with the
// factor A_a A_b taken out, the ratios of A's there reduce to 1).
// res[0] = value; with D res[1..3] = d/dR_a,{x,y,z}.
// ---------------------------------------------------------------------------
template <int LA, int LB, int IA, int IB, bool D, int L>
SHG_HD SHG_INL void pair_elem(const RTab<L> &R, const double *O, const double X[3], double *res)
{
    ElemTerms<LA, LB, D> T;
    elem_terms<LA, LB, IA, IB, D>(R, T);
    elem_apply<LA, LB, IA, IB, D>(T, O, X, res);
}

// whole block (host-side use): every element
template <int LA, int LB, bool D>
SHG_HD SHG_INL void pair_block_from_O(const double *O, const double X[3], double *__restrict__ out,
                                      double *__restrict__ dout)
{
    constexpr int NB = 2 * LB + 1, SZ = (2 * LA + 1) * NB;
    RTab<cmax(LA, LB)> R;
    solid_R<cmax(LA, LB)>(X[0], X[1], X[2], R);
    static_for<0, SZ>([&](auto EE) {
        constexpr int E = decltype(EE)::value;
        double res[D ? 4 : 1];
        pair_elem<LA, LB, E / NB, E % NB, D>(R, O, X, res);
        out[E] = res[0];
        if constexpr (D) {
            dout[E] = res[1];
            dout[SZ + E] = res[2];
            dout[2 * SZ + E] = res[3];
        }
    });
}

// ---------------------------------------------------------------------------
// Three-index overlap (a b a~), Sec. II.D. For each L_a in |la-lt|..la+lt
// (step 2) the block (a b a~) is a sum over the Gaunt expansion of two-center
// blocks (L_a, M_a | lb, mb) whose contracted monopole is P^(k)_{La} (eq. Pa_aba)
// instead of O^(k); the primitive radial terms are (0_a'|r_a^{2m}|0_b)^(k)
// (eqs. sra2ms, I_jab, devsra2ms) with alpha' = alpha + alpha~.
// ---------------------------------------------------------------------------
constexpr double cbinom(int n, int k) { return (k < 0 || k > n) ? 0.0 : cfact(n) / (cfact(k) * cfact(n - k)); }
// rising factorial (L)_j = L (L+1) ... (L+j-1) = (L+j-1)!/(L-1)!, equal to 1 for j = 0
// and to 0 for L = 0, j >= 1
constexpr double crising(int L, int j) { double f = 1; for (int i = 0; i < j; ++i) f *= (L + i); return f; }

template <int LA, int LT, int LB, bool D>
struct AabK {
    static constexpr int LAMIN = cabs(LA - LT), LAMAX = LA + LT, NLA = (LAMAX - LAMIN) / 2 + 1;
    static constexpr int PMAX = cmin(LA, LT);
    static constexpr int KMIN = cmax(LAMIN, LB), KT = LAMAX + LB + (D ? 1 : 0), NKT = KT - KMIN + 1;
    static constexpr int PSTRIDE = 32;   // per triple in the P buffer: iLa * 8 + (k - max(La, lb))
};

// (0_a'|r_a^{2m}|0_b)^(k) for m = 0..PMAX and k = KMIN..KT:
//   pi^(3/2) e^{-rho R^2} / (2^m c^(m+3/2)) sum_i binom(k,i) (-rho)^(k-i) sum_{j>=i} d^i I_j / d(R^2)^i
//   I_j = 2^j (2m+1)!! binom(m,j) / (2j+1)!! * (beta^2/c)^j R^(2j),  c = alpha'+beta, rho = alpha' beta / c
template <int PMAX, int KMIN, int KT>
SHG_HD SHG_INL void sra2m(double ap, double b, double R2, double (&t)[PMAX + 1][KT - KMIN + 1])
{
    const double c = ap + b, ic = 1.0 / c, rho = ap * b * ic, u = b * b * ic;
    double nr[KT + 1];
    nr[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= KT; ++k) nr[k] = nr[k - 1] * (-rho);
    double base = PI_1_5 * exp(-rho * R2) * ic * sqrt(ic);
    static_for<0, PMAX + 1>([&](auto MM) {
        constexpr int M = decltype(MM)::value;
        double C[M + 1];
        double uj = 1.0;
#pragma unroll
        for (int j = 0; j <= M; ++j) {
            C[j] = (cpow2(j) * cdfact(2 * M + 1) * cbinom(M, j) / cdfact(2 * j + 1)) * uj;
            uj *= u;
        }
        double S[M + 1];   // S^(i)(R^2) = sum_{j>=i} C_j j!/(j-i)! (R^2)^(j-i)
#pragma unroll
        for (int i = 0; i <= M; ++i) {
            double acc = C[M] * (cfact(M) / cfact(M - i));
#pragma unroll
            for (int j = M - 1; j >= i; --j) acc = fma(acc, R2, C[j] * (cfact(j) / cfact(j - i)));
            S[i] = acc;
        }
#pragma unroll
        for (int k = KMIN; k <= KT; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i <= (M < k ? M : k); ++i) acc = fma(cbinom(k, i) * nr[k - i], S[i], acc);
            t[M][k - KMIN] = base * acc;
        }
        base *= 0.5 * ic;
    });
}

// P[iLa][k - max(La, lb)] += contribution of one primitive triple (eq. Pa_aba):
//   lambda K_La N_la N_lb N_lt c_alpha c_beta c_alpha~ / ((2 alpha')^La (2 beta)^lb)
//   * sum_j binom(p,j) (La)_j / alpha'^j (0_a'|r_a^{2(p-j)}|0_b)^(k),  p = (la+lt-La)/2
// `wabt` = N_la c_alpha * N_lt c_alpha~ * N_lb c_beta / (2 beta)^lb.
template <int LA, int LT, int LB, bool D>
SHG_HD SHG_INL void aab_accumulate(double ap, double b, double R2, double wabt,
                                   double (&P)[AabK<LA, LT, LB, D>::NLA][8])
{
    using AK = AabK<LA, LT, LB, D>;
    double t[AK::PMAX + 1][AK::NKT];
    sra2m<AK::PMAX, AK::KMIN, AK::KT>(ap, b, R2, t);
    const double iap = 1.0 / ap, i2ap = 0.5 * iap;
    static_for<0, AK::NLA>([&](auto II) {
        constexpr int I = decltype(II)::value;
        constexpr int LAc = AK::LAMIN + 2 * I, p = (LA + LT - LAc) / 2;
        constexpr double lamK = csqrt(4.0 * PI * (2 * LAc + 1) / ((2.0 * LA + 1) * (2 * LT + 1)));
        constexpr int KLO = cmax(LAc, LB), KHI = LAc + LB + (D ? 1 : 0);
        double coef = wabt * lamK;
#pragma unroll
        for (int q = 0; q < LAc; ++q) coef *= i2ap;
#pragma unroll
        for (int k = KLO; k <= KHI; ++k) {
            double sacc = 0.0, apj = 1.0;
#pragma unroll
            for (int j = 0; j <= p; ++j) {
                sacc = fma(cbinom(p, j) * crising(LAc, j) * apj, t[p - j][k - AK::KMIN], sacc);
                apj *= iap;
            }
            P[I][k - KLO] = fma(coef, sacc, P[I][k - KLO]);
        }
    });
}

}  // namespace shg
