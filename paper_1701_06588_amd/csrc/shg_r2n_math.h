// shg_r2n_math.h -- contracted monopole T^(k) of (a|r_a^{2n}|b) (Sec. II.C,
// eq. T_rab2_deriv) in double-double arithmetic, host and device.
//
// Per primitive pair, with x = R^2, c = alpha + beta, rho = alpha beta / c and
// u = beta^2 / c, the sum over j of eq. T_rab2_deriv folds into one function
// e^{-rho x} Q(x) with a degree-n polynomial
//   Q(x) = sum_M binom(n, n-M) (l_a)_{n-M} alpha^{-(n-M)} (2c)^{-M} S_M(x),
//   S_M(x) = sum_j 2^j (2M+1)!!/(2j+1)!! binom(M, j) u^j x^j      (eq. sra2ms)
// (all terms positive), and its k-th R^2 derivative is
//   pi^{3/2} c^{-3/2} e^{-rho x} sum_i binom(k, i) (-rho)^{k-i} Q^(i)(x).
// The alternating sum cancels strongly when l_a and n are large and the
// exponents diffuse (a plain double evaluation loses ~3e-8 relative at n = 5), so c, 1/c,
// rho, u, 1/alpha, the coefficients of Q, its derivatives and the alternating
// sum are carried as unevaluated sums of two doubles (error-free transforms
// with fma); the common factor pi^{3/2} c^{-3/2} e^{-rho x} w_a w_b stays a
// double (it scales every term alike).
#pragma once
#include "shg_math.h"

namespace shg {

struct dd {
    double hi, lo;
};

SHG_HD SHG_INL dd dd_two_sum(double a, double b)
{
#pragma clang fp contract(off)
    const double s = a + b, bb = s - a;
    return dd{s, (a - (s - bb)) + (b - bb)};
}

SHG_HD SHG_INL dd dd_quick(double a, double b)
{
#pragma clang fp contract(off)
    const double s = a + b;
    return dd{s, b - (s - a)};
}

SHG_HD SHG_INL dd dd_add(dd x, dd y)
{
#pragma clang fp contract(off)
    dd s = dd_two_sum(x.hi, y.hi);
    const dd t = dd_two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = dd_quick(s.hi, s.lo);
    s.lo += t.lo;
    return dd_quick(s.hi, s.lo);
}

SHG_HD SHG_INL dd dd_mul(dd x, dd y)
{
#pragma clang fp contract(off)
    const double p = x.hi * y.hi;
    double e = fma(x.hi, y.hi, -p);
    e += x.hi * y.lo + x.lo * y.hi;
    return dd_quick(p, e);
}

SHG_HD SHG_INL dd dd_mul_d(dd x, double d)
{
#pragma clang fp contract(off)
    const double p = x.hi * d;
    double e = fma(x.hi, d, -p);
    e += x.lo * d;
    return dd_quick(p, e);
}

// 1 / x: double quotient plus one correction step on the dd residual
SHG_HD SHG_INL dd dd_recip(dd x)
{
#pragma clang fp contract(off)
    const double q1 = 1.0 / x.hi;
    const dd r = dd_add(dd{1.0, 0.0}, dd_mul_d(x, -q1));
    const double q2 = r.hi * q1;
    return dd_quick(q1, q2);
}

// T[k - KLO] += w_a w_b * (k-th R^2 derivative of the primitive monopole), k = KLO..KHI
template <int LA, int NR, int KLO, int KHI>
SHG_HD SHG_INL void r2n_accumulate(double al, double be, double x, double wab, dd (&T)[KHI - KLO + 1])
{
    const dd c = dd_two_sum(al, be);
    const dd ic = dd_recip(c);
    const dd rho = dd_mul_d(dd_mul_d(ic, al), be);
    const dd u = dd_mul_d(dd_mul_d(ic, be), be);
    const dd ial = dd_recip(dd{al, 0.0});
    const dd hic = dd_mul_d(ic, 0.5);
    // powers: alpha^-j, (2c)^-M, u^j
    dd pa[NR + 1], ph[NR + 1], pu[NR + 1];
    pa[0] = ph[0] = pu[0] = dd{1.0, 0.0};
#pragma unroll
    for (int j = 1; j <= NR; ++j) {
        pa[j] = dd_mul(pa[j - 1], ial);
        ph[j] = dd_mul(ph[j - 1], hic);
        pu[j] = dd_mul(pu[j - 1], u);
    }
    // coefficients of Q (exact integer constants times positive dd factors)
    dd Q[NR + 1];
#pragma unroll
    for (int j = 0; j <= NR; ++j) {
        dd acc{0.0, 0.0};
#pragma unroll
        for (int M = j; M <= NR; ++M) {
            const double k0 = cbinom(NR, NR - M) * crising(LA, NR - M) * cpow2(j) * (cdfact(2 * M + 1) / cdfact(2 * j + 1)) *
                              cbinom(M, j);
            acc = dd_add(acc, dd_mul_d(dd_mul(pa[NR - M], ph[M]), k0));
        }
        Q[j] = dd_mul(acc, pu[j]);
    }
    // Q^(i)(x), i = 0..NR, by Horner
    dd Qd[NR + 1];
#pragma unroll
    for (int i = 0; i <= NR; ++i) {
        dd acc = dd_mul_d(Q[NR], cfact(NR) / cfact(NR - i));
#pragma unroll
        for (int j = NR - 1; j >= i; --j) acc = dd_add(dd_mul_d(acc, x), dd_mul_d(Q[j], cfact(j) / cfact(j - i)));
        Qd[i] = acc;
    }
    // (-rho)^p
    dd nr[KHI + 1];
    nr[0] = dd{1.0, 0.0};
#pragma unroll
    for (int p = 1; p <= KHI; ++p) nr[p] = dd_mul(nr[p - 1], dd{-rho.hi, -rho.lo});
    const double ich = 1.0 / c.hi;
    const double base = wab * PI_1_5 * exp(-rho.hi * x) * ich * sqrt(ich);
#pragma unroll
    for (int k = KLO; k <= KHI; ++k) {
        dd acc{0.0, 0.0};
#pragma unroll
        for (int i = 0; i <= (NR < k ? NR : k); ++i) acc = dd_add(acc, dd_mul_d(dd_mul(nr[k - i], Qd[i]), cbinom(k, i)));
        T[k - KLO] = dd_add(T[k - KLO], dd_mul_d(acc, base));
    }
}

}  // namespace shg
