// shg_bound.h -- conservative analytic bound on max|block| of a shell pair
// (values, and with derivatives the d/dR_a elements too), used to skip
// negligible pairs. With X = R_a - R_b, R = |X| and eq. final_r12int_ab,
//   |block| <= sum_j |O^(la+lb-j)| Cq(la, lb, j) R^(la+lb-2j)
// where Cq bounds A_a A_b |Qhat_j| / R^(la+lb-2j) over all (m_a, m_b) using
// |R^{c/s}_{l,m}(X)| <= R^l / sqrt((l-|m|)!(l+|m|)!) (|C_lm(X)| <= R^l), and
// |O^(k)| <= sum |w_a w_b| |(0|O|0)^(k)| is bounded per operator (Table S1)
// with |w| sums over the primitives (per-shell statistics, k_shell_stats):
//   Coulomb  F_k(T) <= 1/(2k+1) and F_k(T) <= (2k-1)!!/2^(k+1) sqrt(pi/T^(2k+1)),
//            alpha + beta >= 2 sqrt(alpha beta):
//            near = 2 pi^(5/2) 2^-(k+1/2) / (2k+1) * Sc_a(k) Sc_b(k),  Sc(k) = sum|w| a^(k/2-5/4)
//            far  = 2 pi^3 (2k-1)!!/2^(k+1) * Sf_a Sf_b / R^(2k+1),   Sf    = sum|w| a^(-3/2)
//   erf      <= the Coulomb bound; erfc <= twice the Coulomb bound
//   overlap  pi^(3/2) 2^(-3/2-k) So_a(k) So_b(k) e^{-rho_min R^2},  So(k) = sum|w| a^(k/2-3/4)
//   Gaussian pi^3 omega^(-3/2) 2^(-3/2-k) So_a(k) So_b(k) e^{-omega rho_min R^2/(rho_min+omega)}
// (rho_min from the most diffuse exponents: rho and the exponent are increasing
// in both). For derivatives, d/dX_i [O^(k)(R^2) P_j(X)] = 2 X_i O^(k+1) P_j +
// O^(k) d_i P_j with P_j homogeneous of degree pw = la+lb-2j; on the unit sphere
// Bernstein's inequality bounds the tangential gradient by pw max|P_j| and the
// radial part is pw P_j / R, so |d_i P_j| <= sqrt(2) pw Cq R^(pw-1).
#pragma once
#include "shg_math.h"

namespace shg {

constexpr int STAT = 16;        // doubles per shell in the statistics table (one 128-byte line)
constexpr int KB = 10;          // k = 0..9 moments
constexpr int BK = 11;          // k = 0..10 in the per-k constants

// constants of the bound (host-built, device-resident)
struct BoundTab {
    double cq[5][5][5];   // Cq(la, lb, j)
    double co[BK];        // overlap:  pi^(3/2) 2^(-3/2-k)
    double cn[BK];        // Coulomb near: 2 pi^(5/2) 2^-(k+1/2) / (2k+1)
    double cf[BK];        // Coulomb far:  2 pi^3 (2k-1)!! 2^-(k+1)
};

// bound of a shell pair with angular momenta (la, lb), per-shell statistics sa
// and sb (alpha_min, alpha_max, sum|w|, Sf, S[KB] with S = So for the overlap and
// the Gaussian operator, Sc for the Coulomb-like ones) and squared distance
// R2; returns the bound on max|block| and, with deriv, on the d/dR_a elements
// too (their maximum); *vbound receives the value bound alone, *R_out and
// *rmin_out R and the smallest reduced exponent
__device__ __forceinline__ double shell_pair_bound(int la, int lb, const double *__restrict__ sa,
                                                   const double *__restrict__ sb, double R2, int op, double omega,
                                                   int deriv, const BoundTab *__restrict__ bt, double *vbound,
                                                   double *R_out, double *rmin_out)
{
    const double R = sqrt(R2);
    const double rmin = sa[0] * sb[0] / (sa[0] + sb[0]);
    const int jm = la < lb ? la : lb, klo = la > lb ? la : lb;
    const bool gl = op == OP_OVERLAP || op == OP_GAUSS;
    // factors of the bound on |O^(k)| (k-th R^2-derivative of the contracted radial term):
    //   overlap/Gaussian  co[k] So_a[k] So_b[k] e
    //   Coulomb-like      min(cn[k] Sc_a[k] Sc_b[k], cf[k] Sf_a Sf_b R^-(2k+1)) fac
    double e = 0.0, sf = 0.0, iR2 = 0.0, rp = 0.0;
    const double fac = op == OP_ERFC ? 2.0 : 1.0;
    if (gl) {
        if (op == OP_OVERLAP) {
            e = exp(-rmin * R2);
        } else {
            const double iw = 1.0 / omega;
            e = PI * PI * PI * iw * sqrt(iw) * exp(-omega * rmin * R2 / (rmin + omega)) / PI_1_5;
        }
    } else {
        sf = sa[3] * sb[3];
        const double iR = R > 0 ? 1.0 / R : 0.0;
        iR2 = iR * iR;
        rp = iR;   // R^-(2k+1) at k = klo
        for (int k = 0; k < klo; ++k) rp *= iR2;
    }
    // ob(k) for increasing k; rp advances with it
    auto ob_next = [&](int k) {
        double v;
        if (gl) {
            v = bt->co[k] * sa[4 + k] * sb[4 + k] * e;
        } else {
            const double nearb = bt->cn[k] * sa[4 + k] * sb[4 + k];
            const double farb = R > 0 ? bt->cf[k] * sf * rp : 1e300;
            v = fmin(nearb, farb) * fac;
            rp *= iR2;
        }
        return v;
    };
    // j from jm down to 0: k = la + lb - j rises from klo, the power pw = la + lb - 2j rises by 2
    const int pw0 = la + lb - 2 * jm;
    double Rpw = 1.0, Rpw1 = 0.0;   // R^pw and R^(pw-1)
    for (int p = 0; p < pw0; ++p) {
        Rpw1 = Rpw;
        Rpw *= R;
    }
    double ok = ob_next(klo);
    double bound = 0.0, dbound = 0.0;
    for (int j = jm; j >= 0; --j) {
        const int k = la + lb - j, pw = la + lb - 2 * j;
        const double cq = bt->cq[la][lb][j];
        bound += ok * cq * Rpw;
        double okn = 0.0;
        if (deriv || j > 0) okn = ob_next(k + 1);
        if (deriv) {
            double t = okn * 2.0 * R * Rpw;
            if (pw > 0) t += ok * 1.4142135623730951 * pw * Rpw1;
            dbound += t * cq;
        }
        ok = okn;
        Rpw1 = Rpw * R;
        Rpw = Rpw1 * R;
    }
    *vbound = bound;
    *R_out = R;
    *rmin_out = rmin;
    return deriv ? fmax(bound, dbound) : bound;
}

}  // namespace shg
