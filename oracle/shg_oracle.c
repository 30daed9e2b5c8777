/*
 * shg_oracle.c -- CPU oracle for contracted solid-harmonic-Gaussian integrals.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header, table or helper with the GPU engine.
 *
 * What it computes is the plain definition of each integral, by a route that
 * does not use the solid-harmonic (SHG) rearrangement at all:
 *
 *   (a|O|b) = double integral of phi_a(r1) O(r1 - r2) phi_b(r2)
 *                                     (Sec. II.B, eq. contractedr12int)
 *   (a|r_a^{2n}|b) = integral of phi_a(r) |r - A|^{2n} phi_b(r)   (Sec. II.C)
 *   (a b a~) = integral of phi_a(r) phi_a~(r) phi_b(r)
 *                                     (Sec. II.D, eq. aba_integrals)
 *
 * with phi a contracted, normalised real spherical-harmonic Gaussian
 * (Sec. II.A, eq. contracted_phi). Steps:
 *
 *  1. primitive integrals over unnormalised Cartesian Gaussians
 *     x_A^i y_A^j z_A^k exp(-alpha r_A^2):
 *       - overlap: the one-dimensional Obara-Saika recurrence, separately per
 *         Cartesian direction (Sec. III notes the overlap recursion separates);
 *       - the non-local operators 1/r, erf(wr)/r, erfc(wr)/r, exp(-wr^2) and
 *         exp(-wr^2)/r: an
 *         Obara-Saika style vertical recurrence on an auxiliary index n, where
 *         [0|0]^(n) is the n-th derivative of the s-s integral with respect to
 *         R_ab^2 (Table S1 of the supplement);
 *       - (a b a~): the two Cartesians on A are merged into one Cartesian with
 *         summed powers and exponent alpha + alpha~ (Sec. III), then overlap;
 *       - (a|r_a^{2n}|b): r_a^{2n} is expanded into Cartesian monomials on A
 *         (multinomial theorem) merged into the Cartesian of a, then overlap;
 *       - derivatives with respect to A from d/dA_x of the Cartesian primitive:
 *         2 alpha [a+1_x| - a_x [a-1_x|;
 *  2. contraction with the raw coefficients c_alpha;
 *  3. Cartesian -> real solid harmonic transform from the closed-form
 *     expansion of the real solid harmonics S_lm (Helgaker, Jorgensen, Olsen,
 *     Molecular Electronic-Structure Theory, eqs. 6.4.47-6.4.50). Component
 *     m = -l..l; m < 0 are the sine components; S_11 = x, S_1-1 = y, S_10 = z
 *     (the convention of Sec. II.A with the prefactor A_lm of eq. A);
 *  4. normalisation by the oracle's own numerically computed self-overlap of
 *     each shell (it does not use the closed-form N_l of eq. N_l).
 *
 * The arithmetic type `real` is double by default and long double when built
 * with -DORACLE_LONG_DOUBLE (the arbiter of disagreements) and __float128 with
 * -DORACLE_QUAD (113-bit significand, for (a|r_a^{2n}|b) at large n, whose
 * Cartesian expansion cancels beyond what long double resolves).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#if defined(ORACLE_QUAD)
#include <quadmath.h>
typedef __float128 real;
#define R_EXP expq
#define R_SQRT sqrtq
#define R_ERF erfq
#define R_FABS fabsq
#define R_POW powq
#define R_EPS 1e-34Q
#elif defined(ORACLE_LONG_DOUBLE)
typedef long double real;
#define R_EXP expl
#define R_SQRT sqrtl
#define R_ERF erfl
#define R_FABS fabsl
#define R_POW powl
#define R_EPS 1e-21L
#else
typedef double real;
#define R_EXP exp
#define R_SQRT sqrt
#define R_ERF erf
#define R_FABS fabs
#define R_POW pow
#define R_EPS 1e-17
#endif

static const real PI_R = 3.141592653589793238462643383279502884L;

enum { OP_OVERLAP = 0, OP_COULOMB = 1, OP_ERF = 2, OP_ERFC = 3, OP_GAUSS = 4,
       OP_OVERLAP_VRR = 5 /* overlap through the generic recurrence (self-check) */,
       OP_GCOULOMB = 6 /* exp(-w r^2)/r */ };

#define LCART_MAX 12   /* largest Cartesian degree handled (l_a + l_a~ + 1 <= 10) */
#define NMAX_AUX 16    /* largest auxiliary index of the vertical recurrence */

/* ------------------------------------------------------------------------- */
/* Boys function F_n(T) = int_0^1 exp(-T t^2) t^(2n) dt (supplement, eq. 3).   */
/* Small T: the convergent series exp(-T) sum_i (2T)^i / ((2n+1)(2n+3)...(2n+2i+1))
 * for F_nmax and the downward recurrence F_n = (2T F_{n+1} + e^-T)/(2n+1).
 * Large T: F_0 = sqrt(pi/T) erf(sqrt T) / 2 and the upward recurrence
 * F_{n+1} = ((2n+1) F_n - e^-T) / (2T), both from integrating by parts.     */
/* ------------------------------------------------------------------------- */
static void boys(int nmax, real T, real *F)
{
    real e = R_EXP(-T);
    if (T < 40) {
        real term = 1 / (real)(2 * nmax + 1), sum = term;
        for (int i = 1; i < 100000; ++i) {
            term *= 2 * T / (real)(2 * nmax + 2 * i + 1);
            sum += term;
            if (term < R_EPS * sum) break;
        }
        F[nmax] = e * sum;
        for (int n = nmax - 1; n >= 0; --n) F[n] = (2 * T * F[n + 1] + e) / (real)(2 * n + 1);
    } else {
        real st = R_SQRT(T);
        F[0] = R_SQRT(PI_R) / (2 * st) * R_ERF(st);
        for (int n = 0; n < nmax; ++n) F[n + 1] = ((2 * n + 1) * F[n] - e) / (2 * T);
    }
}

/* ------------------------------------------------------------------------- */
/* s-s integral (0_a|O|0_b) and its derivatives with respect to R_ab^2        */
/* (Table S1): g[n] = (d/dR^2)^n (0_a|O|0_b), n = 0..nmax.                    */
/* ------------------------------------------------------------------------- */
static void ss_derivs(int op, real w, real a, real b, real R2, int nmax, real *g)
{
    real p = a + b, rho = a * b / p, T = rho * R2;
    real F[NMAX_AUX + 2], F2[NMAX_AUX + 2];
    switch (op) {
    case OP_OVERLAP:
    case OP_OVERLAP_VRR: {
        real pre = R_POW(PI_R / p, (real)1.5) * R_EXP(-T), f = 1;
        for (int n = 0; n <= nmax; ++n) { g[n] = pre * f; f *= -rho; }
        break;
    }
    case OP_COULOMB: {
        real pre = 2 * R_POW(PI_R, (real)2.5) / (a * b * R_SQRT(p)), f = 1;
        boys(nmax, T, F);
        for (int n = 0; n <= nmax; ++n) { g[n] = pre * f * F[n]; f *= -rho; }
        break;
    }
    case OP_ERF:
    case OP_ERFC: {
        real pre = 2 * R_POW(PI_R, (real)2.5) / (a * b * R_SQRT(p));
        real w2 = w * w, s = w2 / (w2 + rho);
        real pre2 = pre * w / R_SQRT(w2 + rho);
        boys(nmax, T * s, F2);
        if (op == OP_ERFC) boys(nmax, T, F);
        real f = 1, f2 = 1;
        for (int n = 0; n <= nmax; ++n) {
            real v = pre2 * f2 * F2[n];
            g[n] = (op == OP_ERF) ? v : pre * f * F[n] - v;
            f *= -rho;
            f2 *= -rho * s;
        }
        break;
    }
    case OP_GCOULOMB: {
        /* e^{-w T/q} F_0(rho T/q) times a constant (Table S1); its n-th R^2
         * derivative by the Leibniz rule, with d/dx F_j = -F_{j+1} */
        real q = rho + w, x = rho * T / q;
        real pre = R_POW(PI_R / p, (real)1.5) * 2 * PI_R / q * R_EXP(-w * T / q);
        real ea = -w * rho / q, fb = -rho * rho / q;
        boys(nmax, x, F);
        for (int n = 0; n <= nmax; ++n) {
            real acc = 0, c = 1;   /* binom(n, j) */
            for (int j = 0; j <= n; ++j) {
                acc += c * R_POW(ea, (real)(n - j)) * R_POW(fb, (real)j) * F[j];
                c = c * (n - j) / (j + 1);
            }
            g[n] = pre * acc;
        }
        break;
    }
    case OP_GAUSS: {
        real q = rho + w;
        real pre = R_POW(PI_R * PI_R / (p * q), (real)1.5) * R_EXP(-w * T / q), f = 1;
        for (int n = 0; n <= nmax; ++n) { g[n] = pre * f; f *= -w * rho / q; }
        break;
    }
    default:
        for (int n = 0; n <= nmax; ++n) g[n] = 0;
    }
}

/* ------------------------------------------------------------------------- */
/* Cartesian component bookkeeping                                            */
/* ------------------------------------------------------------------------- */
static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian powers of component i of degree l, in the order
 * (l,0,0), (l-1,1,0), (l-1,0,1), (l-2,2,0), ... */
static void cart_pow(int l, int i, int *ax, int *ay, int *az)
{
    int k = 0;
    *ax = *ay = *az = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (k == i) { *ax = x; *ay = y; *az = l - x - y; return; }
            ++k;
        }
}

static int cart_index(int ax, int ay, int az)
{
    int l = ax + ay + az, k = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (x == ax && y == ay) return k;
            ++k;
        }
    return -1;
}

/* all Cartesian triples with degree <= L, degree-major; index tables */
typedef struct {
    int L, n;
    int pw[(LCART_MAX + 1) * (LCART_MAX + 2) * (LCART_MAX + 3) / 6][3];
    int idx[LCART_MAX + 1][LCART_MAX + 1][LCART_MAX + 1];
} cart_set;

static void cart_set_init(cart_set *s, int L)
{
    s->L = L;
    s->n = 0;
    memset(s->idx, -1, sizeof(s->idx));
    for (int l = 0; l <= L; ++l)
        for (int i = 0; i < ncart(l); ++i) {
            int x, y, z;
            cart_pow(l, i, &x, &y, &z);
            s->pw[s->n][0] = x; s->pw[s->n][1] = y; s->pw[s->n][2] = z;
            s->idx[x][y][z] = s->n++;
        }
}

static int cs_get(const cart_set *s, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0) return -1;
    return s->idx[x][y][z];
}

/* ------------------------------------------------------------------------- */
/* Real solid harmonics as Cartesian polynomials (closed form, see header).   */
/* T[(m+l)*ncart(l) + i] = coefficient of Cartesian component i in S_lm.     */
/* ------------------------------------------------------------------------- */
static real fact_r(int n) { real f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }
static real binom_r(int n, int k)
{
    if (k < 0 || k > n) return 0;
    return fact_r(n) / (fact_r(k) * fact_r(n - k));
}

static void solid_harmonic_cart(int l, real *T)
{
    int nc = ncart(l);
    memset(T, 0, sizeof(real) * (size_t)(2 * l + 1) * nc);
    for (int m = -l; m <= l; ++m) {
        int am = abs(m);
        int wm = (m < 0) ? 1 : 0;            /* 2 v_m */
        real Nlm = R_SQRT(2 * fact_r(l + am) * fact_r(l - am) / (m == 0 ? 2 : 1))
                   / (R_POW(2, am) * fact_r(l));
        for (int t = 0; t <= (l - am) / 2; ++t)
            for (int u = 0; u <= t; ++u)
                for (int w = wm; w <= am; w += 2) {  /* w = 2v */
                    int sgn_exp = t + (w - wm) / 2;
                    real C = ((sgn_exp & 1) ? -1 : 1) * R_POW((real)0.25, t) * binom_r(l, t) *
                             binom_r(l - t, am + t) * binom_r(t, u) * binom_r(am, w);
                    int px = 2 * t + am - 2 * u - w, py = 2 * u + w, pz = l - 2 * t - am;
                    if (px < 0 || py < 0 || pz < 0) continue;
                    T[(m + l) * nc + cart_index(px, py, pz)] += Nlm * C;
                }
    }
}

/* ------------------------------------------------------------------------- */
/* Primitive Cartesian integrals                                              */
/* ------------------------------------------------------------------------- */

/* 1-D overlap table S[i][j] = int (x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2) dx,
 * Obara-Saika: S_{i+1,j} = X_PA S_ij + (i S_{i-1,j} + j S_{i,j-1}) / 2p and the
 * analogous step in j; S_00 = sqrt(pi/p) exp(-ab/p (A-B)^2). */
static void overlap_1d(real a, real b, real A, real B, int imax, int jmax, real *S /*[imax+1][jmax+1]*/)
{
    real p = a + b, P = (a * A + b * B) / p, XPA = P - A, XPB = P - B;
    int J = jmax + 1;
    S[0] = R_SQRT(PI_R / p) * R_EXP(-a * b / p * (A - B) * (A - B));
    for (int i = 0; i <= imax; ++i)
        for (int j = 0; j <= jmax; ++j) {
            if (i == 0 && j == 0) continue;
            real v;
            if (i > 0) {
                v = XPA * S[(i - 1) * J + j];
                if (i > 1) v += (i - 1) * S[(i - 2) * J + j] / (2 * p);
                if (j > 0) v += j * S[(i - 1) * J + j - 1] / (2 * p);
            } else {
                v = XPB * S[i * J + j - 1];
                if (j > 1) v += (j - 1) * S[i * J + j - 2] / (2 * p);
            }
            S[i * J + j] = v;
        }
}

/* Generic two-center vertical recurrence, for a non-local operator whose s-s
 * integral depends on R^2 = |A-B|^2 only.  With X = A - B and
 * [a|b]^(n) the integral in which the s-s factor is replaced by its n-th
 * derivative with respect to R^2:
 *
 *  [a+1_i|b]^(n) =  X_i/alpha [a|b]^(n+1)
 *                 + a_i/(2 alpha) ( [a-1_i|b]^(n) + [a-1_i|b]^(n+1) / alpha )
 *                 - b_i/(2 alpha beta) [a|b-1_i]^(n+1)
 *  [a|b+1_i]^(n) = -X_i/beta [a|b]^(n+1)
 *                 - a_i/(2 alpha beta) [a-1_i|b]^(n+1)
 *                 + b_i/(2 beta) ( [a|b-1_i]^(n) + [a|b-1_i]^(n+1) / beta )
 *
 * It follows from x_A^(i+1) e^{-alpha x_A^2} = (d/dA_x + i)(x_A^(i-1) ...)/(2 alpha)
 * form of the Cartesian Gaussian (each Cartesian primitive is a constant-
 * coefficient polynomial in d/dA applied to the s Gaussian) and
 * d/dA_x g^(n)(|A-B|^2) = 2 X_x g^(n+1).
 * V has layout [ia][ib][n] over the index sets sa (degree <= La), sb (<= Lb). */
static void vrr_two_center(int op, real w, real a, real b, const real *X, const cart_set *sa,
                           const cart_set *sb, int N, real *V)
{
    int nb = sb->n, NN = N + 1;
#define VV(ia, ib, n) V[((size_t)(ia) * nb + (ib)) * NN + (n)]
    real R2 = X[0] * X[0] + X[1] * X[1] + X[2] * X[2];
    real g[NMAX_AUX + 2];
    ss_derivs(op, w, a, b, R2, N, g);
    for (int s = 0; s <= sa->L + sb->L; ++s)
        for (int ia = 0; ia < sa->n; ++ia) {
            const int *pa = sa->pw[ia];
            int la = pa[0] + pa[1] + pa[2];
            int lb = s - la;
            if (lb < 0 || lb > sb->L) continue;
            for (int ib = 0; ib < sb->n; ++ib) {
                const int *pb = sb->pw[ib];
                if (pb[0] + pb[1] + pb[2] != lb) continue;
                for (int n = 0; n <= N - s; ++n) {
                    real v;
                    if (s == 0) {
                        v = g[n];
                    } else if (la > 0) {
                        int d = (pa[0] > 0) ? 0 : (pa[1] > 0 ? 1 : 2);
                        int am[3] = {pa[0], pa[1], pa[2]};
                        am[d] -= 1;                       /* a = am + 1_d */
                        int i0 = cs_get(sa, am[0], am[1], am[2]);
                        v = X[d] / a * VV(i0, ib, n + 1);
                        if (am[d] > 0) {
                            int amm[3] = {am[0], am[1], am[2]};
                            amm[d] -= 1;
                            int i1 = cs_get(sa, amm[0], amm[1], amm[2]);
                            v += am[d] / (2 * a) * (VV(i1, ib, n) + VV(i1, ib, n + 1) / a);
                        }
                        if (pb[d] > 0) {
                            int bm[3] = {pb[0], pb[1], pb[2]};
                            bm[d] -= 1;
                            int j1 = cs_get(sb, bm[0], bm[1], bm[2]);
                            v -= pb[d] / (2 * a * b) * VV(i0, j1, n + 1);
                        }
                    } else {
                        int d = (pb[0] > 0) ? 0 : (pb[1] > 0 ? 1 : 2);
                        int bm[3] = {pb[0], pb[1], pb[2]};
                        bm[d] -= 1;                       /* b = bm + 1_d, a = 0 */
                        int j0 = cs_get(sb, bm[0], bm[1], bm[2]);
                        v = -X[d] / b * VV(ia, j0, n + 1);
                        if (bm[d] > 0) {
                            int bmm[3] = {bm[0], bm[1], bm[2]};
                            bmm[d] -= 1;
                            int j1 = cs_get(sb, bmm[0], bmm[1], bmm[2]);
                            v += bm[d] / (2 * b) * (VV(ia, j1, n) + VV(ia, j1, n + 1) / b);
                        }
                    }
                    VV(ia, ib, n) = v;
                }
            }
        }
#undef VV
}

/* Primitive Cartesian blocks for shell a of degree la and shell b of degree lb,
 * components in cart_pow order: P[ia][ib] for degree la, and when Pp/Pm are
 * non-NULL also the blocks of degree la+1 and la-1 (needed for d/dA).  Uses
 * the 1-D overlap recurrence (op == overlap) or the generic vertical
 * recurrence.  A is the center of a (exponent a), B that of b. */
typedef struct {
    cart_set sa, sb;
    real *V;
    size_t vcap;
} work_t;

static void extract_block(const work_t *wk, int N, int la, int lb, real *P)
{
    int na = ncart(la), nb = ncart(lb);
    for (int i = 0; i < na; ++i) {
        int ax, ay, az;
        cart_pow(la, i, &ax, &ay, &az);
        int ia = cs_get(&wk->sa, ax, ay, az);
        for (int j = 0; j < nb; ++j) {
            int bx, by, bz;
            cart_pow(lb, j, &bx, &by, &bz);
            int ib = cs_get(&wk->sb, bx, by, bz);
            P[i * nb + j] = wk->V[((size_t)ia * wk->sb.n + ib) * (N + 1)];
        }
    }
}

static void overlap_block(const real *Sx, const real *Sy, const real *Sz, int J, int la, int lb,
                          real *P)
{
    int na = ncart(la), nb = ncart(lb);
    for (int i = 0; i < na; ++i) {
        int ax, ay, az;
        cart_pow(la, i, &ax, &ay, &az);
        for (int j = 0; j < nb; ++j) {
            int bx, by, bz;
            cart_pow(lb, j, &bx, &by, &bz);
            P[i * nb + j] = Sx[ax * J + bx] * Sy[ay * J + by] * Sz[az * J + bz];
        }
    }
}

static void prim_blocks(work_t *wk, int op, real w, real a, real b, const real *A, const real *B,
                        int la, int lb, real *P, real *Pp, real *Pm)
{
    int Lhi = la + (Pp ? 1 : 0);
    if (op == OP_OVERLAP) {
        real Sx[(LCART_MAX + 1) * (LCART_MAX + 1)], Sy[(LCART_MAX + 1) * (LCART_MAX + 1)],
            Sz[(LCART_MAX + 1) * (LCART_MAX + 1)];
        overlap_1d(a, b, A[0], B[0], Lhi, lb, Sx);
        overlap_1d(a, b, A[1], B[1], Lhi, lb, Sy);
        overlap_1d(a, b, A[2], B[2], Lhi, lb, Sz);
        overlap_block(Sx, Sy, Sz, lb + 1, la, lb, P);
        if (Pp) overlap_block(Sx, Sy, Sz, lb + 1, la + 1, lb, Pp);
        if (Pm && la > 0) overlap_block(Sx, Sy, Sz, lb + 1, la - 1, lb, Pm);
        return;
    }
    real X[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
    if (wk->sa.L != Lhi) cart_set_init(&wk->sa, Lhi);
    if (wk->sb.L != lb) cart_set_init(&wk->sb, lb);
    int N = Lhi + lb;
    size_t need = (size_t)wk->sa.n * wk->sb.n * (N + 1);
    if (need > wk->vcap) {
        free(wk->V);
        wk->V = (real *)malloc(need * sizeof(real));
        wk->vcap = need;
    }
    vrr_two_center(op, w, a, b, X, &wk->sa, &wk->sb, N, wk->V);
    extract_block(wk, N, la, lb, P);
    if (Pp) extract_block(wk, N, la + 1, lb, Pp);
    if (Pm && la > 0) extract_block(wk, N, la - 1, lb, Pm);
}

/* ------------------------------------------------------------------------- */
/* Shell table                                                                */
/* ------------------------------------------------------------------------- */
typedef struct {
    const double *center;
    const int32_t *l, *nprim;
    const int64_t *prim_off;
    const double *exps, *coefs;
} shells_t;

/* contracted, transformed block (2la+1) x (2lb+1) for shells a (at A) and b
 * (at B), unnormalised; dA (nullable) receives d/dA_{x,y,z} as 3 blocks. */
static void contracted_pair(work_t *wk, int op, real w, const shells_t *sh, int sa_, int sb_,
                            const double *Aover, const double *Bover, real *out, real *dA)
{
    int la = sh->l[sa_], lb = sh->l[sb_];
    int na = ncart(la), nb = ncart(lb), nap = ncart(la + 1), nam = la > 0 ? ncart(la - 1) : 0;
    real A[3], B[3];
    for (int d = 0; d < 3; ++d) {
        A[d] = Aover ? Aover[d] : sh->center[3 * sa_ + d];
        B[d] = Bover ? Bover[d] : sh->center[3 * sb_ + d];
    }
    real *C = (real *)calloc((size_t)na * nb, sizeof(real));
    real *Cd = dA ? (real *)calloc((size_t)3 * na * nb, sizeof(real)) : NULL;
    real *P = (real *)malloc(sizeof(real) * (size_t)na * nb);
    real *Pp = dA ? (real *)malloc(sizeof(real) * (size_t)nap * nb) : NULL;
    real *Pm = (dA && la > 0) ? (real *)malloc(sizeof(real) * (size_t)nam * nb) : NULL;
    for (int i = 0; i < sh->nprim[sa_]; ++i)
        for (int j = 0; j < sh->nprim[sb_]; ++j) {
            real a = sh->exps[sh->prim_off[sa_] + i], b = sh->exps[sh->prim_off[sb_] + j];
            real cc = (real)sh->coefs[sh->prim_off[sa_] + i] * (real)sh->coefs[sh->prim_off[sb_] + j];
            prim_blocks(wk, op, w, a, b, A, B, la, lb, P, Pp, Pm);
            for (int k = 0; k < na * nb; ++k) C[k] += cc * P[k];
            if (dA) {
                for (int ic = 0; ic < na; ++ic) {
                    int p[3];
                    cart_pow(la, ic, &p[0], &p[1], &p[2]);
                    for (int d = 0; d < 3; ++d) {
                        int q[3] = {p[0], p[1], p[2]};
                        q[d] += 1;
                        int iu = cart_index(q[0], q[1], q[2]);
                        int idn = -1;
                        if (p[d] > 0) {
                            q[d] -= 2;
                            idn = cart_index(q[0], q[1], q[2]);
                        }
                        for (int jc = 0; jc < nb; ++jc) {
                            real v = 2 * a * Pp[iu * nb + jc];
                            if (idn >= 0) v -= p[d] * Pm[idn * nb + jc];
                            Cd[(size_t)d * na * nb + ic * nb + jc] += cc * v;
                        }
                    }
                }
            }
        }
    real *Ta = (real *)malloc(sizeof(real) * (size_t)(2 * la + 1) * na);
    real *Tb = (real *)malloc(sizeof(real) * (size_t)(2 * lb + 1) * nb);
    solid_harmonic_cart(la, Ta);
    solid_harmonic_cart(lb, Tb);
    int ma_n = 2 * la + 1, mb_n = 2 * lb + 1;
    for (int comp = 0; comp < (dA ? 4 : 1); ++comp) {
        const real *src = comp == 0 ? C : Cd + (size_t)(comp - 1) * na * nb;
        real *dst = comp == 0 ? out : dA + (size_t)(comp - 1) * ma_n * mb_n;
        for (int ma = 0; ma < ma_n; ++ma)
            for (int mb = 0; mb < mb_n; ++mb) {
                real s = 0;
                for (int i = 0; i < na; ++i) {
                    real ta = Ta[ma * na + i];
                    if (ta == 0) continue;
                    for (int j = 0; j < nb; ++j) s += ta * Tb[mb * nb + j] * src[i * nb + j];
                }
                dst[ma * mb_n + mb] = s;
            }
    }
    free(C); free(Cd); free(P); free(Pp); free(Pm); free(Ta); free(Tb);
}

/* Numerical normalisation: 1/sqrt of the contracted self-overlap of one real
 * component (all 2l+1 components share it). */
static real shell_norm(work_t *wk, const shells_t *sh, int s)
{
    int l = sh->l[s];
    real *blk = (real *)malloc(sizeof(real) * (size_t)(2 * l + 1) * (2 * l + 1));
    const double *c = sh->center + 3 * s;
    contracted_pair(wk, OP_OVERLAP, 0, sh, s, s, c, c, blk, NULL);
    real v = blk[l * (2 * l + 1) + l];
    free(blk);
    return 1 / R_SQRT(v);
}

static void work_init(work_t *wk)
{
    memset(wk, 0, sizeof(*wk));
    wk->sa.L = -1;
    wk->sb.L = -1;
}

/* ------------------------------------------------------------------------- */
/* Exported API (host pointers).  Return 0 on success, -1 on bad arguments.  */
/* ------------------------------------------------------------------------- */
int shgo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads used by the OpenMP loops of the calls that follow (timing only) */
void shgo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int shgo_real_bytes(void) { return (int)sizeof(real); }

void shgo_boys(int nmax, double T, double *F)
{
    real f[NMAX_AUX * 4 + 2];
    if (nmax < 0 || nmax > NMAX_AUX * 4) return;
    boys(nmax, (real)T, f);
    for (int n = 0; n <= nmax; ++n) F[n] = (double)f[n];
}

void shgo_ss_derivs(int op, double w, double a, double b, double R2, int nmax, double *g)
{
    real v[NMAX_AUX + 2];
    if (nmax < 0 || nmax > NMAX_AUX) return;
    ss_derivs(op, w, a, b, R2, nmax, v);
    for (int n = 0; n <= nmax; ++n) g[n] = (double)v[n];
}

/* coefficients of the real solid harmonics: T[(m+l)*ncart + i], Cartesian
 * component i has powers pw[3*i..3*i+2] */
int shgo_solid_harmonic(int l, double *T, int32_t *pw)
{
    if (l < 0 || l > LCART_MAX) return -1;
    int nc = ncart(l);
    real *t = (real *)malloc(sizeof(real) * (size_t)(2 * l + 1) * nc);
    solid_harmonic_cart(l, t);
    for (int k = 0; k < (2 * l + 1) * nc; ++k) T[k] = (double)t[k];
    for (int i = 0; i < nc; ++i) {
        int x, y, z;
        cart_pow(l, i, &x, &y, &z);
        pw[3 * i] = x; pw[3 * i + 1] = y; pw[3 * i + 2] = z;
    }
    free(t);
    return 0;
}

/* primitive Cartesian block for tests: P[ia][ib], components in shgo_solid_harmonic order */
int shgo_prim_cart(int op, double w, double a, double b, const double *A, const double *B, int la,
                   int lb, double *P)
{
    if (la < 0 || lb < 0 || la > 10 || lb > 10 || la + lb > NMAX_AUX) return -1;
    work_t wk;
    work_init(&wk);
    real Ar[3] = {A[0], A[1], A[2]}, Br[3] = {B[0], B[1], B[2]};
    int n = ncart(la) * ncart(lb);
    real *p = (real *)malloc(sizeof(real) * n);
    prim_blocks(&wk, op, w, a, b, Ar, Br, la, lb, p, NULL, NULL);
    for (int k = 0; k < n; ++k) P[k] = (double)p[k];
    free(p);
    free(wk.V);
    return 0;
}

static int check_shells(int32_t nshell, const int32_t *l, const int32_t *nprim, int lmax)
{
    for (int i = 0; i < nshell; ++i)
        if (l[i] < 0 || l[i] > lmax || nprim[i] < 1) return -1;
    return 0;
}

/* (a|O|b) for n pairs; out[out_off[i] + ma*(2lb+1) + mb]; dout (nullable)
 * receives d/dR_a at dout[3*out_off[i] + d*(2la+1)(2lb+1) + ...]. */
int shgo_pairs(int32_t nshell, const double *center, const int32_t *l, const int32_t *nprim,
               const int64_t *prim_off, const double *exps, const double *coefs, int op,
               double omega, const int32_t *pairs, int64_t n, const int64_t *out_off, double *out,
               double *dout)
{
    if (n < 0 || op < 0 || op > 6) return -1;
    if (n == 0) return 0;
    if (check_shells(nshell, l, nprim, 8)) return -1;
    shells_t sh = {center, l, nprim, prim_off, exps, coefs};
    real *norm = (real *)malloc(sizeof(real) * (size_t)nshell);
    char *need = (char *)calloc((size_t)nshell, 1);
    for (int64_t i = 0; i < n; ++i) {
        if (pairs[2 * i] < 0 || pairs[2 * i] >= nshell || pairs[2 * i + 1] < 0 ||
            pairs[2 * i + 1] >= nshell) {
            free(norm); free(need);
            return -1;
        }
        need[pairs[2 * i]] = need[pairs[2 * i + 1]] = 1;
    }
#pragma omp parallel
    {
        work_t wk;
        work_init(&wk);
#pragma omp for schedule(dynamic, 16)
        for (int s = 0; s < nshell; ++s)
            if (need[s]) norm[s] = shell_norm(&wk, &sh, s);
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n; ++i) {
            int a = pairs[2 * i], b = pairs[2 * i + 1];
            int sz = (2 * l[a] + 1) * (2 * l[b] + 1);
            real *blk = (real *)malloc(sizeof(real) * (size_t)sz * 4);
            contracted_pair(&wk, op, omega, &sh, a, b, NULL, NULL, blk, dout ? blk + sz : NULL);
            real f = norm[a] * norm[b];
            for (int k = 0; k < sz; ++k) out[out_off[i] + k] = (double)(f * blk[k]);
            if (dout)
                for (int k = 0; k < 3 * sz; ++k) dout[3 * out_off[i] + k] = (double)(f * blk[sz + k]);
            free(blk);
        }
        free(wk.V);
    }
    free(norm);
    free(need);
    return 0;
}

/* (a b a~): a = orb[t0] and a~ = aux[t1] on center A (must coincide), b = orb[t2].
 * out[out_off + (ma*(2lt+1) + mt)*(2lb+1) + mb]; dout (nullable) d/dR_A
 * (moves a and a~ together) at 3*out_off, x, y, z blocks. */
int shgo_aab(int32_t norb, const double *oc, const int32_t *ol, const int32_t *onp,
             const int64_t *ooff, const double *oexp, const double *ocoef, int32_t naux,
             const double *xc, const int32_t *xl, const int32_t *xnp, const int64_t *xoff,
             const double *xexp, const double *xcoef, const int32_t *tri, int64_t n,
             const int64_t *out_off, double *out, double *dout)
{
    if (n < 0) return -1;
    if (n == 0) return 0;
    if (check_shells(norb, ol, onp, 8) || check_shells(naux, xl, xnp, 8)) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int a = tri[3 * i], t = tri[3 * i + 1], b = tri[3 * i + 2];
        if (a < 0 || a >= norb || t < 0 || t >= naux || b < 0 || b >= norb) return -1;
        for (int d = 0; d < 3; ++d)
            if (oc[3 * a + d] != xc[3 * t + d]) return -1;
        if (ol[a] + xl[t] + 1 > LCART_MAX - 1) return -1;
    }
    shells_t so = {oc, ol, onp, ooff, oexp, ocoef};
    shells_t sx = {xc, xl, xnp, xoff, xexp, xcoef};
    real *no = (real *)malloc(sizeof(real) * (size_t)norb);
    real *nx = (real *)malloc(sizeof(real) * (size_t)naux);
#pragma omp parallel
    {
        work_t wk;
        work_init(&wk);
#pragma omp for schedule(dynamic, 16)
        for (int s = 0; s < norb; ++s) no[s] = shell_norm(&wk, &so, s);
#pragma omp for schedule(dynamic, 16)
        for (int s = 0; s < naux; ++s) nx[s] = shell_norm(&wk, &sx, s);
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n; ++i) {
            int a = tri[3 * i], t = tri[3 * i + 1], b = tri[3 * i + 2];
            int la = ol[a], lt = xl[t], lb = ol[b];
            int na = ncart(la), nt = ncart(lt), nb = ncart(lb);
            int ma_n = 2 * la + 1, mt_n = 2 * lt + 1, mb_n = 2 * lb + 1;
            int L = la + lt;
            real A[3] = {oc[3 * a], oc[3 * a + 1], oc[3 * a + 2]};
            real B[3] = {oc[3 * b], oc[3 * b + 1], oc[3 * b + 2]};
            /* Cartesian blocks C[ia][it][ib] (value) and dC[d][ia][it][ib] */
            size_t csz = (size_t)na * nt * nb;
            real *C = (real *)calloc(csz * 4, sizeof(real));
            int J = lb + 1, I = L + 2;
            real *Sx = (real *)malloc(sizeof(real) * I * J);
            real *Sy = (real *)malloc(sizeof(real) * I * J);
            real *Sz = (real *)malloc(sizeof(real) * I * J);
            for (int pa = 0; pa < onp[a]; ++pa)
                for (int pt = 0; pt < xnp[t]; ++pt)
                    for (int pb = 0; pb < onp[b]; ++pb) {
                        real al = oexp[ooff[a] + pa] + xexp[xoff[t] + pt];
                        real be = oexp[ooff[b] + pb];
                        real cc = (real)ocoef[ooff[a] + pa] * (real)xcoef[xoff[t] + pt] *
                                  (real)ocoef[ooff[b] + pb];
                        overlap_1d(al, be, A[0], B[0], L + 1, lb, Sx);
                        overlap_1d(al, be, A[1], B[1], L + 1, lb, Sy);
                        overlap_1d(al, be, A[2], B[2], L + 1, lb, Sz);
                        const real *S1[3] = {Sx, Sy, Sz};
                        for (int ia = 0; ia < na; ++ia) {
                            int p[3];
                            cart_pow(la, ia, &p[0], &p[1], &p[2]);
                            for (int it = 0; it < nt; ++it) {
                                int q[3];
                                cart_pow(lt, it, &q[0], &q[1], &q[2]);
                                int m[3] = {p[0] + q[0], p[1] + q[1], p[2] + q[2]};
                                for (int ib = 0; ib < nb; ++ib) {
                                    int r[3];
                                    cart_pow(lb, ib, &r[0], &r[1], &r[2]);
                                    real s1[3], d1[3];
                                    for (int d = 0; d < 3; ++d) {
                                        s1[d] = S1[d][m[d] * J + r[d]];
                                        /* d/dA of x_A^m e^{-al x_A^2}: 2 al x^(m+1) - m x^(m-1) */
                                        d1[d] = 2 * al * S1[d][(m[d] + 1) * J + r[d]];
                                        if (m[d] > 0) d1[d] -= m[d] * S1[d][(m[d] - 1) * J + r[d]];
                                    }
                                    size_t k = ((size_t)ia * nt + it) * nb + ib;
                                    C[k] += cc * s1[0] * s1[1] * s1[2];
                                    C[csz + k] += cc * d1[0] * s1[1] * s1[2];
                                    C[2 * csz + k] += cc * s1[0] * d1[1] * s1[2];
                                    C[3 * csz + k] += cc * s1[0] * s1[1] * d1[2];
                                }
                            }
                        }
                    }
            real *Ta = (real *)malloc(sizeof(real) * ma_n * na);
            real *Tt = (real *)malloc(sizeof(real) * mt_n * nt);
            real *Tb = (real *)malloc(sizeof(real) * mb_n * nb);
            solid_harmonic_cart(la, Ta);
            solid_harmonic_cart(lt, Tt);
            solid_harmonic_cart(lb, Tb);
            real f = no[a] * nx[t] * no[b];
            size_t osz = (size_t)ma_n * mt_n * mb_n;
            real *tmp1 = (real *)malloc(sizeof(real) * ma_n * nt * nb);
            real *tmp2 = (real *)malloc(sizeof(real) * ma_n * mt_n * nb);
            for (int comp = 0; comp < (dout ? 4 : 1); ++comp) {
                const real *src = C + comp * csz;
                for (int ma = 0; ma < ma_n; ++ma)
                    for (int k = 0; k < nt * nb; ++k) {
                        real s = 0;
                        for (int ia = 0; ia < na; ++ia) s += Ta[ma * na + ia] * src[(size_t)ia * nt * nb + k];
                        tmp1[ma * nt * nb + k] = s;
                    }
                for (int ma = 0; ma < ma_n; ++ma)
                    for (int mt = 0; mt < mt_n; ++mt)
                        for (int ib = 0; ib < nb; ++ib) {
                            real s = 0;
                            for (int it = 0; it < nt; ++it)
                                s += Tt[mt * nt + it] * tmp1[(ma * nt + it) * nb + ib];
                            tmp2[(ma * mt_n + mt) * nb + ib] = s;
                        }
                for (int k = 0; k < ma_n * mt_n; ++k)
                    for (int mb = 0; mb < mb_n; ++mb) {
                        real s = 0;
                        for (int ib = 0; ib < nb; ++ib) s += Tb[mb * nb + ib] * tmp2[k * nb + ib];
                        double v = (double)(f * s);
                        if (comp == 0) out[out_off[i] + k * mb_n + mb] = v;
                        else dout[3 * out_off[i] + (comp - 1) * osz + k * mb_n + mb] = v;
                    }
            }
            free(C); free(Sx); free(Sy); free(Sz); free(Ta); free(Tt); free(Tb); free(tmp1); free(tmp2);
        }
        free(wk.V);
    }
    free(no);
    free(nx);
    return 0;
}

/* (a|r_a^{2n}|b) (Sec. II.C, eq. ara2nb_def): the local operator r_a^{2n} =
 * (x_A^2 + y_A^2 + z_A^2)^n is centred on A, so it is expanded by the
 * multinomial theorem into sum_{i+j+k=n} n!/(i!j!k!) x_A^{2i} y_A^{2j} z_A^{2k}
 * and each term merged into the Cartesian factor of a; then the plain overlap
 * of the merged Cartesian Gaussians. d/dR_A moves a and the operator together
 * (both depend on r - A): the derivative of the merged Cartesian as for a
 * plain Gaussian. a and b come from the same shell table; out, out_off, dout
 * as in shgo_pairs; n in [0, 8]. */
int shgo_r2n(int32_t nshell, const double *center, const int32_t *l, const int32_t *nprim,
             const int64_t *prim_off, const double *exps, const double *coefs, int nr,
             const int32_t *pairs, int64_t n, const int64_t *out_off, double *out, double *dout)
{
    if (n < 0 || nr < 0 || nr > 8) return -1;
    if (n == 0) return 0;
    if (check_shells(nshell, l, nprim, 8)) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (pairs[2 * i] < 0 || pairs[2 * i] >= nshell || pairs[2 * i + 1] < 0 || pairs[2 * i + 1] >= nshell)
            return -1;
    shells_t sh = {center, l, nprim, prim_off, exps, coefs};
    real *norm = (real *)malloc(sizeof(real) * (size_t)nshell);
    /* multinomial terms of (x^2 + y^2 + z^2)^nr */
    int nterm = 0;
    int tp[45][3];
    real tc[45];
    for (int i = 0; i <= nr; ++i)
        for (int j = 0; j <= nr - i; ++j) {
            int k = nr - i - j;
            tp[nterm][0] = 2 * i; tp[nterm][1] = 2 * j; tp[nterm][2] = 2 * k;
            tc[nterm++] = fact_r(nr) / (fact_r(i) * fact_r(j) * fact_r(k));
        }
#pragma omp parallel
    {
        work_t wk;
        work_init(&wk);
#pragma omp for schedule(dynamic, 16)
        for (int s = 0; s < nshell; ++s) norm[s] = shell_norm(&wk, &sh, s);
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n; ++i) {
            int a = pairs[2 * i], b = pairs[2 * i + 1];
            int la = l[a], lb = l[b], na = ncart(la), nb = ncart(lb);
            int ma_n = 2 * la + 1, mb_n = 2 * lb + 1;
            const double *A = center + 3 * a, *B = center + 3 * b;
            size_t csz = (size_t)na * nb;
            real *Cc = (real *)calloc(csz * 4, sizeof(real));
            int I = la + 2 * nr + 2, J = lb + 1;
            real *Sx = (real *)malloc(sizeof(real) * I * J);
            real *Sy = (real *)malloc(sizeof(real) * I * J);
            real *Sz = (real *)malloc(sizeof(real) * I * J);
            for (int pa = 0; pa < nprim[a]; ++pa)
                for (int pb = 0; pb < nprim[b]; ++pb) {
                    real al = exps[prim_off[a] + pa], be = exps[prim_off[b] + pb];
                    real cc = (real)coefs[prim_off[a] + pa] * (real)coefs[prim_off[b] + pb];
                    overlap_1d(al, be, A[0], B[0], I - 1, lb, Sx);
                    overlap_1d(al, be, A[1], B[1], I - 1, lb, Sy);
                    overlap_1d(al, be, A[2], B[2], I - 1, lb, Sz);
                    const real *S1[3] = {Sx, Sy, Sz};
                    for (int ia = 0; ia < na; ++ia) {
                        int p[3];
                        cart_pow(la, ia, &p[0], &p[1], &p[2]);
                        for (int ib = 0; ib < nb; ++ib) {
                            int r[3];
                            cart_pow(lb, ib, &r[0], &r[1], &r[2]);
                            size_t k = (size_t)ia * nb + ib;
                            for (int t = 0; t < nterm; ++t) {
                                real s1[3], d1[3];
                                for (int d = 0; d < 3; ++d) {
                                    int m = p[d] + tp[t][d];
                                    s1[d] = S1[d][m * J + r[d]];
                                    d1[d] = 2 * al * S1[d][(m + 1) * J + r[d]];
                                    if (m > 0) d1[d] -= m * S1[d][(m - 1) * J + r[d]];
                                }
                                real f = cc * tc[t];
                                Cc[k] += f * s1[0] * s1[1] * s1[2];
                                Cc[csz + k] += f * d1[0] * s1[1] * s1[2];
                                Cc[2 * csz + k] += f * s1[0] * d1[1] * s1[2];
                                Cc[3 * csz + k] += f * s1[0] * s1[1] * d1[2];
                            }
                        }
                    }
                }
            real *Ta = (real *)malloc(sizeof(real) * ma_n * na);
            real *Tb = (real *)malloc(sizeof(real) * mb_n * nb);
            solid_harmonic_cart(la, Ta);
            solid_harmonic_cart(lb, Tb);
            real f = norm[a] * norm[b];
            size_t osz = (size_t)ma_n * mb_n;
            for (int comp = 0; comp < (dout ? 4 : 1); ++comp) {
                const real *src = Cc + comp * csz;
                for (int ma = 0; ma < ma_n; ++ma)
                    for (int mb = 0; mb < mb_n; ++mb) {
                        real s = 0;
                        for (int ia = 0; ia < na; ++ia) {
                            real ta = Ta[ma * na + ia];
                            if (ta == 0) continue;
                            for (int ib = 0; ib < nb; ++ib) s += ta * Tb[mb * nb + ib] * src[(size_t)ia * nb + ib];
                        }
                        double v = (double)(f * s);
                        if (comp == 0) out[out_off[i] + ma * mb_n + mb] = v;
                        else dout[3 * out_off[i] + (comp - 1) * osz + ma * mb_n + mb] = v;
                    }
            }
            free(Cc); free(Sx); free(Sy); free(Sz); free(Ta); free(Tb);
        }
        free(wk.V);
    }
    free(norm);
    return 0;
}
