// shg_monopole.hip -- two-center integrals whose contracted radial term is
// computed by a kernel of its own and then fed to the shared tile in its
// precomputed-monopole mode (pair items, blocks straight to out_off):
//
//  * (a|r_a^{2n}|b) and d/dR_a (Sec. II.C, eqs. ara2nb and T_rab2_deriv).
//    The operator r_a^{2n} is centred on A, so the contracted radial term is
//    the monopole T^(k) of eq. T_rab2_deriv (a binomial sum over the
//    primitive (0_a|r_a^{2m}|0_b)^(k), eq. sra2ms and its R^2 derivatives)
//    and the block follows eq. ara2nb, which has the form of eq.
//    final_r12int_ab with T^(k) in place of O^(k); d/dR_a (a and the operator
//    move together) follows eq. dev_ab the same way. T^(k) is accumulated in
//    double-double (shg_r2n_math.h).
//  * the Gaussian-damped Coulomb operator exp(-omega r^2)/r (Table S1): O^(k)
//    of eq. O_rab2_deriv with the R^2 derivatives of its s-s integral, a
//    Leibniz sum over Boys functions F_j whose terms all share one sign.
//
// Per call:
//   k_classify / k_scan_bins / k_scatter   class-sorted pair ids (shared with
//                                          the two-center path)
//   per class (la, lb), in chunks of at most MONO_CHUNK pairs:
//     k_r2n_radial<la,lb,D> or k_gc_radial<la,lb,D>
//                            G lanes per pair: the contracted radial terms for
//                            k = max(la,lb) .. la+lb+D, xor butterfly
//     k_tile<la,lb,D>        precomputed-monopole mode: angular part and
//                            assembly, LDS-staged coalesced stores
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "shg_ctx.h"
#include "shg_r2n_math.h"

using namespace shg;

namespace {

constexpr int R2N_MAX = 5;
constexpr int R2N_TSTRIDE = MONO_TSTRIDE;  // doubles per pair in the radial-term buffer (NK <= 6)
constexpr int64_t MONO_CHUNK = 1 << 20;
constexpr int RG = 8, RTPB = 256;         // lanes per pair, threads per block

struct R2nArgs {
    const int32_t *pairs, *order;
    const double *center;
    const int32_t *nprim;
    const int64_t *prim_off;
    const double *exps, *w;   // folded weights N_l c / (2 alpha)^l
    double *T;                // [pos - start][R2N_TSTRIDE]
    int64_t start, count;
    int nr;                   // r_a^{2n}: n
    double omega;             // exp(-omega r^2)/r: omega
    const double *tab;        // Boys grid
};

// T^(k) for k = KLO..KHI of one pair (eq. T_rab2_deriv), accumulated over the
// primitive pairs in double-double (r2n_accumulate) and rounded once at the end
template <int LA, int LB, bool D, int NR>
__device__ __forceinline__ void r2n_pair(const R2nArgs &a, int64_t slot, int g)
{
    constexpr int KLO = cmax(LA, LB), KHI = LA + LB + (D ? 1 : 0), NK = KHI - KLO + 1;
    const bool live = slot < a.count;
    const int64_t pos = a.start + (live ? slot : 0);
    const int p = a.order[pos];
    const int sa = a.pairs[2 * (int64_t)p], sb = a.pairs[2 * (int64_t)p + 1];
    const double X0 = a.center[3 * sa] - a.center[3 * sb];
    const double X1 = a.center[3 * sa + 1] - a.center[3 * sb + 1];
    const double X2 = a.center[3 * sa + 2] - a.center[3 * sb + 2];
    const double R2 = fma(X0, X0, fma(X1, X1, X2 * X2));
    const int64_t oa = a.prim_off[sa], ob = a.prim_off[sb];
    const int kb = a.nprim[sb];
    const int P = live ? a.nprim[sa] * kb : 0;
    dd T[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) T[k] = dd{0.0, 0.0};
    for (int q = g; q < P; q += RG) {
        const int ia = q / kb, ib = q - ia * kb;
        r2n_accumulate<LA, NR, KLO, KHI>(a.exps[oa + ia], a.exps[ob + ib], R2, a.w[oa + ia] * a.w[ob + ib], T);
    }
#pragma unroll
    for (int m = 1; m < RG; m <<= 1)
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const dd o{__shfl_xor(T[k].hi, m, RG), __shfl_xor(T[k].lo, m, RG)};
            T[k] = dd_add(T[k], o);
        }
    if (live && g == 0) {
        double *dst = a.T + (pos - a.start) * R2N_TSTRIDE;
#pragma unroll
        for (int k = 0; k < NK; ++k) dst[k] = T[k].hi + T[k].lo;
    }
}

template <int LA, int LB, bool D>
__global__ __launch_bounds__(RTPB) void k_r2n_radial(R2nArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * RTPB + threadIdx.x;
    const int64_t slot = t / RG;
    const int g = (int)(t % RG);
    switch (a.nr) {
    case 0: r2n_pair<LA, LB, D, 0>(a, slot, g); break;
    case 1: r2n_pair<LA, LB, D, 1>(a, slot, g); break;
    case 2: r2n_pair<LA, LB, D, 2>(a, slot, g); break;
    case 3: r2n_pair<LA, LB, D, 3>(a, slot, g); break;
    case 4: r2n_pair<LA, LB, D, 4>(a, slot, g); break;
    default: r2n_pair<LA, LB, D, 5>(a, slot, g); break;
    }
}

// O^(k), k = KLO..KHI, of exp(-omega r^2)/r for one pair: per primitive pair
// with c = a + b, rho = a b / c, T = rho R^2, q = rho + omega, the s-s
// integral is (pi/c)^{3/2} (2 pi / q) e^{-omega T / q} F_0(rho T / q) and its
// k-th R^2 derivative sum_j binom(k, j) e^{k-j} f^j F_j(rho T / q) times the
// same prefactor, e = -omega rho / q, f = -rho^2 / q (Table S1)
template <int LA, int LB, bool D>
__device__ __forceinline__ void gc_pair(const R2nArgs &a, int64_t slot, int g)
{
    constexpr int KLO = cmax(LA, LB), KHI = LA + LB + (D ? 1 : 0), NK = KHI - KLO + 1;
    const bool live = slot < a.count;
    const int64_t pos = a.start + (live ? slot : 0);
    const int p = a.order[pos];
    const int sa = a.pairs[2 * (int64_t)p], sb = a.pairs[2 * (int64_t)p + 1];
    const double X0 = a.center[3 * sa] - a.center[3 * sb];
    const double X1 = a.center[3 * sa + 1] - a.center[3 * sb + 1];
    const double X2 = a.center[3 * sa + 2] - a.center[3 * sb + 2];
    const double R2 = fma(X0, X0, fma(X1, X1, X2 * X2));
    const int64_t oa = a.prim_off[sa], ob = a.prim_off[sb];
    const int kb = a.nprim[sb];
    const int P = live ? a.nprim[sa] * kb : 0;
    double O[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) O[k] = 0.0;
    for (int q = g; q < P; q += RG) {
        const int ia = q / kb, ib = q - ia * kb;
        const double al = a.exps[oa + ia], be = a.exps[ob + ib];
        const double c = al + be, ic = 1.0 / c, rho = al * be * ic, T = rho * R2;
        const double qq = rho + a.omega, iq = 1.0 / qq;
        const double pre = a.w[oa + ia] * a.w[ob + ib] * PI_1_5 * ic * sqrt(ic) * (2.0 * PI) * iq *
                           exp(-a.omega * T * iq);
        const double e = -a.omega * rho * iq, f = -rho * rho * iq;
        double F[KHI + 1];
        boys<0, KHI>(rho * T * iq, a.tab, F);
        double pe[KHI + 1], pf[KHI + 1];
        pe[0] = pf[0] = 1.0;
#pragma unroll
        for (int k = 1; k <= KHI; ++k) {
            pe[k] = pe[k - 1] * e;
            pf[k] = pf[k - 1] * f;
        }
#pragma unroll
        for (int k = KLO; k <= KHI; ++k) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j <= k; ++j) s = fma(cbinom(k, j) * pe[k - j] * pf[j], F[j], s);
            O[k - KLO] = fma(pre, s, O[k - KLO]);
        }
    }
#pragma unroll
    for (int m = 1; m < RG; m <<= 1)
#pragma unroll
        for (int k = 0; k < NK; ++k) O[k] += __shfl_xor(O[k], m, RG);
    if (live && g == 0) {
        double *dst = a.T + (pos - a.start) * R2N_TSTRIDE;
#pragma unroll
        for (int k = 0; k < NK; ++k) dst[k] = O[k];
    }
}

template <int LA, int LB, bool D>
__global__ __launch_bounds__(RTPB) void k_gc_radial(R2nArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * RTPB + threadIdx.x;
    gc_pair<LA, LB, D>(a, t / RG, (int)(t % RG));
}

typedef void (*rad_fn)(hipStream_t, const R2nArgs &);

template <int LA, int LB, bool D>
void launch_r2n_radial(hipStream_t s, const R2nArgs &a)
{
    unsigned g = (unsigned)((a.count * RG + RTPB - 1) / RTPB);
    hipLaunchKernelGGL((k_r2n_radial<LA, LB, D>), dim3(g), dim3(RTPB), 0, s, a);
}

template <int LA, int LB, bool D>
void launch_gc_radial(hipStream_t s, const R2nArgs &a)
{
    unsigned g = (unsigned)((a.count * RG + RTPB - 1) / RTPB);
    hipLaunchKernelGGL((k_gc_radial<LA, LB, D>), dim3(g), dim3(RTPB), 0, s, a);
}

template <int... I>
const rad_fn *make_r2n_table(std::integer_sequence<int, I...>)
{
    // index (la * 5 + lb) * 2 + D
    static const rad_fn t[] = {&launch_r2n_radial<I / 10, (I / 2) % 5, (I % 2) == 1>...};
    return t;
}

template <int... I>
const rad_fn *make_gc_table(std::integer_sequence<int, I...>)
{
    static const rad_fn t[] = {&launch_gc_radial<I / 10, (I / 2) % 5, (I % 2) == 1>...};
    return t;
}

const rad_fn *r2n_table()
{
    static const rad_fn *t = make_r2n_table(std::make_integer_sequence<int, NCLASS * 2>{});
    return t;
}

const rad_fn *gc_table()
{
    static const rad_fn *t = make_gc_table(std::make_integer_sequence<int, NCLASS * 2>{});
    return t;
}

// binning, then per class and chunk the radial kernel of `rtab` and the tile
int monopole_pairs(shg_ctx *c, const char *what, const rad_fn *rtab, int nr, double omega, const shg_shells *sh,
                   const int32_t *pairs, int64_t n, const int64_t *out_off, double *out, double *dout)
{
    if (n < 0) return set_err(c, SHG_EINVAL, "%s: n < 0", what);
    if (n >= (int64_t)1 << 31) return set_err(c, SHG_EINVAL, "%s: n >= 2^31 pairs per call", what);
    int rc = check_shells(c, sh, what);
    if (rc) return rc;
    if (n == 0) return 0;
    if (!pairs || !out_off || !out) return set_err(c, SHG_EINVAL, "%s: NULL pointer argument", what);
    const bool deriv = dout != nullptr;
    const int D = deriv ? 1 : 0;
    if ((rc = grow(c, c->keys, c->keys_cap, (size_t)n))) return rc;
    if ((rc = grow(c, c->order, c->order_cap, (size_t)n))) return rc;
    const int64_t chunk = std::min<int64_t>(MONO_CHUNK, n);
    if ((rc = grow(c, c->Pbuf[0], c->Pbuf_cap[0], (size_t)(chunk * R2N_TSTRIDE)))) return rc;
    hipStream_t s = c->stream;
    int32_t *hist = c->bins, *cursor = c->bins + (NBINS_MAX + 1);
    hipLaunchKernelGGL(k_fill_i32, dim3((NBINS + 1 + 255) / 256), dim3(256), 0, s, hist, 0, NBINS + 1);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, c->err, 0, 1);
    if ((rc = prep_shells(c, sh, LMAX, c->w, c->w_cap))) return rc;
    const unsigned gb = (unsigned)((n + 256 * 16 - 1) / (256 * 16));
    hipLaunchKernelGGL(k_classify, dim3(gb), dim3(256), 0, s, n, pairs, sh->nshell, sh->l, sh->nprim, c->keys, hist,
                       c->err);
    hipLaunchKernelGGL(k_scan_bins, dim3(1), dim3(256), 0, s, hist, NBINS, cursor, cursor);
    HIP_TRY(c, hipMemcpyAsync(c->host_rb, cursor, (NBINS + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(c->host_rb + NBINS + 1, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_scatter, dim3(gb), dim3(256), 0, s, n, c->keys, cursor, c->order, nullptr, nullptr,
                       nullptr);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(s));
    if ((rc = decode_err(c, c->host_rb[NBINS + 1], what))) return rc;

    for (int la = 0; la <= LMAX; ++la)
        for (int lb = 0; lb <= LMAX; ++lb) {
            const int cls = la * (LMAX + 1) + lb;
            const int64_t b0 = c->host_rb[cls * 64], b1 = c->host_rb[(cls + 1) * 64];
            for (int64_t c0 = b0; c0 < b1; c0 += chunk) {
                const int64_t cn = std::min<int64_t>(chunk, b1 - c0);
                R2nArgs ra{pairs, c->order, sh->center, sh->nprim, sh->prim_off, sh->exps, c->w, c->Pbuf[0],
                           c0, cn, nr, omega, c->boys};
                rtab[cls * 2 + D](s, ra);
                TileArgs ta{};
                ta.order = c->order;
                ta.center = sh->center;
                ta.out = out;
                ta.dout = dout;
                ta.triples = pairs;
                ta.tstride = 2;
                ta.ooff = out_off;
                ta.P = c->Pbuf[0];
                ta.pstride = R2N_TSTRIDE;
                ta.poff = 0;
                ta.ybase = c0;
                tile_table(la)[lb * 2 + D](s, ta, c0, cn, TileShape{64, sched_rows(la, lb, deriv)});
            }
        }
    HIP_TRY(c, hipGetLastError());
    return 0;
}

}  // namespace

namespace shg {
void gc_radial_range(hipStream_t s, int cls, bool deriv, const shg_shells *sh, const int32_t *pairs,
                     const int32_t *order, const double *w, const double *tab, double omega, double *T, int64_t start,
                     int64_t count)
{
    R2nArgs ra{pairs, order, sh->center, sh->nprim, sh->prim_off, sh->exps, w, T + start * R2N_TSTRIDE,
               start, count, 0, omega, tab};
    gc_table()[cls * 2 + (deriv ? 1 : 0)](s, ra);
}

void r2n_radial_range(hipStream_t s, int cls, bool deriv, const shg_shells *sh, const int32_t *pairs,
                      const int32_t *order, const double *w, int nr, double *T, int64_t start, int64_t count)
{
    R2nArgs ra{pairs, order, sh->center, sh->nprim, sh->prim_off, sh->exps, w, T + start * R2N_TSTRIDE,
               start, count, nr, 0.0, nullptr};
    r2n_table()[cls * 2 + (deriv ? 1 : 0)](s, ra);
}

int gcoulomb_pairs(shg_ctx *c, const char *what, double omega, const shg_shells *sh, const int32_t *pairs, int64_t n,
                   const int64_t *out_off, double *out, double *dout)
{
    return monopole_pairs(c, what, gc_table(), 0, omega, sh, pairs, n, out_off, out, dout);
}
}  // namespace shg

extern "C" int shg_pairs_r2n(shg_ctx *c, const shg_shells *sh, int nr, const int32_t *pairs, int64_t n,
                             const int64_t *out_off, double *out, double *dout)
{
    const char *what = "shg_pairs_r2n";
    if (!c) return SHG_EINVAL;
    if (nr < 0 || nr > R2N_MAX) return set_err(c, SHG_EINVAL, "%s: n = %d outside [0, %d]", what, nr, R2N_MAX);
    return monopole_pairs(c, what, r2n_table(), nr, 0.0, sh, pairs, n, out_off, out, dout);
}
