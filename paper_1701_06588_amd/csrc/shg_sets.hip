// shg_sets.hip -- family basis sets (Sec. III): shg_set_pairs.
//
// Per call:
//   k_prep_set_funcs   validation; N_l and folded weights w = N_l c / (2 alpha)^l
//                      of every contracted function (one wave per set)
//   k_set_count        per set pair: validation, radial-scratch size, l-block
//                      items counted per bin (la, lb, na, nb) in LDS
//   k_scan_part/top/apply  set-pair offsets into the radial scratch; bin starts
//   k_set_scatter      item records in bin order (one global atomic per bin and
//                      workgroup)
//   k_set_radial       one wave per set pair: primitive radial terms for every
//                      primitive pair (orders up to the pair's largest),
//                      O^(k) = C_a^T G^(k) C_b one k at a time through LDS
//   k_setblk<la,lb,D>  per non-empty bin: the l-block elements (shg_sets.h)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "shg_ctx.h"
#include "shg_sets.h"

using namespace shg;

namespace {

constexpr int SET_NBIN = (LMAX + 1) * (LMAX + 1) * 81;   // (la, lb, na - 1, nb - 1), na, nb <= 9
constexpr int SET_TPB = 256;

__device__ __forceinline__ int set_bin(int la, int lb, int na, int nb)
{
    return ((la * (LMAX + 1) + lb) * 9 + na - 1) * 9 + nb - 1;
}

// validation of each set and the folded weights of its functions; one wave per set
__global__ void k_prep_set_funcs(shg_sets s, double *w, int32_t *err)
{
    const int si = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (si >= s.nset) return;
    const int K = s.nexp[si], nf = s.nfun[si];
    const int64_t e0 = s.exp_off[si], f0 = s.fun_off[si];
    if (K < 1 || K > SET_KMAX || e0 < 0 || e0 + K > s.nexp_total) {
        if (lane == 0) atomicOr(err, ERR_SHELL_K);
        return;
    }
    if (nf < 1 || nf > SET_FMAX || f0 < 0 || f0 + nf > s.nfun_total) {
        if (lane == 0) atomicOr(err, ERR_SET_FUN);
        return;
    }
    bool bad = false;
    for (int k = 0; k < K; ++k) {
        const double e = s.exps[e0 + k];
        bad |= !(e > 0.0) || !(e < 1e300);
    }
    if (bad) {
        if (lane == 0) atomicOr(err, ERR_SHELL_EXP);
        return;
    }
    int lprev = 0;
    for (int f = 0; f < nf; ++f) {
        const int l = s.fun_l[f0 + f];
        const int64_t co = s.coef_off[f0 + f];
        if (l < lprev || l > LMAX || co < 0 || co + K > s.ncoef_total) {
            if (lane == 0) atomicOr(err, l > LMAX || l < 0 ? ERR_SHELL_L : ERR_SET_FUN);
            return;
        }
        lprev = l;
    }
    for (int f = 0; f < nf; ++f) {
        const int l = s.fun_l[f0 + f];
        const int64_t co = s.coef_off[f0 + f];
        double t = 0.0;
        if (lane < K * K) {
            const int qa = lane / K, qb = lane - qa * K;
            t = shell_norm_term(l, s.exps[e0 + qa], s.exps[e0 + qb], s.coefs[co + qa], s.coefs[co + qb]);
        }
        for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
        if (lane < K) {
            const double N = shell_norm_from_sum(l, t);
            double a2 = 2.0 * s.exps[e0 + lane], p = 1.0;
            for (int q = 0; q < l; ++q) p *= a2;
            w[co + lane] = N * s.coefs[co + lane] / p;
        }
    }
}

// radial terms of one function with angular momentum l against every function of B
__device__ __forceinline__ int set_row_scratch(const shg_sets &s, int64_t fb0, int nfb, int l, int deriv)
{
    int t = 0;
    for (int j = 0; j < nfb; ++j) t += set_nk(l, s.fun_l[fb0 + j], deriv);
    return t;
}

// walks the l-block items of set pair (sa, sb) in a fixed order: A's functions
// grouped by l, then B's, each group cut into chunks of at most the bin's
// function counts; f(bin, fa, fb, row0, col0, o0, orow) per item, with o0 the
// offset of its first function pair in the set pair's radial terms and orow
// their row stride. The radial terms of a set pair are stored function pair
// by function pair, row-major over (fa, fb), set_nk orders each.
template <class F>
__device__ __forceinline__ void for_items(const shg_sets &s, int sa, int sb, int deriv, F &&f)
{
    const int64_t fa0 = s.fun_off[sa], fb0 = s.fun_off[sb];
    const int nfa = s.nfun[sa], nfb = s.nfun[sb];
    int row = 0;
    int64_t orow0 = 0;
    for (int ia = 0; ia < nfa;) {
        const int la = s.fun_l[fa0 + ia];
        int ja = ia;
        while (ja < nfa && s.fun_l[fa0 + ja] == la) ++ja;
        const int na_tot = ja - ia;
        const int srow = set_row_scratch(s, fb0, nfb, la, deriv);
        int col = 0;
        int64_t ocol = 0;
        for (int ib = 0; ib < nfb;) {
            const int lb = s.fun_l[fb0 + ib];
            int jb = ib;
            while (jb < nfb && s.fun_l[fb0 + jb] == lb) ++jb;
            const int nb_tot = jb - ib;
            const int nk = set_nk(la, lb, deriv);
            const int fpm = set_fp_max(la, lb, deriv != 0);
            const int nbc = min(nb_tot, fpm), nac = min(na_tot, max(1, fpm / nbc));
            for (int a0 = 0; a0 < na_tot; a0 += nac)
                for (int b0 = 0; b0 < nb_tot; b0 += nbc) {
                    const int na = min(nac, na_tot - a0), nb = min(nbc, nb_tot - b0);
                    f(set_bin(la, lb, na, nb), ia + a0, ib + b0, row + a0 * (2 * la + 1), col + b0 * (2 * lb + 1),
                      orow0 + (int64_t)a0 * srow + ocol + (int64_t)b0 * nk, srow);
                }
            col += nb_tot * (2 * lb + 1);
            ocol += (int64_t)nb_tot * nk;
            ib = jb;
        }
        row += na_tot * (2 * la + 1);
        orow0 += (int64_t)na_tot * srow;
        ia = ja;
    }
}

// per set pair: validation, radial-scratch size (set_nk doubles per function pair) and
// item counts per bin (LDS histogram, one global atomic per non-empty bin)
__global__ __launch_bounds__(SET_TPB) void k_set_count(int64_t n, const int32_t *sp, shg_sets s, int deriv,
                                                       int64_t *osz, int32_t *hist, int32_t *err)
{
    __shared__ int32_t lh[SET_NBIN];
    for (int b = threadIdx.x; b < SET_NBIN; b += SET_TPB) lh[b] = 0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * SET_TPB + threadIdx.x;
    if (p < n) {
        const int sa = sp[2 * p], sb = sp[2 * p + 1];
        if (sa < 0 || sa >= s.nset || sb < 0 || sb >= s.nset) {
            atomicOr(err, ERR_PAIR_INDEX);
            osz[p] = 0;
        } else {
            int64_t t = 0;
            for_items(s, sa, sb, deriv, [&](int bin, int, int, int, int, int64_t, int) { atomicAdd(&lh[bin], 1); });
            for (int fa = 0; fa < s.nfun[sa]; ++fa)
                t += set_row_scratch(s, s.fun_off[sb], s.nfun[sb], s.fun_l[s.fun_off[sa] + fa], deriv);
            osz[p] = t;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < SET_NBIN; b += SET_TPB)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// item records in bin order: counts per bin in LDS, one range per bin and
// workgroup reserved with a global atomic, then each item placed
__global__ __launch_bounds__(SET_TPB) void k_set_scatter(int64_t n, const int32_t *sp, shg_sets s, int deriv,
                                                         const int64_t *out_off, const int64_t *obase,
                                                         const int64_t *nsgf, int32_t *cursor, SetItem *items)
{
    __shared__ int32_t cnt[SET_NBIN];
    __shared__ int32_t gb[SET_NBIN];
    for (int b = threadIdx.x; b < SET_NBIN; b += SET_TPB) cnt[b] = 0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * SET_TPB + threadIdx.x;
    bool ok = false;
    int sa = 0, sb = 0;
    if (p < n) {
        sa = sp[2 * p];
        sb = sp[2 * p + 1];
        ok = sa >= 0 && sa < s.nset && sb >= 0 && sb < s.nset;
    }
    if (ok) for_items(s, sa, sb, deriv, [&](int bin, int, int, int, int, int64_t, int) { atomicAdd(&cnt[bin], 1); });
    __syncthreads();
    for (int b = threadIdx.x; b < SET_NBIN; b += SET_TPB) {
        if (cnt[b]) gb[b] = atomicAdd(&cursor[b], cnt[b]);
        cnt[b] = 0;
    }
    __syncthreads();
    if (ok) {
        const int ld = (int)nsgf[sb];
        const int64_t blk = nsgf[sa] * nsgf[sb];
        for_items(s, sa, sb, deriv, [&](int bin, int fa, int fb, int row0, int col0, int64_t o0, int orow) {
            const int32_t pos = gb[bin] + atomicAdd(&cnt[bin], 1);
            items[pos] = SetItem{sa, sb, fa, fb, row0, col0, ld, orow, out_off[p], obase[p] + o0, blk, 0};
        });
    }
}

// spherical functions per set
__global__ void k_set_nsgf(shg_sets s, int64_t *nsgf)
{
    const int si = blockIdx.x * blockDim.x + threadIdx.x;
    if (si >= s.nset) return;
    int64_t t = 0;
    const int nf = min(max(s.nfun[si], 0), SET_FMAX);
    for (int f = 0; f < nf; ++f) t += 2 * s.fun_l[s.fun_off[si] + f] + 1;
    nsgf[si] = t;
}

// exclusive scan of n int64 values (sizes of the set pairs' radial scratch),
// out[n] = total, in three launches: k_scan_part sums each chunk of
// SCAN_CHUNK values, k_scan_top scans the chunk sums in one workgroup, and
// k_scan_apply scans each chunk again from its start value
constexpr int SCAN_T = 256, SCAN_V = 8, SCAN_CHUNK = SCAN_T * SCAN_V;

// exclusive scan over the 256 threads of a workgroup (x = the thread's value);
// returns the thread's start, *total the sum
__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t *lds, int64_t *total)
{
    const int t = threadIdx.x;
    lds[t] = x;
    __syncthreads();
    for (int d = 1; d < SCAN_T; d <<= 1) {
        const int64_t v = t >= d ? lds[t - d] : 0;
        __syncthreads();
        lds[t] += v;
        __syncthreads();
    }
    const int64_t incl = lds[t];
    *total = lds[SCAN_T - 1];
    __syncthreads();
    return incl - x;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_part(int64_t n, const int64_t *in, int64_t *part)
{
    __shared__ int64_t lds[SCAN_T];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    int64_t x = 0;
    for (int v = 0; v < SCAN_V; ++v) {
        const int64_t i = base + (int64_t)v * SCAN_T + threadIdx.x;   // coalesced
        if (i < n) x += in[i];
    }
    int64_t tot;
    (void)block_excl_scan(x, lds, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// one workgroup: exclusive scan of the nblk chunk sums in place, total to *total_out
__global__ __launch_bounds__(SCAN_T) void k_scan_top(int64_t nblk, int64_t *part, int64_t *total_out)
{
    __shared__ int64_t lds[SCAN_T];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nblk; b0 += SCAN_T) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t x = i < nblk ? part[i] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(x, lds, &tot);
        if (i < nblk) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(int64_t n, const int64_t *in, const int64_t *part,
                                                       int64_t *out)
{
    __shared__ int64_t lds[SCAN_T];
    // each thread takes SCAN_V consecutive values of the chunk
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_V;
    int64_t v[SCAN_V], x = 0;
#pragma unroll
    for (int k = 0; k < SCAN_V; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        x += v[k];
    }
    int64_t tot;
    int64_t acc = part[blockIdx.x] + block_excl_scan(x, lds, &tot);
#pragma unroll
    for (int k = 0; k < SCAN_V; ++k) {
        if (base + k < n) out[base + k] = acc;
        acc += v[k];
    }
}

// one wave per set pair (a workgroup of its own, so the barriers below are
// the wave's): G^(k)[alpha][beta] of every primitive pair (a lane each) for
// k = 0..kmax, then per k T[alpha][fb] = sum_beta G^(k) w_b[fb][beta] and
// O^(k)[fa][fb] = sum_alpha w_a[fa][alpha] T[alpha][fb] for the function pairs
// that need this k (eq. O_rab2_deriv as C_a^T G C_b)
template <int K>
__device__ __forceinline__ void set_radial_k(int op, double ea, double eb, double R2, double omega, const double *tab,
                                             double *g)
{
    double gk[K + 1];
    radial_rt<0, K>(op, ea, eb, R2, omega, tab, gk);
#pragma unroll
    for (int k = 0; k <= K; ++k) g[k] = gk[k];
}

__global__ __launch_bounds__(64) void k_set_radial(int64_t n, const int32_t *sp, shg_sets s, const double *w, int op,
                                                   double omega, int deriv, const double *tab, const int64_t *obase,
                                                   double *O)
{
    __shared__ double sG[SET_KS][64];
    __shared__ double sT[SET_KMAX * SET_FMAX];
    __shared__ double sWa[SET_FMAX * SET_KMAX], sWb[SET_FMAX * SET_KMAX];
    __shared__ int sRow[SET_FMAX], sCol[LMAX + 1][SET_FMAX];   // radial-term offsets: row of fa, column of (l_a, fb)
    const int lane = threadIdx.x;
    const int64_t p = blockIdx.x;
    if (p >= n) return;   // uniform over the workgroup
    const int sa = sp[2 * p], sb = sp[2 * p + 1];
    const int ka = s.nexp[sa], kb = s.nexp[sb], nfa = s.nfun[sa], nfb = s.nfun[sb];
    const int64_t fa0 = s.fun_off[sa], fb0 = s.fun_off[sb], ea0 = s.exp_off[sa], eb0 = s.exp_off[sb];
    // functions are sorted by l: the last of each set has the largest
    const int kmax = s.fun_l[fa0 + nfa - 1] + s.fun_l[fb0 + nfb - 1] + (deriv ? 1 : 0);
    const double X0 = s.center[3 * sa] - s.center[3 * sb], X1 = s.center[3 * sa + 1] - s.center[3 * sb + 1],
                 X2 = s.center[3 * sa + 2] - s.center[3 * sb + 2];
    const double R2 = fma(X0, X0, fma(X1, X1, X2 * X2));
    if (lane < ka * kb) {
        const int ia = lane / kb, ib = lane - ia * kb;
        const double ea = s.exps[ea0 + ia], eb = s.exps[eb0 + ib];
        double g[SET_KS];
        switch (kmax) {   // only the orders this set pair needs
        case 0: set_radial_k<0>(op, ea, eb, R2, omega, tab, g); break;
        case 1: set_radial_k<1>(op, ea, eb, R2, omega, tab, g); break;
        case 2: set_radial_k<2>(op, ea, eb, R2, omega, tab, g); break;
        case 3: set_radial_k<3>(op, ea, eb, R2, omega, tab, g); break;
        case 4: set_radial_k<4>(op, ea, eb, R2, omega, tab, g); break;
        case 5: set_radial_k<5>(op, ea, eb, R2, omega, tab, g); break;
        case 6: set_radial_k<6>(op, ea, eb, R2, omega, tab, g); break;
        case 7: set_radial_k<7>(op, ea, eb, R2, omega, tab, g); break;
        case 8: set_radial_k<8>(op, ea, eb, R2, omega, tab, g); break;
        default: set_radial_k<9>(op, ea, eb, R2, omega, tab, g); break;
        }
        for (int k = 0; k <= kmax; ++k) sG[k][lane] = g[k];
    }
    for (int e = lane; e < nfa * ka; e += 64) {
        const int f = e / ka, q = e - f * ka;
        sWa[e] = w[s.coef_off[fa0 + f] + q];
    }
    for (int e = lane; e < nfb * kb; e += 64) {
        const int f = e / kb, q = e - f * kb;
        sWb[e] = w[s.coef_off[fb0 + f] + q];
    }
    if (lane <= LMAX) {
        int t = 0;
        for (int fb = 0; fb < nfb; ++fb) {
            sCol[lane][fb] = t;
            t += set_nk(lane, s.fun_l[fb0 + fb], deriv);
        }
        if (lane == 0) {   // rows: the running sum of each function's full row (its column total)
            int r = 0;
            for (int fa = 0; fa < nfa; ++fa) {
                sRow[fa] = r;
                r += set_row_scratch(s, fb0, nfb, s.fun_l[fa0 + fa], deriv);
            }
        }
    }
    __syncthreads();
    double *dst = O + obase[p];
    for (int k = 0; k <= kmax; ++k) {
        for (int e = lane; e < ka * nfb; e += 64) {
            const int ia = e / nfb, fb = e - ia * nfb;
            double t = 0.0;
            for (int ib = 0; ib < kb; ++ib) t = fma(sG[k][ia * kb + ib], sWb[fb * kb + ib], t);
            sT[e] = t;
        }
        __syncthreads();
        for (int e = lane; e < nfa * nfb; e += 64) {
            const int fa = e / nfb, fb = e - fa * nfb;
            const int la = s.fun_l[fa0 + fa], lb = s.fun_l[fb0 + fb];
            const int klo = la > lb ? la : lb;
            if (k >= klo && k <= la + lb + (deriv ? 1 : 0)) {
                double o = 0.0;
                for (int ia = 0; ia < ka; ++ia) o = fma(sWa[fa * ka + ia], sT[ia * nfb + fb], o);
                dst[sRow[fa] + sCol[la][fb] + (k - klo)] = o;
            }
        }
        __syncthreads();
    }
}

}  // namespace

extern "C" int shg_set_pairs(shg_ctx *c, const shg_sets *sets, shg_op op, double omega, const int32_t *set_pairs,
                             int64_t n, const int64_t *out_off, double *out, double *dout)
{
    const char *what = "shg_set_pairs";
    if (!c) return SHG_EINVAL;
    if ((int)op < 0 || (int)op > 4) return set_err(c, SHG_EINVAL, "%s: unknown operator %d", what, (int)op);
    if ((op == SHG_ERF || op == SHG_ERFC || op == SHG_GAUSS) && !(omega > 0.0 && omega < 1e300))
        return set_err(c, SHG_EINVAL, "%s: omega must be positive and finite for this operator", what);
    if (!sets) return set_err(c, SHG_EINVAL, "%s: set table is NULL", what);
    if (sets->nset < 0 || sets->nexp_total < 0 || sets->nfun_total < 0 || sets->ncoef_total < 0 || n < 0)
        return set_err(c, SHG_EINVAL, "%s: negative count", what);
    if (n >= (int64_t)1 << 31) return set_err(c, SHG_EINVAL, "%s: n >= 2^31 set pairs per call", what);
    if (n == 0) return 0;
    if (sets->nset > 0 && (!sets->center || !sets->nexp || !sets->exp_off || !sets->exps || !sets->nfun ||
                           !sets->fun_off || !sets->fun_l || !sets->coef_off || !sets->coefs))
        return set_err(c, SHG_EINVAL, "%s: NULL array in the set table", what);
    if (!set_pairs || !out_off || !out) return set_err(c, SHG_EINVAL, "%s: NULL pointer argument", what);
    const int deriv = dout ? 1 : 0;
    hipStream_t s = c->stream;
    int rc = 0;
    if ((rc = grow(c, c->set_w, c->set_w_cap, (size_t)sets->ncoef_total + 1))) return rc;
    // osz [n], obase [n + 1], then the scan's chunk sums
    if ((rc = grow(c, c->set_osz, c->set_osz_cap, (size_t)n * 2 + 2 + (size_t)(n / SCAN_CHUNK + 1)))) return rc;
    if ((rc = grow(c, c->set_nsgf, c->set_nsgf_cap, (size_t)sets->nset + 1))) return rc;
    int64_t *osz = c->set_osz, *obase = c->set_osz + n + 1;
    int32_t *hist = c->bins, *cursor = c->bins + (NBINS_MAX + 1);
    static_assert(SET_NBIN <= NBINS_MAX, "set bins fit the histogram");
    hipLaunchKernelGGL(k_fill_i32, dim3((SET_NBIN + 1 + 255) / 256), dim3(256), 0, s, hist, 0, SET_NBIN + 1);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, c->err, 0, 1);
    if (sets->nset > 0)
        hipLaunchKernelGGL(k_prep_set_funcs, dim3((sets->nset + 3) / 4), dim3(256), 0, s, *sets, c->set_w, c->err);
    // validation first: the item walk reads the function lists it checks
    HIP_TRY(c, hipMemcpyAsync(c->host_rb, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if ((rc = decode_err(c, c->host_rb[0], what))) return rc;
    if (sets->nset > 0)
        hipLaunchKernelGGL(k_set_nsgf, dim3((sets->nset + 255) / 256), dim3(256), 0, s, *sets, c->set_nsgf);
    const unsigned gb = (unsigned)((n + SET_TPB - 1) / SET_TPB);
    hipLaunchKernelGGL(k_set_count, dim3(gb), dim3(SET_TPB), 0, s, n, set_pairs, *sets, deriv, osz, hist, c->err);
    const int64_t nchunk = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    int64_t *part = obase + n + 1;   // nchunk values after the scan's n + 1
    hipLaunchKernelGGL(k_scan_part, dim3((unsigned)nchunk), dim3(SCAN_T), 0, s, n, osz, part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, s, nchunk, part, obase + n);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nchunk), dim3(SCAN_T), 0, s, n, osz, part, obase);
    hipLaunchKernelGGL(k_scan_bins, dim3(1), dim3(256), 0, s, hist, SET_NBIN, cursor, cursor);
    HIP_TRY(c, hipMemcpyAsync(c->host_rb, cursor, (SET_NBIN + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(c->host_rb + SET_NBIN + 1, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    int64_t o_total = 0;
    HIP_TRY(c, hipMemcpyAsync(&o_total, obase + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(s));
    if ((rc = decode_err(c, c->host_rb[SET_NBIN + 1], what))) return rc;
    std::vector<int32_t> starts(c->host_rb, c->host_rb + SET_NBIN + 1);
    const int64_t nitems = starts[SET_NBIN];
    if ((rc = grow(c, c->set_items, c->set_items_cap, (size_t)nitems + 1))) return rc;
    if ((rc = grow(c, c->set_O, c->set_O_cap, (size_t)o_total + 1))) return rc;
    hipLaunchKernelGGL(k_set_scatter, dim3(gb), dim3(SET_TPB), 0, s, n, set_pairs, *sets, deriv, out_off, obase,
                       c->set_nsgf, cursor, c->set_items);
    hipLaunchKernelGGL(k_set_radial, dim3((unsigned)n), dim3(64), 0, s, n, set_pairs, *sets, c->set_w, (int)op, omega,
                       deriv, c->boys, obase, c->set_O);
    SetBlkArgs ba{c->set_items, sets->center, c->set_O, out, dout, 1, 1};
    for (int la = 0; la <= LMAX; ++la)
        for (int lb = 0; lb <= LMAX; ++lb)
            for (int na = 1; na <= 9; ++na)
                for (int nb = 1; nb <= 9; ++nb) {
                    const int bin = ((la * (LMAX + 1) + lb) * 9 + na - 1) * 9 + nb - 1;
                    const int64_t b0 = starts[bin], b1 = starts[bin + 1];
                    if (b1 <= b0) continue;
                    ba.na = na;
                    ba.nb = nb;
                    setblk_table(la)[lb * 2 + deriv](s, ba, b0, b1 - b0);
                }
    HIP_TRY(c, hipGetLastError());
    return 0;
}
