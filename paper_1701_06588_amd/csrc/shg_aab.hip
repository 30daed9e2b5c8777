// shg_aab.hip -- three-index overlap (a b a~) (Sec. II.D) and its d/dR_A.
//
// Per call:
//   k_prep_shells     weights of the orbital and auxiliary shell tables
//   k_aab_classify    class key (la, la~, lb) per triple + validation; LDS histogram
//   k_scan_bins / k_scatter (shared with the two-center path)
//   per class, in chunks of at most ctx->aab_chunk triples (default 2^17), spread over
//   AAB_NSTREAM streams (own scratch each; fork/join with events on the
//   context stream, so the call stays ordered on it):
//     k_aab_radial    G lanes per triple: P^(k)_{La} for every La of the class from
//                     the primitive triples (eqs. Pa_aba, devsra2ms)
//     k_tile<La,lb,D> (three-index mode) the two-center blocks Y_La = (La Ma | lb mb)
//                     with P_La as contracted monopole (eq. final (a b a~) formula),
//                     into scratch
//     k_aab_gaunt     out[ma][ma~][mb] = sum_{La,Ma} G^{La,la,la~}_{Ma,ma,ma~} Y_La[Ma][mb]
//                     (real Gaunt coefficients, eq. CG_expansion), coalesced stores
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "gaunt_table.h"
#include "shg_ctx.h"

using namespace shg;

namespace {

constexpr int AAB_LA = 3, AAB_LT = 6, AAB_LB = 3;
constexpr int AAB_NCLASS = (AAB_LA + 1) * (AAB_LT + 1) * (AAB_LB + 1);
constexpr int AAB_PSTRIDE = 32;   // radial-term doubles per triple: at most 4 L_a values x 8 orders
constexpr int RAD_G = 8, RAD_TPB = 256;

__device__ __forceinline__ int aab_key(int la, int lt, int lb) { return (la * (AAB_LT + 1) + lt) * (AAB_LB + 1) + lb; }

__global__ __launch_bounds__(256) void k_aab_classify(int64_t n, const int32_t *tri, int norb, const double *oc,
                                                      const int32_t *ol, int naux, const double *xc,
                                                      const int32_t *xl, int32_t *keys, int32_t *hist, int32_t *err)
{
    __shared__ int32_t lh[AAB_NCLASS + 1];
    for (int b = threadIdx.x; b <= AAB_NCLASS; b += 256) lh[b] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * 256 * 16;
    int bad = 0;
    for (int it = 0; it < 16; ++it) {
        int64_t i = base + (int64_t)it * 256 + threadIdx.x;
        if (i >= n) break;
        int a = tri[3 * i], t = tri[3 * i + 1], b = tri[3 * i + 2];
        int key = AAB_NCLASS;
        if (a < 0 || a >= norb || t < 0 || t >= naux || b < 0 || b >= norb) {
            bad |= ERR_PAIR_INDEX;
        } else if (oc[3 * a] != xc[3 * t] || oc[3 * a + 1] != xc[3 * t + 1] || oc[3 * a + 2] != xc[3 * t + 2]) {
            bad |= ERR_AAB_CENTER;
        } else {
            int la = ol[a], lt = xl[t], lb = ol[b];
            if (la < 0 || la > AAB_LA || lt < 0 || lt > AAB_LT || lb < 0 || lb > AAB_LB)
                bad |= ERR_AAB_L;
            else
                key = aab_key(la, lt, lb);
        }
        keys[i] = key;
        atomicAdd(&lh[key], 1);
    }
    if (bad) atomicOr(err, bad);
    __syncthreads();
    for (int b = threadIdx.x; b <= AAB_NCLASS; b += 256)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

struct AabRadArgs {
    const int32_t *tri, *order;
    const double *oc;
    const int32_t *onp;
    const int64_t *ooff;
    const double *oexp, *ow;     // orbital exponents and weights N c / (2 alpha)^l
    const int32_t *xnp;
    const int64_t *xoff;
    const double *xexp, *xw;     // auxiliary exponents and weights
    double *P;                   // [L_a index][pos - pbase][8]: each L_a tile reads one contiguous slab
    int64_t pbase, start, count;
};

// G lanes per triple; lane g takes primitive triples q = g, g+G, ...; xor butterfly
template <int LA, int LT, int LB, bool D>
__global__ __launch_bounds__(RAD_TPB) void k_aab_radial(AabRadArgs a)
{
    using AK = AabK<LA, LT, LB, D>;
    const int64_t t = (int64_t)blockIdx.x * RAD_TPB + threadIdx.x;
    const int64_t slot = t / RAD_G;
    const int g = (int)(t % RAD_G);
    const bool live = slot < a.count;
    const int64_t pos = a.start + (live ? slot : 0);
    const int p = a.order[pos];
    const int sa = a.tri[3 * (int64_t)p], st = a.tri[3 * (int64_t)p + 1], sb = a.tri[3 * (int64_t)p + 2];
    const double X0 = a.oc[3 * sa] - a.oc[3 * sb], X1 = a.oc[3 * sa + 1] - a.oc[3 * sb + 1],
                 X2 = a.oc[3 * sa + 2] - a.oc[3 * sb + 2];
    const double R2 = X0 * X0 + X1 * X1 + X2 * X2;
    const int ka = a.onp[sa], kt = a.xnp[st], kb = a.onp[sb];
    const int64_t oa = a.ooff[sa], ot = a.xoff[st], ob = a.ooff[sb];
    const int NP = live ? ka * kt * kb : 0;
    double P[AK::NLA][8];
#pragma unroll
    for (int i = 0; i < AK::NLA; ++i)
#pragma unroll
        for (int k = 0; k < 8; ++k) P[i][k] = 0.0;
    // the triple's primitive data staged once in LDS (lane g loads primitive g of
    // each shell, K <= KMAX < RAD_G, all loads independent): exponents, and the
    // weights with the a and a~ weights' (2 alpha)^l factors taken out
    __shared__ double sE[3][RAD_TPB / RAD_G][KMAX], sW[3][RAD_TPB / RAD_G][KMAX];
    static_assert(KMAX <= RAD_G, "one primitive per lane");
    const int ls = threadIdx.x / RAD_G;
    if (live) {
        if (g < ka) {
            const double e = a.oexp[oa + g];
            double f = a.ow[oa + g];
#pragma unroll
            for (int k = 0; k < LA; ++k) f *= 2.0 * e;
            sE[0][ls][g] = e;
            sW[0][ls][g] = f;
        }
        if (g < kt) {
            const double e = a.xexp[ot + g];
            double f = a.xw[ot + g];
#pragma unroll
            for (int k = 0; k < LT; ++k) f *= 2.0 * e;
            sE[1][ls][g] = e;
            sW[1][ls][g] = f;
        }
        if (g < kb) {
            sE[2][ls][g] = a.oexp[ob + g];
            sW[2][ls][g] = a.ow[ob + g];
        }
    }
    __syncthreads();
    for (int q = g; q < NP; q += RAD_G) {
        const int ib = q % kb, r = q / kb, it = r % kt, ia = r / kt;
        aab_accumulate<LA, LT, LB, D>(sE[0][ls][ia] + sE[1][ls][it], sE[2][ls][ib], R2,
                                      sW[0][ls][ia] * sW[1][ls][it] * sW[2][ls][ib], P);
    }
#pragma unroll
    for (int m = 1; m < RAD_G; m <<= 1)
#pragma unroll
        for (int i = 0; i < AK::NLA; ++i)
#pragma unroll
            for (int k = 0; k < 8; ++k) P[i][k] += __shfl_xor(P[i][k], m, RAD_G);
    if (live && g == 0) {
#pragma unroll
        for (int i = 0; i < AK::NLA; ++i) {
            double *dst = a.P + ((int64_t)i * a.count + (pos - a.pbase)) * 8;
#pragma unroll
            for (int k = 0; k < 8; ++k) dst[k] = P[i][k];
        }
    }
}

typedef void (*aab_rad_fn)(hipStream_t, const AabRadArgs &);

template <int LA, int LT, int LB, bool D>
void launch_aab_radial(hipStream_t s, const AabRadArgs &a)
{
    unsigned g = (unsigned)((a.count * RAD_G + RAD_TPB - 1) / RAD_TPB);
    hipLaunchKernelGGL((k_aab_radial<LA, LT, LB, D>), dim3(g), dim3(RAD_TPB), 0, s, a);
}

template <int... I>
const aab_rad_fn *make_rad_table(std::integer_sequence<int, I...>)
{
    // index ((la * 7 + lt) * 4 + lb) * 2 + D
    static const aab_rad_fn t[] = {&launch_aab_radial<I / 56, (I / 8) % 7, (I / 2) % 4, (I % 2) == 1>...};
    return t;
}

const aab_rad_fn *rad_table()
{
    static const aab_rad_fn *t = make_rad_table(std::make_integer_sequence<int, AAB_NCLASS * 2>{});
    return t;
}

struct GauntArgs {
    const int32_t *order;
    const int64_t *out_off;
    const int32_t *gidx;    // {start, count} per (ma, mt) of the class's (la, lt)
    const int32_t *glm;     // {L, M}
    const double *gg;
    const double *Yv, *Yd;
    double *out, *dout;
    int64_t start, count, ys;
    int la, lt, lb, nc, lamin;
};

// A group is GQ triples; a pass is one group and one component (value or one
// of x, y, z). Each workgroup stages the class's Gaunt lists (at most 2 terms
// per L_a value) in LDS once and then runs passes: it stages the pass's Y
// blocks (every L_a of the class) and computes out[ma][mt][mb] = sum over the
// list of (ma, mt) of G * Y_L[M][mb], a thread per (triple, ma, mt) row of NB
// values. The class is a template parameter so that all index arithmetic is by
// constants.
constexpr int GQ = 8;
constexpr int GAUNT_GRID = 2048;   // workgroups per launch at most (eight per CU)

template <int LA, int LT, int LB, int NC>
__global__ __launch_bounds__(256) void k_aab_gaunt(GauntArgs a)
{
    constexpr int NA = 2 * LA + 1, NT = 2 * LT + 1, NB = 2 * LB + 1, NAT = NA * NT, SZ = NAT * NB;
    constexpr int LAMIN = LA > LT ? LA - LT : LT - LA, NLA = (LA + LT - LAMIN) / 2 + 1, GMAX = NAT * 2 * NLA;
    // offset of the L_a block with index n (L_a = LAMIN + 2n) in a triple's Y: sum of (2L'+1) NB, L' < L_a
    constexpr auto loffc = [](int n) constexpr { return NB * (n * (2 * LAMIN + 1) + 2 * n * (n - 1)); };
    constexpr int YS = loffc(NLA), NIT = (GQ * YS + 255) / 256;
    __shared__ int2 s_idx[NAT];
    __shared__ int2 s_lm[GMAX];
    __shared__ double s_g[GMAX];
    __shared__ double sY[GQ * YS];
    __shared__ int64_t s_off[GQ];
    const int tid = threadIdx.x;
    const int2 *gidx = (const int2 *)a.gidx;
    const int g0 = gidx[0].x;
    const int gn = min(GMAX, gidx[NAT - 1].x + gidx[NAT - 1].y - g0);   // lists are contiguous in (ma, mt)
    for (int t = tid; t < NAT; t += 256) {
        const int2 e = gidx[t];
        s_idx[t] = make_int2(e.x - g0, e.y);
    }
    for (int t = tid; t < gn; t += 256) {
        s_lm[t] = ((const int2 *)a.glm)[g0 + t];
        s_g[t] = a.gg[g0 + t];
    }
    // a workgroup takes groups blockIdx.x, blockIdx.x + gridDim.x, ... and runs
    // the NC components of each group as consecutive passes: the derivative
    // components of a Y row are adjacent segments that share cache lines at
    // their edges, so a line fetched for one pass is still in this CU's L2 for
    // the next, and the group's output rows are written from one XCD
    const int64_t ngt = (a.count + GQ - 1) / GQ;
    // a pass's Y values (NIT per thread) and output offsets are loaded into
    // registers one pass ahead: their loads are in flight while the previous
    // pass's rows are computed and stored
    double yv[NIT];
    int64_t offv = 0;
    const auto load_pass = [&](int64_t g, int c) {
        const int64_t q0 = g * GQ;
        const int nq = (int)min((int64_t)GQ, a.count - q0);
        if (tid < nq) offv = a.out_off[a.order[a.start + q0 + tid]];
        // the group's Y values sit in one window of Yv (c = 0) or Yd: a uniform
        // base and 32-bit offsets (a triple's Y stride is YS)
        const double *base = c == 0 ? a.Yv + q0 * YS : a.Yd + 3 * q0 * YS;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int t = tid + it * 256;
            if (t < nq * YS) {
                const int ql = t / YS, r = t - ql * YS;
                int nL = 0;
#pragma unroll
                for (int n = 1; n < NLA; ++n) nL += r >= loffc(n) ? 1 : 0;
                const int L = LAMIN + 2 * nL;
                const int o = c == 0 ? t : 3 * ql * YS + 3 * loffc(nL) + (c - 1) * (2 * L + 1) * NB + (r - loffc(nL));
                yv[it] = base[o];
            }
        }
    };
    int64_t g = blockIdx.x;
    int c = 0;
    if (g < ngt) load_pass(g, 0);
    while (g < ngt) {
        const int64_t q0 = g * GQ;
        const int nq = (int)min((int64_t)GQ, a.count - q0);
        __syncthreads();   // the previous pass's rows are written (and the lists staged)
        if (tid < nq) s_off[tid] = offv;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int t = tid + it * 256;
            if (t < nq * YS) sY[t] = yv[it];
        }
        __syncthreads();
        int64_t gnext = g;
        int cnext = c + 1;
        if (cnext == NC) {
            cnext = 0;
            gnext += gridDim.x;
        }
        if (gnext < ngt) load_pass(gnext, cnext);
        // a thread takes one (triple, ma, mt) row: all NB values of mb at once, so
        // each Gaunt term's coefficient and (L, M) are read once for NB products;
        // consecutive threads write consecutive rows (contiguous stores)
        for (int e = tid; e < nq * NAT; e += 256) {
            const int ql = e / NAT, amt = e - ql * NAT;
            const int2 se = s_idx[amt];
            const double *y = sY + ql * YS;
            double v[NB];
#pragma unroll
            for (int mb = 0; mb < NB; ++mb) v[mb] = 0.0;
            for (int k = se.x; k < se.x + se.y && k < gn; ++k) {
                const int L = s_lm[k].x, M = s_lm[k].y;
                const double g = s_g[k];
                const int n = (L - LAMIN) / 2;
                const double *yl = y + NB * (n * (2 * LAMIN + 1) + 2 * n * (n - 1)) + (M + L) * NB;
#pragma unroll
                for (int mb = 0; mb < NB; ++mb) v[mb] = fma(g, yl[mb], v[mb]);
            }
            const int64_t off = s_off[ql];
            double *dst = c == 0 ? a.out + off + amt * NB : a.dout + 3 * off + (int64_t)(c - 1) * SZ + amt * NB;
#pragma unroll
            for (int mb = 0; mb < NB; ++mb) dst[mb] = v[mb];
        }
        g = gnext;
        c = cnext;
    }
}

typedef void (*gaunt_fn)(hipStream_t, unsigned grid, const GauntArgs &);

template <int LA, int LT, int LB, int NC>
void launch_gaunt(hipStream_t s, unsigned grid, const GauntArgs &a)
{
    hipLaunchKernelGGL((k_aab_gaunt<LA, LT, LB, NC>), dim3(grid), dim3(256), 0, s, a);
}

template <int... I>
const gaunt_fn *make_gaunt_table(std::integer_sequence<int, I...>)
{
    // index ((la * 7 + lt) * 4 + lb) * 2 + D
    static const gaunt_fn t[] = {&launch_gaunt<I / 56, (I / 8) % 7, (I / 2) % 4, (I % 2) ? 4 : 1>...};
    return t;
}

const gaunt_fn *gaunt_table()
{
    static const gaunt_fn *t = make_gaunt_table(std::make_integer_sequence<int, AAB_NCLASS * 2>{});
    return t;
}

int upload_gaunt(shg_ctx *c)
{
    if (c->gaunt_idx) return 0;
    GauntTable G = build_gaunt_table(AAB_LA, AAB_LT);
    std::vector<int32_t> idx, lm;
    std::vector<double> gg;
    const int maxmm = (2 * AAB_LA + 1) * (2 * AAB_LT + 1);
    idx.assign((size_t)(AAB_LA + 1) * (AAB_LT + 1) * maxmm * 2, 0);
    for (int la = 0; la <= AAB_LA; ++la)
        for (int lt = 0; lt <= AAB_LT; ++lt)
            for (int ma = -la; ma <= la; ++ma)
                for (int mt = -lt; mt <= lt; ++mt) {
                    const auto &ent = G.at(la, lt, ma, mt);
                    if ((int)ent.size() > 2 * ((la < lt ? la : lt) + 1))
                        return set_err(c, SHG_EDEVICE, "shg_aab: Gaunt list longer than two terms per L");
                    size_t slot = ((size_t)(la * (AAB_LT + 1) + lt) * maxmm + (ma + la) * (2 * lt + 1) + (mt + lt)) * 2;
                    idx[slot] = (int32_t)gg.size();
                    idx[slot + 1] = (int32_t)ent.size();
                    for (const auto &e : ent) {
                        lm.push_back(e.L);
                        lm.push_back(e.M);
                        gg.push_back(e.g);
                    }
                }
    HIP_TRY(c, hipMalloc((void **)&c->gaunt_idx, idx.size() * sizeof(int32_t)));
    HIP_TRY(c, hipMalloc((void **)&c->gaunt_lm, lm.size() * sizeof(int32_t)));
    HIP_TRY(c, hipMalloc((void **)&c->gaunt_g, gg.size() * sizeof(double)));
    HIP_TRY(c, hipMemcpy(c->gaunt_idx, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->gaunt_lm, lm.data(), lm.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->gaunt_g, gg.data(), gg.size() * sizeof(double), hipMemcpyHostToDevice));
    return 0;
}

}  // namespace

extern "C" int shg_aab(shg_ctx *c, const shg_shells *orb, const shg_shells *aux, const int32_t *triples, int64_t n,
                       const int64_t *out_off, double *out, double *dout)
{
    const char *what = "shg_aab";
    if (!c) return SHG_EINVAL;
    if (n < 0) return set_err(c, SHG_EINVAL, "%s: n < 0", what);
    if (n >= (int64_t)1 << 31) return set_err(c, SHG_EINVAL, "%s: n >= 2^31 triples per call", what);
    int rc = check_shells(c, orb, what);
    if (!rc) rc = check_shells(c, aux, what);
    if (rc) return rc;
    if (n == 0) return 0;
    if (!triples || !out_off || !out) return set_err(c, SHG_EINVAL, "%s: NULL pointer argument", what);
    if ((rc = upload_gaunt(c))) return rc;
    const bool deriv = dout != nullptr;
    const int D = deriv ? 1 : 0, NC = deriv ? 4 : 1;
    hipStream_t s = c->stream;
    if ((rc = grow(c, c->keys, c->keys_cap, (size_t)n))) return rc;
    if ((rc = grow(c, c->order, c->order_cap, (size_t)n))) return rc;
    int32_t *hist = c->bins, *cursor = c->bins + (NBINS_MAX + 1);
    hipLaunchKernelGGL(k_fill_i32, dim3((AAB_NCLASS + 1 + 255) / 256), dim3(256), 0, s, hist, 0, AAB_NCLASS + 1);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, c->err, 0, 1);
    if ((rc = prep_shells(c, orb, AAB_LA, c->w, c->w_cap))) return rc;
    if ((rc = prep_shells(c, aux, AAB_LT, c->w2, c->w2_cap))) return rc;
    unsigned gb = (unsigned)((n + 256 * 16 - 1) / (256 * 16));
    hipLaunchKernelGGL(k_aab_classify, dim3(gb), dim3(256), 0, s, n, triples, orb->nshell, orb->center, orb->l,
                       aux->nshell, aux->center, aux->l, c->keys, hist, c->err);
    hipLaunchKernelGGL(k_scan_bins, dim3(1), dim3(256), 0, s, hist, AAB_NCLASS, cursor, cursor);
    HIP_TRY(c, hipMemcpyAsync(c->host_rb, cursor, (AAB_NCLASS + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(c->host_rb + AAB_NCLASS + 1, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_scatter, dim3(gb), dim3(256), 0, s, n, c->keys, cursor, c->order, nullptr, nullptr,
                       nullptr);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(s));
    if ((rc = decode_err(c, c->host_rb[AAB_NCLASS + 1], what))) return rc;
    std::vector<int32_t> starts(c->host_rb, c->host_rb + AAB_NCLASS + 1);

    // work items (class, chunk); the host work below (sizes, layout checks,
    // scratch growth) ends before the fork, so no error return leaves a side
    // stream un-joined
    struct Item {
        int key, la, lt, lb, lamin, lamax, w;
        int64_t c0, cn, ys;
        double cost;
    };
    std::vector<Item> items;
    for (int la = 0; la <= AAB_LA; ++la)
        for (int lt = 0; lt <= AAB_LT; ++lt)
            for (int lb = 0; lb <= AAB_LB; ++lb) {
                const int key = (la * (AAB_LT + 1) + lt) * (AAB_LB + 1) + lb;
                const int64_t b0 = starts[key], b1 = starts[key + 1];
                if (b1 <= b0) continue;
                const int lamin = la > lt ? la - lt : lt - la, lamax = la + lt, NB = 2 * lb + 1;
                int64_t ys = 0;
                for (int L = lamin; L <= lamax; L += 2) ys += (int64_t)(2 * L + 1) * NB;
                if (ys != (int64_t)NB * (((lamax - lamin) / 2 + 1) * (2 * lamin + 1) +
                                         2 * ((lamax - lamin) / 2 + 1) * ((lamax - lamin) / 2)))
                    return set_err(c, SHG_EDEVICE, "shg_aab: inconsistent Y block layout");
                for (int64_t c0 = b0; c0 < b1; c0 += c->aab_chunk) {
                    const int64_t cn = std::min<int64_t>(c->aab_chunk, b1 - c0);
                    // Y blocks written and read, output blocks written
                    const double cost = (double)cn * NC * (double)(ys + (2 * la + 1) * (2 * lt + 1) * NB);
                    items.push_back({key, la, lt, lb, lamin, lamax, 0, c0, cn, ys, cost});
                }
            }
    // largest first onto the least loaded stream
    std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
    const int nw = (int)std::min<size_t>(AAB_NSTREAM, items.size());
    double load[AAB_NSTREAM] = {};
    int64_t need_p[AAB_NSTREAM] = {}, need_y[AAB_NSTREAM] = {};
    for (Item &it : items) {
        int w = 0;
        for (int v = 1; v < nw; ++v)
            if (load[v] < load[w]) w = v;
        it.w = w;
        load[w] += it.cost;
        need_p[w] = std::max<int64_t>(need_p[w], it.cn * AAB_PSTRIDE);
        need_y[w] = std::max<int64_t>(need_y[w], it.cn * it.ys);
    }
    for (int w = 0; w < nw; ++w) {
        if ((rc = grow(c, c->Pbuf[w], c->Pbuf_cap[w], (size_t)need_p[w]))) return rc;
        if ((rc = grow(c, c->Yv[w], c->Yv_cap[w], (size_t)need_y[w]))) return rc;
        if (deriv && (rc = grow(c, c->Yd[w], c->Yd_cap[w], (size_t)(3 * need_y[w])))) return rc;
        if (!c->aab_ev[w]) HIP_TRY(c, hipEventCreateWithFlags(&c->aab_ev[w], hipEventDisableTiming));
        if (w > 0 && !c->aab_side[w - 1])
            HIP_TRY(c, hipStreamCreateWithFlags(&c->aab_side[w - 1], hipStreamNonBlocking));
    }
    hipStream_t ws[AAB_NSTREAM] = {s};
    for (int w = 1; w < nw; ++w) ws[w] = c->aab_side[w - 1];
    // fork: the side streams start after the binning on the context stream
    if (nw > 1) {
        HIP_TRY(c, hipEventRecord(c->aab_ev[0], s));
        for (int w = 1; w < nw; ++w) HIP_TRY(c, hipStreamWaitEvent(ws[w], c->aab_ev[0], 0));
    }
    const aab_rad_fn *rtab = rad_table();
    const int maxmm = (2 * AAB_LA + 1) * (2 * AAB_LT + 1);
    hipError_t first = hipSuccess;
    for (const Item &it : items) {
        hipStream_t sw = ws[it.w];
        const int NB = 2 * it.lb + 1;
        AabRadArgs ra{triples, c->order, orb->center, orb->nprim, orb->prim_off, orb->exps, c->w,
                      aux->nprim, aux->prim_off, aux->exps, c->w2, c->Pbuf[it.w], it.c0, it.c0, it.cn};
        rtab[it.key * 2 + D](sw, ra);
        int64_t loff = 0;
        for (int L = it.lamin, iL = 0; L <= it.lamax; L += 2, ++iL) {
            TileArgs ta{};
            ta.order = c->order;
            ta.center = orb->center;
            ta.out = c->Yv[it.w];
            ta.dout = deriv ? c->Yd[it.w] : nullptr;
            ta.triples = triples;
            ta.tstride = 3;
            ta.P = c->Pbuf[it.w];
            ta.pstride = 8;                    // P is [L_a index][triple][8]
            ta.poff = (int)(iL * 8 * it.cn);
            ta.ybase = it.c0;
            ta.ys = it.ys;
            ta.yoff = loff;
            TileShape shp{64, sched_rows(L, it.lb, deriv)};
            tile_table(L)[it.lb * 2 + D](sw, ta, it.c0, it.cn, shp);
            loff += (int64_t)(2 * L + 1) * NB;
        }
        GauntArgs ga{c->order, out_off, c->gaunt_idx + (size_t)(it.la * (AAB_LT + 1) + it.lt) * maxmm * 2,
                     c->gaunt_lm, c->gaunt_g, c->Yv[it.w], deriv ? c->Yd[it.w] : nullptr, out, dout, it.c0, it.cn,
                     it.ys, it.la, it.lt, it.lb, NC, it.lamin};
        const int64_t groups = (it.cn + GQ - 1) / GQ;
        gaunt_table()[it.key * 2 + D](sw, (unsigned)std::min<int64_t>(groups, GAUNT_GRID), ga);
        const hipError_t e = hipGetLastError();
        if (first == hipSuccess) first = e;
    }
    // join: the context stream continues after every side stream's work
    for (int w = 1; w < nw; ++w) {
        const hipError_t e1 = hipEventRecord(c->aab_ev[w], ws[w]);
        const hipError_t e2 = hipStreamWaitEvent(s, c->aab_ev[w], 0);
        if (first == hipSuccess) first = e1 != hipSuccess ? e1 : e2;
    }
    if (first != hipSuccess) return set_err(c, SHG_EDEVICE, "%s: launch failed: %s", what, hipGetErrorString(first));
    HIP_TRY(c, hipGetLastError());
    return 0;
}

extern "C" int shg_set_aab_chunk(shg_ctx *c, int64_t chunk)
{
    if (!c) return SHG_EINVAL;
    if (chunk < 1 || chunk > ((int64_t)1 << 24))
        return set_err(c, SHG_EINVAL, "shg_set_aab_chunk: chunk must be in [1, 2^24]");
    c->aab_chunk = chunk;
    return 0;
}
