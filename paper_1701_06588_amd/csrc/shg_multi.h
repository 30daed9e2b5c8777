// shg_multi.h -- persistent kernel evaluating several operators on one pair
// list in a single pass.
//
// The angular factors of a block element (the Qhat sums of eq.
// final_r12int_ab and of the derivative recurrences) depend on X = R_a - R_b
// only, not on the operator; the operator enters through the contracted
// radial terms O^(k) (eq. O_rab2_deriv). A tile of 64 pairs therefore
//   phase 1  contracts O^(k) of every operator (4 lanes per pair, butterfly),
//            reading each primitive pair's exponents and weights once
//   phase 2  lanes = pairs, waves take fixed shares of the elements; per
//            element the operator-independent terms are formed once and
//            combined with each operator's O^(k) (elem_terms / elem_apply, the
//            same floating-point order as the single-operator path, so blocks
//            are bitwise those of shg_pairs_deriv), and stored straight to
//            every operator's output
// One barrier after phase 1 and one at the end of a tile; tiles come from the
// plan's tile queue through an atomic counter, the next index
// requested at tile start and handed over through LDS after phase 1.
#pragma once
#include "shg_kernels.h"
#include "shg_persist.h"

namespace shg {

constexpr int MULTI_MAX = 5;

struct MultiOps {
    int nops;
    int op[MULTI_MAX];
    double omega[MULTI_MAX];
    double *out[MULTI_MAX];
    double *dout[MULTI_MAX];
};

// per pair in LDS: O^(k) of every operator (stride NK), then X
constexpr int MULTI_SO = MULTI_MAX * 6 + 3;   // 33 doubles (odd: conflict-free)

template <int LA, int LB, bool D, int L, int NK>
__device__ __forceinline__ void reg_fence_multi(RTab<L> &R, double (&O)[MULTI_MAX][NK], double (&X)[3])
{
    static_for<0, L + 1>([&](auto LL) {
        constexpr int l = decltype(LL)::value;
        if constexpr (row_used(l, LA, LB, D)) {
#pragma unroll
            for (int m = 0; m <= l; ++m) asm volatile("" : "+v"(R.c[ridx(l, m)]));
#pragma unroll
            for (int m = 1; m <= l; ++m) asm volatile("" : "+v"(R.s[ridx(l, m)]));
        }
    });
#pragma unroll
    for (int o = 0; o < MULTI_MAX; ++o)
#pragma unroll
        for (int k = 0; k < NK; ++k) asm volatile("" : "+v"(O[o][k]));
    asm volatile("" : "+v"(X[0]), "+v"(X[1]), "+v"(X[2]));
}

template <int LA, int LB, bool D, class Hook>
__device__ __forceinline__ void tile_multi(const TileArgs &a, const MultiOps &m, int64_t tstart, int tcount,
                                           double *sO, int64_t *sOff, const Hook &after_p1)
{
    using PK = PairK<LA, LB, D>;
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, SZ = NA * NB, NC = D ? 4 : 1, NK = PK::NK;
    const int tid = threadIdx.x;
    const int nops = m.nops;

    // ---- phase 1: every operator's O^(k), 4 lanes per pair ----
    {
        constexpr int G = 4;
        const int i = tid / G, g = tid % G;
        const bool live = i < tcount;
        const PairRec rc = a.rec[tstart + (live ? i : 0)];
        const int sa = rc.a, sb = rc.b;
        const double X0 = a.center[3 * sa] - a.center[3 * sb];
        const double X1 = a.center[3 * sa + 1] - a.center[3 * sb + 1];
        const double X2 = a.center[3 * sa + 2] - a.center[3 * sb + 2];
        const double R2 = fma(X0, X0, fma(X1, X1, X2 * X2));   // fixed rounding order
        const int64_t oa = a.prim_off[sa], ob = a.prim_off[sb];
        const int kb = a.nprim[sb];
        const int P = live ? a.nprim[sa] * kb : 0;
        double O[MULTI_MAX][NK];
#pragma unroll
        for (int o = 0; o < MULTI_MAX; ++o)
#pragma unroll
            for (int k = 0; k < NK; ++k) O[o][k] = 0.0;
        for (int q = g; q < P; q += G) {
            const int ia = q / kb, ib = q - ia * kb;
            const double ea = a.exps[oa + ia], eb = a.exps[ob + ib];
            const double ww = a.w[oa + ia] * a.w[ob + ib];
#pragma unroll
            for (int o = 0; o < MULTI_MAX; ++o) {
                if (o < nops) {
                    double gk[NK];
                    radial_rt<PK::KLO, PK::KHI>(m.op[o], ea, eb, R2, m.omega[o], a.tab, gk);
#pragma unroll
                    for (int k = 0; k < NK; ++k) O[o][k] = fma(ww, gk[k], O[o][k]);
                }
            }
        }
        for (int s = 1; s < G; s <<= 1)
#pragma unroll
            for (int o = 0; o < MULTI_MAX; ++o)
                if (o < nops)
#pragma unroll
                    for (int k = 0; k < NK; ++k) O[o][k] += __shfl_xor(O[o][k], s, G);
        if (live && g == 0) {
#pragma unroll
            for (int o = 0; o < MULTI_MAX; ++o)
                if (o < nops)
#pragma unroll
                    for (int k = 0; k < NK; ++k) sO[i * MULTI_SO + o * NK + k] = O[o][k];
            sO[i * MULTI_SO + MULTI_MAX * 6] = X0;
            sO[i * MULTI_SO + MULTI_MAX * 6 + 1] = X1;
            sO[i * MULTI_SO + MULTI_MAX * 6 + 2] = X2;
            sOff[i] = rc.off;
        }
    }
    after_p1();
    __syncthreads();

    // ---- phase 2: lanes = pairs, wave w takes the elements E with E % 4 == w ----
    const int lane = tid & 63, wave = tid >> 6;
    const bool live = lane < tcount;
    double X[3], O[MULTI_MAX][NK];
    const int il = live ? lane : 0;
#pragma unroll
    for (int o = 0; o < MULTI_MAX; ++o)
#pragma unroll
        for (int k = 0; k < NK; ++k) O[o][k] = (live && o < nops) ? sO[il * MULTI_SO + o * NK + k] : 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) X[d] = live ? sO[il * MULTI_SO + MULTI_MAX * 6 + d] : 0.0;
    const int64_t off = live ? sOff[il] : 0;
    RTab<cmax(LA, LB)> R;
    solid_R<cmax(LA, LB)>(X[0], X[1], X[2], R);
    const auto run = [&](auto WW) {
        constexpr int W = decltype(WW)::value;
        static_for<0, SZ>([&](auto EE) {
            constexpr int E = decltype(EE)::value;
            if constexpr (E % 4 == W) {
                reg_fence_multi<LA, LB, D>(R, O, X);
                ElemTerms<LA, LB, D> T;
                elem_terms<LA, LB, E / NB, E % NB, D>(R, T);
#pragma unroll
                for (int o = 0; o < MULTI_MAX; ++o) {
                    if (o < nops) {
                        double res[NC];
                        elem_apply<LA, LB, E / NB, E % NB, D>(T, O[o], X, res);
                        if (live) {
                            m.out[o][off + E] = res[0];
#pragma unroll
                            for (int c = 1; c < NC; ++c) m.dout[o][3 * off + (c - 1) * SZ + E] = res[c];
                        }
                    }
                }
            }
        });
    };
    switch (wave) {
    case 0: run(IC<0>{}); break;
    case 1: run(IC<1>{}); break;
    case 2: run(IC<2>{}); break;
    default: run(IC<3>{}); break;
    }
    __syncthreads();   // LDS of this tile is read before the next tile's phase 1 writes it
}

template <bool D>
__global__ __launch_bounds__(TILE_THREADS) void k_multi(TileArgs a, MultiOps m, const QTile *__restrict__ q,
                                                        int ntiles, int *counter)
{
    __shared__ double sO[64 * MULTI_SO];
    __shared__ int64_t sOff[64];
    __shared__ int s_t[2];
    if (threadIdx.x == 0) s_t[0] = atomicAdd(counter, 1);
    __syncthreads();
    for (int k = 0;; ++k) {
        const int t = s_t[k & 1];
        if (t >= ntiles) break;
        int nxt = 0;
        if (threadIdx.x == 0) nxt = atomicAdd(counter, 1);
        const auto hand_over = [&]() {
            if (threadIdx.x == 0) s_t[(k + 1) & 1] = nxt;
        };
        const QTile tile = q[t];
        static_for<0, NCLASS>([&](auto CC) {
            constexpr int C = decltype(CC)::value;
            if (tile.cls == C)
                tile_multi<C / (LMAX + 1), C % (LMAX + 1), D>(a, m, tile.start, tile.count, sO, sOff, hand_over);
        });
    }
}

typedef void (*multi_fn)(hipStream_t, int grid, const TileArgs &, const MultiOps &, const QTile *, int, int *);
typedef int (*multi_occ_fn)();

template <bool D>
void launch_multi(hipStream_t s, int grid, const TileArgs &a, const MultiOps &m, const QTile *q, int ntiles,
                  int *counter)
{
    hipLaunchKernelGGL(k_multi<D>, dim3(grid), dim3(TILE_THREADS), 0, s, a, m, q, ntiles, counter);
}

template <bool D>
int multi_occupancy()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_multi<D>, TILE_THREADS, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb > 0 ? nb : 1;
}

// defined in shg_multi_d0.hip / shg_multi_d1.hip
void multi_entry_d0(multi_fn *f, multi_occ_fn *occ);
void multi_entry_d1(multi_fn *f, multi_occ_fn *occ);

}  // namespace shg
