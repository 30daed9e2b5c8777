// shg_sets.h -- family basis sets (Sec. III): the contracted functions of a set
// share one set of exponents, so for a pair of sets (A, B)
//   * the primitive radial terms (0_a|O|0_b)^(k) (Table S1) are evaluated once
//     per primitive pair of the set pair, for every k the set pair needs, and
//     contracted for all function pairs at once as the matrix product
//     O^(k) = C_a^T G^(k) C_b (eq. O_rab2_deriv with the folded weights of each
//     function as the columns of C): k_set_radial, one wave per set pair;
//   * the angular factors of an element (Qhat of eq. final_r12int_ab and of the
//     derivative recurrences) depend on (la, lb) and X = R_a - R_b only, so for
//     an l-block -- the functions of A with l = la against those of B with
//     l = lb -- they are formed once per element and applied to every function
//     pair of the block: k_setblk<la, lb, D>, a lane per l-block item, tiles of
//     64 items of one (la, lb, na, nb) bin, elements split over the waves,
//     results staged in LDS and copied out row segment by row segment.
// The output block of a set pair is (sum_a (2la+1)) x (sum_b (2lb+1)) row-major,
// functions in set order (grouped by l), components m = -l..l.
#pragma once
#include "shg_kernels.h"

namespace shg {

constexpr int SET_KMAX = 8;     // exponents per set (K_a K_b <= 64: a lane per primitive pair)
constexpr int SET_FMAX = 16;    // contracted functions per set
constexpr int SET_KS = 10;      // radial orders of a set pair: k = 0..9
constexpr int SET_STAGE = 80;   // staged doubles per item and pass: na nb rows NB NC <= 80

// an l-block item: functions fa_rel0 .. fa_rel0+na-1 of set sa (l = la) against
// fb_rel0 .. fb_rel0+nb-1 of set sb (l = lb); na, nb come from the item's bin
struct __align__(16) SetItem {
    int32_t sa, sb;
    int32_t fa_rel0, fb_rel0;   // first function of the item, relative to its set
    int32_t row0, col0;         // block row / column of its first component
    int32_t ld, orow;           // row stride of the set-pair block (nsgf of B); of the item's radial terms
    int64_t off;                // element offset of the set-pair block in out (dout: 3 off)
    int64_t obase;              // radial terms of the item's first function pair: function pair (i, j)
                                // of the item at obase + i orow + j NK, NK orders each
    int64_t blk;                // elements of the set-pair block (derivative block stride)
    int64_t pad;
};

struct SetBlkArgs {
    const SetItem *items;       // class-sorted
    const double *center;       // [nset][3]
    const double *O;            // radial scratch
    double *out, *dout;
    int na, nb;                 // functions per item on each side (uniform in a launch)
};

// rows of the base block per pass: as many as fit SET_STAGE / 2 for one function pair
constexpr int set_rows(int la, int lb, bool D)
{
    int rows = 2 * la + 1;
    while (rows > 1 && rows * (2 * lb + 1) * (D ? 4 : 1) > SET_STAGE / 2) --rows;
    return rows;
}
// function pairs an item may carry for (lb, D)
constexpr int set_fp_max(int la, int lb, bool D)
{
    int f = SET_STAGE / (set_rows(la, lb, D) * (2 * lb + 1) * (D ? 4 : 1));
    return f > 9 ? 9 : f;
}

// radial orders a function pair (la, lb) needs: k = max(la, lb) .. la + lb + deriv
__host__ __device__ constexpr int set_nk(int la, int lb, int deriv) { return (la < lb ? la : lb) + 1 + deriv; }

constexpr int SETBLK_TP = 64;

template <int LA, int LB, bool D>
__global__ __launch_bounds__(TILE_THREADS) void k_setblk(SetBlkArgs a, int64_t start, int64_t count)
{
    using PK = PairK<LA, LB, D>;
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NC = D ? 4 : 1, NK = PK::NK;
    constexpr int RP = set_rows(LA, LB, D), NPASS = (NA + RP - 1) / RP;
    constexpr int FPM = set_fp_max(LA, LB, D);
    constexpr int SO = FPM * NK + 3;                    // per item: O of each function pair, then X
    constexpr int PS = SET_STAGE | 1;                   // staged doubles per item (odd stride)
    __shared__ double sO[SETBLK_TP * SO];
    __shared__ double sT[SETBLK_TP * PS];
    __shared__ SetItem sIt[SETBLK_TP];
    __shared__ double *sDst[SETBLK_TP][NC];
    const int tid = threadIdx.x;
    const int64_t tstart = start + (int64_t)blockIdx.x * SETBLK_TP;
    const int tcount = (int)min((int64_t)SETBLK_TP, start + count - tstart);
    const int na = a.na, nb = a.nb, nfp = na * nb;

    // ---- phase 1: per item X, destinations, and the contracted radial terms of its function pairs ----
    if (tid < tcount) {
        const SetItem it = a.items[tstart + tid];
        sIt[tid] = it;
#pragma unroll
        for (int d = 0; d < 3; ++d) sO[tid * SO + FPM * NK + d] = a.center[3 * it.sa + d] - a.center[3 * it.sb + d];
        sDst[tid][0] = a.out + it.off + (int64_t)it.row0 * it.ld + it.col0;
        if constexpr (D) {
#pragma unroll
            for (int c = 1; c < NC; ++c)
                sDst[tid][c] = a.dout + 3 * it.off + (c - 1) * it.blk + (int64_t)it.row0 * it.ld + it.col0;
        }
    }
    __syncthreads();
    for (int e = tid; e < tcount * nfp * NK; e += TILE_THREADS) {
        const int i = e / (nfp * NK), r = e - i * (nfp * NK);
        const int f = r / NK, k = r - f * NK;
        const int fa = f / nb, fb = f - fa * nb;
        const SetItem &it = sIt[i];
        sO[i * SO + r] = a.O[it.obase + (int64_t)fa * it.orow + fb * NK + k];
    }
    __syncthreads();

    // ---- phase 2: lanes = items, waves split the elements of a pass ----
    const int lane = tid & 63, wave = tid >> 6;
    const bool live = lane < tcount;
    const int il = live ? lane : 0;
    double X[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) X[d] = sO[il * SO + FPM * NK + d];
    RTab<cmax(LA, LB)> R;
    solid_R<cmax(LA, LB)>(X[0], X[1], X[2], R);
    static_for<0, NPASS>([&](auto PP) {
        constexpr int R0 = decltype(PP)::value * RP, R1 = cmin(NA, R0 + RP), NR = R1 - R0;
        const auto run = [&](auto WW) {
            constexpr int W = decltype(WW)::value;
            static_for<R0 * NB, R1 * NB>([&](auto EE) {
                constexpr int E = decltype(EE)::value;
                if constexpr ((E - R0 * NB) % 4 == W) {
                    ElemTerms<LA, LB, D> T;
                    elem_terms<LA, LB, E / NB, E % NB, D>(R, T);
                    for (int f = 0; f < nfp; ++f) {
                        const int fa = f / nb, fb = f - fa * nb;
                        double O[NK];
#pragma unroll
                        for (int k = 0; k < NK; ++k) O[k] = sO[il * SO + f * NK + k];
                        double res[NC];
                        elem_apply<LA, LB, E / NB, E % NB, D>(T, O, X, res);
                        if (live) {
                            // staged as [c][fa][row][fb][mb]: a row segment over (fb, mb) is contiguous
                            const int rr = E / NB - R0, mb = E % NB;
#pragma unroll
                            for (int c = 0; c < NC; ++c)
                                sT[lane * PS + ((c * na + fa) * NR + rr) * (nb * NB) + fb * NB + mb] = res[c];
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
        __syncthreads();
        // ---- phase 3: copy row segments (nb NB doubles each) to the set-pair blocks ----
        const int seg = nb * NB, per = NC * na * NR * seg;
        for (int e = tid; e < tcount * per; e += TILE_THREADS) {
            const int i = e / per, rem = e - i * per;
            const int q = rem / seg, j = rem - q * seg;          // q = (c, fa, rr)
            const int c = q / (na * NR), fr = q - c * (na * NR);
            const int fa = fr / NR, rr = fr - fa * NR;
            const int row = fa * NA + R0 + rr;
            sDst[i][c][(int64_t)row * sIt[i].ld + j] = sT[i * PS + rem];
        }
        __syncthreads();
    });
}

typedef void (*setblk_fn)(hipStream_t, const SetBlkArgs &, int64_t start, int64_t count);

template <int LA, int LB, bool D>
void launch_setblk(hipStream_t s, const SetBlkArgs &a, int64_t start, int64_t count)
{
    const unsigned g = (unsigned)((count + SETBLK_TP - 1) / SETBLK_TP);
    hipLaunchKernelGGL((k_setblk<LA, LB, D>), dim3(g), dim3(TILE_THREADS), 0, s, a, start, count);
}

// per-l_a dispatch tables: setblk_table_la<l_a>()[lb * 2 + D]
const setblk_fn *setblk_table_la0();
const setblk_fn *setblk_table_la1();
const setblk_fn *setblk_table_la2();
const setblk_fn *setblk_table_la3();
const setblk_fn *setblk_table_la4();
inline const setblk_fn *setblk_table(int la)
{
    switch (la) {
    case 0: return setblk_table_la0();
    case 1: return setblk_table_la1();
    case 2: return setblk_table_la2();
    case 3: return setblk_table_la3();
    default: return setblk_table_la4();
    }
}

}  // namespace shg
