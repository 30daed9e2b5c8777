// shg_kernels.h -- HIP kernels of the two-center path and their launchers.
//
// Per call the plain path is:
//   k_prep_shells    N_l and folded weights per shell                (shell preparation)
//   k_classify       class key (la, lb, Ka, Kb) per pair, LDS-aggregated histogram
//   k_scan_bins      exclusive scan of the histogram
//   k_scatter        class-sorted order of the pairs and, per sorted position, a
//                    16-byte record (shell ids, output offset) so that the tile
//                    kernels read their pairs with coalesced loads
//   k_tile<la,lb,D>  one launch per class; a workgroup owns a tile of TP shell pairs:
//     phase 1  G = 256/TP lanes per shell pair evaluate the radial terms of the
//              primitive pairs (Table S1; Boys by Taylor grid + recurrence) and
//              contract them into O^(k) (eq. O_rab2_deriv); butterfly reduction
//              inside the lane group, result in LDS
//     phase 2  lanes = pairs, waves split the block elements: solid harmonics of
//              X = R_a - R_b, Qtilde and the element value and d/dR_a
//              (eqs. final_r12int_ab, dev_ab, cartesian_dev_x/y/z), written to an
//              LDS tile of `rows_pp` block rows
//     phase 3  the workgroup copies the LDS tile to the caller's blocks with
//              consecutive lanes on consecutive doubles (coalesced stores)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shg_bound.h"
#include "shg_math.h"

namespace shg {

constexpr int LMAX = 4;        // two-center / orbital shells
constexpr int KMAX = 7;
constexpr int NCLASS = (LMAX + 1) * (LMAX + 1);
constexpr int NBINS = NCLASS * 64;      // (la, lb, Ka-1, Kb-1)
constexpr int TILE_THREADS = 256;

// class-sorted pair record: shells of the pair and offset of its block
struct __align__(16) PairRec {
    int32_t a, b;
    int64_t off;
};

struct TileArgs {
    const PairRec *rec;        // [sorted position] (two-center mode)
    const int32_t *order;      // class-sorted item ids (three-index mode)
    const double *center;      // [nshell][3]
    const int32_t *nprim;
    const int64_t *prim_off;
    const double *exps;
    const double *w;           // folded weights N_l c / (2 alpha)^l
    const double *tab;         // Boys grid
    double *out, *dout;
    double omega;
    int op;
    // precomputed-monopole mode (triples != nullptr): items are rows of
    // `tstride` shell indices, a first and b last ((a, a~, b) triples of the
    // three-index overlap, (a, b) pairs of (a|r_a^{2n}|b)); phase 1 loads
    // O^(k) from P[(pos - ybase) * pstride + poff + k] and block `pos` goes to
    // out[ooff[item]] when ooff is set, else to out[(pos - ybase) * ys + yoff]
    // (scratch Y blocks of one chunk of a triple class)
    const int32_t *triples;
    const double *P;
    int pstride, poff;
    int64_t ybase, ys, yoff;
    const int64_t *ooff;
    int tstride;
    // in-kernel screening (screened plans; two-center mode): with sstat set, a
    // pair whose analytic bound (shg_bound.h, per-shell statistics sstat) is
    // below stau -- or, with skeep set, whose decision flag skeep[pos] is 0 --
    // gets zero radial terms, so its block and d/dR_a blocks are written as
    // zeros; without skeep the decision is stored as sflag[pos] (1 kept, 0 skipped)
    const double *sstat;
    const BoundTab *sbt;
    const uint8_t *skeep;
    uint8_t *sflag;
    double stau;
};

// tile shape: TP pairs (64, 128 or 256) and rows_pp block rows per LDS pass
struct TileShape {
    int tp, rows_pp;
};

template <int KLO, int KHI>
__device__ __forceinline__ void radial_rt(int op, double a, double b, double R2, double omega,
                                          const double *__restrict__ tab, double (&g)[KHI - KLO + 1])
{
    switch (op) {
    case OP_OVERLAP: radial<OP_OVERLAP, KLO, KHI>(a, b, R2, omega, tab, g); break;
    case OP_COULOMB: radial<OP_COULOMB, KLO, KHI>(a, b, R2, omega, tab, g); break;
    case OP_ERF: radial<OP_ERF, KLO, KHI>(a, b, R2, omega, tab, g); break;
    case OP_ERFC: radial<OP_ERFC, KLO, KHI>(a, b, R2, omega, tab, g); break;
    default: radial<OP_GAUSS, KLO, KHI>(a, b, R2, omega, tab, g); break;
    }
}

// Makes the harmonics table, the contracted radial terms and X opaque to the
// optimiser: placed between block elements it stops values of one element from
// being shared with (and kept live for) the next, which bounds the register
// footprint of the large classes at the cost of recomputing a few W entries.
constexpr bool row_used(int l, int LA, int LB, bool D)
{
    int jm = cmin(LA, LB) + (D ? 1 : 0);
    return (l <= LA && l >= LA - jm) || (l <= LB && l >= LB - jm);
}

template <int LA, int LB, bool D, int L, int NK>
__device__ __forceinline__ void reg_fence(RTab<L> &R, double (&O)[NK], double (&X)[3])
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
    for (int k = 0; k < NK; ++k) asm volatile("" : "+v"(O[k]));
    asm volatile("" : "+v"(X[0]), "+v"(X[1]), "+v"(X[2]));
}

// LDS of a tile: per pair 9 doubles (O^(k), k < 6, and X), two block pointers,
// and the staged rows with an odd per-pair stride (conflict-free 8-byte
// accesses when consecutive lanes take consecutive pairs)
constexpr int SO_STRIDE = 9;
// 64-pair tiles of the two-center mode first stage every pair's exponents and
// folded weights (both shells, KMAX each) in the staging area, after 256 bytes
// of screening flags, so the radial loop reads them from LDS
constexpr int STG_STRIDE = 4 * KMAX + 1;   // odd: conflict-free
constexpr int STG_OFF = 256;
inline constexpr int tile_smem_bytes_rt(int tp, int rows_pp, int lb, bool D)
{
    const int rows = tp * (((D ? 4 : 1) * rows_pp * (2 * lb + 1)) | 1) * 8;
    const int stage = tp == 64 ? STG_OFF + tp * STG_STRIDE * 8 : 0;
    return tp * SO_STRIDE * 8 + tp * 16 + (rows > stage ? rows : stage);
}
template <int LA, int LB, bool D>
constexpr int tile_smem_bytes(int tp, int rows_pp)
{
    return tile_smem_bytes_rt(tp, rows_pp, LB, D);
}

// compiled tile schedule (tp = 64): block rows per LDS pass. The persistent
// kernel holds two workgroups per CU (its register use), so each two-center
// class stages as many rows as fit in half the LDS (whole blocks without
// derivatives); measured faster than the per-class tuned shapes. The L_a blocks
// of the three-index overlap (l_a = 5..9, launched per class) take the rows
// that fit the LDS share of their register-limited occupancy (two workgroups
// per CU from l_a = 7 with derivatives, three otherwise).
constexpr int sched_rows(int la, int lb, bool D)
{
    // (2,2) stages four rows so that the light classes (la + lb <= 4) fit 53 KiB:
    // three workgroups per CU for their persistent kernel
    constexpr int rows_d[5][5] = {{1, 1, 1, 1, 1}, {3, 3, 3, 3, 3}, {5, 5, 4, 5, 4}, {7, 7, 7, 5, 4}, {9, 9, 7, 5, 4}};
    if (la <= 4) return D ? rows_d[la][lb] : 2 * la + 1;
    const int budget = (D && la >= 7) ? 80 * 1024 - 256 : 53 * 1024;
    int rows = 2 * la + 1;
    while (rows > 1 && tile_smem_bytes_rt(64, rows, lb, D) > budget) --rows;
    return rows;
}

// One tile of `tcount` (<= shape.tp) class-(LA,LB) pairs starting at sorted
// position `tstart`. smem: dynamic LDS of tile_smem_bytes(tp, rows_pp).
struct NoHook {
    __device__ void operator()() const {}
};

// `after_p1` runs once per thread after phase 1 and before the first barrier.
// FIXED_ROWS > 0 selects the compiled schedule: tp = 64 and FIXED_ROWS block
// rows per pass, every pass's element list and the waves' shares of it fixed
// at compile time (no per-element tests at run time); `shape` is then unused.
template <int LA, int LB, bool D, int FIXED_ROWS = 0, class Hook = NoHook>
__device__ __forceinline__ void tile_pairs(const TileArgs &a, int64_t tstart, int tcount, TileShape shape,
                                           char *smem, const Hook &after_p1 = Hook())
{
    using PK = PairK<LA, LB, D>;
    static_assert(PK::NK + 3 <= SO_STRIDE, "O^(k) and X must fit the per-pair LDS slot");
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, SZ = NA * NB, NC = D ? 4 : 1;
    const int TP = FIXED_ROWS > 0 ? 64 : shape.tp, rows_pp = FIXED_ROWS > 0 ? FIXED_ROWS : shape.rows_pp;
    double *sO = (double *)smem;                   // [TP][SO_STRIDE]: O^(k), then X
    double **sPv = (double **)(sO + TP * SO_STRIDE);    // [TP] block of the pair in out
    double **sPd = sPv + TP;                       // [TP] its d/dR_a blocks in dout
    double *sT = (double *)(sPd + TP);             // [TP][odd stride]
    const int tid = threadIdx.x;

    // ---- phase 1: radial terms and contraction, G lanes per shell pair ----
    // (classes with l_a > LMAX only occur as L_a blocks of the three-index overlap)
    if (LA > LMAX || a.triples) {
        // precomputed mode: O^(k) = P^(k)_La of a triple (k_aab_radial) or T^(k)
        // of a pair under r_a^{2n} (k_r2n_radial)
        for (int i = tid; i < tcount; i += TILE_THREADS) {
            const int64_t pos = tstart + i;
#pragma unroll
            for (int k = 0; k < PK::NK; ++k)
                sO[i * SO_STRIDE + k] = a.P[(pos - a.ybase) * a.pstride + a.poff + k];
            const int p = a.order[pos];
            const int64_t row = (int64_t)a.tstride * p;
            const int sa = a.triples[row], sb = a.triples[row + a.tstride - 1];
#pragma unroll
            for (int d = 0; d < 3; ++d) sO[i * SO_STRIDE + 6 + d] = a.center[3 * sa + d] - a.center[3 * sb + d];
            const int64_t off = a.ooff ? a.ooff[p] : (pos - a.ybase) * a.ys + a.yoff;
            sPv[i] = a.out + off;
            sPd[i] = a.dout ? a.dout + 3 * off : nullptr;
        }
    } else if constexpr (LA <= LMAX) {
        const int G = TILE_THREADS / TP;
        const int i = tid / G, g = tid - (tid / G) * G;
        const bool live = i < tcount;
        // screening (a.sstat set): one thread per pair decides, from the bound or the
        // model's flag, before any radial work; the flags pass through the first
        // 256 bytes of the staging area, which is free until phase 2
        int *sSkip = (int *)sT;
        const auto screen = [&]() {
            for (int q = tid; q < tcount; q += TILE_THREADS) {
                bool sk;
                if (a.skeep) {
                    sk = a.skeep[tstart + q] == 0;
                } else {
                    const PairRec r = a.rec[tstart + q];
                    const double Y0 = a.center[3 * r.a] - a.center[3 * r.b];
                    const double Y1 = a.center[3 * r.a + 1] - a.center[3 * r.b + 1];
                    const double Y2 = a.center[3 * r.a + 2] - a.center[3 * r.b + 2];
                    double vb, Rr, rm;
                    sk = shell_pair_bound(LA, LB, a.sstat + (size_t)r.a * STAT, a.sstat + (size_t)r.b * STAT,
                                          fma(Y0, Y0, fma(Y1, Y1, Y2 * Y2)), a.op, a.omega, D ? 1 : 0, a.sbt, &vb,
                                          &Rr, &rm) < a.stau;
                }
                if (a.sflag) a.sflag[tstart + q] = sk ? 0 : 1;
                sSkip[q] = sk ? 1 : 0;
            }
        };
        // screening inputs of this thread's pair (64-pair tiles: thread q decides pair
        // q), loaded together with the pairs' own data
        const bool bthread = TP == 64 && a.sstat && !a.skeep && tid < tcount;
        PairRec rq{};
        if (bthread) rq = a.rec[tstart + tid];
        const PairRec rc = a.rec[tstart + (live ? i : 0)];
        const int sa = rc.a, sb = rc.b;
        const double X0 = a.center[3 * sa] - a.center[3 * sb];
        const double X1 = a.center[3 * sa + 1] - a.center[3 * sb + 1];
        const double X2 = a.center[3 * sa + 2] - a.center[3 * sb + 2];
        const double R2 = fma(X0, X0, fma(X1, X1, X2 * X2));   // fixed rounding order
        const int64_t oa = a.prim_off[sa], ob = a.prim_off[sb];
        const int ka = a.nprim[sa], kb = a.nprim[sb];
        double O[PK::NK];
#pragma unroll
        for (int k = 0; k < PK::NK; ++k) O[k] = 0.0;
        if (TP == 64) {
            // the pair's lanes stage its exponents and weights with independent
            // loads, so the loop below waits on memory only for the Boys table;
            // the screening decisions are taken while those loads are in flight
            static_assert(TILE_THREADS / 64 == 4 && (KMAX + 3) / 4 == 2, "two staged values per lane and shell");
            // the bound reads statistics entries 0 .. 4 + la + lb + 1 of both shells
            constexpr int NST = 4 + LA + LB + 2;
            static_assert(NST <= STAT, "bound statistics of one shell");
            double qa[NST], qb[NST], QX = 0, QY = 0, QZ = 0;
            if (bthread) {
#pragma unroll
                for (int e = 0; e < NST; ++e) {
                    qa[e] = a.sstat[(size_t)rq.a * STAT + e];
                    qb[e] = a.sstat[(size_t)rq.b * STAT + e];
                }
                QX = a.center[3 * rq.a] - a.center[3 * rq.b];
                QY = a.center[3 * rq.a + 1] - a.center[3 * rq.b + 1];
                QZ = a.center[3 * rq.a + 2] - a.center[3 * rq.b + 2];
            }
            double *sP = (double *)((char *)sT + STG_OFF) + i * STG_STRIDE;
            double va[2][2], vb[2][2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int q = g + 4 * u;
                if (live && q < ka) {
                    va[u][0] = a.exps[oa + q];
                    va[u][1] = a.w[oa + q];
                }
                if (live && q < kb) {
                    vb[u][0] = a.exps[ob + q];
                    vb[u][1] = a.w[ob + q];
                }
            }
            if (bthread) {
                double vbd, Rr, rm;
                const bool sk = shell_pair_bound(LA, LB, qa, qb, fma(QX, QX, fma(QY, QY, QZ * QZ)), a.op, a.omega,
                                                 D ? 1 : 0, a.sbt, &vbd, &Rr, &rm) < a.stau;
                a.sflag[tstart + tid] = sk ? 0 : 1;
                sSkip[tid] = sk ? 1 : 0;
            } else if (a.sstat && a.skeep && tid < tcount) {
                sSkip[tid] = a.skeep[tstart + tid] == 0 ? 1 : 0;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int q = g + 4 * u;
                if (live && q < ka) {
                    sP[q] = va[u][0];
                    sP[2 * KMAX + q] = va[u][1];
                }
                if (live && q < kb) {
                    sP[KMAX + q] = vb[u][0];
                    sP[3 * KMAX + q] = vb[u][1];
                }
            }
            __syncthreads();
            // a skipped pair gets no primitive work: its O^(k) stay zero, and so does its block
            const int P = live && !(a.sstat && sSkip[i] != 0) ? ka * kb : 0;
            for (int q = g; q < P; q += G) {
                const int ia = q / kb, ib = q - ia * kb;
                double gk[PK::NK];
                radial_rt<PK::KLO, PK::KHI>(a.op, sP[ia], sP[KMAX + ib], R2, a.omega, a.tab, gk);
                const double ww = sP[2 * KMAX + ia] * sP[3 * KMAX + ib];
#pragma unroll
                for (int k = 0; k < PK::NK; ++k) O[k] = fma(ww, gk[k], O[k]);
            }
        } else {
            bool skip = false;
            if (a.sstat) {
                screen();
                __syncthreads();
                skip = live && sSkip[i] != 0;
            }
            const int P = live && !skip ? ka * kb : 0;
            for (int q = g; q < P; q += G) {
                const int ia = q / kb, ib = q - ia * kb;
                double gk[PK::NK];
                radial_rt<PK::KLO, PK::KHI>(a.op, a.exps[oa + ia], a.exps[ob + ib], R2, a.omega, a.tab, gk);
                const double ww = a.w[oa + ia] * a.w[ob + ib];
#pragma unroll
                for (int k = 0; k < PK::NK; ++k) O[k] = fma(ww, gk[k], O[k]);
            }
        }
        for (int m = 1; m < G; m <<= 1)
#pragma unroll
            for (int k = 0; k < PK::NK; ++k) O[k] += __shfl_xor(O[k], m, G);
        if (live && g == 0) {
#pragma unroll
            for (int k = 0; k < PK::NK; ++k) sO[i * SO_STRIDE + k] = O[k];
            sO[i * SO_STRIDE + 6] = X0;
            sO[i * SO_STRIDE + 7] = X1;
            sO[i * SO_STRIDE + 8] = X2;
            sPv[i] = a.out + rc.off;
            sPd[i] = a.dout ? a.dout + 3 * rc.off : nullptr;
        }
    }
    after_p1();
    __syncthreads();

    // ---- phase 2: angular part; lanes = pairs, waves split the elements ----
    const int lane = tid & 63, wave = tid >> 6;
    const int PW = TP / 64, EW = (TILE_THREADS / 64) / PW;
    const int pg = wave % PW, es = wave / PW;
    const int i = pg * 64 + lane;
    const bool live = i < tcount;
    double X[3], O[PK::NK];
    {
        const int il = live ? i : 0;
#pragma unroll
        for (int k = 0; k < PK::NK; ++k) O[k] = live ? sO[il * SO_STRIDE + k] : 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) X[d] = live ? sO[il * SO_STRIDE + 6 + d] : 0.0;
    }
    RTab<cmax(LA, LB)> R;
    solid_R<cmax(LA, LB)>(X[0], X[1], X[2], R);

    if constexpr (FIXED_ROWS > 0) {
        // compiled schedule: tp = 64, so es = wave and i = lane
        constexpr int NPASS = (NA + FIXED_ROWS - 1) / FIXED_ROWS;
        static_for<0, NPASS>([&](auto PP) {
            constexpr int R0 = decltype(PP)::value * FIXED_ROWS;
            constexpr int R1 = cmin(NA, R0 + FIXED_ROWS);
            constexpr int SEG = (R1 - R0) * NB, PER = NC * SEG, PS = PER | 1;
            const auto run = [&](auto WW) {
                constexpr int W = decltype(WW)::value;
                static_for<R0 * NB, R1 * NB>([&](auto EE) {
                    constexpr int E = decltype(EE)::value;
                    if constexpr ((E - R0 * NB) % 4 == W) {
                        reg_fence<LA, LB, D>(R, O, X);
                        double res[NC];
                        pair_elem<LA, LB, E / NB, E % NB, D>(R, O, X, res);
                        if (live) {
#pragma unroll
                            for (int c = 0; c < NC; ++c) sT[i * PS + c * SEG + (E - R0 * NB)] = res[c];
                        }
                    }
                });
            };
            switch (es) {
            case 0: run(IC<0>{}); break;
            case 1: run(IC<1>{}); break;
            case 2: run(IC<2>{}); break;
            default: run(IC<3>{}); break;
            }
            __syncthreads();
            const int total = tcount * PER;
            for (int f = tid; f < total; f += TILE_THREADS) {
                const int ii = f / PER, rem = f - ii * PER;
                const int c = NC == 4 ? rem / SEG : 0;
                double *dst = c == 0 ? sPv[ii] : sPd[ii] + (c - 1) * SZ;
                dst[R0 * NB + rem - c * SEG] = sT[ii * PS + rem];
            }
            __syncthreads();
        });
    } else {
        for (int r0 = 0; r0 < NA; r0 += rows_pp) {
            const int r1 = min(NA, r0 + rows_pp);
            const int SEG = (r1 - r0) * NB;
            const int per = NC * SEG, PS = per | 1;
            static_for<0, SZ>([&](auto EE) {
                constexpr int E = decltype(EE)::value;
                constexpr int IA = E / NB, IB = E % NB;
                if (IA >= r0 && IA < r1 && ((E - r0 * NB) % EW) == es) {
                    reg_fence<LA, LB, D>(R, O, X);
                    double res[NC];
                    pair_elem<LA, LB, IA, IB, D>(R, O, X, res);
                    if (live) {
    #pragma unroll
                        for (int c = 0; c < NC; ++c) sT[i * PS + c * SEG + (E - r0 * NB)] = res[c];
                    }
                }
            });
            __syncthreads();
            // ---- phase 3: coalesced copy of the LDS tile into the blocks ----
            // thread f takes staged value f = ii * per + rem; (ii, rem) advance by a
            // fixed step instead of being divided out per value, and the destination
            // is selected without branching
            const int total = tcount * per;
            const int qs = TILE_THREADS / per, rs = TILE_THREADS - qs * per;
            const int rowoff = r0 * NB;
            int ii = tid / per, rem = tid - ii * per;
    #pragma unroll 2
            for (int f = tid; f < total; f += TILE_THREADS) {
                int c = 0;
                if constexpr (NC == 4) c = (rem >= SEG) + (rem >= 2 * SEG) + (rem >= 3 * SEG);
                double *dst = c == 0 ? sPv[ii] : sPd[ii] + (c - 1) * SZ;
                dst[rowoff + rem - c * SEG] = sT[ii * PS + rem];
                ii += qs;
                rem += rs;
                if (rem >= per) {
                    rem -= per;
                    ++ii;
                }
            }
            __syncthreads();
        }
    }
}

template <int LA, int LB, bool D>
__global__ __launch_bounds__(TILE_THREADS) void k_tile(TileArgs a, int64_t start, int64_t count, TileShape shape)
{
    extern __shared__ __align__(16) char smem[];
    const int64_t tstart = start + (int64_t)blockIdx.x * shape.tp;
    const int tcount = (int)min((int64_t)shape.tp, start + count - tstart);
    constexpr int FR = sched_rows(LA, LB, D);
    if constexpr (LA > LMAX) {
        // L_a blocks of the three-index overlap: launched with the compiled schedule only
        tile_pairs<LA, LB, D, FR>(a, tstart, tcount, shape, smem);
    } else {
        if (shape.tp == 64 && shape.rows_pp == FR)
            tile_pairs<LA, LB, D, FR>(a, tstart, tcount, shape, smem);
        else
            tile_pairs<LA, LB, D>(a, tstart, tcount, shape, smem);
    }
}

typedef void (*tile_fn)(hipStream_t, const TileArgs &, int64_t start, int64_t count, TileShape shape);

template <int LA, int LB, bool D>
void launch_tile(hipStream_t s, const TileArgs &a, int64_t start, int64_t count, TileShape shape)
{
    unsigned g = (unsigned)((count + shape.tp - 1) / shape.tp);
    size_t smem = (size_t)tile_smem_bytes<LA, LB, D>(shape.tp, shape.rows_pp);
    static bool attr_set = false;   // allow up to the full 160 KiB of LDS per workgroup
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_tile<LA, LB, D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_tile<LA, LB, D>), dim3(g), dim3(TILE_THREADS), smem, s, a, start, count, shape);
}

// default tile shape of class (la, lb, D) under an LDS budget (bytes)
inline TileShape default_shape(int la, int lb, bool D, int tp, int lds_budget)
{
    int NA = 2 * la + 1;
    int rows = NA;
    while (rows > 1 && tile_smem_bytes_rt(tp, rows, lb, D) > lds_budget) --rows;
    int passes = (NA + rows - 1) / rows;
    rows = (NA + passes - 1) / passes;
    return TileShape{tp, rows};
}

// dispatch tables (one translation unit per l_a): tile_table_la<l_a>()[lb * 2 + D];
// l_a = 0..4 cover lb = 0..4 (two-center classes), l_a = 5..9 cover lb = 0..3
// (the L_a blocks of the three-index overlap)
const tile_fn *tile_table_la0();
const tile_fn *tile_table_la1();
const tile_fn *tile_table_la2();
const tile_fn *tile_table_la3();
const tile_fn *tile_table_la4();
const tile_fn *tile_table_la5();
const tile_fn *tile_table_la6();
const tile_fn *tile_table_la7();
const tile_fn *tile_table_la8();
const tile_fn *tile_table_la9();
inline const tile_fn *tile_table(int la)
{
    switch (la) {
    case 0: return tile_table_la0();
    case 1: return tile_table_la1();
    case 2: return tile_table_la2();
    case 3: return tile_table_la3();
    case 4: return tile_table_la4();
    case 5: return tile_table_la5();
    case 6: return tile_table_la6();
    case 7: return tile_table_la7();
    case 8: return tile_table_la8();
    default: return tile_table_la9();
    }
}

}  // namespace shg
