// shg_kernels.h -- HIP kernels of the plain per-class path and their launchers.
//
// Per call the path is:
//   k_prep_shells    N_l and folded weights per shell          (shell preparation)
//   k_classify       class key (la, lb, Ka, Kb) per pair, histogram
//   k_scan_bins      exclusive scan of the histogram
//   k_scatter        class-sorted order of the pairs
//   k_contract<...>  one thread per shell pair: radial terms of every primitive
//                    pair (Table S1, Boys by Taylor grid + recurrence) and their
//                    contraction into O^(k) (eq. O_rab2_deriv), kept in registers
//   k_assemble<...>  one thread per shell pair and block row (grid.y = row):
//                    solid harmonics of X = R_a - R_b, Qtilde, block values and
//                    d/dR_a (eqs. final_r12int_ab, dev_ab, cartesian_dev_x/y/z)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shg_math.h"

namespace shg {

constexpr int LMAX = 4;        // two-center / orbital shells
constexpr int KMAX = 7;
constexpr int NCLASS = (LMAX + 1) * (LMAX + 1);
constexpr int NBINS = NCLASS * 64;      // (la, lb, Ka-1, Kb-1)
constexpr int OSTRIDE = 8;              // doubles per pair in the O^(k) scratch buffer
constexpr int CONTRACT_TPB = 128;
constexpr int ASSEMBLE_TPB = 64;

struct ContractArgs {
    const int32_t *pairs;      // [n][2]
    const int32_t *order;      // class-sorted pair ids
    const double *center;      // [nshell][3]
    const int32_t *nprim;
    const int64_t *prim_off;
    const double *exps;
    const double *w;           // folded weights N_l c / (2 alpha)^l
    const double *tab;         // Boys grid
    double omega;
    double *Obuf;              // [sorted position][OSTRIDE]
    int64_t start, count;
};

struct AssembleArgs {
    const int32_t *pairs;
    const int32_t *order;
    const double *center;
    const int64_t *out_off;
    const double *Obuf;
    double *out, *dout;
    int64_t start, count;
};

template <int LA, int LB, int OP, bool D>
__global__ __launch_bounds__(CONTRACT_TPB) void k_contract(ContractArgs a)
{
    int64_t t = (int64_t)blockIdx.x * CONTRACT_TPB + threadIdx.x;
    if (t >= a.count) return;
    int64_t pos = a.start + t;
    int p = a.order[pos];
    int sa = a.pairs[2 * (int64_t)p], sb = a.pairs[2 * (int64_t)p + 1];
    double X0 = a.center[3 * sa] - a.center[3 * sb];
    double X1 = a.center[3 * sa + 1] - a.center[3 * sb + 1];
    double X2 = a.center[3 * sa + 2] - a.center[3 * sb + 2];
    double R2 = X0 * X0 + X1 * X1 + X2 * X2;
    int64_t oa = a.prim_off[sa], ob = a.prim_off[sb];
    double O[PairK<LA, LB, D>::NK];
    contract_pair<LA, LB, OP, D>(a.exps + oa, a.w + oa, a.nprim[sa], a.exps + ob, a.w + ob, a.nprim[sb], R2,
                                 a.omega, a.tab, O);
#pragma unroll
    for (int k = 0; k < PairK<LA, LB, D>::NK; ++k) a.Obuf[pos * OSTRIDE + k] = O[k];
}

template <int LA, int LB, bool D>
__global__ __launch_bounds__(ASSEMBLE_TPB) void k_assemble(AssembleArgs a)
{
    int64_t t = (int64_t)blockIdx.x * ASSEMBLE_TPB + threadIdx.x;
    if (t >= a.count) return;
    int64_t pos = a.start + t;
    int p = a.order[pos];
    int sa = a.pairs[2 * (int64_t)p], sb = a.pairs[2 * (int64_t)p + 1];
    double X[3] = {a.center[3 * sa] - a.center[3 * sb], a.center[3 * sa + 1] - a.center[3 * sb + 1],
                   a.center[3 * sa + 2] - a.center[3 * sb + 2]};
    double O[PairK<LA, LB, D>::NK];
#pragma unroll
    for (int k = 0; k < PairK<LA, LB, D>::NK; ++k) O[k] = a.Obuf[pos * OSTRIDE + k];
    RTab<cmax(LA, LB)> R;
    solid_R<cmax(LA, LB)>(X[0], X[1], X[2], R);
    constexpr int NB = 2 * LB + 1, SZ = (2 * LA + 1) * NB;
    int64_t off = a.out_off[p];
    const int row = blockIdx.y;   // uniform across the wave
    static_for<0, 2 * LA + 1>([&](auto IAA) {
        constexpr int IA = decltype(IAA)::value;
        if (row == IA)
            pair_row<LA, LB, IA, D>(R, O, X, a.out + off + IA * NB, D ? a.dout + 3 * off + IA * NB : nullptr, SZ);
    });
}

typedef void (*contract_fn)(hipStream_t, const ContractArgs &);
typedef void (*assemble_fn)(hipStream_t, const AssembleArgs &);

template <int LA, int LB, int OP, bool D>
void launch_contract(hipStream_t s, const ContractArgs &a)
{
    unsigned g = (unsigned)((a.count + CONTRACT_TPB - 1) / CONTRACT_TPB);
    hipLaunchKernelGGL((k_contract<LA, LB, OP, D>), dim3(g), dim3(CONTRACT_TPB), 0, s, a);
}

template <int LA, int LB, bool D>
void launch_assemble(hipStream_t s, const AssembleArgs &a)
{
    unsigned g = (unsigned)((a.count + ASSEMBLE_TPB - 1) / ASSEMBLE_TPB);
    hipLaunchKernelGGL((k_assemble<LA, LB, D>), dim3(g, 2 * LA + 1), dim3(ASSEMBLE_TPB), 0, s, a);
}

// dispatch tables, defined in the per-operator / per-l_a translation units:
// contract_table(op)[(la * 5 + lb) * 2 + D], assemble_table(la)[lb * 2 + D]
const contract_fn *contract_table_op0();
const contract_fn *contract_table_op1();
const contract_fn *contract_table_op2();
const contract_fn *contract_table_op3();
const contract_fn *contract_table_op4();
const assemble_fn *assemble_table_la0();
const assemble_fn *assemble_table_la1();
const assemble_fn *assemble_table_la2();
const assemble_fn *assemble_table_la3();
const assemble_fn *assemble_table_la4();

}  // namespace shg
