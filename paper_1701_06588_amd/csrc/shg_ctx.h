// shg_ctx.h -- library-private context and helpers shared by the translation
// units of libshg.so (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../../include/shg.h"
#include "shg_kernels.h"
#include "shg_sets.h"

// error bits raised on the device
enum { ERR_SHELL_L = 1, ERR_SHELL_K = 2, ERR_SHELL_EXP = 4, ERR_PAIR_INDEX = 8, ERR_AAB_CENTER = 16,
       ERR_AAB_L = 32, ERR_SET_FUN = 64 };

using shg::NCLASS;
using shg::LMAX;
using shg::TileShape;

// the three-index overlap spreads its (class, chunk) work items over the
// context stream and AAB_NSTREAM - 1 side streams, each with its own scratch
constexpr int AAB_NSTREAM = 4;

struct shg_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    double *boys = nullptr;          // Boys grid
    // growable scratch
    double *w = nullptr;  size_t w_cap = 0;          // folded weights
    double *w2 = nullptr; size_t w2_cap = 0;         // second shell table (aab aux)
    int32_t *keys = nullptr; size_t keys_cap = 0;
    int32_t *order = nullptr; size_t order_cap = 0;
    shg::PairRec *rec = nullptr; size_t rec_cap = 0;   // class-sorted pair records
    TileShape shape[5][LMAX + 1][LMAX + 1][2];      // tile shape per (op, la, lb, deriv), autotuned
    char arch[64] = {0};
    double tune_ms[5][LMAX + 1][LMAX + 1][2] = {};
    // optional per-launch timing with HIP events (shg_profile_*)
    int prof_on = 0;
    hipEvent_t ev[NCLASS + 3] = {};   // [0] binning start, [1] binning end, [2+cls], [NCLASS+2] classes start
    double prof_ms[NCLASS][2] = {};
    int64_t prof_launches[NCLASS][2] = {}, prof_pairs[NCLASS][2] = {};
    double prof_bin_ms = 0;
    int64_t prof_bin_calls = 0;
    // three-index overlap: Gaunt table (uploaded on first use) and scratch
    int32_t *gaunt_idx = nullptr;    // [(la*7 + lt)][(ma+la)(2lt+1) + mt+lt] -> {start, count}
    int32_t *gaunt_lm = nullptr;     // entries: {L, M}
    double *gaunt_g = nullptr;       // entries: coefficient
    double *Pbuf[AAB_NSTREAM] = {}; size_t Pbuf_cap[AAB_NSTREAM] = {};   // P^(k)_La per triple
    double *Yv[AAB_NSTREAM] = {}; size_t Yv_cap[AAB_NSTREAM] = {};       // two-center blocks (La|lb) per triple
    double *Yd[AAB_NSTREAM] = {}; size_t Yd_cap[AAB_NSTREAM] = {};       // and their d/dR_a
    hipStream_t aab_side[AAB_NSTREAM - 1] = {};   // default priority, non-blocking
    int64_t aab_chunk = (int64_t)1 << 17;          // triples per (class, chunk) work item
    hipEvent_t aab_ev[AAB_NSTREAM] = {};          // [0] fork from the context stream, [w] join of side stream w
    double *stats = nullptr; size_t stats_cap = 0;  // per-shell screening statistics
    void *bound_tab = nullptr;       // constants of the analytic bound (device)
    // family sets (shg_set_pairs): folded weights, radial-scratch sizes and
    // offsets, spherical functions per set, l-block items, radial scratch
    double *set_w = nullptr; size_t set_w_cap = 0;
    int64_t *set_osz = nullptr; size_t set_osz_cap = 0;
    int64_t *set_nsgf = nullptr; size_t set_nsgf_cap = 0;
    shg::SetItem *set_items = nullptr; size_t set_items_cap = 0;
    double *set_O = nullptr; size_t set_O_cap = 0;
    int32_t *bins = nullptr;         // [2][NBINS_MAX + 1]: histogram, then cursors
    int32_t *err = nullptr;          // device error flag
    int32_t *host_rb = nullptr;      // pinned read-back: class starts + error
    void *noalloc_scratch = nullptr;  // this device's fixed scratch (shg_pairs_noalloc)
    hipError_t noalloc_err = hipSuccess;
    char msg[512] = {0};
};

namespace shg {

extern char g_create_msg[512];
constexpr int NBINS_MAX = 8192;

inline int set_err(shg_ctx *c, int code, const char *fmt, ...)
{
    char *dst = c ? c->msg : g_create_msg;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(ctx, call)                                                                     \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_err(ctx, SHG_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

template <class T>
inline int grow(shg_ctx *c, T *&p, size_t &cap, size_t need)
{
    if (need <= cap) return 0;
    if (p) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipFree(p));
        p = nullptr;
        cap = 0;
    }
    size_t n = need + need / 4 + 64;
    hipError_t e = hipMalloc((void **)&p, n * sizeof(T));
    if (e != hipSuccess) {
        p = nullptr;
        return set_err(c, SHG_ENOMEM, "hipMalloc(%zu bytes) failed: %s", n * sizeof(T), hipGetErrorString(e));
    }
    cap = n;
    return 0;
}


// helpers and small kernels defined in shg_api.hip
int check_shells(shg_ctx *c, const shg_shells *sh, const char *what);
int prep_shells(shg_ctx *c, const shg_shells *sh, int lmax, double *&w, size_t &cap);
int decode_err(shg_ctx *c, int32_t e, const char *what);
__global__ void k_fill_i32(int32_t *p, int32_t v, int n);
__global__ void k_prep_shells(int nshell, const int32_t *l, const int32_t *nprim, const int64_t *prim_off,
                              const double *exps, const double *coefs, int64_t nprim_total, int lmax, double *w,
                              int32_t *err);
__global__ void k_classify(int64_t n, const int32_t *pairs, int nshell, const int32_t *l, const int32_t *nprim,
                           int32_t *keys, int32_t *hist, int32_t *err);
__global__ void k_scan_bins(const int32_t *hist, int nb, int32_t *starts, int32_t *cursor);
__global__ void k_scatter(int64_t n, const int32_t *keys, int32_t *cursor, int32_t *order, const int32_t *pairs,
                          const int64_t *out_off, PairRec *rec);
// exp(-omega r^2)/r pairs through the precomputed-monopole tiles (shg_monopole.hip);
// gc_radial_range writes the radial terms of sorted positions [start, start +
// count) of one class to T[pos * MONO_TSTRIDE + k]
constexpr int MONO_TSTRIDE = 8;
void gc_radial_range(hipStream_t s, int cls, bool deriv, const shg_shells *sh, const int32_t *pairs,
                     const int32_t *order, const double *w, const double *tab, double omega, double *T, int64_t start,
                     int64_t count);
// the same for (a|r_a^{2n}|b), 0 <= nr <= 5
void r2n_radial_range(hipStream_t s, int cls, bool deriv, const shg_shells *sh, const int32_t *pairs,
                      const int32_t *order, const double *w, int nr, double *T, int64_t start, int64_t count);
int gcoulomb_pairs(shg_ctx *c, const char *what, double omega, const shg_shells *sh, const int32_t *pairs, int64_t n,
                   const int64_t *out_off, double *out, double *dout);
// screening stage of a screened plan (shg_screen.hip): per-shell statistics
// from the folded weights, then (keep non-NULL) keep[i] (0: skip) for the n
// class-sorted records, the kept flags counted into bsum[i / 4096] (bsum
// nullable, zeroed by the caller); kernels only, graph-capturable; work: n * 15
// floats with a model
int plan_screen_enqueue(shg_ctx *c, hipStream_t s, const shg_shells *sh, const double *w, double *stats,
                        const PairRec *rec, int64_t n, int nops, const int *ops, const double *omegas, int deriv,
                        double tau, shg_mlp *mlp, float *work, uint8_t *keep, int32_t *bsum);
size_t plan_screen_stats_doubles(int nshell);
// uploads the bound's constants (once per context; not during stream capture)
int screen_prepare(shg_ctx *c);
// whether a model predicts operator op (and, with deriv, the d/dR_a blocks too)
bool mlp_covers(const shg_mlp *m, int op, int deriv);

}  // namespace shg
