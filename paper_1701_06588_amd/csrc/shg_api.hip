// shg_api.hip -- C ABI of libshg.so (declared in include/shg.h): context,
// shell preparation, class binning of the pair list and the per-class launches.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/shg.h"
#include "boys_table.h"
#include "shg_ctx.h"
#include "shg_kernels.h"

using namespace shg;

namespace shg {
char g_create_msg[512];
}

namespace shg {
// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t v, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// N_l (eq. N_l) and w_alpha = N_l c_alpha / (2 alpha)^l (eq. O_rab2), with validation
__global__ void k_prep_shells(int nshell, const int32_t *l, const int32_t *nprim, const int64_t *prim_off,
                              const double *exps, const double *coefs, int64_t nprim_total, int lmax, double *w,
                              int32_t *err)
{
    // one wave per shell: lane q < K^2 takes the primitive pair (q / K, q % K)
    // of the self-overlap sum, a butterfly adds them up
    const int i = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (i >= nshell) return;
    const int li = l[i], K = nprim[i];
    const int64_t o = prim_off[i];
    if (li < 0 || li > lmax) { if (lane == 0) atomicOr(err, ERR_SHELL_L); return; }
    if (K < 1 || K > KMAX || o < 0 || o + K > nprim_total) { if (lane == 0) atomicOr(err, ERR_SHELL_K); return; }
    bool bad = false;
    for (int k = 0; k < K; ++k) {
        double e = exps[o + k];
        bad |= !(e > 0.0) || !(e < 1e300);
    }
    if (bad) { if (lane == 0) atomicOr(err, ERR_SHELL_EXP); return; }
    double t = 0.0;
    if (lane < K * K) {
        const int qa = lane / K, qb = lane - qa * K;
        t = shell_norm_term(li, exps[o + qa], exps[o + qb], coefs[o + qa], coefs[o + qb]);
    }
    for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
    if (lane < K) {
        const double N = shell_norm_from_sum(li, t);
        double a2 = 2.0 * exps[o + lane], p = 1.0;
        for (int q = 0; q < li; ++q) p *= a2;
        w[o + lane] = N * coefs[o + lane] / p;
    }
}

// class key of each pair: ((la*5 + lb)*8 + Ka-1)*8 + Kb-1; invalid pairs -> NBINS
// sentinel. Counts are aggregated per workgroup in LDS before one global
// atomic per non-empty bin.
constexpr int BIN_TPB = 256, BIN_ITEMS = 16;

__global__ __launch_bounds__(BIN_TPB) void k_classify(int64_t n, const int32_t *pairs, int nshell,
                                                      const int32_t *l, const int32_t *nprim, int32_t *keys,
                                                      int32_t *hist, int32_t *err)
{
    __shared__ int32_t lh[NBINS + 1];
    for (int b = threadIdx.x; b <= NBINS; b += BIN_TPB) lh[b] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * BIN_TPB * BIN_ITEMS;
    int bad = 0;
    for (int it = 0; it < BIN_ITEMS; ++it) {
        int64_t i = base + (int64_t)it * BIN_TPB + threadIdx.x;
        if (i >= n) break;
        int a = pairs[2 * i], b = pairs[2 * i + 1];
        int key = NBINS;
        if (a < 0 || a >= nshell || b < 0 || b >= nshell) {
            bad = 1;
        } else {
            int la = l[a], lb = l[b], ka = nprim[a], kb = nprim[b];
            if (la >= 0 && la <= LMAX && lb >= 0 && lb <= LMAX && ka >= 1 && ka <= KMAX && kb >= 1 && kb <= KMAX)
                key = ((la * (LMAX + 1) + lb) * 8 + ka - 1) * 8 + kb - 1;
        }
        keys[i] = key;
        atomicAdd(&lh[key], 1);
    }
    if (bad) atomicOr(err, ERR_PAIR_INDEX);
    __syncthreads();
    for (int b = threadIdx.x; b <= NBINS; b += BIN_TPB)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// exclusive scan of nb+1 bins by one workgroup of 256 threads; also writes the
// cursors (copy of the starts) used by the scatter
__global__ __launch_bounds__(256) void k_scan_bins(const int32_t *hist, int nb, int32_t *starts, int32_t *cursor)
{
    __shared__ int32_t part[256];
    int t = threadIdx.x;
    int per = (nb + 1 + 255) / 256;
    int lo = t * per, hi = min(lo + per, nb + 1);
    int32_t s = 0;
    for (int i = lo; i < hi; ++i) s += hist[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int32_t acc = 0;
        for (int i = 0; i < 256; ++i) { int32_t v = part[i]; part[i] = acc; acc += v; }
    }
    __syncthreads();
    int32_t acc = part[t];
    for (int i = lo; i < hi; ++i) { starts[i] = acc; cursor[i] = acc; acc += hist[i]; }
}

// class-sorted order: each workgroup ranks its items per bin in LDS, reserves
// one contiguous range per non-empty bin with a single global atomic, then
// writes the pair ids and (rec non-null) the pair records (order inside a bin
// is unspecified; results do not depend on it)
__global__ __launch_bounds__(BIN_TPB) void k_scatter(int64_t n, const int32_t *keys, int32_t *cursor,
                                                     int32_t *order, const int32_t *pairs, const int64_t *out_off,
                                                     PairRec *rec)
{
    __shared__ int32_t cnt[NBINS + 1];
    __shared__ int32_t gbase[NBINS + 1];
    for (int b = threadIdx.x; b <= NBINS; b += BIN_TPB) cnt[b] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * BIN_TPB * BIN_ITEMS;
    int32_t rank[BIN_ITEMS], key[BIN_ITEMS];
#pragma unroll
    for (int it = 0; it < BIN_ITEMS; ++it) {
        int64_t i = base + (int64_t)it * BIN_TPB + threadIdx.x;
        key[it] = -1;
        if (i < n) {
            key[it] = keys[i];
            rank[it] = atomicAdd(&cnt[key[it]], 1);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b <= NBINS; b += BIN_TPB)
        if (cnt[b]) gbase[b] = atomicAdd(&cursor[b], cnt[b]);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < BIN_ITEMS; ++it) {
        int64_t i = base + (int64_t)it * BIN_TPB + threadIdx.x;
        if (key[it] >= 0) {
            const int32_t pos = gbase[key[it]] + rank[it];
            order[pos] = (int32_t)i;
            if (rec) rec[pos] = PairRec{pairs[2 * i], pairs[2 * i + 1], out_off[i]};
        }
    }
}

}  // namespace shg

// ---------------------------------------------------------------------------
// fixed scratch of shg_pairs_noalloc: one array per device, held until the
// process ends; host code uses the address hipGetSymbolAddress gives for the
// current device (never the array's name, which on the host is only a stand-in)
// ---------------------------------------------------------------------------
namespace {
constexpr size_t NOALLOC_W_BYTES = (size_t)SHG_NOALLOC_MAX_PRIMS * sizeof(double);
constexpr size_t NOALLOC_KEYS_BYTES = (size_t)SHG_NOALLOC_MAX_PAIRS * sizeof(int32_t);
constexpr size_t NOALLOC_REC_BYTES = (size_t)SHG_NOALLOC_MAX_PAIRS * sizeof(PairRec);
constexpr size_t NOALLOC_BYTES = NOALLOC_W_BYTES + 2 * NOALLOC_KEYS_BYTES + NOALLOC_REC_BYTES;
static_assert(NOALLOC_W_BYTES % 256 == 0 && NOALLOC_KEYS_BYTES % 256 == 0, "256-byte aligned sub-arrays");

static __device__ __align__(256) double scratch[NOALLOC_BYTES / sizeof(double)];

constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEV] = {};
hipError_t g_scratch_err[NOALLOC_MAX_DEV] = {};
bool g_scratch_done[NOALLOC_MAX_DEV] = {};

// address of the current device's copy of `scratch` (looked up once per device)
hipError_t noalloc_scratch_address(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= NOALLOC_MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *p = nullptr;
        g_scratch_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[device] = g_scratch_err[device] == hipSuccess ? p : nullptr;
        g_scratch_done[device] = true;
    }
    *ptr = g_scratch_ptr[device];
    return g_scratch_err[device];
}
}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int shg_create(shg_ctx **out, void *hip_stream)
{
    if (!out) return set_err(nullptr, SHG_EINVAL, "shg_create: ctx pointer is NULL");
    *out = nullptr;
    shg_ctx *c = new (std::nothrow) shg_ctx();
    if (!c) return set_err(nullptr, SHG_ENOMEM, "shg_create: out of host memory");
    c->stream = (hipStream_t)hip_stream;
    for (int la = 0; la <= LMAX; ++la)
        for (int lb = 0; lb <= LMAX; ++lb)
            for (int d = 0; d < 2; ++d)
                for (int op = 0; op < 5; ++op) c->shape[op][la][lb][d] = default_shape(la, lb, d == 1, 64, 48 * 1024);
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, c->device);
        if (e == hipSuccess) {
            strncpy(c->arch, prop.gcnArchName, sizeof(c->arch) - 1);
            char *colon = strchr(c->arch, ':');
            if (colon) *colon = 0;
        }
    }
    // the fixed scratch of shg_pairs_noalloc (this device's copy); a failure is
    // kept and reported by that entry point only
    if (e == hipSuccess) c->noalloc_err = noalloc_scratch_address(c->device, &c->noalloc_scratch);
    std::vector<double> tab((size_t)BOYS_NPTS * BOYS_STRIDE);
    build_boys_table(tab.data());
    if (e == hipSuccess) e = hipMalloc((void **)&c->boys, tab.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(c->boys, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void **)&c->bins, 2 * (NBINS_MAX + 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&c->err, 64 * sizeof(int32_t));
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->host_rb, (NBINS_MAX + 64) * sizeof(int32_t));
    if (e != hipSuccess) {
        set_err(nullptr, SHG_EDEVICE, "shg_create: %s", hipGetErrorString(e));
        shg_destroy(c);
        return SHG_EDEVICE;
    }
    *out = c;
    return 0;
}

extern "C" void shg_destroy(shg_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (int i = 0; i < NCLASS + 3; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    (void)hipFree(c->boys);
    (void)hipFree(c->w);
    (void)hipFree(c->w2);
    (void)hipFree(c->keys);
    (void)hipFree(c->order);
    (void)hipFree(c->rec);
    (void)hipFree(c->bins);
    (void)hipFree(c->stats);
    (void)hipFree(c->bound_tab);
    (void)hipFree(c->set_w);
    (void)hipFree(c->set_osz);
    (void)hipFree(c->set_nsgf);
    (void)hipFree(c->set_items);
    (void)hipFree(c->set_O);
    for (int w = 0; w < AAB_NSTREAM; ++w) {
        (void)hipFree(c->Pbuf[w]);
        (void)hipFree(c->Yv[w]);
        (void)hipFree(c->Yd[w]);
        if (c->aab_ev[w]) (void)hipEventDestroy(c->aab_ev[w]);
        if (w > 0 && c->aab_side[w - 1]) {
            (void)hipStreamSynchronize(c->aab_side[w - 1]);
            (void)hipStreamDestroy(c->aab_side[w - 1]);
        }
    }
    (void)hipFree(c->gaunt_idx);
    (void)hipFree(c->gaunt_lm);
    (void)hipFree(c->gaunt_g);
    (void)hipFree(c->err);
    if (c->host_rb) (void)hipHostFree(c->host_rb);
    delete c;
}

extern "C" const char *shg_last_error(const shg_ctx *c) { return c ? c->msg : g_create_msg; }

// ---------------------------------------------------------------------------
// helpers shared by the entry points
// ---------------------------------------------------------------------------
namespace shg {
int check_shells(shg_ctx *c, const shg_shells *sh, const char *what)
{
    if (!sh) return set_err(c, SHG_EINVAL, "%s: shell table is NULL", what);
    if (sh->nshell < 0 || sh->nprim_total < 0)
        return set_err(c, SHG_EINVAL, "%s: negative nshell or nprim_total", what);
    if (sh->nshell > 0 && (!sh->center || !sh->l || !sh->nprim || !sh->prim_off || !sh->exps || !sh->coefs))
        return set_err(c, SHG_EINVAL, "%s: NULL array in the shell table", what);
    return 0;
}

int prep_shells(shg_ctx *c, const shg_shells *sh, int lmax, double *&w, size_t &cap)
{
    int rc = grow(c, w, cap, (size_t)sh->nprim_total + 1);
    if (rc) return rc;
    if (sh->nshell > 0)
        hipLaunchKernelGGL(k_prep_shells, dim3((sh->nshell + 3) / 4), dim3(256), 0, c->stream, sh->nshell,
                           sh->l, sh->nprim, sh->prim_off, sh->exps, sh->coefs, sh->nprim_total, lmax, w, c->err);
    return 0;
}

int decode_err(shg_ctx *c, int32_t e, const char *what)
{
    if (!e) return 0;
    return set_err(c, SHG_EINVAL, "%s: invalid input:%s%s%s%s%s%s%s", what, (e & ERR_SHELL_L) ? " shell l out of range;" : "",
                   (e & ERR_SHELL_K) ? " contraction length outside [1,7] or prim_off out of range;" : "",
                   (e & ERR_SHELL_EXP) ? " exponent not positive and finite;" : "",
                   (e & ERR_PAIR_INDEX) ? " shell index outside [0, nshell);" : "",
                   (e & ERR_AAB_CENTER) ? " a and a~ of a triple are on different centers;" : "",
                   (e & ERR_AAB_L) ? " l of a triple outside the supported range;" : "",
                   (e & ERR_SET_FUN) ? " set functions: count outside [1,16], offsets out of range or l not"
                                       " grouped in non-decreasing order;" : "");
}

}  // namespace shg

// device scratch of one plain evaluation: folded weights (one per primitive),
// class keys, class-sorted ids and pair records (one each per pair)
struct PairScratch {
    double *w;
    int32_t *keys, *order;
    PairRec *rec;
};

static int pairs_validate(shg_ctx *c, const char *what, const shg_shells *sh, shg_op op, double omega,
                          const int32_t *pairs, int64_t n, const int64_t *out_off, double *out, double *dout,
                          bool deriv)
{
    if ((int)op < 0 || (int)op > 4) return set_err(c, SHG_EINVAL, "%s: unknown operator %d", what, (int)op);
    if ((op == SHG_ERF || op == SHG_ERFC || op == SHG_GAUSS) && !(omega > 0.0 && omega < 1e300))
        return set_err(c, SHG_EINVAL, "%s: omega must be positive and finite for this operator", what);
    if (n < 0) return set_err(c, SHG_EINVAL, "%s: n < 0", what);
    if (n >= (int64_t)1 << 31) return set_err(c, SHG_EINVAL, "%s: n >= 2^31 pairs per call", what);
    int rc = check_shells(c, sh, what);
    if (rc) return rc;
    if (n > 0 && (!pairs || !out_off || !out || (deriv && !dout)))
        return set_err(c, SHG_EINVAL, "%s: NULL pointer argument", what);
    return 0;
}

// binning and per-class launches of one validated call (n > 0) with the given scratch
static int pairs_run(shg_ctx *c, const char *what, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs,
                     int64_t n, const int64_t *out_off, double *out, double *dout, bool deriv, const PairScratch &ps)
{
    int rc = 0;
    hipStream_t s = c->stream;
    int32_t *hist = c->bins, *cursor = c->bins + (NBINS_MAX + 1);
    if (c->prof_on) HIP_TRY(c, hipEventRecord(c->ev[0], s));
    hipLaunchKernelGGL(k_fill_i32, dim3((NBINS + 1 + 255) / 256), dim3(256), 0, s, hist, 0, NBINS + 1);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, c->err, 0, 1);
    if (sh->nshell > 0)
        hipLaunchKernelGGL(k_prep_shells, dim3((sh->nshell + 3) / 4), dim3(256), 0, s, sh->nshell, sh->l, sh->nprim,
                           sh->prim_off, sh->exps, sh->coefs, sh->nprim_total, LMAX, ps.w, c->err);
    unsigned gb = (unsigned)((n + BIN_TPB * BIN_ITEMS - 1) / (BIN_TPB * BIN_ITEMS));
    hipLaunchKernelGGL(k_classify, dim3(gb), dim3(BIN_TPB), 0, s, n, pairs, sh->nshell, sh->l, sh->nprim, ps.keys,
                       hist, c->err);
    // the scan leaves the bin starts in `cursor`; they are read back (class
    // starts are every 64th bin) before the scatter advances the cursors
    hipLaunchKernelGGL(k_scan_bins, dim3(1), dim3(256), 0, s, hist, NBINS, cursor, cursor);
    HIP_TRY(c, hipMemcpyAsync(c->host_rb, cursor, (NBINS + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(c->host_rb + NBINS + 1, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_scatter, dim3(gb), dim3(BIN_TPB), 0, s, n, ps.keys, cursor, ps.order, pairs, out_off, ps.rec);
    if (c->prof_on) HIP_TRY(c, hipEventRecord(c->ev[1], s));
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(s));
    if ((rc = decode_err(c, c->host_rb[NBINS + 1], what))) return rc;

    const tile_fn *ttab[5] = {tile_table_la0(), tile_table_la1(), tile_table_la2(), tile_table_la3(),
                              tile_table_la4()};
    const int D = deriv ? 1 : 0;
    TileArgs ta{ps.rec, ps.order, sh->center, sh->nprim, sh->prim_off, sh->exps, ps.w, c->boys, out, dout,
                omega, (int)op};
    int prev = NCLASS + 2;   // event before the next class launch
    int used[NCLASS];
    int nused = 0;
    if (c->prof_on) HIP_TRY(c, hipEventRecord(c->ev[NCLASS + 2], s));
    for (int la = 0; la <= LMAX; ++la)
        for (int lb = 0; lb <= LMAX; ++lb) {
            int cls = la * (LMAX + 1) + lb;
            int64_t b0 = c->host_rb[cls * 64], b1 = c->host_rb[(cls + 1) * 64];
            if (b1 <= b0) continue;
            ttab[la][lb * 2 + D](s, ta, b0, b1 - b0, c->shape[op][la][lb][D]);
            if (c->prof_on) {
                HIP_TRY(c, hipEventRecord(c->ev[2 + cls], s));
                c->prof_launches[cls][D] += 1;
                c->prof_pairs[cls][D] += b1 - b0;
                used[nused++] = cls;
            }
        }
    if (c->prof_on) {
        // per-class kernel time = gap between consecutive events on the stream
        HIP_TRY(c, hipStreamSynchronize(s));
        float ms = 0;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        c->prof_bin_ms += ms;
        c->prof_bin_calls += 1;
        for (int u = 0; u < nused; ++u) {
            int cls = used[u];
            HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[prev], c->ev[2 + cls]));
            c->prof_ms[cls][D] += ms;
            prev = 2 + cls;
        }
    }
    HIP_TRY(c, hipGetLastError());
    return 0;
}

static int pairs_common(shg_ctx *c, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs, int64_t n,
                        const int64_t *out_off, double *out, double *dout, bool deriv)
{
    const char *what = deriv ? "shg_pairs_deriv" : "shg_pairs";
    if (!c) return SHG_EINVAL;
    int rc = pairs_validate(c, what, sh, op, omega, pairs, n, out_off, out, dout, deriv);
    if (rc || n == 0) return rc;
    if ((rc = grow(c, c->keys, c->keys_cap, (size_t)n))) return rc;
    if ((rc = grow(c, c->order, c->order_cap, (size_t)n))) return rc;
    if ((rc = grow(c, c->rec, c->rec_cap, (size_t)n))) return rc;
    if ((rc = grow(c, c->w, c->w_cap, (size_t)sh->nprim_total + 1))) return rc;
    return pairs_run(c, what, sh, op, omega, pairs, n, out_off, out, dout, deriv,
                     PairScratch{c->w, c->keys, c->order, c->rec});
}

extern "C" int shg_pairs(shg_ctx *c, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs, int64_t n,
                         const int64_t *out_off, double *out)
{
    if (c && op == SHG_GCOULOMB) {
        if (!(omega > 0.0 && omega < 1e300))
            return set_err(c, SHG_EINVAL, "shg_pairs: omega must be positive and finite for this operator");
        return gcoulomb_pairs(c, "shg_pairs", omega, sh, pairs, n, out_off, out, nullptr);
    }
    return pairs_common(c, sh, op, omega, pairs, n, out_off, out, nullptr, false);
}

extern "C" int shg_pairs_deriv(shg_ctx *c, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs,
                               int64_t n, const int64_t *out_off, double *out, double *dout)
{
    if (c && op == SHG_GCOULOMB) {
        if (!(omega > 0.0 && omega < 1e300))
            return set_err(c, SHG_EINVAL, "shg_pairs_deriv: omega must be positive and finite for this operator");
        if (!dout) return set_err(c, SHG_EINVAL, "shg_pairs_deriv: NULL pointer argument");
        return gcoulomb_pairs(c, "shg_pairs_deriv", omega, sh, pairs, n, out_off, out, dout);
    }
    return pairs_common(c, sh, op, omega, pairs, n, out_off, out, dout, true);
}

extern "C" int shg_pairs_noalloc(shg_ctx *c, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs,
                                 int64_t n, const int64_t *out_off, double *out, double *dout)
{
    const char *what = "shg_pairs_noalloc";
    if (!c) return SHG_EINVAL;
    const bool deriv = dout != nullptr;
    int rc = pairs_validate(c, what, sh, op, omega, pairs, n, out_off, out, dout, deriv);
    if (rc || n == 0) return rc;
    if (n > SHG_NOALLOC_MAX_PAIRS)
        return set_err(c, SHG_EINVAL, "%s: n = %lld exceeds SHG_NOALLOC_MAX_PAIRS = %d", what, (long long)n,
                       SHG_NOALLOC_MAX_PAIRS);
    if (sh->nprim_total > SHG_NOALLOC_MAX_PRIMS)
        return set_err(c, SHG_EINVAL, "%s: nprim_total = %lld exceeds SHG_NOALLOC_MAX_PRIMS = %d", what,
                       (long long)sh->nprim_total, SHG_NOALLOC_MAX_PRIMS);
    if (c->noalloc_err != hipSuccess || !c->noalloc_scratch)
        return set_err(c, SHG_EDEVICE, "%s: no address for the fixed scratch array: %s", what,
                       hipGetErrorString(c->noalloc_err != hipSuccess ? c->noalloc_err : hipErrorInvalidSymbol));
    char *base = (char *)c->noalloc_scratch;
    PairScratch ps{(double *)base, (int32_t *)(base + NOALLOC_W_BYTES),
                   (int32_t *)(base + NOALLOC_W_BYTES + NOALLOC_KEYS_BYTES),
                   (PairRec *)(base + NOALLOC_W_BYTES + 2 * NOALLOC_KEYS_BYTES)};
    return pairs_run(c, what, sh, op, omega, pairs, n, out_off, out, dout, deriv, ps);
}

extern "C" int shg_profile_enable(shg_ctx *c, int on)
{
    if (!c) return SHG_EINVAL;
    if (on && !c->ev[0])
        for (int i = 0; i < NCLASS + 3; ++i) HIP_TRY(c, hipEventCreate(&c->ev[i]));
    c->prof_on = on ? 1 : 0;
    memset(c->prof_ms, 0, sizeof(c->prof_ms));
    memset(c->prof_launches, 0, sizeof(c->prof_launches));
    memset(c->prof_pairs, 0, sizeof(c->prof_pairs));
    c->prof_bin_ms = 0;
    c->prof_bin_calls = 0;
    return 0;
}

extern "C" int shg_profile_read(const shg_ctx *c, int la, int lb, int deriv, double *ms, int64_t *launches,
                                int64_t *pairs)
{
    if (!c || !ms || !launches || !pairs) return SHG_EINVAL;
    if (la < 0) {   // binning stage (shell preparation, classification, scan, scatter)
        *ms = c->prof_bin_ms;
        *launches = c->prof_bin_calls;
        *pairs = 0;
        return 0;
    }
    if (la > LMAX || lb < 0 || lb > LMAX || (deriv != 0 && deriv != 1)) return SHG_EINVAL;
    int cls = la * (LMAX + 1) + lb;
    *ms = c->prof_ms[cls][deriv];
    *launches = c->prof_launches[cls][deriv];
    *pairs = c->prof_pairs[cls][deriv];
    return 0;
}

static int check_shape(shg_ctx *c, int op, int la, int lb, int deriv, int tp, int rows_pp)
{
    if (op < 0 || op > 4 || la < 0 || la > LMAX || lb < 0 || lb > LMAX || (deriv != 0 && deriv != 1))
        return set_err(c, SHG_EINVAL, "tile shape: class out of range");
    if (tp != 64 && tp != 128 && tp != 256) return set_err(c, SHG_EINVAL, "tile shape: tp must be 64, 128 or 256");
    if (rows_pp < 1 || rows_pp > 2 * la + 1) return set_err(c, SHG_EINVAL, "tile shape: rows_pp outside [1, 2la+1]");
    long bytes = tile_smem_bytes_rt(tp, rows_pp, lb, deriv != 0);
    if (bytes > 160 * 1024) return set_err(c, SHG_EINVAL, "tile shape: needs %ld bytes of LDS (> 160 KiB)", bytes);
    return 0;
}

extern "C" int shg_set_tile_shape(shg_ctx *c, int op, int la, int lb, int deriv, int tp, int rows_pp)
{
    if (!c) return SHG_EINVAL;
    int rc = check_shape(c, op, la, lb, deriv, tp, rows_pp);
    if (rc) return rc;
    c->shape[op][la][lb][deriv] = TileShape{tp, rows_pp};
    return 0;
}

extern "C" int shg_get_tile_shape(const shg_ctx *c, int op, int la, int lb, int deriv, int *tp, int *rows_pp)
{
    if (!c || !tp || !rows_pp || op < 0 || op > 4 || la < 0 || la > LMAX || lb < 0 || lb > LMAX ||
        (deriv != 0 && deriv != 1))
        return SHG_EINVAL;
    *tp = c->shape[op][la][lb][deriv].tp;
    *rows_pp = c->shape[op][la][lb][deriv].rows_pp;
    return 0;
}

// ---------------------------------------------------------------------------
// autotuner: times every admissible tile shape of every class present in the
// caller's pair list and keeps the fastest; the cache file is a small JSON
// list keyed by (GPU architecture, op, la, lb, deriv)
// ---------------------------------------------------------------------------
extern "C" int shg_autotune(shg_ctx *c, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs,
                            int64_t n, const int64_t *out_off, double *out, double *dout, int reps)
{
    if (!c) return SHG_EINVAL;
    if (reps < 1) reps = 1;
    const bool deriv = dout != nullptr;
    // bin (and evaluate once with the current shapes; this validates the input)
    int rc = pairs_common(c, sh, op, omega, pairs, n, out_off, out, dout, deriv);
    if (rc || n == 0) return rc;
    hipStream_t s = c->stream;
    const int D = deriv ? 1 : 0;
    const tile_fn *ttab[5] = {tile_table_la0(), tile_table_la1(), tile_table_la2(), tile_table_la3(),
                              tile_table_la4()};
    TileArgs ta{c->rec, c->order, sh->center, sh->nprim, sh->prim_off, sh->exps, c->w, c->boys, out, dout,
                omega, (int)op};
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    for (int la = 0; la <= LMAX; ++la)
        for (int lb = 0; lb <= LMAX; ++lb) {
            int cls = la * (LMAX + 1) + lb;
            int64_t b0 = c->host_rb[cls * 64], b1 = c->host_rb[(cls + 1) * 64];
            if (b1 <= b0) continue;
            float best = 1e30f;
            TileShape bs = c->shape[op][la][lb][D];
            const int rows_c[5] = {1, 2, 3, 5, 2 * la + 1};
            for (int tp = 64; tp <= 256; tp *= 2)
                for (int r = 0; r < 5; ++r) {
                    int rows = rows_c[r];
                    bool dup = false;
                    for (int q = 0; q < r; ++q) dup |= rows_c[q] == rows;
                    if (dup || rows > 2 * la + 1) continue;
                    if (check_shape(c, op, la, lb, D, tp, rows)) continue;
                    TileShape sh_try{tp, rows};
                    ttab[la][lb * 2 + D](s, ta, b0, b1 - b0, sh_try);   // warm-up
                    HIP_TRY(c, hipEventRecord(e0, s));
                    for (int k = 0; k < reps; ++k) ttab[la][lb * 2 + D](s, ta, b0, b1 - b0, sh_try);
                    HIP_TRY(c, hipEventRecord(e1, s));
                    HIP_TRY(c, hipEventSynchronize(e1));
                    float ms = 0;
                    HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best) { best = ms; bs = sh_try; }
                }
            c->shape[op][la][lb][D] = bs;
            c->tune_ms[op][la][lb][D] = best / reps;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_err(c, 0, "");
    // leave the caller's buffers holding results of the selected shapes
    return pairs_common(c, sh, op, omega, pairs, n, out_off, out, dout, deriv);
}

extern "C" int shg_tuning_save(const shg_ctx *c, const char *path)
{
    if (!c || !path) return SHG_EINVAL;
    FILE *f = fopen(path, "w");
    if (!f) return SHG_EINVAL;
    fprintf(f, "{\"arch\": \"%s\", \"shapes\": [\n", c->arch);
    bool first = true;
    for (int op = 0; op < 5; ++op)
        for (int la = 0; la <= LMAX; ++la)
            for (int lb = 0; lb <= LMAX; ++lb)
                for (int d = 0; d < 2; ++d) {
                    if (c->tune_ms[op][la][lb][d] <= 0) continue;
                    const TileShape &t = c->shape[op][la][lb][d];
                    fprintf(f, "%s  {\"op\": %d, \"la\": %d, \"lb\": %d, \"deriv\": %d, \"tp\": %d, \"rows_pp\": %d, "
                               "\"ms\": %.6f}",
                            first ? "" : ",\n", op, la, lb, d, t.tp, t.rows_pp, c->tune_ms[op][la][lb][d]);
                    first = false;
                }
    fprintf(f, "\n]}\n");
    fclose(f);
    return 0;
}

// Applies the entries of a cache written by shg_tuning_save for this GPU's
// architecture; malformed or out-of-range entries are skipped (defaults stay).
// Returns the number of entries applied (>= 0) or SHG_EINVAL if the file
// cannot be read.
extern "C" int shg_tuning_load(shg_ctx *c, const char *path)
{
    if (!c || !path) return SHG_EINVAL;
    FILE *f = fopen(path, "r");
    if (!f) return SHG_EINVAL;
    std::vector<char> buf;
    char tmp[4096];
    size_t k;
    while ((k = fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + k);
    fclose(f);
    buf.push_back(0);
    const char *txt = buf.data();
    char arch[64] = {0};
    const char *pa = strstr(txt, "\"arch\"");
    if (!pa || sscanf(pa, "\"arch\": \"%63[^\"]\"", arch) != 1 || strcmp(arch, c->arch) != 0) return 0;
    int applied = 0;
    for (const char *p = strchr(txt, '{'); p; p = strchr(p + 1, '{')) {
        int op, la, lb, d, tp, rows;
        double ms;
        if (sscanf(p, "{\"op\": %d, \"la\": %d, \"lb\": %d, \"deriv\": %d, \"tp\": %d, \"rows_pp\": %d, \"ms\": %lf}",
                   &op, &la, &lb, &d, &tp, &rows, &ms) != 7)
            continue;
        if (check_shape(c, op, la, lb, d, tp, rows)) continue;
        c->shape[op][la][lb][d] = TileShape{tp, rows};
        c->tune_ms[op][la][lb][d] = ms;
        ++applied;
    }
    set_err(c, 0, "");
    return applied;
}


