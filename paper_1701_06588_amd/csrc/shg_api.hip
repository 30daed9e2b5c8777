// shg_api.hip -- C ABI of libshg.so (declared in include/shg.h): context,
// shell preparation, class binning of the pair list and the per-class launches.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../../include/shg.h"
#include "boys_table.h"
#include "shg_kernels.h"

using namespace shg;

// error bits raised on the device
enum { ERR_SHELL_L = 1, ERR_SHELL_K = 2, ERR_SHELL_EXP = 4, ERR_PAIR_INDEX = 8, ERR_AAB_CENTER = 16,
       ERR_AAB_L = 32 };

struct shg_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    double *boys = nullptr;          // Boys grid
    // growable scratch
    double *w = nullptr;  size_t w_cap = 0;          // folded weights
    double *w2 = nullptr; size_t w2_cap = 0;         // second shell table (aab aux)
    int32_t *keys = nullptr; size_t keys_cap = 0;
    int32_t *order = nullptr; size_t order_cap = 0;
    double *Obuf = nullptr; size_t Obuf_cap = 0;
    int32_t *bins = nullptr;         // [2][NBINS_MAX + 1]: histogram, then cursors
    int32_t *err = nullptr;          // device error flag
    int32_t *host_rb = nullptr;      // pinned read-back: class starts + error
    char msg[512] = {0};
};

static char g_create_msg[512];
static constexpr int NBINS_MAX = 8192;

static int set_err(shg_ctx *c, int code, const char *fmt, ...)
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
static int grow(shg_ctx *c, T *&p, size_t &cap, size_t need)
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
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nshell) return;
    int li = l[i], K = nprim[i];
    int64_t o = prim_off[i];
    if (li < 0 || li > lmax) { atomicOr(err, ERR_SHELL_L); return; }
    if (K < 1 || K > KMAX || o < 0 || o + K > nprim_total) { atomicOr(err, ERR_SHELL_K); return; }
    for (int k = 0; k < K; ++k) {
        double e = exps[o + k];
        if (!(e > 0.0) || !(e < 1e300)) { atomicOr(err, ERR_SHELL_EXP); return; }
    }
    double N = shell_norm(li, K, exps + o, coefs + o);
    for (int k = 0; k < K; ++k) {
        double a2 = 2.0 * exps[o + k], p = 1.0;
        for (int q = 0; q < li; ++q) p *= a2;
        w[o + k] = N * coefs[o + k] / p;
    }
}

// class key of each pair: ((la*5 + lb)*8 + Ka-1)*8 + Kb-1; invalid pairs -> NBINS sentinel
__global__ void k_classify(int64_t n, const int32_t *pairs, int nshell, const int32_t *l, const int32_t *nprim,
                           int32_t *keys, int32_t *hist, int32_t *err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = pairs[2 * i], b = pairs[2 * i + 1];
    int key = NBINS;
    if (a < 0 || a >= nshell || b < 0 || b >= nshell) {
        atomicOr(err, ERR_PAIR_INDEX);
    } else {
        int la = l[a], lb = l[b], ka = nprim[a], kb = nprim[b];
        if (la >= 0 && la <= LMAX && lb >= 0 && lb <= LMAX && ka >= 1 && ka <= KMAX && kb >= 1 && kb <= KMAX)
            key = ((la * (LMAX + 1) + lb) * 8 + ka - 1) * 8 + kb - 1;
    }
    keys[i] = key;
    atomicAdd(&hist[key], 1);
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

__global__ void k_scatter(int64_t n, const int32_t *keys, int32_t *cursor, int32_t *order)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int pos = atomicAdd(&cursor[keys[i]], 1);
    order[pos] = (int32_t)i;
}

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
    hipError_t e = hipGetDevice(&c->device);
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
    (void)hipFree(c->boys);
    (void)hipFree(c->w);
    (void)hipFree(c->w2);
    (void)hipFree(c->keys);
    (void)hipFree(c->order);
    (void)hipFree(c->Obuf);
    (void)hipFree(c->bins);
    (void)hipFree(c->err);
    if (c->host_rb) (void)hipHostFree(c->host_rb);
    delete c;
}

extern "C" const char *shg_last_error(const shg_ctx *c) { return c ? c->msg : g_create_msg; }

// ---------------------------------------------------------------------------
// helpers shared by the entry points
// ---------------------------------------------------------------------------
static int check_shells(shg_ctx *c, const shg_shells *sh, const char *what)
{
    if (!sh) return set_err(c, SHG_EINVAL, "%s: shell table is NULL", what);
    if (sh->nshell < 0 || sh->nprim_total < 0)
        return set_err(c, SHG_EINVAL, "%s: negative nshell or nprim_total", what);
    if (sh->nshell > 0 && (!sh->center || !sh->l || !sh->nprim || !sh->prim_off || !sh->exps || !sh->coefs))
        return set_err(c, SHG_EINVAL, "%s: NULL array in the shell table", what);
    return 0;
}

static int prep_shells(shg_ctx *c, const shg_shells *sh, int lmax, double *&w, size_t &cap)
{
    int rc = grow(c, w, cap, (size_t)sh->nprim_total + 1);
    if (rc) return rc;
    if (sh->nshell > 0)
        hipLaunchKernelGGL(k_prep_shells, dim3((sh->nshell + 255) / 256), dim3(256), 0, c->stream, sh->nshell,
                           sh->l, sh->nprim, sh->prim_off, sh->exps, sh->coefs, sh->nprim_total, lmax, w, c->err);
    return 0;
}

static int decode_err(shg_ctx *c, int32_t e, const char *what)
{
    if (!e) return 0;
    return set_err(c, SHG_EINVAL, "%s: invalid input:%s%s%s%s%s%s", what, (e & ERR_SHELL_L) ? " shell l out of range;" : "",
                   (e & ERR_SHELL_K) ? " contraction length outside [1,7] or prim_off out of range;" : "",
                   (e & ERR_SHELL_EXP) ? " exponent not positive and finite;" : "",
                   (e & ERR_PAIR_INDEX) ? " shell index outside [0, nshell);" : "",
                   (e & ERR_AAB_CENTER) ? " a and a~ of a triple are on different centers;" : "",
                   (e & ERR_AAB_L) ? " l of a triple outside the supported range;" : "");
}

static int pairs_common(shg_ctx *c, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs, int64_t n,
                        const int64_t *out_off, double *out, double *dout, bool deriv)
{
    const char *what = deriv ? "shg_pairs_deriv" : "shg_pairs";
    if (!c) return SHG_EINVAL;
    if ((int)op < 0 || (int)op > 4) return set_err(c, SHG_EINVAL, "%s: unknown operator %d", what, (int)op);
    if ((op == SHG_ERF || op == SHG_ERFC || op == SHG_GAUSS) && !(omega > 0.0 && omega < 1e300))
        return set_err(c, SHG_EINVAL, "%s: omega must be positive and finite for this operator", what);
    if (n < 0) return set_err(c, SHG_EINVAL, "%s: n < 0", what);
    if (n >= (int64_t)1 << 31) return set_err(c, SHG_EINVAL, "%s: n >= 2^31 pairs per call", what);
    int rc = check_shells(c, sh, what);
    if (rc) return rc;
    if (n == 0) return 0;
    if (!pairs || !out_off || !out || (deriv && !dout)) return set_err(c, SHG_EINVAL, "%s: NULL pointer argument", what);

    if ((rc = grow(c, c->keys, c->keys_cap, (size_t)n))) return rc;
    if ((rc = grow(c, c->order, c->order_cap, (size_t)n))) return rc;
    if ((rc = grow(c, c->Obuf, c->Obuf_cap, (size_t)n * OSTRIDE))) return rc;
    hipStream_t s = c->stream;
    int32_t *hist = c->bins, *cursor = c->bins + (NBINS_MAX + 1);
    hipLaunchKernelGGL(k_fill_i32, dim3((NBINS + 1 + 255) / 256), dim3(256), 0, s, hist, 0, NBINS + 1);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, c->err, 0, 1);
    if ((rc = prep_shells(c, sh, LMAX, c->w, c->w_cap))) return rc;
    unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_classify, dim3(g), dim3(256), 0, s, n, pairs, sh->nshell, sh->l, sh->nprim, c->keys, hist,
                       c->err);
    // the scan leaves the bin starts in `cursor`; they are read back (class
    // starts are every 64th bin) before the scatter advances the cursors
    hipLaunchKernelGGL(k_scan_bins, dim3(1), dim3(256), 0, s, hist, NBINS, cursor, cursor);
    HIP_TRY(c, hipMemcpyAsync(c->host_rb, cursor, (NBINS + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(c->host_rb + NBINS + 1, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, s, n, c->keys, cursor, c->order);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(s));
    if ((rc = decode_err(c, c->host_rb[NBINS + 1], what))) return rc;

    const contract_fn *ctab[5] = {contract_table_op0(), contract_table_op1(), contract_table_op2(),
                                  contract_table_op3(), contract_table_op4()};
    const assemble_fn *atab[5] = {assemble_table_la0(), assemble_table_la1(), assemble_table_la2(),
                                  assemble_table_la3(), assemble_table_la4()};
    const int D = deriv ? 1 : 0;
    for (int la = 0; la <= LMAX; ++la)
        for (int lb = 0; lb <= LMAX; ++lb) {
            int cls = la * (LMAX + 1) + lb;
            int64_t b0 = c->host_rb[cls * 64], b1 = c->host_rb[(cls + 1) * 64];
            if (b1 <= b0) continue;
            ContractArgs ca{pairs, c->order, sh->center, sh->nprim, sh->prim_off, sh->exps, c->w, c->boys, omega,
                            c->Obuf, b0, b1 - b0};
            ctab[op][(la * 5 + lb) * 2 + D](s, ca);
            AssembleArgs aa{pairs, c->order, sh->center, out_off, c->Obuf, out, dout, b0, b1 - b0};
            atab[la][lb * 2 + D](s, aa);
        }
    HIP_TRY(c, hipGetLastError());
    return 0;
}

extern "C" int shg_pairs(shg_ctx *c, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs, int64_t n,
                         const int64_t *out_off, double *out)
{
    return pairs_common(c, sh, op, omega, pairs, n, out_off, out, nullptr, false);
}

extern "C" int shg_pairs_deriv(shg_ctx *c, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs,
                               int64_t n, const int64_t *out_off, double *out, double *dout)
{
    return pairs_common(c, sh, op, omega, pairs, n, out_off, out, dout, true);
}

extern "C" int shg_aab(shg_ctx *c, const shg_shells *orb, const shg_shells *aux, const int32_t *triples, int64_t n,
                       const int64_t *out_off, double *out, double *dout)
{
    if (!c) return SHG_EINVAL;
    (void)orb; (void)aux; (void)triples; (void)n; (void)out_off; (void)out; (void)dout;
    return set_err(c, SHG_EINVAL, "shg_aab: not built yet");
}
