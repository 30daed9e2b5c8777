// shg_swap.hip -- swap symmetry of the two-center blocks (Sec. V): for an
// operator that depends on |r1 - r2| only, the block of the swapped pair
// (b, a), each function keeping its center, is the transpose of the block of
// (a, b); d/dR_b of (a|O|b) is -d/dR_a (translation invariance), so the
// derivative blocks of (b, a) with respect to its first center are minus the
// transposed derivative blocks of (a, b). A caller that needs both orders
// evaluates one and fills the other here, a copy instead of an evaluation.
//
#include <hip/hip_runtime.h>

#include "shg_ctx.h"

using namespace shg;

namespace {

constexpr int SW_TPB = 256, SW_PAIRS = 64, SW_U = 8;

// q = floor(r / d) for 0 <= r < 2^12, 1 <= d <= 81 from a float reciprocal: (r + 0.5) / d
// is at least 0.5 / d > 2^-8 away from an integer, far above the float rounding error
__device__ __forceinline__ int small_div(int r, float rd) { return (int)(((float)r + 0.5f) * rd); }

// A workgroup takes 64 pairs: their metadata is loaded at once (one round of
// latency) into LDS with a prefix over the block sizes, then all 256 threads
// walk the concatenated destination elements, SW_U loads in flight per thread
// before the matching stores (stores contiguous within each destination
// block, loads gathered within the source block).
__global__ __launch_bounds__(SW_TPB) void k_swap_blocks(int64_t n, const int32_t *pairs, int nshell,
                                                        const int32_t *l, const int64_t *src_off,
                                                        const int64_t *dst_off, double *out, double *dout,
                                                        int32_t *err)
{
    __shared__ int64_t s_src[SW_PAIRS], s_dst[SW_PAIRS];
    __shared__ int s_na[SW_PAIRS], s_nb[SW_PAIRS], s_beg[SW_PAIRS + 1];
    __shared__ float s_rna[SW_PAIRS], s_rsz[SW_PAIRS];
    const int64_t base = (int64_t)blockIdx.x * SW_PAIRS;
    const int cnt = (int)min<int64_t>(SW_PAIRS, n - base);
    const int t = threadIdx.x;
    if (t < SW_PAIRS) {
        int na = 1, nb = 1, sz = 0;
        int64_t so = 0, d0 = 0;
        if (t < cnt) {
            const int64_t i = base + t;
            const int a = pairs[2 * i], b = pairs[2 * i + 1];
            if (a < 0 || a >= nshell || b < 0 || b >= nshell) {
                atomicOr(err, ERR_PAIR_INDEX);
            } else {
                const int la = l[a], lb = l[b];
                if (la < 0 || la > LMAX || lb < 0 || lb > LMAX) {
                    atomicOr(err, ERR_SHELL_L);
                } else {
                    na = 2 * la + 1;
                    nb = 2 * lb + 1;
                    sz = na * nb;
                    so = src_off[i];
                    d0 = dst_off[i];
                }
            }
        }
        s_na[t] = na;
        s_nb[t] = nb;
        s_rna[t] = 1.0f / (float)na;
        s_rsz[t] = sz ? 1.0f / (float)sz : 0.0f;
        s_src[t] = so;
        s_dst[t] = d0;
        s_beg[t + 1] = sz;
    }
    __syncthreads();
    if (t == 0) {
        s_beg[0] = 0;
        for (int p = 1; p <= SW_PAIRS; ++p) s_beg[p] += s_beg[p - 1];
    }
    __syncthreads();
    const int total = s_beg[SW_PAIRS];
    // values: destination element r of pair p is (mb, ma) = (r / NA, r % NA)
    int cur = 0;
    for (int e0 = 0; e0 < total; e0 += SW_TPB * SW_U) {
        double v[SW_U];
        int64_t di[SW_U];
#pragma unroll
        for (int u = 0; u < SW_U; ++u) {
            const int e = e0 + u * SW_TPB + t;
            di[u] = -1;
            if (e < total) {
                while (s_beg[cur + 1] <= e) ++cur;
                const int r = e - s_beg[cur], na = s_na[cur], mb = small_div(r, s_rna[cur]), ma = r - mb * na;
                v[u] = out[s_src[cur] + ma * s_nb[cur] + mb];
                di[u] = s_dst[cur] + r;
            }
        }
#pragma unroll
        for (int u = 0; u < SW_U; ++u)
            if (di[u] >= 0) out[di[u]] = v[u];
    }
    if (!dout) return;
    // derivatives: three blocks per pair, element e of pair p in [3 beg_p, 3 beg_{p+1})
    cur = 0;
    for (int e0 = 0; e0 < 3 * total; e0 += SW_TPB * SW_U) {
        double v[SW_U];
        int64_t di[SW_U];
#pragma unroll
        for (int u = 0; u < SW_U; ++u) {
            const int e = e0 + u * SW_TPB + t;
            di[u] = -1;
            if (e < 3 * total) {
                while (3 * s_beg[cur + 1] <= e) ++cur;
                const int sz = s_beg[cur + 1] - s_beg[cur], r3 = e - 3 * s_beg[cur], c = small_div(r3, s_rsz[cur]),
                          r = r3 - c * sz;
                const int na = s_na[cur], mb = small_div(r, s_rna[cur]), ma = r - mb * na;
                v[u] = -dout[3 * s_src[cur] + c * sz + ma * s_nb[cur] + mb];
                di[u] = 3 * s_dst[cur] + r3;
            }
        }
#pragma unroll
        for (int u = 0; u < SW_U; ++u)
            if (di[u] >= 0) dout[di[u]] = v[u];
    }
}

}  // namespace

extern "C" int shg_pairs_swap(shg_ctx *c, const shg_shells *sh, const int32_t *pairs, int64_t n,
                              const int64_t *src_off, const int64_t *dst_off, double *out, double *dout)
{
    const char *what = "shg_pairs_swap";
    if (!c) return SHG_EINVAL;
    if (n < 0) return set_err(c, SHG_EINVAL, "%s: n < 0", what);
    if (n >= (int64_t)1 << 31) return set_err(c, SHG_EINVAL, "%s: n >= 2^31 pairs per call", what);
    int rc = check_shells(c, sh, what);
    if (rc) return rc;
    hipStream_t s = c->stream;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, c->err, 0, 1);   // what shg_pairs_swap_check reads
    if (n == 0) {
        HIP_TRY(c, hipGetLastError());
        return 0;
    }
    if (!pairs || !src_off || !dst_off || !out) return set_err(c, SHG_EINVAL, "%s: NULL pointer argument", what);
    hipLaunchKernelGGL(k_swap_blocks, dim3((unsigned)((n + SW_PAIRS - 1) / SW_PAIRS)), dim3(SW_TPB), 0, s, n, pairs,
                       sh->nshell, sh->l, src_off, dst_off, out, dout, c->err);
    HIP_TRY(c, hipGetLastError());
    return 0;
}

extern "C" int shg_pairs_swap_check(shg_ctx *c)
{
    if (!c) return SHG_EINVAL;
    HIP_TRY(c, hipMemcpyAsync(c->host_rb, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return decode_err(c, c->host_rb[0], "shg_pairs_swap");
}
