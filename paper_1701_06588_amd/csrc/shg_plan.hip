// shg_plan.hip -- batched path: a plan bins a fixed pair list once, orders its
// tiles into a work queue and records the evaluation in a hipGraph that can be
// replayed (picking up new centers, exponents or coefficients written into the
// same device buffers) without any host synchronisation.
//
// Two execution modes, chosen at creation (SHG_PLAN_PERSISTENT) or by
// shg_plan_autotune:
//   per-class   the per-class k_tile launches of the plain path, graph-captured
//   persistent  one k_persist launch over a tile work queue
// A screened plan decides on every execution, on the device, which pairs are
// evaluated; nothing is read back to the host. By default the persistent
// kernel tests each pair's analytic bound (or reads the learned predictor's
// decision) before its radial sum and stores a skipped pair's block as zeros.
// With SHG_PLAN_COMPACT a stage runs first: bound or predictor per pair, a
// scan that compacts the kept class-sorted records, the tile queue built from
// the kept counts, the skipped blocks zeroed; the persistent kernel then reads
// the number of tiles from device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "shg_ctx.h"
#include "shg_persist.h"

using namespace shg;

struct shg_plan {
    shg_ctx *ctx = nullptr;
    shg_shells sh{};
    int op = 0;
    double omega = 0;
    const int32_t *pairs = nullptr;
    int64_t n = 0;
    const int64_t *out_off = nullptr;
    double *out = nullptr, *dout = nullptr;
    int deriv = 0;
    int mode = 0;                     // 0 per-class launches, 1 persistent
    int qorder = 2;                   // tile order: 0 heaviest first, 1 alternating ends, 2 round robin
    int32_t *order = nullptr;         // class-sorted pair ids (plan-owned)
    PairRec *rec = nullptr;           // class-sorted pair records (plan-owned; compacting: the kept ones)
    double *w = nullptr;              // folded weights (plan-owned)
    QTile *queue = nullptr;
    int ntiles = 0;                   // screened: the most tiles a queue can hold
    // persistent mode: heavy classes (the first nt_h tiles of the queue) and light
    // classes each run by a kernel of their own group (split), or one kernel of
    // all classes (compacting screened plans)
    int split = 0, nt_h = 0, grid_h = 0, grid_l = 0;
    size_t smem_h = 0, smem_l = 0;
    int *counter = nullptr;           // [0] tile counter; screened plans: the meta block below
    // screening on the device (screened plans); meta: [0] tile counter; compacting
    // mode [1] tiles, [2] kept, [3] skipped,
    // [META_KS + c] kept start of class c, [META_TS + k] first tile of the k-th
    // class of the queue order
    int screened = 0;
    int compact = 0;                  // screened: compaction stage (else in-kernel skipping)
    double tau = 0;
    shg_mlp *mlp = nullptr;
    PairRec *rec_all = nullptr;       // class-sorted records of every pair
    uint8_t *keep = nullptr;          // [n] decision per sorted position (1 kept)
    int32_t *bsum = nullptr;          // [2][nblk + 1]: kept per scan block, exclusive scan
    int32_t *skip = nullptr;          // [n] sorted positions of the skipped pairs (compacting mode)
    double *stats = nullptr;          // per-shell screening statistics
    float *swork = nullptr;           // model inference scratch (n * 15 floats)
    int64_t cls_all[NCLASS + 1] = {}; // class starts of the unscreened sorted order
    int grid = 0;
    size_t smem = 0;
    TileShape shapes[NCLASS] = {};    // per-class launches (tuned shapes)
    int64_t cls_start[NCLASS + 1] = {};
    hipStream_t cap_stream = nullptr;
    // two recorded graphs: the stage (shell preparation, radial or screening
    // stage) and the evaluation kernels, launched back to back
    hipGraph_t graph = nullptr, graph_k = nullptr;
    hipGraphExec_t exec = nullptr, exec_k = nullptr;
    // kernel timing (shg_plan_time_kernels): event pairs around the evaluation graph
    int timing = 0;
    std::vector<hipEvent_t> tev;      // 2 per timed execution
    int tev_used = 0;
    double *T = nullptr;              // precomputed-monopole operators: radial terms per sorted position
    int nr = 0;                       // (a|r_a^{2n}|b): n
};

// plan operator code of (a|r_a^{2n}|b) (outside the shg_op range)
constexpr int PLAN_OP_R2N = 16;
static bool plan_mono(int op) { return op == SHG_GCOULOMB || op == PLAN_OP_R2N; }

__global__ void k_make_recs(int64_t n, const int32_t *order, const int32_t *pairs, const int64_t *out_off, PairRec *rec);

// tile arguments of a plan: two-center mode, or for exp(-omega r^2)/r the
// precomputed-monopole mode over the plan's radial-term buffer
static TileArgs plan_tile_args(const shg_plan *p)
{
    TileArgs ta{p->rec, p->order, p->sh.center, p->sh.nprim, p->sh.prim_off, p->sh.exps, p->w, p->ctx->boys, p->out,
                p->dout, p->omega, p->op};
    if (p->screened && !p->compact) {
        ta.sstat = p->stats;
        ta.sbt = (const BoundTab *)p->ctx->bound_tab;
        ta.skeep = p->mlp ? p->keep : nullptr;    // the model's flags, from the stage
        ta.sflag = p->mlp ? nullptr : p->keep;    // else the kernel records the bound's decisions
        ta.stau = p->tau;
    }
    if (plan_mono(p->op)) {
        ta.triples = p->pairs;
        ta.tstride = 2;
        ta.ooff = p->out_off;
        ta.P = p->T;
        ta.pstride = MONO_TSTRIDE;
        ta.poff = 0;
        ta.ybase = 0;
    }
    return ta;
}

// the radial stage of the operators evaluated in precomputed-monopole mode
static void plan_radial(const shg_plan *p, hipStream_t s)
{
    if (!plan_mono(p->op)) return;
    for (int cls = 0; cls < NCLASS; ++cls) {
        const int64_t b0 = p->cls_start[cls], b1 = p->cls_start[cls + 1];
        if (b1 <= b0) continue;
        if (p->op == SHG_GCOULOMB)
            gc_radial_range(s, cls, p->deriv != 0, &p->sh, p->pairs, p->order, p->w, p->ctx->boys, p->omega, p->T,
                            b0, b1 - b0);
        else
            r2n_radial_range(s, cls, p->deriv != 0, &p->sh, p->pairs, p->order, p->w, p->nr, p->T, b0, b1 - b0);
    }
}

// ---------------------------------------------------------------------------
// device screening stage of screened plans
// ---------------------------------------------------------------------------
constexpr int META_KS = 8, META_TS = META_KS + NCLASS + 1, META_N = META_TS + NCLASS + 1;
constexpr int SCAN_TPB = 256, SCAN_ITEMS = 16, SCAN_BLK = SCAN_TPB * SCAN_ITEMS;

// the unscreened class starts and the queue's class order (heaviest first)
struct ScreenShape {
    int32_t cls_all[NCLASS + 1];
    int32_t cls_seq[NCLASS];
    int32_t nblk;
    int32_t qorder;   // 0 heaviest first, 1 alternating ends
};

// one workgroup: exclusive scan of the kept counts of the scan blocks (written
// by the screening stage), the kept and skipped totals, the kept start of the
// classes that begin at the end of the list; clears the tile counter
__global__ __launch_bounds__(256) void k_keep_scan(ScreenShape ss, const int32_t *bsum, int32_t *bscan, int32_t *meta)
{
    __shared__ int32_t part[256];
    const int t = threadIdx.x, nb = ss.nblk;
    const int per = (nb + 255) / 256;
    const int lo = min(nb, t * per), hi = min(nb, lo + per);
    int32_t acc = 0;
    for (int b = lo; b < hi; ++b) acc += bsum[b];
    part[t] = acc;
    __syncthreads();
    if (t == 0) {
        int32_t run = 0;
        for (int i = 0; i < 256; ++i) {
            const int32_t v = part[i];
            part[i] = run;
            run += v;
        }
        part[0] = run;   // (thread 0 already holds its own prefix, 0)
    }
    __syncthreads();
    const int32_t total = part[0];
    acc = t == 0 ? 0 : part[t];
    for (int b = lo; b < hi; ++b) {
        bscan[b] = acc;
        acc += bsum[b];
    }
    if (t <= NCLASS && ss.cls_all[t] >= ss.cls_all[NCLASS]) meta[META_KS + t] = total;
    if (t == 0) {
        bscan[nb] = total;
        meta[0] = 0;
        meta[2] = total;
        meta[3] = ss.cls_all[NCLASS] - total;
    }
}

// stable compaction: kept sorted position i -> rec[kept before i] = rec_all[i];
// skipped position i -> skip[skipped before i] = i; the kept start of every
// class that begins inside the list. A thread owns SCAN_ITEMS consecutive
// positions of its block (one 16-byte load of their flags).
__global__ __launch_bounds__(SCAN_TPB) void k_compact(int64_t n, ScreenShape ss, const uint8_t *keep,
                                                      const int32_t *bscan, const PairRec *rec_all, PairRec *rec,
                                                      int32_t *skip, int32_t *meta)
{
    static_assert(SCAN_ITEMS == 16, "one 16-byte load of flags per thread");
    __shared__ int32_t wsum[SCAN_TPB / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLK + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t flags = 0;
    if (base + SCAN_ITEMS <= n) {
        const uint4 v = *(const uint4 *)(keep + base);
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 16; ++q) flags |= (((w4[q >> 2] >> (8 * (q & 3))) & 0xffu) != 0 ? 1u : 0u) << q;
    } else {
        for (int q = 0; q < 16 && base + q < n; ++q) flags |= (keep[base + q] != 0 ? 1u : 0u) << q;
    }
    const int cnt = __popc(flags);
    // inclusive scan of the per-thread counts within the wave, then across waves
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t inc = cnt;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t v = __shfl_up(inc, d, 64);
        if (lane >= d) inc += v;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int32_t wbase = 0;
    for (int q = 0; q < wv; ++q) wbase += wsum[q];
    const int32_t kept0 = bscan[blockIdx.x] + wbase + inc - cnt;   // kept before this thread's first position
    // kept starts of the classes beginning in this thread's positions
    for (int c = 0; c <= NCLASS; ++c) {
        const int32_t pos = ss.cls_all[c];
        if (pos >= base && pos < base + SCAN_ITEMS && pos < n)
            meta[META_KS + c] = kept0 + __popc(flags & ((1u << (pos - base)) - 1u));
    }
    int32_t kept = kept0;
    int64_t skipped = base - kept0;
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const int64_t i = base + q;
        if (i >= n) break;
        if ((flags >> q) & 1u) rec[kept++] = rec_all[i];
        else skip[skipped++] = (int32_t)i;
    }
}

// tile queue of the kept pairs: 64-pair tiles, classes in queue order
// (heaviest first; alternately from the two ends with qorder 1); the tile
// count goes to meta[1] for the persistent kernel
__global__ void k_build_queue(ScreenShape ss, int32_t *meta, int max_tiles, QTile *q)
{
    int32_t ks[NCLASS + 1], ts[NCLASS + 1];
#pragma unroll
    for (int c = 0; c <= NCLASS; ++c) ks[c] = meta[META_KS + c];
    int32_t ntiles = 0;
#pragma unroll
    for (int k = 0; k < NCLASS; ++k) {
        const int c = ss.cls_seq[k];
        ts[k] = ntiles;
        ntiles += (ks[c + 1] - ks[c] + 63) / 64;
    }
    ts[NCLASS] = ntiles;
    if (blockIdx.x == 0 && threadIdx.x == 0) meta[1] = ntiles;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < max_tiles; j += gridDim.x * blockDim.x) {
        if (j >= ntiles) break;
        const int src = ss.qorder == 1 ? ((j & 1) ? ntiles - 1 - (j >> 1) : (j >> 1)) : j;
        int k = 0;
        while (k + 1 < NCLASS && ts[k + 1] <= src) ++k;
        const int c = ss.cls_seq[k];
        const int32_t u = src - ts[k];
        q[j] = QTile{c, min(64, ks[c + 1] - ks[c] - 64 * u), (int64_t)ks[c] + 64 * (int64_t)u};
    }
}

// skipped blocks (values and d/dR_a) set to zero, one wave per pair
__global__ void k_zero_skipped(const int32_t *meta, const int32_t *skip, const PairRec *rec_all, const int32_t *l,
                               double *out, double *dout)
{
    const int64_t nskip = meta[3];
    const int lane = threadIdx.x & 63;
    for (int64_t j = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; j < nskip;
         j += (int64_t)gridDim.x * (blockDim.x / 64)) {
        const PairRec r = rec_all[skip[j]];
        const int sz = (2 * l[r.a] + 1) * (2 * l[r.b] + 1);
        for (int e = lane; e < sz; e += 64) out[r.off + e] = 0.0;
        if (dout)
            for (int e = lane; e < 3 * sz; e += 64) dout[3 * r.off + e] = 0.0;
    }
}

static ScreenShape plan_screen_shape(const shg_plan *p)
{
    ScreenShape ss{};
    for (int c = 0; c <= NCLASS; ++c) ss.cls_all[c] = (int32_t)p->cls_all[c];
    std::vector<std::pair<double, int>> cls_cost;
    for (int cls = 0; cls < NCLASS; ++cls) {
        const int la = cls / (LMAX + 1), lb = cls % (LMAX + 1);
        cls_cost.push_back({-((double)(2 * la + 1) * (2 * lb + 1) * (p->deriv ? 4 : 1) + 4.0 * (la + lb + 1)), cls});
    }
    std::stable_sort(cls_cost.begin(), cls_cost.end());
    for (int q = 0; q < NCLASS; ++q) ss.cls_seq[q] = cls_cost[q].second;
    ss.nblk = (int32_t)((p->n + SCAN_BLK - 1) / SCAN_BLK);
    ss.qorder = p->qorder == 0 ? 0 : 1;
    return ss;
}

// screening stage. In-kernel mode: per-shell statistics (and with a model the
// decision flags), skip count and tile counter cleared; the persistent kernel
// decides per pair. Compaction mode: decisions, compaction, tile queue, skipped
// blocks zeroed.
static int plan_screen_stage(shg_plan *p, hipStream_t s)
{
    shg_ctx *c = p->ctx;
    const int64_t n = p->n;
    if (n == 0) return 0;
    if (!p->compact) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, p->counter, 0, p->split ? 2 : 1);
        int rc = plan_screen_enqueue(c, s, &p->sh, p->w, p->stats, p->rec_all, n, 1, &p->op, &p->omega, p->deriv,
                                     p->tau, p->mlp, p->swork, p->mlp ? p->keep : nullptr, nullptr);
        if (rc) return rc;
        HIP_TRY(c, hipGetLastError());
        return 0;
    }
    const ScreenShape ss = plan_screen_shape(p);
    int32_t *bscan = p->bsum + ss.nblk + 1;
    hipLaunchKernelGGL(k_fill_i32, dim3((ss.nblk + 1 + 255) / 256), dim3(256), 0, s, p->bsum, 0, ss.nblk + 1);
    int rc = plan_screen_enqueue(c, s, &p->sh, p->w, p->stats, p->rec_all, n, 1, &p->op, &p->omega, p->deriv, p->tau,
                                 p->mlp, p->swork, p->keep, p->bsum);
    if (rc) return rc;
    hipLaunchKernelGGL(k_keep_scan, dim3(1), dim3(256), 0, s, ss, p->bsum, bscan, p->counter);
    hipLaunchKernelGGL(k_compact, dim3(ss.nblk), dim3(SCAN_TPB), 0, s, n, ss, p->keep, bscan, p->rec_all, p->rec,
                       p->skip, p->counter);
    const unsigned qgrid = (unsigned)std::max(1, std::min((p->ntiles + 255) / 256, 1024));
    hipLaunchKernelGGL(k_build_queue, dim3(qgrid), dim3(256), 0, s, ss, p->counter, p->ntiles, p->queue);
    const unsigned zgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 3) / 4, 2048));
    hipLaunchKernelGGL(k_zero_skipped, dim3(zgrid), dim3(256), 0, s, p->counter, p->skip, p->rec_all, p->sh.l, p->out,
                       p->dout);
    HIP_TRY(c, hipGetLastError());
    return 0;
}

static void persist_entry(int deriv, int group, persist_fn *f, persist_occ_fn *occ)
{
    if (deriv) persist_entry_d1(group, f, occ);
    else persist_entry_d0(group, f, occ);
}

static void plan_launch_persist(const shg_plan *p, hipStream_t s, const TileArgs &ta)
{
    persist_fn f;
    persist_occ_fn occ;
    if (!p->split) {
        persist_entry(p->deriv, PG_ALL, &f, &occ);
        // a compacting screened plan's kernel reads the number of tiles from counter[1]
        f(s, p->grid, p->smem, ta, p->queue, p->screened && p->compact ? -1 : p->ntiles, p->counter);
        return;
    }
    // heavy tiles first, on tile counter [0]; the light ones after, on counter [1]
    if (p->nt_h > 0) {
        persist_entry(p->deriv, PG_HEAVY, &f, &occ);
        f(s, p->grid_h, p->smem_h, ta, p->queue, p->nt_h, p->counter);
    }
    if (p->ntiles > p->nt_h) {
        persist_entry(p->deriv, PG_LIGHT, &f, &occ);
        f(s, p->grid_l, p->smem_l, ta, p->queue + p->nt_h, p->ntiles - p->nt_h, p->counter + 1);
    }
}

// shell preparation and the stage before the evaluation kernels (radial terms
// of the precomputed-monopole operators, or screening; the tile counter)
static int plan_enqueue_stage(shg_plan *p, hipStream_t s)
{
    shg_ctx *c = p->ctx;
    const shg_shells *sh = &p->sh;
    if (sh->nshell > 0)
        hipLaunchKernelGGL(k_prep_shells, dim3((sh->nshell + 3) / 4), dim3(256), 0, s, sh->nshell, sh->l, sh->nprim,
                           sh->prim_off, sh->exps, sh->coefs, sh->nprim_total, LMAX, p->w, c->err);
    plan_radial(p, s);
    if (p->screened) {
        int rc = plan_screen_stage(p, s);   // also clears the tile counter
        if (rc) return rc;
    } else if (p->mode == 1 && p->ntiles > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, p->counter, 0, p->split ? 2 : 1);
    }
    HIP_TRY(c, hipGetLastError());
    return 0;
}

// the evaluation kernels: the persistent kernel or the per-class launches
static int plan_enqueue_kernels(shg_plan *p, hipStream_t s)
{
    const TileArgs ta = plan_tile_args(p);
    if (p->mode == 1) {
        if (p->ntiles > 0) plan_launch_persist(p, s, ta);
    } else {
        for (int cls = 0; cls < NCLASS; ++cls) {
            int64_t b0 = p->cls_start[cls], b1 = p->cls_start[cls + 1];
            if (b1 <= b0) continue;
            tile_table(cls / (LMAX + 1))[(cls % (LMAX + 1)) * 2 + p->deriv](s, ta, b0, b1 - b0, p->shapes[cls]);
        }
    }
    HIP_TRY(p->ctx, hipGetLastError());
    return 0;
}

static int plan_enqueue(shg_plan *p, hipStream_t s)
{
    int rc = plan_enqueue_stage(p, s);
    return rc ? rc : plan_enqueue_kernels(p, s);
}

static void plan_free_graph(shg_plan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->exec_k) (void)hipGraphExecDestroy(p->exec_k);
    if (p->graph_k) (void)hipGraphDestroy(p->graph_k);
    p->exec = p->exec_k = nullptr;
    p->graph = p->graph_k = nullptr;
}

static int capture_one(shg_plan *p, int (*enq)(shg_plan *, hipStream_t), hipGraph_t *graph, hipGraphExec_t *exec)
{
    shg_ctx *c = p->ctx;
    HIP_TRY(c, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enq(p, p->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return set_err(c, SHG_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    *graph = g;
    HIP_TRY(c, hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
    return 0;
}

static int plan_capture(shg_plan *p)
{
    shg_ctx *c = p->ctx;
    plan_free_graph(p);
    if (!p->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    int rc = capture_one(p, plan_enqueue_stage, &p->graph, &p->exec);
    if (!rc) rc = capture_one(p, plan_enqueue_kernels, &p->graph_k, &p->exec_k);
    return rc;
}

// builds the tile queue of the persistent kernels: tiles of 64 pairs and the
// compiled schedule of each class (its LDS need sets the dynamic LDS of the
// launch). Split plans queue the heavy classes' tiles first, then the light
// ones; the tile order applies within each part.
static int plan_build_queue(shg_plan *p)
{
    shg_ctx *c = p->ctx;
    const bool split = !(p->screened && p->compact);
    std::vector<QTile> q;
    size_t smem_g[3] = {0, 0, 0};
    int nt_g[3] = {0, 0, 0};
    constexpr int TP = 64;
    const int groups[2] = {PG_HEAVY, PG_LIGHT};
    for (int gi = 0; gi < (split ? 2 : 1); ++gi) {
        const int group = split ? groups[gi] : PG_ALL;
        std::vector<std::pair<double, int>> cls_cost;
        for (int cls = 0; cls < NCLASS; ++cls) {
            int la = cls / (LMAX + 1), lb = cls % (LMAX + 1);
            if (!persist_has(group, la, lb)) continue;
            double per_pair = (double)(2 * la + 1) * (2 * lb + 1) * (p->deriv ? 4 : 1) + 4.0 * (la + lb + 1);
            cls_cost.push_back({-per_pair, cls});
        }
        std::sort(cls_cost.begin(), cls_cost.end());
        std::vector<QTile> g;
        for (auto &cc : cls_cost) {
            int cls = cc.second;
            int64_t b0 = p->cls_start[cls], b1 = p->cls_start[cls + 1];
            int la = cls / (LMAX + 1), lb = cls % (LMAX + 1);
            if (b1 > b0) {
                size_t b = (size_t)tile_smem_bytes_rt(TP, sched_rows(la, lb, p->deriv != 0), lb, p->deriv != 0);
                smem_g[group] = std::max(smem_g[group], b);
            }
            for (int64_t s0 = b0; s0 < b1; s0 += TP)
                g.push_back(QTile{cls, (int32_t)std::min<int64_t>(TP, b1 - s0), s0});
        }
        if (p->qorder == 1) {
            // alternate from the two ends of the heaviest-first order: co-resident
            // workgroups then mix arithmetic-heavy tiles with light, load/store-bound
            // ones, and the launch ends on tiles of middle weight
            std::vector<QTile> z;
            z.reserve(g.size());
            size_t lo = 0, hi = g.size();
            while (lo < hi) {
                z.push_back(g[lo++]);
                if (lo < hi) z.push_back(g[--hi]);
            }
            g.swap(z);
        } else if (p->qorder == 2) {
            // round robin over the classes, heaviest class first in every round
            std::vector<std::vector<QTile>> per(NCLASS);
            std::vector<int> cls_seq;
            for (const auto &t : g) {
                if (per[t.cls].empty()) cls_seq.push_back(t.cls);
                per[t.cls].push_back(t);
            }
            std::vector<QTile> z;
            z.reserve(g.size());
            std::vector<size_t> pos(NCLASS, 0);
            while (z.size() < g.size())
                for (int cls : cls_seq)
                    if (pos[cls] < per[cls].size()) z.push_back(per[cls][pos[cls]++]);
            g.swap(z);
        }
        nt_g[group] = (int)g.size();
        q.insert(q.end(), g.begin(), g.end());
    }
    if (q.size() >= (size_t)1 << 31) return set_err(c, SHG_EINVAL, "plan: too many tiles");
    if (p->queue) { HIP_TRY(c, hipFree(p->queue)); p->queue = nullptr; }
    p->ntiles = (int)q.size();
    p->split = split ? 1 : 0;
    p->nt_h = nt_g[PG_HEAVY];
    p->smem_h = smem_g[PG_HEAVY];
    p->smem_l = smem_g[PG_LIGHT];
    p->smem = split ? std::max(p->smem_h, p->smem_l) : smem_g[PG_ALL];
    if (p->smem > (size_t)PERSIST_MAX_SMEM && p->mode == 1)
        return set_err(c, SHG_EINVAL, "plan: tile shapes need %zu bytes of LDS, more than the persistent kernel allows",
                       p->smem);
    if (!q.empty()) {
        HIP_TRY(c, hipMalloc((void **)&p->queue, q.size() * sizeof(QTile)));
        HIP_TRY(c, hipMemcpy(p->queue, q.data(), q.size() * sizeof(QTile), hipMemcpyHostToDevice));
    }
    hipDeviceProp_t prop;
    HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
    // the occupancy queries also raise the kernels' LDS limits, before any graph capture
    const auto grid_of = [&](int group, size_t smem, int nt) {
        persist_fn f;
        persist_occ_fn occ;
        persist_entry(p->deriv, group, &f, &occ);
        return std::max(1, std::min(nt, prop.multiProcessorCount * occ(smem)));
    };
    if (split) {
        p->grid_h = grid_of(PG_HEAVY, p->smem_h, p->nt_h);
        p->grid_l = grid_of(PG_LIGHT, p->smem_l, p->ntiles - p->nt_h);
    }
    p->grid = grid_of(PG_ALL, p->smem, p->ntiles);
    return 0;
}

static int plan_create_impl(shg_ctx *c, const shg_shells *sh, int op, double omega, int nr, const int32_t *pairs,
                            int64_t n, const int64_t *out_off, double *out, double *dout, unsigned flags,
                            shg_plan **plan)
{
    const bool deriv = dout != nullptr;
    if (flags & ~(SHG_PLAN_PERSISTENT | SHG_PLAN_NO_GRAPH))
        return set_err(c, SHG_EINVAL, "plan: flags 0x%x not known here (SHG_PLAN_COMPACT is for screened plans)",
                       flags & ~(SHG_PLAN_PERSISTENT | SHG_PLAN_NO_GRAPH));
    // evaluate once through the plain path: validates the input and bins the pairs
    int rc = op == PLAN_OP_R2N ? shg_pairs_r2n(c, sh, nr, pairs, n, out_off, out, dout)
             : deriv           ? shg_pairs_deriv(c, sh, (shg_op)op, omega, pairs, n, out_off, out, dout)
                               : shg_pairs(c, sh, (shg_op)op, omega, pairs, n, out_off, out);
    if (rc) return rc;
    shg_plan *p = new (std::nothrow) shg_plan();
    if (!p) return set_err(c, SHG_ENOMEM, "shg_plan_create: out of host memory");
    p->ctx = c;
    p->sh = *sh;
    p->op = op;
    p->nr = nr;
    p->omega = omega;
    p->pairs = pairs;
    p->n = n;
    p->out_off = out_off;
    p->out = out;
    p->dout = dout;
    p->deriv = deriv ? 1 : 0;
    p->mode = (flags & SHG_PLAN_PERSISTENT) ? 1 : 0;
    for (int cls = 0; cls <= NCLASS; ++cls) p->cls_start[cls] = n > 0 ? c->host_rb[cls * 64] : 0;
    // tuned shapes of the nearest in-kernel operator
    const int sop = op == SHG_GCOULOMB ? (int)SHG_COULOMB : op == PLAN_OP_R2N ? (int)SHG_OVERLAP : op;
    for (int cls = 0; cls < NCLASS; ++cls) p->shapes[cls] = c->shape[sop][cls / (LMAX + 1)][cls % (LMAX + 1)][p->deriv];
    auto fail = [&](int code) { shg_plan_destroy(p); return code; };
    hipError_t e = hipMalloc((void **)&p->order, std::max<int64_t>(n, 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&p->rec, std::max<int64_t>(n, 1) * sizeof(PairRec));
    if (e == hipSuccess) e = hipMalloc((void **)&p->w, std::max<int64_t>(sh->nprim_total, 1) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&p->counter, 64 * sizeof(int));
    if (e == hipSuccess && plan_mono(op))
        e = hipMalloc((void **)&p->T, std::max<int64_t>(n, 1) * MONO_TSTRIDE * sizeof(double));
    if (e != hipSuccess) return fail(set_err(c, SHG_ENOMEM, "shg_plan_create: %s", hipGetErrorString(e)));
    if (n > 0) {
        e = hipMemcpyAsync(p->order, c->order, n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess && plan_mono(op)) {
            // the precomputed-monopole path leaves no pair records in the context
            hipLaunchKernelGGL(k_make_recs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, p->order,
                               pairs, out_off, p->rec);
            e = hipGetLastError();
        } else if (e == hipSuccess) {
            e = hipMemcpyAsync(p->rec, c->rec, n * sizeof(PairRec), hipMemcpyDeviceToDevice, c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(set_err(c, SHG_EDEVICE, "shg_plan_create: %s", hipGetErrorString(e)));
    }
    if ((rc = plan_build_queue(p))) return fail(rc);
    if (!(flags & SHG_PLAN_NO_GRAPH) && (rc = plan_capture(p))) return fail(rc);
    *plan = p;
    return 0;
}

extern "C" int shg_plan_create(shg_ctx *c, const shg_shells *sh, shg_op op, double omega, const int32_t *pairs,
                               int64_t n, const int64_t *out_off, double *out, double *dout, unsigned flags,
                               shg_plan **plan)
{
    if (!c || !plan) return SHG_EINVAL;
    *plan = nullptr;
    if ((int)op < 0 || (int)op > 5) return set_err(c, SHG_EINVAL, "shg_plan_create: unknown operator %d", (int)op);
    return plan_create_impl(c, sh, (int)op, omega, 0, pairs, n, out_off, out, dout, flags, plan);
}

extern "C" int shg_plan_create_r2n(shg_ctx *c, const shg_shells *sh, int nr, const int32_t *pairs, int64_t n,
                                   const int64_t *out_off, double *out, double *dout, unsigned flags, shg_plan **plan)
{
    if (!c || !plan) return SHG_EINVAL;
    *plan = nullptr;
    return plan_create_impl(c, sh, PLAN_OP_R2N, 0.0, nr, pairs, n, out_off, out, dout, flags, plan);
}

// records of the pairs in `order` (precomputed-monopole plans)
__global__ void k_make_recs(int64_t n, const int32_t *order, const int32_t *pairs, const int64_t *out_off, PairRec *rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p = order[i];
    rec[i] = PairRec{pairs[2 * p], pairs[2 * p + 1], out_off[p]};
}

// reads the decision of the last execution back: kept and skipped counts and
// the kept class starts (synchronises the context stream)
static int plan_read_flags(const shg_plan *p, std::vector<uint8_t> &f)
{
    f.resize(p->n);
    if (p->n > 0 && hipMemcpy(f.data(), p->keep, p->n, hipMemcpyDeviceToHost) != hipSuccess)
        return set_err(p->ctx, SHG_EDEVICE, "plan: read-back failed");
    return 0;
}

static int plan_read_meta(const shg_plan *p, int64_t *kept, int64_t *skipped, int64_t *ks)
{
    shg_ctx *c = p->ctx;
    int32_t m[META_N];
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(m, p->counter, sizeof(m), hipMemcpyDeviceToHost));
    if (p->compact) {
        if (kept) *kept = m[2];
        if (skipped) *skipped = m[3];
        if (ks)
            for (int cls = 0; cls <= NCLASS; ++cls) ks[cls] = m[META_KS + cls];
        return 0;
    }
    // in-kernel mode: one decision flag per class-sorted position
    std::vector<uint8_t> f;
    if (int rc = plan_read_flags(p, f)) return rc;
    std::vector<int64_t> cnt(NCLASS, 0);
    int64_t ns = 0;
    for (int cls = 0; cls < NCLASS; ++cls)
        for (int64_t q = p->cls_all[cls]; q < p->cls_all[cls + 1]; ++q) cnt[cls] += f[q] == 0;
    for (int cls = 0; cls < NCLASS; ++cls) ns += cnt[cls];
    if (kept) *kept = p->n - ns;
    if (skipped) *skipped = ns;
    if (ks) {
        ks[0] = 0;
        for (int cls = 0; cls < NCLASS; ++cls) ks[cls + 1] = ks[cls] + (p->cls_all[cls + 1] - p->cls_all[cls]) - cnt[cls];
    }
    return 0;
}

extern "C" int shg_plan_create_screened(shg_ctx *c, const shg_shells *sh, shg_op op, double omega,
                                        const int32_t *pairs, int64_t n, const int64_t *out_off, double *out,
                                        double *dout, unsigned flags, double tau, shg_mlp *mlp, shg_plan **plan,
                                        int64_t *n_skipped)
{
    const char *what = "shg_plan_create_screened";
    if (!c || !plan) return SHG_EINVAL;
    *plan = nullptr;
    if (!(tau > 0.0) || !(tau < 1e300)) return set_err(c, SHG_EINVAL, "%s: tau must be positive and finite", what);
    if ((int)op < 0 || (int)op > 4) return set_err(c, SHG_EINVAL, "%s: operator %d cannot be screened", what, (int)op);
    if (flags & SHG_PLAN_NO_GRAPH) return set_err(c, SHG_EINVAL, "%s: screened plans are always recorded", what);
    shg_plan *p = nullptr;
    int rc = shg_plan_create(c, sh, op, omega, pairs, n, out_off, out, dout,
                             ((flags & ~SHG_PLAN_COMPACT) | SHG_PLAN_PERSISTENT | SHG_PLAN_NO_GRAPH), &p);
    if (rc) return rc;
    auto fail = [&](int code) { shg_plan_destroy(p); return code; };
    if (p->smem > (size_t)PERSIST_MAX_SMEM)
        return fail(set_err(c, SHG_EINVAL, "%s: the persistent kernel cannot take these tiles", what));
    p->screened = 1;
    p->compact = (flags & SHG_PLAN_COMPACT) ? 1 : 0;
    if (p->compact) {
        p->split = 0;     // its queue is built on the device for the all-class kernel,
        p->qorder = 1;    // in the first two orders only
    }
    p->mode = 1;
    p->tau = tau;
    p->mlp = mlp;
    for (int cls = 0; cls <= NCLASS; ++cls) p->cls_all[cls] = p->cls_start[cls];
    const int64_t nb = (n + SCAN_BLK - 1) / SCAN_BLK;
    hipError_t e = hipSuccess;
    if (n > 0) {
        e = hipMalloc((void **)&p->rec_all, n * sizeof(PairRec));
        if (e == hipSuccess) e = hipMalloc((void **)&p->keep, ((n + 15) / 16 * 16) * sizeof(uint8_t));
        if (e == hipSuccess && p->compact) e = hipMalloc((void **)&p->skip, n * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc((void **)&p->bsum, 2 * (nb + 1) * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc((void **)&p->stats, plan_screen_stats_doubles(sh->nshell) * sizeof(double));
        if (e == hipSuccess && mlp) e = hipMalloc((void **)&p->swork, (size_t)n * 15 * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(p->rec_all, p->rec, n * sizeof(PairRec), hipMemcpyDeviceToDevice);
    }
    if (e == hipSuccess) {
        (void)hipFree(p->counter);
        p->counter = nullptr;
        e = hipMalloc((void **)&p->counter, META_N * sizeof(int32_t));
    }
    if (e != hipSuccess) return fail(set_err(c, SHG_ENOMEM, "%s: %s", what, hipGetErrorString(e)));
    if ((rc = screen_prepare(c))) return fail(rc);
    if ((rc = plan_capture(p))) return fail(rc);
    // the first execution zeroes the skipped blocks (the plain evaluation of the
    // creation wrote every block) and gives the skip count
    if ((rc = shg_plan_execute(p))) return fail(rc);
    int64_t ns = 0;
    if ((rc = plan_read_meta(p, nullptr, &ns, nullptr))) return fail(rc);
    if (n_skipped) *n_skipped = ns;
    *plan = p;
    return 0;
}

constexpr int PLAN_TIMED_MAX = 1024;

extern "C" int shg_plan_execute(shg_plan *p)
{
    if (!p) return SHG_EINVAL;
    shg_ctx *c = p->ctx;
    const bool timed = p->timing && p->tev_used < PLAN_TIMED_MAX;
    if (timed && (size_t)(2 * p->tev_used + 2) > p->tev.size()) {
        for (int k = 0; k < 2; ++k) {
            hipEvent_t ev;
            HIP_TRY(c, hipEventCreate(&ev));
            p->tev.push_back(ev);
        }
    }
    if (p->exec) HIP_TRY(c, hipGraphLaunch(p->exec, c->stream));
    else if (int rc = plan_enqueue_stage(p, c->stream)) return rc;
    if (timed) HIP_TRY(c, hipEventRecord(p->tev[2 * p->tev_used], c->stream));
    if (p->exec_k) HIP_TRY(c, hipGraphLaunch(p->exec_k, c->stream));
    else if (int rc = plan_enqueue_kernels(p, c->stream)) return rc;
    if (timed) {
        HIP_TRY(c, hipEventRecord(p->tev[2 * p->tev_used + 1], c->stream));
        ++p->tev_used;
    }
    return 0;
}

extern "C" int shg_plan_time_kernels(shg_plan *p, int on)
{
    if (!p) return SHG_EINVAL;
    p->timing = on ? 1 : 0;
    p->tev_used = 0;
    return 0;
}

extern "C" int shg_plan_kernel_time(shg_plan *p, double *ms_sum, int64_t *executions)
{
    if (!p || !ms_sum || !executions) return SHG_EINVAL;
    shg_ctx *c = p->ctx;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double tot = 0;
    for (int i = 0; i < p->tev_used; ++i) {
        float ms = 0;
        HIP_TRY(c, hipEventElapsedTime(&ms, p->tev[2 * i], p->tev[2 * i + 1]));
        tot += ms;
    }
    *ms_sum = tot;
    *executions = p->tev_used;
    p->tev_used = 0;
    return 0;
}

extern "C" int shg_plan_set_mode(shg_plan *p, int persistent)
{
    if (!p) return SHG_EINVAL;
    if (p->screened && !persistent)
        return set_err(p->ctx, SHG_EINVAL, "plan: a screened plan runs the persistent kernel only");
    if (persistent && p->smem > (size_t)PERSIST_MAX_SMEM)
        return set_err(p->ctx, SHG_EINVAL, "plan: tile shapes need more LDS than the persistent kernel allows");
    p->mode = persistent ? 1 : 0;
    if (p->exec) {
        HIP_TRY(p->ctx, hipStreamSynchronize(p->ctx->stream));
        return plan_capture(p);
    }
    return 0;
}

extern "C" int shg_plan_autotune(shg_plan *p, int reps, double *ms_per_class, double *ms_persistent)
{
    if (!p) return SHG_EINVAL;
    shg_ctx *c = p->ctx;
    if (reps < 1) reps = 1;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    auto time_mode = [&](int mode, float *ms) {
        p->mode = mode;
        int rc = plan_enqueue(p, c->stream);   // warm-up
        if (rc) return rc;
        HIP_TRY(c, hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r)
            if ((rc = plan_enqueue(p, c->stream))) return rc;
        HIP_TRY(c, hipEventRecord(e1, c->stream));
        HIP_TRY(c, hipEventSynchronize(e1));
        HIP_TRY(c, hipEventElapsedTime(ms, e0, e1));
        *ms /= reps;
        return 0;
    };
    float t_class = 0, t_pers = 0;
    int rc = 0;
    // a screened plan runs the persistent kernel only; a compacting one over a
    // queue built on the device in one of the first two orders
    if (!p->screened && (rc = time_mode(0, &t_class))) return rc;
    const bool can_persist = p->smem <= (size_t)PERSIST_MAX_SMEM;
    if (can_persist) {
        // the persistent kernel with each tile order of the queue
        int best_q = p->qorder;
        float best = 0;
        const int norders = p->screened && p->compact ? 2 : 3;
        for (int qo = 0; qo < norders; ++qo) {
            p->qorder = qo;
            if ((rc = plan_build_queue(p))) return rc;
            float t = 0;
            if ((rc = time_mode(1, &t))) return rc;
            if (qo == 0 || t < best) {
                best = t;
                best_q = qo;
            }
        }
        p->qorder = best_q;
        if ((rc = plan_build_queue(p))) return rc;
        t_pers = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms_per_class) *ms_per_class = p->screened ? -1.0 : t_class;
    if (ms_persistent) *ms_persistent = can_persist ? t_pers : -1.0;
    p->mode = p->screened || (can_persist && t_pers < t_class) ? 1 : 0;
    if (p->exec) {
        if ((rc = plan_capture(p))) return rc;
    }
    // a screened plan leaves the outputs of its last decision in place
    if (p->screened) return shg_plan_execute(p);
    return 0;
}

extern "C" int shg_plan_mode(const shg_plan *p) { return p ? p->mode : SHG_EINVAL; }

extern "C" int shg_plan_tile_order(const shg_plan *p) { return p ? p->qorder : SHG_EINVAL; }

extern "C" int shg_plan_set_tile_order(shg_plan *p, int order)
{
    if (!p) return SHG_EINVAL;
    if (order < 0 || order > (p->screened && p->compact ? 1 : 2))
        return set_err(p->ctx, SHG_EINVAL, "plan: tile order %d not available for this plan", order);
    HIP_TRY(p->ctx, hipStreamSynchronize(p->ctx->stream));
    p->qorder = order;
    int rc = plan_build_queue(p);
    if (!rc && p->exec) rc = plan_capture(p);
    return rc;
}

// ids of the pairs the last execution of a screened plan skipped (host array
// of capacity cap; synchronises the context stream); returns their number
// (the full count even when cap is smaller); 0 for unscreened plans
extern "C" int64_t shg_plan_skipped(const shg_plan *p, int32_t *ids, int64_t cap)
{
    if (!p) return SHG_EINVAL;
    if (!p->screened || p->n == 0) return 0;
    int64_t ns = 0;
    int rc = plan_read_meta(p, nullptr, &ns, nullptr);
    if (rc) return rc;
    if (ids && cap > 0 && ns > 0) {
        const int64_t m = std::min(ns, cap);
        std::vector<int32_t> pos, order(p->n);
        if (p->compact) {
            pos.resize(m);
            if (hipMemcpy(pos.data(), p->skip, m * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
                return set_err(p->ctx, SHG_EDEVICE, "shg_plan_skipped: read-back failed");
        } else {
            std::vector<uint8_t> f;
            if ((rc = plan_read_flags(p, f))) return rc;
            for (int64_t q = 0; q < p->n && (int64_t)pos.size() < m; ++q)
                if (f[q] == 0) pos.push_back((int32_t)q);
        }
        if (hipMemcpy(order.data(), p->order, p->n * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
            return set_err(p->ctx, SHG_EDEVICE, "shg_plan_skipped: read-back failed");
        for (int64_t i = 0; i < m; ++i) ids[i] = order[pos[i]];
    }
    return ns;
}

// kept pairs and their algorithmic bytes (output values [+ d/dR_a] + 8 bytes of
// pair indices + 8 bytes of offset per pair), host pointers; a screened plan
// reports its last execution (synchronises the context stream)
extern "C" int shg_plan_stats(const shg_plan *p, int64_t *kept, int64_t *alg_bytes)
{
    if (!p || !kept || !alg_bytes) return SHG_EINVAL;
    int64_t starts[NCLASS + 1];
    for (int cls = 0; cls <= NCLASS; ++cls) starts[cls] = p->cls_start[cls];
    if (p->screened && p->n > 0) {
        int rc = plan_read_meta(p, nullptr, nullptr, starts);
        if (rc) return rc;
    }
    int64_t k = 0, b = 0;
    for (int cls = 0; cls < NCLASS; ++cls) {
        int64_t cnt = starts[cls + 1] - starts[cls];
        int la = cls / (LMAX + 1), lb = cls % (LMAX + 1);
        k += cnt;
        b += cnt * ((int64_t)8 * (2 * la + 1) * (2 * lb + 1) * (p->deriv ? 4 : 1) + 16);
    }
    *kept = k;
    *alg_bytes = b;
    return 0;
}

// average duration (ms) of the evaluation kernels alone (persistent kernel or
// the per-class launches, without the shell preparation or screening stage),
// timed with HIP events over `reps` enqueues on the ctx stream; synchronous. A
// screened plan runs its kernel on the tile queue of its last execution.
extern "C" int shg_plan_kernel_ms(shg_plan *p, int reps, double *ms)
{
    if (!p || !ms || reps < 1) return SHG_EINVAL;
    shg_ctx *c = p->ctx;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    const TileArgs ta = plan_tile_args(p);
    double tot = 0;
    for (int r = 0; r < reps; ++r) {
        if (p->mode >= 1)
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, p->counter, 0, p->split ? 2 : 1);
        HIP_TRY(c, hipEventRecord(e0, c->stream));
        plan_radial(p, c->stream);
        if (p->mode == 1) {
            if (p->ntiles > 0) plan_launch_persist(p, c->stream, ta);
        } else {
            for (int cls = 0; cls < NCLASS; ++cls) {
                int64_t b0 = p->cls_start[cls], b1 = p->cls_start[cls + 1];
                if (b1 > b0)
                    tile_table(cls / (LMAX + 1))[(cls % (LMAX + 1)) * 2 + p->deriv](c->stream, ta, b0, b1 - b0,
                                                                                   p->shapes[cls]);
            }
        }
        HIP_TRY(c, hipEventRecord(e1, c->stream));
        HIP_TRY(c, hipEventSynchronize(e1));
        float t = 0;
        HIP_TRY(c, hipEventElapsedTime(&t, e0, e1));
        tot += t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = tot / reps;
    return 0;
}

extern "C" void shg_plan_destroy(shg_plan *p)
{
    if (!p) return;
    if (p->ctx) (void)hipStreamSynchronize(p->ctx->stream);
    plan_free_graph(p);
    for (hipEvent_t ev : p->tev) (void)hipEventDestroy(ev);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    (void)hipFree(p->order);
    (void)hipFree(p->rec);
    (void)hipFree(p->T);
    (void)hipFree(p->w);
    (void)hipFree(p->queue);
    (void)hipFree(p->counter);
    (void)hipFree(p->rec_all);
    (void)hipFree(p->keep);
    (void)hipFree(p->skip);
    (void)hipFree(p->bsum);
    (void)hipFree(p->stats);
    (void)hipFree(p->swork);
    delete p;
}
