// shg_plan.hip -- batched path: a plan bins a fixed pair list once, orders its
// tiles into a work queue and records the evaluation in a hipGraph that can be
// replayed (picking up new centers, exponents or coefficients written into the
// same device buffers) without any host synchronisation.
//
// Two execution modes, chosen at creation (SHG_PLAN_PERSISTENT) or by
// shg_plan_autotune:
//   per-class   the per-class k_tile launches of the plain path, graph-captured
//   persistent  one k_persist launch over a tile work queue
// A multi-operator plan (shg_plan_create_multi) evaluates several operators on
// the pair list with one k_multi launch over the same queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "shg_ctx.h"
#include "shg_multi.h"
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
    int mode = 0;                     // 0 per-class launches, 1 persistent, 2 multi-operator
    int qorder = 1;                   // tile order: 0 heaviest first, 1 alternating ends, 2 round robin
    int nops = 0;                     // > 0: multi-operator plan
    MultiOps mops{};
    int32_t *order = nullptr;         // class-sorted pair ids (plan-owned)
    PairRec *rec = nullptr;           // class-sorted pair records (plan-owned)
    double *w = nullptr;              // folded weights (plan-owned)
    QTile *queue = nullptr;
    int ntiles = 0;
    int *counter = nullptr;
    int grid = 0;
    size_t smem = 0;
    TileShape shapes[NCLASS] = {};    // per-class launches (tuned shapes)
    int64_t cls_start[NCLASS + 1] = {};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<int32_t> skipped;     // pair ids removed by screening
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

static int plan_enqueue(shg_plan *p, hipStream_t s)
{
    shg_ctx *c = p->ctx;
    const shg_shells *sh = &p->sh;
    if (sh->nshell > 0)
        hipLaunchKernelGGL(k_prep_shells, dim3((sh->nshell + 3) / 4), dim3(256), 0, s, sh->nshell, sh->l, sh->nprim,
                           sh->prim_off, sh->exps, sh->coefs, sh->nprim_total, LMAX, p->w, c->err);
    plan_radial(p, s);
    const TileArgs ta = plan_tile_args(p);
    if (p->nops > 0) {
        if (p->ntiles > 0) {
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, p->counter, 0, 1);
            multi_fn f;
            multi_occ_fn occ;
            if (p->deriv) multi_entry_d1(&f, &occ);
            else multi_entry_d0(&f, &occ);
            f(s, p->grid, ta, p->mops, p->queue, p->ntiles, p->counter);
        }
    } else if (p->mode == 0) {
        for (int cls = 0; cls < NCLASS; ++cls) {
            int64_t b0 = p->cls_start[cls], b1 = p->cls_start[cls + 1];
            if (b1 <= b0) continue;
            tile_table(cls / (LMAX + 1))[(cls % (LMAX + 1)) * 2 + p->deriv](s, ta, b0, b1 - b0, p->shapes[cls]);
        }
    } else if (p->ntiles > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, p->counter, 0, 1);
        persist_fn f;
        persist_occ_fn occ;
        if (p->deriv) persist_entry_d1(&f, &occ);
        else persist_entry_d0(&f, &occ);
        f(s, p->grid, p->smem, ta, p->queue, p->ntiles, p->counter);
    }
    HIP_TRY(c, hipGetLastError());
    return 0;
}

static void plan_free_graph(shg_plan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

static int plan_capture(shg_plan *p)
{
    shg_ctx *c = p->ctx;
    plan_free_graph(p);
    if (!p->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIP_TRY(c, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = plan_enqueue(p, p->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return set_err(c, SHG_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    p->graph = g;
    HIP_TRY(c, hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return 0;
}

// builds the tile queue of the persistent kernels: tiles
// of 64 pairs and the compiled schedule of each class (its LDS need is the
// dynamic LDS of the launch)
static int plan_build_queue(shg_plan *p)
{
    shg_ctx *c = p->ctx;
    std::vector<QTile> q;
    std::vector<std::pair<double, int>> cls_cost;
    for (int cls = 0; cls < NCLASS; ++cls) {
        int la = cls / (LMAX + 1), lb = cls % (LMAX + 1);
        double per_pair = (double)(2 * la + 1) * (2 * lb + 1) * (p->deriv ? 4 : 1) + 4.0 * (la + lb + 1);
        cls_cost.push_back({-per_pair, cls});
    }
    std::sort(cls_cost.begin(), cls_cost.end());
    size_t smem = 0;
    constexpr int TP = 64;
    for (auto &cc : cls_cost) {
        int cls = cc.second;
        int64_t b0 = p->cls_start[cls], b1 = p->cls_start[cls + 1];
        int la = cls / (LMAX + 1), lb = cls % (LMAX + 1);
        if (b1 > b0) {
            size_t b = (size_t)tile_smem_bytes_rt(TP, sched_rows(la, lb, p->deriv != 0), lb, p->deriv != 0);
            smem = std::max(smem, b);
        }
        for (int64_t s0 = b0; s0 < b1; s0 += TP) q.push_back(QTile{cls, (int32_t)std::min<int64_t>(TP, b1 - s0), s0});
    }
    if (p->qorder == 1) {
        // alternate from the two ends of the heaviest-first order: co-resident
        // workgroups then mix arithmetic-heavy tiles with light, load/store-bound
        // ones, and the launch ends on tiles of middle weight
        std::vector<QTile> z;
        z.reserve(q.size());
        size_t lo = 0, hi = q.size();
        while (lo < hi) {
            z.push_back(q[lo++]);
            if (lo < hi) z.push_back(q[--hi]);
        }
        q.swap(z);
    } else if (p->qorder == 2) {
        // round robin over the classes, heaviest class first in every round
        std::vector<std::vector<QTile>> per(NCLASS);
        std::vector<int> cls_seq;
        for (const auto &t : q) {
            if (per[t.cls].empty()) cls_seq.push_back(t.cls);
            per[t.cls].push_back(t);
        }
        std::vector<QTile> z;
        z.reserve(q.size());
        std::vector<size_t> pos(NCLASS, 0);
        while (z.size() < q.size())
            for (int cls : cls_seq)
                if (pos[cls] < per[cls].size()) z.push_back(per[cls][pos[cls]++]);
        q.swap(z);
    }
    if (q.size() >= (size_t)1 << 31) return set_err(c, SHG_EINVAL, "plan: too many tiles");
    if (p->queue) { HIP_TRY(c, hipFree(p->queue)); p->queue = nullptr; }
    p->ntiles = (int)q.size();
    p->smem = smem;
    if (smem > (size_t)PERSIST_MAX_SMEM && p->mode == 1)
        return set_err(c, SHG_EINVAL, "plan: tile shapes need %zu bytes of LDS, more than the persistent kernel allows",
                       smem);
    if (!q.empty()) {
        HIP_TRY(c, hipMalloc((void **)&p->queue, q.size() * sizeof(QTile)));
        HIP_TRY(c, hipMemcpy(p->queue, q.data(), q.size() * sizeof(QTile), hipMemcpyHostToDevice));
    }
    persist_fn f;
    persist_occ_fn occ;
    if (p->deriv) persist_entry_d1(&f, &occ);
    else persist_entry_d0(&f, &occ);
    hipDeviceProp_t prop;
    HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
    // the per-class kernels raise their LDS limit on first launch; make sure that
    // happened before a graph capture by launching nothing here but the query
    int per_cu = occ(p->smem);
    p->grid = std::max(1, std::min(p->ntiles, prop.multiProcessorCount * per_cu));
    return 0;
}

static int plan_create_impl(shg_ctx *c, const shg_shells *sh, int op, double omega, int nr, const int32_t *pairs,
                            int64_t n, const int64_t *out_off, double *out, double *dout, unsigned flags,
                            shg_plan **plan)
{
    const bool deriv = dout != nullptr;
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

// records of the pairs in `order` (after screening removed some)
__global__ void k_make_recs(int64_t n, const int32_t *order, const int32_t *pairs, const int64_t *out_off, PairRec *rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p = order[i];
    rec[i] = PairRec{pairs[2 * p], pairs[2 * p + 1], out_off[p]};
}

__global__ void k_zero_blocks(int64_t ns, const int32_t *ids, const int32_t *pairs, const int32_t *l,
                              const int64_t *out_off, double *out, double *dout)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (i >= ns) return;
    const int p = ids[i];
    const int sz = (2 * l[pairs[2 * (int64_t)p]] + 1) * (2 * l[pairs[2 * (int64_t)p + 1]] + 1);
    const int64_t off = out_off[p];
    for (int e = threadIdx.x % 64; e < sz; e += 64) out[off + e] = 0.0;
    if (dout)
        for (int e = threadIdx.x % 64; e < 3 * sz; e += 64) dout[3 * off + e] = 0.0;
}

// keeps the pairs with hkeep[id] != 0: stable compaction of the class-sorted
// order and records, skipped ids collected, their blocks zeroed in every
// output of the plan, tile queue rebuilt
static int plan_compact(shg_plan *p, const std::vector<int32_t> &hkeep, const std::vector<int32_t> &horder,
                        int64_t *nskip_out)
{
    shg_ctx *c = p->ctx;
    std::vector<int32_t> korder, skipped;
    korder.reserve(p->n);
    int64_t new_start[NCLASS + 1];
    for (int cls = 0; cls < NCLASS; ++cls) {
        new_start[cls] = (int64_t)korder.size();
        for (int64_t q = p->cls_start[cls]; q < p->cls_start[cls + 1]; ++q) {
            int32_t id = horder[q];
            if (hkeep[id]) korder.push_back(id);
            else skipped.push_back(id);
        }
    }
    new_start[NCLASS] = (int64_t)korder.size();
    const int64_t nskip = (int64_t)skipped.size();
    p->skipped = skipped;
    if (!korder.empty()) {
        const int64_t nk = (int64_t)korder.size();
        HIP_TRY(c, hipMemcpy(p->order, korder.data(), nk * sizeof(int32_t), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_make_recs, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, c->stream, nk, p->order,
                           p->pairs, p->out_off, p->rec);
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    for (int cls = 0; cls <= NCLASS; ++cls) p->cls_start[cls] = new_start[cls];
    if (nskip > 0) {
        int32_t *ids = nullptr;
        HIP_TRY(c, hipMalloc((void **)&ids, nskip * sizeof(int32_t)));
        HIP_TRY(c, hipMemcpy(ids, skipped.data(), nskip * sizeof(int32_t), hipMemcpyHostToDevice));
        const int nout = p->nops > 0 ? p->nops : 1;
        for (int o = 0; o < nout; ++o) {
            double *out = p->nops > 0 ? p->mops.out[o] : p->out;
            double *dout = p->nops > 0 ? p->mops.dout[o] : p->dout;
            hipLaunchKernelGGL(k_zero_blocks, dim3((unsigned)((nskip + 3) / 4)), dim3(256), 0, c->stream, nskip, ids,
                               p->pairs, p->sh.l, p->out_off, out, dout);
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        (void)hipFree(ids);
    }
    *nskip_out = nskip;
    return plan_build_queue(p);
}

extern "C" int shg_plan_create_screened(shg_ctx *c, const shg_shells *sh, shg_op op, double omega,
                                        const int32_t *pairs, int64_t n, const int64_t *out_off, double *out,
                                        double *dout, unsigned flags, double tau, shg_mlp *mlp, shg_plan **plan,
                                        int64_t *n_skipped)
{
    if (!c || !plan) return SHG_EINVAL;
    *plan = nullptr;
    if (!(tau > 0.0)) return set_err(c, SHG_EINVAL, "shg_plan_create_screened: tau must be positive");
    shg_plan *p = nullptr;
    int rc = shg_plan_create(c, sh, op, omega, pairs, n, out_off, out, dout, flags | SHG_PLAN_NO_GRAPH, &p);
    if (rc) return rc;
    auto fail = [&](int code) { shg_plan_destroy(p); return code; };
    int64_t nskip = 0;
    if (n > 0) {
        int32_t *keep = nullptr;
        float *work = nullptr;
        HIP_TRY(c, hipMalloc((void **)&keep, n * sizeof(int32_t)));
        if (hipMalloc((void **)&work, (size_t)n * 15 * sizeof(float)) != hipSuccess) {
            (void)hipFree(keep);
            return fail(set_err(c, SHG_ENOMEM, "shg_plan_create_screened: out of device memory"));
        }
        rc = screen_pairs(c, sh, op, omega, pairs, n, p->deriv, tau, mlp, keep, work);
        std::vector<int32_t> hkeep(n), horder(n);
        if (!rc && (hipMemcpy(hkeep.data(), keep, n * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess ||
                    hipMemcpy(horder.data(), p->order, n * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess))
            rc = set_err(c, SHG_EDEVICE, "shg_plan_create_screened: read-back failed");
        (void)hipFree(work);
        (void)hipFree(keep);
        if (rc) return fail(rc);
        if ((rc = plan_compact(p, hkeep, horder, &nskip))) return fail(rc);
    }
    if (!(flags & SHG_PLAN_NO_GRAPH) && (rc = plan_capture(p))) return fail(rc);
    if (n_skipped) *n_skipped = nskip;
    *plan = p;
    return 0;
}

extern "C" int shg_plan_create_multi(shg_ctx *c, const shg_shells *sh, int nops, const shg_op *ops,
                                     const double *omegas, const int32_t *pairs, int64_t n, const int64_t *out_off,
                                     double *const *outs, double *const *douts, double tau, shg_plan **plan,
                                     int64_t *n_skipped)
{
    const char *what = "shg_plan_create_multi";
    if (!c || !plan) return SHG_EINVAL;
    *plan = nullptr;
    if (nops < 1 || nops > MULTI_MAX) return set_err(c, SHG_EINVAL, "%s: 1 to %d operators", what, MULTI_MAX);
    if (!ops || !omegas || !outs) return set_err(c, SHG_EINVAL, "%s: NULL pointer argument", what);
    if (tau < 0.0 || !(tau < 1e300)) return set_err(c, SHG_EINVAL, "%s: tau must be >= 0 and finite", what);
    const bool deriv = douts != nullptr;
    for (int o = 0; o < nops; ++o)
        if (!outs[o] || (deriv && !douts[o])) return set_err(c, SHG_EINVAL, "%s: NULL output pointer", what);
    for (int o = 0; o < nops; ++o)
        if ((int)ops[o] < 0 || (int)ops[o] > 4)
            return set_err(c, SHG_EINVAL, "%s: operator %d is not available in plans", what, (int)ops[o]);
    // every operator once through the plain path: validation and the exact blocks
    int rc = 0;
    for (int o = 0; o < nops; ++o) {
        rc = deriv ? shg_pairs_deriv(c, sh, ops[o], omegas[o], pairs, n, out_off, outs[o], douts[o])
                   : shg_pairs(c, sh, ops[o], omegas[o], pairs, n, out_off, outs[o]);
        if (rc) return rc;
    }
    shg_plan *p = nullptr;
    rc = shg_plan_create(c, sh, ops[0], omegas[0], pairs, n, out_off, outs[0], deriv ? douts[0] : nullptr,
                         SHG_PLAN_NO_GRAPH, &p);
    if (rc) return rc;
    auto fail = [&](int code) { shg_plan_destroy(p); return code; };
    p->nops = nops;
    p->mode = 2;
    p->mops.nops = nops;
    for (int o = 0; o < MULTI_MAX; ++o) {
        const int oo = o < nops ? o : 0;
        p->mops.op[o] = (int)ops[oo];
        p->mops.omega[o] = omegas[oo];
        p->mops.out[o] = outs[oo];
        p->mops.dout[o] = deriv ? douts[oo] : nullptr;
    }
    int64_t nskip = 0;
    if (tau > 0.0 && n > 0) {
        // a pair is skipped only when every operator's bound is below tau
        int32_t *keep = nullptr;
        float *work = nullptr;
        HIP_TRY(c, hipMalloc((void **)&keep, n * sizeof(int32_t)));
        if (hipMalloc((void **)&work, (size_t)n * 15 * sizeof(float)) != hipSuccess) {
            (void)hipFree(keep);
            return fail(set_err(c, SHG_ENOMEM, "%s: out of device memory", what));
        }
        std::vector<int32_t> hkeep(n, 0), tmp(n), horder(n);
        for (int o = 0; o < nops && !rc; ++o) {
            rc = screen_pairs(c, sh, ops[o], omegas[o], pairs, n, p->deriv, tau, nullptr, keep, work);
            if (!rc && hipMemcpy(tmp.data(), keep, n * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
                rc = set_err(c, SHG_EDEVICE, "%s: read-back failed", what);
            for (int64_t i = 0; i < n && !rc; ++i) hkeep[i] |= tmp[i];
        }
        if (!rc && hipMemcpy(horder.data(), p->order, n * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
            rc = set_err(c, SHG_EDEVICE, "%s: read-back failed", what);
        (void)hipFree(work);
        (void)hipFree(keep);
        if (rc) return fail(rc);
        if ((rc = plan_compact(p, hkeep, horder, &nskip))) return fail(rc);
    }
    multi_fn f;
    multi_occ_fn occ;
    if (p->deriv) multi_entry_d1(&f, &occ);
    else multi_entry_d0(&f, &occ);
    hipDeviceProp_t prop;
    HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
    p->grid = std::max(1, std::min(p->ntiles, prop.multiProcessorCount * occ()));
    if ((rc = plan_capture(p))) return fail(rc);
    if (n_skipped) *n_skipped = nskip;
    *plan = p;
    return 0;
}

extern "C" int shg_plan_execute(shg_plan *p)
{
    if (!p) return SHG_EINVAL;
    shg_ctx *c = p->ctx;
    if (p->exec) {
        HIP_TRY(c, hipGraphLaunch(p->exec, c->stream));
        return 0;
    }
    return plan_enqueue(p, c->stream);
}

extern "C" int shg_plan_set_mode(shg_plan *p, int persistent)
{
    if (!p) return SHG_EINVAL;
    if (p->nops > 0) return set_err(p->ctx, SHG_EINVAL, "plan: a multi-operator plan has one mode");
    if (persistent && p->smem > (size_t)PERSIST_MAX_SMEM)
        return set_err(p->ctx, SHG_EINVAL, "plan: tile shapes need more LDS than the persistent kernel allows");
    p->mode = persistent ? 1 : 0;
    if (p->graph || p->exec) {
        HIP_TRY(p->ctx, hipStreamSynchronize(p->ctx->stream));
        return plan_capture(p);
    }
    return 0;
}

extern "C" int shg_plan_kernel_ms(shg_plan *p, int reps, double *ms);

extern "C" int shg_plan_autotune(shg_plan *p, int reps, double *ms_per_class, double *ms_persistent)
{
    if (!p) return SHG_EINVAL;
    shg_ctx *c = p->ctx;
    if (reps < 1) reps = 1;
    if (p->nops > 0) {   // one mode: report its time
        double ms = 0;
        int rc = shg_plan_kernel_ms(p, reps, &ms);
        if (ms_per_class) *ms_per_class = -1.0;
        if (ms_persistent) *ms_persistent = ms;
        return rc;
    }
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
    int rc = time_mode(0, &t_class);
    if (rc) return rc;
    const bool can_persist = p->smem <= (size_t)PERSIST_MAX_SMEM;
    if (can_persist) {
        // the persistent kernel with each tile order of the queue
        int best_q = p->qorder;
        float best = 0;
        for (int qo = 0; qo < 3; ++qo) {
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
    if (ms_per_class) *ms_per_class = t_class;
    if (ms_persistent) *ms_persistent = can_persist ? t_pers : -1.0;
    p->mode = (can_persist && t_pers < t_class) ? 1 : 0;
    if (p->graph || p->exec) return plan_capture(p);
    return 0;
}

extern "C" int shg_plan_mode(const shg_plan *p) { return p ? p->mode : SHG_EINVAL; }

extern "C" int shg_plan_tile_order(const shg_plan *p) { return p ? p->qorder : SHG_EINVAL; }

// ids of the pairs a screened plan skips (host array of capacity cap); returns
// their number (the full count even when cap is smaller)
extern "C" int64_t shg_plan_skipped(const shg_plan *p, int32_t *ids, int64_t cap)
{
    if (!p) return SHG_EINVAL;
    int64_t n = (int64_t)p->skipped.size();
    if (ids)
        for (int64_t i = 0; i < n && i < cap; ++i) ids[i] = p->skipped[i];
    return n;
}

// kept pairs and their algorithmic bytes (output values [+ d/dR_a] + 8 bytes of
// pair indices + 8 bytes of offset per pair), host pointers
extern "C" int shg_plan_stats(const shg_plan *p, int64_t *kept, int64_t *alg_bytes)
{
    if (!p || !kept || !alg_bytes) return SHG_EINVAL;
    int64_t k = 0, b = 0;
    for (int cls = 0; cls < NCLASS; ++cls) {
        int64_t cnt = p->cls_start[cls + 1] - p->cls_start[cls];
        int la = cls / (LMAX + 1), lb = cls % (LMAX + 1);
        k += cnt;
        b += cnt * ((int64_t)8 * (2 * la + 1) * (2 * lb + 1) * (p->deriv ? 4 : 1) * (p->nops > 0 ? p->nops : 1) + 16);
    }
    *kept = k;
    *alg_bytes = b;
    return 0;
}

// average duration (ms) of the evaluation kernels alone (persistent kernel or
// the per-class launches, without the shell preparation), timed with HIP events
// over `reps` enqueues on the ctx stream; synchronous
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
        if (p->mode >= 1) hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, p->counter, 0, 1);
        HIP_TRY(c, hipEventRecord(e0, c->stream));
        plan_radial(p, c->stream);
        if (p->nops > 0) {
            multi_fn f;
            multi_occ_fn occ;
            if (p->deriv) multi_entry_d1(&f, &occ);
            else multi_entry_d0(&f, &occ);
            if (p->ntiles > 0) f(c->stream, p->grid, ta, p->mops, p->queue, p->ntiles, p->counter);
        } else if (p->mode == 1) {
            persist_fn f;
            persist_occ_fn occ;
            if (p->deriv) persist_entry_d1(&f, &occ);
            else persist_entry_d0(&f, &occ);
            if (p->ntiles > 0) f(c->stream, p->grid, p->smem, ta, p->queue, p->ntiles, p->counter);
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
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    (void)hipFree(p->order);
    (void)hipFree(p->rec);
    (void)hipFree(p->T);
    (void)hipFree(p->w);
    (void)hipFree(p->queue);
    (void)hipFree(p->counter);
    delete p;
}
