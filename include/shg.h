/*
 * shg.h -- C ABI of libshg.so, the MI355X (gfx950) engine for contracted
 * solid-harmonic-Gaussian (SHG) integrals.
 *
 * Reference: Golze, Benedikter, Iannuzzi, Wilhelm, Hutter, "Fast evaluation of
 * solid harmonic Gaussian integrals for local resolution-of-the-identity
 * methods and range-separated hybrid functionals" (arXiv:1701.06588).
 *
 * Conventions (all entry points):
 *   - units: bohr and bohr^-2; FP64 in and out;
 *   - a shell is one contracted function phi_{l,m} = N_l sum_alpha c_alpha
 *     C_{l,m}(r) exp(-alpha r^2) (Sec. II.A, eqs. SHG_primitive, contracted_phi);
 *     the caller passes RAW coefficients c_alpha, the library applies N_l
 *     (eq. N_l), so results do not depend on the scale of c;
 *   - real components m = -l..l stored at index m + l; m >= 0 is the cosine
 *     and m < 0 the sine component (Sec. II.B, eq. Qref), i.e. the real solid
 *     harmonic A_{l,|m|} R^{c/s}_{l,|m|}(r) (eq. A, Sec. II.F): p = (y, z, x);
 *   - derivatives are with respect to the position of the first center,
 *     d/dR_a (Sec. II.E, eq. dev_ab); d/dR_b = -d/dR_a by translation
 *     invariance;
 *   - every pointer argument below is a DEVICE pointer (allocated by the
 *     caller, e.g. with torch) unless stated otherwise; the library never
 *     frees caller memory;
 *   - calls are asynchronous on the context's stream, except that the plain
 *     entry points read back a few bytes (the class histogram and an error
 *     flag) and therefore synchronise that stream once per call;
 *   - return 0 on success, a negative SHG_E* code on error; no exception ever
 *     crosses the ABI; shg_last_error() gives a message for the last failure.
 */
#ifndef SHG_H
#define SHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHG_EINVAL  (-1)   /* bad argument (l, K, exponent, operator, omega, index, NULL) */
#define SHG_ENOMEM  (-2)   /* device or host allocation failed */
#define SHG_EDEVICE (-3)   /* HIP runtime error; text in shg_last_error() */

#define SHG_LMAX_ORB 4     /* largest l of a two-center shell and of an orbital shell */
#define SHG_LMAX_AUX 6     /* largest l of an auxiliary (RI) shell in shg_aab */
#define SHG_KMAX     7     /* largest contraction length K of any shell */

/* Operators O(r1 - r2) of the two-center integral (a|O|b), Sec. III and
 * Table S1 of the supplement. omega is the range parameter. */
typedef enum {
    SHG_OVERLAP = 0,   /* delta(r)                       omega ignored */
    SHG_COULOMB = 1,   /* 1/r                            omega ignored */
    SHG_ERF     = 2,   /* erf(omega r)/r   (long range)   omega > 0    */
    SHG_ERFC    = 3,   /* erfc(omega r)/r  (short range)  omega > 0    */
    SHG_GAUSS   = 4,   /* exp(-omega r^2)                 omega > 0    */
    SHG_GCOULOMB = 5   /* exp(-omega r^2)/r               omega > 0;
                          shg_pairs, shg_pairs_deriv and shg_plan_create
                          (not in screened plans, nor in
                          shg_autotune) */
} shg_op;

/* Shell table. All arrays are DEVICE arrays of length nshell (prim arrays of
 * length nprim_total); prim_off[i] is the first primitive of shell i. */
typedef struct {
    int32_t nshell;
    int64_t nprim_total;
    const double  *center;    /* [nshell][3]                                   */
    const int32_t *l;         /* [nshell] 0..lmax                              */
    const int32_t *nprim;     /* [nshell] 1..SHG_KMAX                          */
    const int64_t *prim_off;  /* [nshell]                                      */
    const double  *exps;      /* [nprim_total] > 0                             */
    const double  *coefs;     /* [nprim_total] raw contraction coefficients    */
} shg_shells;

typedef struct shg_ctx shg_ctx;

/* Create a context bound to the current HIP device and to `hip_stream`
 * (a hipStream_t, NULL = default stream). Uploads the Boys-function table.
 * *ctx receives the handle (owned by the caller, release with shg_destroy). */
int  shg_create(shg_ctx **ctx, void *hip_stream);
void shg_destroy(shg_ctx *ctx);
/* Message of the last failed call on ctx (static storage inside ctx; valid until
 * the next call). ctx may be NULL (then: message of the last shg_create). */
const char *shg_last_error(const shg_ctx *ctx);

/* (a|O|b) for n shell pairs (Sec. II.B, eq. final_r12int_ab).
 *   pairs   [n][2] int32   (shell a on center A, shell b on center B)
 *   out_off [n]    int64   element offset of block i in out
 *   out     block i = (2la+1) x (2lb+1) doubles row-major at out[out_off[i]]
 * Shells must satisfy l <= SHG_LMAX_ORB, 1 <= K <= SHG_KMAX, exponents > 0;
 * violations or pair indices outside [0, nshell) return SHG_EINVAL (no block
 * of the call is then guaranteed). n == 0 is a no-op success. */
int shg_pairs(shg_ctx *ctx, const shg_shells *sh, shg_op op, double omega,
              const int32_t *pairs, int64_t n, const int64_t *out_off, double *out);

/* (a|O|b) and d/dR_a (Sec. II.E, eq. dev_ab with the recurrences of
 * Sec. II.F, eqs. cartesian_dev_x/y/z). Values as in shg_pairs; dout holds,
 * for block i, three blocks (x, y, z) of (2la+1)(2lb+1) doubles starting at
 * dout[3*out_off[i]]. */
int shg_pairs_deriv(shg_ctx *ctx, const shg_shells *sh, shg_op op, double omega,
                    const int32_t *pairs, int64_t n, const int64_t *out_off,
                    double *out, double *dout);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Computes
 * exactly what shg_pairs (dout NULL) or shg_pairs_deriv (dout non-NULL)
 * computes, with the same kernels, but keeps the binning scratch (folded
 * weights, class keys, sorted ids, pair records) in a fixed device array of
 * the library instead of context memory grown on demand; the call performs no
 * device or host allocation. The array is 32 MiB, one copy per GPU the library
 * runs on, held until the process ends. Limits: n <= SHG_NOALLOC_MAX_PAIRS
 * (n = 0 is a no-op success) and sh->nprim_total <= SHG_NOALLOC_MAX_PRIMS, else
 * SHG_EINVAL; op SHG_OVERLAP..SHG_GAUSS (SHG_GCOULOMB: SHG_EINVAL). Every
 * call on one GPU shares that GPU's array (across contexts too), so calls
 * that overlap in time on one GPU race; serialise them (one stream, or the
 * call's own synchronisation: like shg_pairs it synchronises the context
 * stream once, after binning). Other arguments and errors as in shg_pairs. */
#define SHG_NOALLOC_MAX_PAIRS (1 << 20)
#define SHG_NOALLOC_MAX_PRIMS (1 << 20)
int shg_pairs_noalloc(shg_ctx *ctx, const shg_shells *sh, shg_op op, double omega,
                      const int32_t *pairs, int64_t n, const int64_t *out_off,
                      double *out, double *dout);

/* (a|r_a^{2n}|b) (Sec. II.C, eq. ara2nb_def, evaluated by eqs. ara2nb and
 * T_rab2_deriv): the local operator r_a^{2n} = |r - R_a|^{2n} centred on a's
 * center, 0 <= nr <= 5 (else SHG_EINVAL; nr = 0 is the overlap).
 *   pairs, out_off, out as in shg_pairs (a and b from the same shell table)
 *   dout    nullable; d/dR_a with a and the operator moving together, x, y, z
 *           blocks at dout[3*out_off[i]]
 * Shells as in shg_pairs. */
int shg_pairs_r2n(shg_ctx *ctx, const shg_shells *sh, int nr, const int32_t *pairs,
                  int64_t n, const int64_t *out_off, double *out, double *dout);

/* ---- family basis sets (Sec. III) ----------------------------------------
 * A set is a group of contracted functions on one center that share the set's
 * K exponents (1 <= K <= SHG_SET_KMAX); each function has its own l
 * (0..SHG_LMAX_ORB) and K raw contraction coefficients. Within a set the
 * functions must be grouped by l in non-decreasing order (MOLOPT order:
 * s, s, p, p, d, ...), 1..SHG_SET_FMAX functions per set. All arrays DEVICE. */
#define SHG_SET_KMAX 8
#define SHG_SET_FMAX 16
typedef struct {
    int32_t nset;
    int64_t nexp_total, nfun_total, ncoef_total;
    const double  *center;    /* [nset][3]                                     */
    const int32_t *nexp;      /* [nset] K                                      */
    const int64_t *exp_off;   /* [nset] first exponent of the set in exps      */
    const double  *exps;      /* [nexp_total] > 0                              */
    const int32_t *nfun;      /* [nset] contracted functions of the set        */
    const int64_t *fun_off;   /* [nset] first function in fun_l / coef_off     */
    const int32_t *fun_l;     /* [nfun_total] l of each function               */
    const int64_t *coef_off;  /* [nfun_total] first of the function's K raw coefficients in coefs */
    const double  *coefs;     /* [ncoef_total]                                 */
} shg_sets;

/* (A|O|B) for n pairs of family sets (Sec. III with eqs. O_rab2_deriv and
 * final_r12int_ab): per set pair the primitive radial terms are evaluated once
 * for all its function pairs and contracted as C_a^T G^(k) C_b, and per
 * (la, lb) the angular factors of each element are formed once for all
 * function pairs with those l.
 *   set_pairs [n][2] int32 (set on A, set on B)
 *   out       block i = nsgf_A x nsgf_B doubles row-major at out[out_off[i]],
 *             nsgf = sum over the set's functions of 2l+1; rows (and columns)
 *             in function order, components m = -l..l within a function
 *   dout      nullable; d/dR_A as x, y, z blocks of nsgf_A x nsgf_B at
 *             dout[3*out_off[i]]
 * Each entry equals the (a|O|b) of shg_pairs for the two functions taken as
 * shells. Operators SHG_OVERLAP..SHG_GAUSS; invalid sets or indices give
 * SHG_EINVAL. Synchronises the context stream twice (validation, binning). */
int shg_set_pairs(shg_ctx *ctx, const shg_sets *sets, shg_op op, double omega,
                  const int32_t *set_pairs, int64_t n, const int64_t *out_off,
                  double *out, double *dout);

/* Swap symmetry (Sec. V): for the operators of shg_op (even functions of
 * r1 - r2) and each function keeping its center, (b|O|a) = (a|O|b)^T, and by
 * translation invariance d/dR_b (b|O|a) = -(d/dR_a (a|O|b))^T. Given the
 * blocks of the pairs (a, b) = pairs[i] already in out (and dout) at
 * src_off[i], writes the blocks of the swapped pairs (b, a) at dst_off[i] of
 * the same buffers: (2lb+1) x (2la+1) row-major, derivatives x, y, z at
 * dout[3*dst_off[i]]; dout nullable. Source and destination blocks must not
 * overlap. Asynchronous: a pair index or l outside range skips that block and
 * is reported by shg_pairs_swap_check (which synchronises the stream). */
int shg_pairs_swap(shg_ctx *ctx, const shg_shells *sh, const int32_t *pairs, int64_t n,
                   const int64_t *src_off, const int64_t *dst_off, double *out, double *dout);
int shg_pairs_swap_check(shg_ctx *ctx);

/* Measurement utility, not part of the method: launches `blocks` workgroups
 * of 256 threads, each thread running `iters` rounds of 8 independent FP64
 * FMA chains with no memory traffic, on the context's stream; out (device,
 * >= blocks*256 doubles) receives one result per thread; *flops (host)
 * receives the floating-point operations of the launch (2 per FMA). The
 * caller times the launch; the ratio is the FP64 rate the device sustains. */
int shg_fp64_ceiling(shg_ctx *ctx, int64_t iters, int blocks, double *out, double *flops);

/* Three-index overlap (a b a~) (Sec. II.D, eq. aba_integrals): a = orb shell
 * t[0] and a~ = aux shell t[1] share center A (their centers must be equal
 * bit for bit, else SHG_EINVAL), b = orb shell t[2].
 *   triples [n][3] int32
 *   out     block i = (2la+1) x (2la~+1) x (2lb+1) doubles at out[out_off[i]]
 *   dout    nullable; d/dR_A (a and a~ move together) as x, y, z blocks at
 *           dout[3*out_off[i]]
 * Orbital shells: l <= SHG_LMAX_ORB - 1 (= 3); aux shells: l <= SHG_LMAX_AUX.
 * The work runs on the context's stream and three library-owned side streams
 * forked from and joined back into it, so to the caller it is ordered on the
 * context's stream like every other call. */
int shg_aab(shg_ctx *ctx, const shg_shells *orb, const shg_shells *aux,
            const int32_t *triples, int64_t n, const int64_t *out_off,
            double *out, double *dout);

/* Work-item size of shg_aab: each (l_a, l_a~, l_b) class is processed in
 * chunks of at most `chunk` triples (1 <= chunk <= 2^24, default 2^17); the
 * chunks' scratch (radial terms and two-center blocks) scales with it.
 * Results do not depend on it. */
int shg_set_aab_chunk(shg_ctx *ctx, int64_t chunk);

/* ---- batched path ------------------------------------------------------- */

/* A plan fixes one evaluation: shell table, operator, pair list, offsets and
 * output buffers (all device pointers, kept by reference, owned by the caller
 * and required to outlive the plan). Creation runs shg_pairs / shg_pairs_deriv
 * once (dout NULL: values only), which validates the input and bins the pairs
 * by class, copies the class-sorted order, builds a tile work queue (round
 * robin over the classes by default) and, unless SHG_PLAN_NO_GRAPH, records the
 * evaluation (shell preparation + class kernels) in a hipGraph. Execution replays it with
 * no host synchronisation and no binning; new centers, exponents or raw
 * coefficients written into the same buffers are picked up, but the shells'
 * l and K and the pair list must not change (they are not re-validated).
 *   flags: SHG_PLAN_PERSISTENT  persistent class-binned kernels over the tile
 *                               queue (64-pair tiles, each class with its
 *                               compiled tile schedule; one kernel for the
 *                               heavy classes la + lb >= 5, then one for the
 *                               light ones) instead of one launch per class
 *                               (with the tuned tile shapes)
 *          SHG_PLAN_NO_GRAPH    enqueue the kernels on every execute */
#define SHG_PLAN_PERSISTENT 1u
#define SHG_PLAN_NO_GRAPH   2u
#define SHG_PLAN_COMPACT    4u   /* screened plans only: see shg_plan_create_screened */
typedef struct shg_plan shg_plan;
int  shg_plan_create(shg_ctx *ctx, const shg_shells *sh, shg_op op, double omega,
                     const int32_t *pairs, int64_t n, const int64_t *out_off,
                     double *out, double *dout, unsigned flags, shg_plan **plan);
int  shg_plan_execute(shg_plan *plan);        /* asynchronous on the ctx stream */
/* Times the per-class launches and the persistent kernel with each of the
 * three tile orders of its queue (heaviest class first; alternating from the
 * two ends of that order; round robin over the classes), `reps` times each
 * with HIP events (synchronous), keeps the fastest (re-recording the graph)
 * and reports the per-class time and the best persistent time (host pointers,
 * nullable; -1 when the persistent kernel cannot take the plan's tiles). */
int  shg_plan_autotune(shg_plan *plan, int reps, double *ms_per_class, double *ms_persistent);
int  shg_plan_set_mode(shg_plan *plan, int persistent);
int  shg_plan_mode(const shg_plan *plan);     /* 0 per-class launches, 1 persistent */
int  shg_plan_tile_order(const shg_plan *plan);  /* 0 heaviest first, 1 alternating ends, 2 round robin */
/* fix the tile order of the persistent queue (0..2; compacting screened plans 0..1)
 * without timing; re-records the graphs; synchronises the context stream */
int  shg_plan_set_tile_order(shg_plan *plan, int order);
/* ids of the pairs the last execution of a screened plan skipped, written to
 * the host array ids (capacity cap, nullable; in no particular order); returns
 * how many there are (0 for unscreened plans). Synchronises the context
 * stream. */
int64_t shg_plan_skipped(const shg_plan *plan, int32_t *ids, int64_t cap);
/* number of pairs a plan evaluates (a screened plan: at its last execution)
 * and their algorithmic bytes (8 (2la+1)(2lb+1)(1 or 4) + 16 per pair); host
 * pointers; synchronises the context stream for screened plans */
int  shg_plan_stats(const shg_plan *plan, int64_t *kept, int64_t *alg_bytes);
/* mean duration in ms of the plan's evaluation kernels alone (no shell
 * preparation), timed with HIP events over `reps` runs; synchronous */
int  shg_plan_kernel_ms(shg_plan *plan, int reps, double *ms);
/* Kernel timing inside replays: with on != 0, every later shg_plan_execute
 * records a HIP event pair on the context stream around the plan's evaluation
 * kernels (the persistent kernel or the per-class launches, recorded as a
 * graph of their own after the stage graph of shell preparation and, for a
 * screened plan, the screening stage), for up to 1024 executions.
 * shg_plan_kernel_time synchronises the context stream, returns (host
 * pointers) the summed milliseconds and the number of timed executions since
 * the last call or since timing was switched on, and restarts the count. */
int  shg_plan_time_kernels(shg_plan *plan, int on);
int  shg_plan_kernel_time(shg_plan *plan, double *ms_sum, int64_t *executions);
void shg_plan_destroy(shg_plan *plan);

/* ---- prescreening ------------------------------------------------------ */

/* Learned predictor of log10 max|block| (12 features -> 3 x 64 SiLU -> 1;
 * bf16 weights, fp32 accumulation; inference on bf16 MFMA, training on the
 * library's own forward/backward/Adam kernels). Parameters: 9217 fp32 master
 * values (layout W1[64][12], b1, W2[64][64], b2, W3[64][64], b3, w4[64], b4). */
typedef struct shg_mlp shg_mlp;
int  shg_mlp_create(shg_ctx *ctx, uint64_t seed, shg_mlp **mlp);      /* He-initialised */
void shg_mlp_destroy(shg_mlp *mlp);
/* host arrays of 9217 floats (nullable): copy out the master parameters and/or
 * replace them (replacing resets the Adam state) */
int  shg_mlp_params(shg_mlp *mlp, float *host_out, const float *host_in);
/* feature standardisation (mean, std) and training range [lo, hi] (host arrays
 * of 12, lo/hi nullable); pairs with a feature outside the range fall back to
 * the analytic bound */
int  shg_mlp_set_norm(shg_mlp *mlp, const float *mean, const float *std, const float *lo, const float *hi);
/* calibration margin (log10 units) added to predictions before comparing with tau */
int  shg_mlp_set_margin(shg_mlp *mlp, float margin);
/* what the model predicts: ops_mask has bit (1 << op) for every shg_op it was
 * trained on (SHG_OVERLAP..SHG_GAUSS), deriv_targets != 0 when its targets are
 * log10 max over the value block and its d/dR_a blocks. Screened plans
 * consult a model only for an operator in its mask, and for plans with
 * derivatives only when deriv_targets is set. Saved with the model. */
int  shg_mlp_set_scope(shg_mlp *mlp, uint32_t ops_mask, int deriv_targets);
/* one Adam step on a batch: X [B][12] and y [B] device fp32; pinball loss at
 * `quantile` on y - prediction; loss_out (device float, nullable) receives
 * the summed per-sample loss */
int  shg_mlp_train_step(shg_mlp *mlp, const float *X, const float *y, int B, float lr, float quantile,
                        float *loss_out);
/* gradient of the mean loss (device [9217], nullable) without updating */
int  shg_mlp_grad(shg_mlp *mlp, const float *X, const float *y, int B, float quantile, float *grad_out,
                  float *loss_out);
/* prediction for n feature rows (device): pred [n] fp32, in_range [n] int32 */
int  shg_mlp_predict(shg_mlp *mlp, const float *X, int64_t n, float *pred, int32_t *in_range);
int  shg_mlp_save(shg_mlp *mlp, const char *path);
int  shg_mlp_load(shg_mlp *mlp, const char *path);

/* The 12 screening features of each pair (device fp32 [n][12]: la, lb,
 * log10 alpha_min/max of a and of b, R, log10(1 + rho_min R^2), log10 of the
 * bound, operator code (shg_op), omega R for erf/erfc (else 0),
 * log10(sum|w_a| sum|w_b|)) and log10 of the conservative analytic bound on
 * max|block| (device fp32 [n]); with deriv != 0 the bound (and the feature)
 * covers the d/dR_a elements too. */
int  shg_screen_features(shg_ctx *ctx, const shg_shells *sh, shg_op op, double omega,
                         const int32_t *pairs, int64_t n, int deriv, float *feat,
                         float *log10_bound);
/* log10 max|element| (clamped at -30) of evaluated blocks (training targets),
 * over the value block and, with dout non-NULL, its d/dR_a blocks too */
int  shg_block_logmax(shg_ctx *ctx, const shg_shells *sh, const int32_t *pairs, int64_t n,
                      const int64_t *out_off, const double *out, const double *dout, float *y);

/* A plan for (a|r_a^{2n}|b) (Sec. II.C, as shg_pairs_r2n, 0 <= nr <= 5):
 * arguments, flags, validation and ownership as in shg_plan_create; the
 * recorded evaluation runs the monopole stage and then the tiles. */
int shg_plan_create_r2n(shg_ctx *ctx, const shg_shells *sh, int nr, const int32_t *pairs, int64_t n,
                        const int64_t *out_off, double *out, double *dout, unsigned flags, shg_plan **plan);

/* Screened plan: as shg_plan_create, always recorded, persistent mode. Every
 * execution decides anew, on the device, which pairs it evaluates, so centers
 * (or exponents, coefficients) written into the shell buffers between
 * executions are screened afresh: a pair is skipped when its analytic bound
 * (values, and with dout the d/dR_a elements too) is below tau, or when a
 * model (mlp non-NULL, whose scope covers op and, with dout, derivatives;
 * features inside its training range) predicts, plus its margin, below
 * log10(tau). Skipped blocks (and their d/dR_a blocks) are set to zero in the
 * same execution; kept blocks are those of the plain path. The execution
 * (graph replay) reads nothing back to the host. Two ways to run it:
 *   default           the persistent kernel evaluates the bound of each pair
 *                     of its tile (or reads the model's decision) before the
 *                     radial sum; a skipped pair gets no primitive work and
 *                     its block is stored as zeros by the tile itself. Best
 *                     when few pairs drop out.
 *   SHG_PLAN_COMPACT  a screening stage (bound or model, a scan compacting the
 *                     kept class-sorted pair records, a tile queue built from
 *                     the kept counts, the skipped blocks zeroed) runs before
 *                     the persistent kernel, which sees kept pairs only. Best
 *                     when most pairs drop out.
 * The model, if any, must outlive the plan. Operators SHG_OVERLAP..SHG_GAUSS;
 * tau > 0. Creation executes once; *n_skipped (host, nullable) receives the
 * number of pairs that execution skipped. */
int  shg_plan_create_screened(shg_ctx *ctx, const shg_shells *sh, shg_op op, double omega,
                              const int32_t *pairs, int64_t n, const int64_t *out_off,
                              double *out, double *dout, unsigned flags, double tau,
                              shg_mlp *mlp, shg_plan **plan, int64_t *n_skipped);

/* ---- tuning and timing ------------------------------------------------- */

/* Tile shape used by the per-class launches of operator op for class
 * (la, lb, deriv): tp shell pairs per workgroup (64, 128 or 256; 256/tp lanes
 * share the radial work of one pair) and rows_pp block rows per LDS staging
 * pass (1..2la+1). Returns SHG_EINVAL for values outside those ranges or tiles
 * needing more than 160 KiB of LDS. Host pointers for the get variant. */
int shg_set_tile_shape(shg_ctx *ctx, int op, int la, int lb, int deriv, int tp, int rows_pp);
int shg_get_tile_shape(const shg_ctx *ctx, int op, int la, int lb, int deriv, int *tp, int *rows_pp);

/* Autotuner: bins the caller's pair list like shg_pairs(_deriv) (dout NULL:
 * values only), then for every class present times each admissible tile shape
 * `reps` times with HIP events and keeps the fastest for (op, class, deriv).
 * Synchronous. On return out/dout hold the results computed with the selected
 * shapes. Arguments and errors as in shg_pairs_deriv. */
int shg_autotune(shg_ctx *ctx, const shg_shells *sh, shg_op op, double omega,
                 const int32_t *pairs, int64_t n, const int64_t *out_off,
                 double *out, double *dout, int reps);
/* Tuning cache (host path): JSON list of the tuned shapes with the GPU
 * architecture name; load applies only entries of the current architecture
 * and returns how many it applied (or SHG_EINVAL if the file is unreadable). */
int shg_tuning_save(const shg_ctx *ctx, const char *path);
int shg_tuning_load(shg_ctx *ctx, const char *path);

/* Per-launch timing with HIP events recorded on the context stream around
 * every class launch of shg_pairs / shg_pairs_deriv (profiled calls also
 * synchronise at their end). shg_profile_enable clears the counters.
 * shg_profile_read returns, for class (la, lb, deriv), the accumulated kernel
 * milliseconds, the number of launches and the pairs they processed; la < 0
 * selects the binning stage (shell preparation, classification, scan,
 * scatter) instead. Host pointers. */
int shg_profile_enable(shg_ctx *ctx, int on);
int shg_profile_read(const shg_ctx *ctx, int la, int lb, int deriv, double *ms, int64_t *launches,
                     int64_t *pairs);

#ifdef __cplusplus
}
#endif
#endif /* SHG_H */
