/*
 * flow.h -- C ABI of the MI355X (gfx950) TV-L1 optical-flow library built on the preconditioned
 * dual solvers of Sun, Tai and Yuan, "Variational Image Motion Estimation by Accelerated Dual
 * Optimization" (arXiv 2011.10979).
 *
 * Problem (Sec. 1, eq:l1:optical:flow and eq:l1:optical:flow:no:w): given two grayscale frames
 * I0 = I(t) and I1 = I(t+1), find a per-pixel displacement d = (u, v), u along columns (x) and v
 * along rows (y), with I1(x + d) ~= I0(x), by minimising the isotropic TV-L1 energy
 *     |grad w|_1 + |grad d|_1 + lambda | grad I^T d + beta w + I_t |_1          (beta >= 0)
 * (the w / illumination block is present only for beta > 0).  The energy is linearised around the
 * current flow and solved on its dual by one of the paper's schemes inside a coarse-to-fine
 * warping pyramid (Sec. 4).
 *
 * Conventions shared by every entry point
 *   - Images and flow fields are row-major FP32 planes of H rows by W columns, each side at most
 *     FLOW_MAX_SIDE (larger sides are refused with FLOW_E_INVAL; device memory bounds the area
 *     long before: a pair's working set is about 100 B per pixel).  `ld` / `ld_*` is the
 *     row pitch in ELEMENTS (>= W).  Pointers tagged "device" must be device memory of the
 *     context's GPU (e.g. torch.cuda tensors); nothing is ever copied from host memory unless a
 *     pointer is tagged "host".
 *   - Input frames hold intensities in [0, 1]; the solver multiplies them by
 *     params.intensity_scale (kappa, default 255: the 8-bit scale of the paper's data) before
 *     forming the data term.
 *   - Every call returns a flow_status; none throws or aborts.  flow_last_error() gives a
 *     thread-local message for the last failing call on the calling thread.
 *   - The caller owns every buffer it passes.  The library never retains a caller pointer after a
 *     call returns (serving tickets: until the ticket is done), never frees it and never writes
 *     to an input.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is stream-ordered on it;
 *     entry points documented as blocking synchronise that stream before returning.
 */
#ifndef FLOWMI_FLOW_H
#define FLOWMI_FLOW_H

#include <stddef.h>
#include <stdint.h>

#define FLOW_MAX_SIDE 131072   /* largest H or W of any plane */

#ifdef __cplusplus
extern "C" {
#endif

typedef enum flow_status {
    FLOW_OK = 0,
    FLOW_E_INVAL = -1,      /* invalid argument (NULL pointer, bad size, parameter out of range) */
    FLOW_E_NOMEM = -2,      /* request exceeds the context's HBM budget, or device allocation failed */
    FLOW_E_HIP = -3,        /* a HIP runtime call failed (message in flow_last_error) */
    FLOW_E_NONFINITE = -4,  /* energy or gap is not finite (outputs are still written) */
    FLOW_E_BUSY = -5,       /* serving queue full / context busy */
    FLOW_E_NOTFOUND = -6    /* unknown ticket */
} flow_status;

/* Solver scheme (Sec. 3.1).
 *   FLOW_PADMM   rpADMMI (tag rpADMMI): dual steps with the proximal weights a c I - c grad grad^* and
 *                a~ c I - c M_s, multipliers relaxed by r = relax in (0, (1+sqrt 5)/2); relax = 1 is
 *                pADMM; beta = 0 with relax = 1 is Zach-pADMM (tag Zach-pADMM).
 *   FLOW_RPADMM2 rpADMMII (tag rpADMMII): relaxation rho = relax in (0, 2) of [SUN].
 *   FLOW_PDR     preconditioned Douglas-Rachford on the saddle-point form (tag pDR) with
 *                gs_sweeps symmetric red-black Gauss-Seidel sweeps as the preconditioner.
 *   FLOW_ALG1    ALG1 of Sec. 4, the first-order primal-dual method the paper compares against, on
 *                the same saddle form: y+ = P(y + alg1_tau grad X bar), X+ = J(X + alg1_sigma div y+)
 *                (eq:resolvent), X bar+ = 2 X+ - X; alg1_tau alg1_sigma 8 <= 1. */
typedef enum flow_scheme { FLOW_PADMM = 0, FLOW_RPADMM2 = 1, FLOW_PDR = 2, FLOW_ALG1 = 3 } flow_scheme;

/* Storage of the image / derivative pyramids: FP32, or FP16 with FP32 arithmetic. */
typedef enum flow_storage { FLOW_STORE_F32 = 0, FLOW_STORE_F16 = 1 } flow_storage;

typedef struct flow_params {
    uint32_t struct_size;     /* sizeof(flow_params); set by flow_params_default */
    int32_t scheme;           /* flow_scheme, default FLOW_PADMM */
    double lambda;            /* data weight > 0, default 0.05 */
    double beta;              /* illumination weight >= 0, default 0 (no w block) */
    double c;                 /* ADMM step > 0, default 0.05 (Sec. 4) */
    double relax;             /* r (PADMM) in (0, 1.618...) or rho (RPADMM2) in (0, 2); default 1 */
    double sigma, tau;        /* pDR steps > 0, defaults 2 and 0.4 (Sec. 4) */
    int32_t gs_sweeps;        /* pDR symmetric sweeps >= 1, default 1 */
    double intensity_scale;   /* kappa > 0, default 255 */
    int32_t levels;           /* pyramid levels >= 1 (factor 1/2, ceil sizes); default 5 */
    int32_t warps;            /* re-linearisations per level >= 1; default 5 */
    int32_t iters;            /* inner iterations per warp >= 0; default 50 */
    int32_t storage;          /* flow_storage, default FLOW_STORE_F32 */
    int32_t use_graph;        /* 1: capture the whole solve in a hipGraph once per shape and replay */
    double tol;               /* > 0: stop a warp's iterations once |gap| / energy <= tol (checked
                                 every check_every iterations; disables graph replay); 0: fixed count */
    int32_t check_every;      /* >= 1 when tol > 0 */
    double alg1_tau;          /* ALG1 dual step > 0, default 0.1 (Sec. 4) */
    double alg1_sigma;        /* ALG1 primal step > 0, default 1 / (8 alg1_tau) = 1.25 */
} flow_params;

/* FP64 scalars of the last warp of the finest level (linearised energy of that warp):
 *   energy   = sum |grad d| (+ sum |grad w|) + lambda sum |rho|     (eq:l1:finite / eq:l1:finite:no:w)
 *   dual     = sum I_t s                                             (eq:dual:l1:flow:cons)
 *   gap      = energy - dual
 *   residual = |A s + B y|_2, the violation of eq:dual:l1:flow:constaint
 *   tv, data = the two parts of energy.
 * For pDR the dual pair is (q, s) = (P(y_bar + 2 tau grad X), Theta) of the last iteration; for ALG1
 * it is (y, Theta) of the last iteration. */
typedef struct flow_result {
    double energy, dual, gap, residual, tv, data;
} flow_result;

/* Per-solve timing, filled when the context's stats are enabled (flow_set_stats).  Times come
 * from hipEvents recorded around each level's block of iteration kernels on the solve stream. */
#define FLOW_MAX_LEVELS 16
typedef struct flow_stats {
    int32_t levels;
    int32_t H[FLOW_MAX_LEVELS], W[FLOW_MAX_LEVELS];
    int64_t iterations[FLOW_MAX_LEVELS];      /* inner iterations run at this level (all warps) */
    double iter_ms[FLOW_MAX_LEVELS];          /* event time of their kernel launches (includes gaps) */
    double total_ms;                          /* event time of the whole solve on the device */
    int64_t px_iter;                          /* pixel-iterations of the solve */
    int32_t graph_replayed;                   /* 1 if the solve ran as a graph replay */
    int64_t level_px[FLOW_MAX_LEVELS];        /* pixels of the level (a batch: summed over its pairs) */
    int64_t launches[FLOW_MAX_LEVELS];        /* iteration-kernel launches at this level (all warps) */
} flow_stats;

typedef struct flow_ctx flow_ctx;

/* Fill *p with the defaults listed above.  FLOW_E_INVAL if p is NULL. */
flow_status flow_params_default(flow_params* p);

/* Create a context on HIP device `device` whose device allocations never exceed
 * hbm_budget_bytes (0 = no limit).  *out receives the context.  FLOW_E_INVAL on a bad device,
 * FLOW_E_HIP on a runtime error. */
flow_status flow_create(flow_ctx** out, int device, size_t hbm_budget_bytes);

/* Release the context and all its device memory, graphs and streams (NULL is a no-op). */
flow_status flow_destroy(flow_ctx* ctx);

/* Plain solve of one pair (the whole coarse-to-fine pipeline of Sec. 4).
 *   I0, I1   device, H x W, pitch ld (elements), intensities in [0, 1]
 *   u, v     device outputs, H x W, pitch ld_uv: the flow in pixels of the finest level
 *   res      host, may be NULL: energy / dual / gap of the final warp
 *   stream   hipStream_t; the call is stream-ordered and blocks until the results are written
 * Errors: FLOW_E_INVAL for NULL device pointers, H or W < 2, ld or ld_uv < W, levels < 1,
 * warps < 1, iters < 0, lambda <= 0, beta < 0, c <= 0, relax outside the Prop. 3.1 range of the
 * scheme, sigma or tau <= 0, gs_sweeps < 1, intensity_scale <= 0, tol < 0, or a coarsest level
 * with a side < 2; FLOW_E_NOMEM if the pair's working set exceeds the budget; FLOW_E_NONFINITE
 * if energy or gap is not finite. */
flow_status flow_solve(flow_ctx* ctx, const float* I0, const float* I1, int32_t H, int32_t W, int64_t ld,
                       const flow_params* p, float* u, float* v, int64_t ld_uv, flow_result* res,
                       void* stream);

/* One pair of a batch: device frames and outputs as in flow_solve (caller-owned, FP32, pitches ld
 * and ld_uv in elements); res is host memory (may be NULL); levels > 0 sets this pair's pyramid
 * depth (0: params->levels), so pairs of very different sizes can each keep coarsest levels of a
 * useful size. */
typedef struct flow_pair {
    const float* I0;
    const float* I1;
    int32_t H, W;
    int64_t ld;
    float* u;
    float* v;
    int64_t ld_uv;
    flow_result* res;
    int32_t levels;
} flow_pair;

/* Solve n pairs of uneven sizes together (the coarse-to-fine solve of Sec. 4 for every pair).
 * Stage s works on pyramid level Lmax-1-s of every pair that has it (all pairs reach level 0 in
 * the last stage); each step of a stage (level start, linearisation, K iterations, energy) is ONE
 * launch over all pairs, the iterations a launch of the K-iteration tile kernel over the tiles of
 * every pair's level, in XCD order or from per-XCD work queues (choice, K and tile width per stage
 * from flow_autotune_batched, else built in).  pDR and ALG1 (Sec. 3.1.2, Sec. 4) take the same
 * stages with their own tile kernels in table order (1024 threads, the built-in K per launch, or
 * the whole warp per launch where every level of a stage fits one tile).  With tol > 0, or a pDR
 * halo that no tile holds (many sweeps), the pairs run as plain solves in turn.  Every pair's
 * arithmetic is independent of the rest of the batch and of the stage choices, so a pair's results
 * are bitwise the same alone or in any batch, and equal to a plain solve that uses small
 * 1024-thread tiles (tb_mode 4) at every level (pDR and ALG1: to the plain tile solve).
 * The context keeps the working set of the last batch (arena, tables, captured graph) for reuse.
 * Errors: FLOW_E_INVAL (any pair invalid: nothing runs), FLOW_E_NOMEM (working set of all pairs
 * above the budget), FLOW_E_NONFINITE (outputs written, some pair's energy not finite).  Blocks
 * until all results are written. */
flow_status flow_solve_batched(flow_ctx* ctx, int32_t n, const flow_pair* pairs, const flow_params* p,
                               void* stream);

/* ------------------------------------------------------------------------------------------------
 * Serving: continuous batching of pairs that arrive over time.
 * ----------------------------------------------------------------------------------------------*/
typedef struct flow_server flow_server;

typedef struct flow_server_stats {
    int64_t submitted, admitted, completed;
    int64_t epochs;                 /* flow_server_step calls that launched work */
    int32_t active, queued;         /* pairs in flight / waiting for admission now */
    int32_t peak_active;
    uint64_t arena_bytes;           /* the serving budget (pairs' working sets) */
    uint64_t bytes_in_use, peak_bytes_in_use;
    int64_t graphs_captured;        /* graphs of an epoch's tile launches captured so far (one per
                                       buffer set and stage choice; every other epoch replays one) */
} flow_server_stats;

/* Device bytes of one pair's working set (pyramids, linearisation, scheme state of every level) for
 * an H x W pair under p with `levels` levels (0: p->levels): what flow_solve, a batch and the
 * serving budget hold per pair.  Host-only. */
flow_status flow_working_set_bytes(int32_t H, int32_t W, const flow_params* p, int32_t levels, uint64_t* bytes);

/* Allocation-free variant of flow_solve, for callers that cannot allocate device memory (code
 * that must not call hipMalloc: serving loops with a fixed footprint, harnesses that forbid
 * allocation).  No context: the whole working set of the solve -- pyramids, linearisation, scheme
 * state, reduction partials -- lives in one static device workspace of FLOW_STATIC_BYTES per GPU,
 * which the library holds from the first call on that GPU until the process ends.  The call makes
 * no device allocation and calls no allocating routine; it runs on the current device with the
 * built-in kernel plan (no autotuning, no graph), so its flow and energy are bitwise those of
 * flow_solve on a context without autotuning.
 *   I0, I1, u, v, ld, ld_uv, p, stream   as for flow_solve (p->use_graph is ignored; p->tol must
 *                                         be 0: a fixed iteration count)
 *   res      host, may be NULL.  Non-NULL: the call blocks until the results are written and
 *            reports FLOW_E_NONFINITE as flow_solve does; NULL: the call only enqueues the work on
 *            `stream` and returns (no host synchronisation, no finiteness check).
 * Every call on one GPU uses that GPU's single workspace, which keeps the last call's contents:
 * calls that overlap on one GPU (concurrent streams or host threads) race and must be serialised
 * by the caller.  Errors: as flow_solve, plus FLOW_E_INVAL for tol != 0 and FLOW_E_NOMEM (before
 * any device work) when the pair's working set exceeds the workspace -- a 1920 x 1080 pADMM pair
 * at beta = 0 with 6 levels fits, see flow_static_bytes. */
#define FLOW_STATIC_BYTES (256ull << 20)
flow_status flow_solve_static(const float* I0, const float* I1, int32_t H, int32_t W, int64_t ld,
                              const flow_params* p, float* u, float* v, int64_t ld_uv, flow_result* res,
                              void* stream);

/* Workspace bytes flow_solve_static needs for an H x W pair under p (*need) and the workspace size
 * (*limit, = FLOW_STATIC_BYTES); either pointer may be NULL.  Host-only. */
flow_status flow_static_bytes(int32_t H, int32_t W, const flow_params* p, uint64_t* need, uint64_t* limit);

/* Create a serving engine on ctx's GPU for solves with parameters p (any scheme, tol = 0, else
 * FLOW_E_INVAL; per-pair pyramid depth from flow_pair.levels, else p->levels).  pDR and ALG1 epochs
 * launch their tile kernels in table order directly; flow_server_submit refuses (FLOW_E_INVAL) a
 * pDR pair with so many sweeps that its halo outgrows a tile at some level.  hbm_budget: bytes of device memory for
 * the working sets of the pairs in flight (0: 8 GiB), allocated once here; a few MB of tables come
 * on top.  max_active: most pairs in flight at once.  Every epoch runs on `stream` (hipStream_t).
 * ctx must outlive the engine.  FLOW_E_NOMEM if the budget cannot be allocated. */
flow_status flow_server_create(flow_ctx* ctx, const flow_params* p, size_t hbm_budget, int32_t max_active,
                               void* stream, flow_server** out);
flow_status flow_server_destroy(flow_server* srv);

/* Queue one pair (device frames and outputs as in flow_solve; res host, may be NULL).  The caller
 * keeps I0, I1, u, v and res valid and untouched until flow_server_poll reports the ticket done,
 * and the frames must be complete on `stream`'s device before the next flow_server_step.
 * FLOW_E_INVAL for a bad pair, FLOW_E_NOMEM if its working set can never fit the budget. */
flow_status flow_server_submit(flow_server* srv, const flow_pair* pair, uint64_t* ticket);

/* Run one epoch (asynchronous on the engine's stream): admit queued pairs, in arrival order, while
 * a slot and room in the budget are free (first-fit; a pair that does not fit holds the queue);
 * advance every admitted pair by one warp of its coarse-to-fine solve (Sec. 4) -- level start where
 * due, linearisation, `iters` iterations -- with one launch per step over all of them
 * (tile launches cover the current level of every pair; pairs at different levels and warps share
 * them); finish the pairs that completed level 0 (energy, flow export).  Released memory and slots
 * return when the epoch's work has completed on the device.  Blocks only when the buffers of the
 * epoch before last are still in use.  A pair's results are bitwise the same alone or in any mix,
 * and equal to flow_solve_batched.  active / queued (may be NULL) receive the counts after it. */
flow_status flow_server_step(flow_server* srv, int32_t* active, int32_t* queued);

/* done = 1 once the ticket's u, v and res are written (the ticket is then collected and later
 * polls return FLOW_E_NOTFOUND); FLOW_E_NONFINITE with done = 1 if its energy is not finite. */
flow_status flow_server_poll(flow_server* srv, uint64_t ticket, int32_t* done);

/* Step until nothing is active or queued, then wait for the device (blocking). */
flow_status flow_server_drain(flow_server* srv);
flow_status flow_server_get_stats(const flow_server* srv, flow_server_stats* out);

/* Batched autotuner: for each stage of this batch, time every tile-launch choice (the general tiles
 * in table order or per-XCD work queues, and the wave-row tiles of 32 / 48 / 64 rows in table order;
 * every K in [2, 10] that is the smallest for its number of launches per warp, ceil(iters / n), or
 * the whole warp where every level of the stage fits one tile; extended tile width 64 or 128, 64 for
 * the wave-row tiles) over one warp's iterations, and keep the
 * fastest for later flow_solve_batched calls on batches whose stage has the same level shapes.
 * The choice changes speed only (results are bitwise the same).  Runs the pipeline on the pairs'
 * frames; blocking. */
flow_status flow_autotune_batched(flow_ctx* ctx, int32_t n, const flow_pair* pairs, const flow_params* p,
                                  void* stream);

/* Set the stage choice of `level` for batches with this batch's stage shapes, as
 * flow_autotune_batched would (for reuse of a measured choice, e.g. the "stages" entries of its
 * report): order 0 general tiles from the tile table / 1 general tiles from work queues / 2049,
 * 3073 or 4097 wave-row tiles of 32 / 48 / 64 rows from the tile table (the report's "nt" where it
 * is one of these), K iterations per tile launch (>= iters: the whole warp in one launch),
 * extended tile width ew in [16, 512] (at most 64 for the wave-row tiles).  For pDR and ALG1 batches
 * `order` is the stage's work-group code (the report's "nt": 1024 / 512 threads, pDR 2048 / 513 with
 * two cells of each colour, the wave-row codes 4098 / 6145 / 3074 / 2050 of pDR and 3074 / 2050 of
 * ALG1, as the scheme and beta allow) and `ew` is not used.  The choice changes speed only.
 * FLOW_E_INVAL if no pair has the level or one of its levels takes no tiles of that K and width
 * (that code and K).
 * Host-only. */
flow_status flow_tune_batched_stage(flow_ctx* ctx, int32_t n, const flow_pair* pairs, const flow_params* p,
                                    int32_t level, int32_t order, int32_t K, int32_t ew);

/* Autotuner: for every pyramid level of an H x W pair under params p, time each iteration-kernel
 * choice over one warp's iterations with HIP events on `stream`, and keep the fastest per level
 * shape for this context's later solves.  ADMM family: one-pass kernel with 2 / 4 / 8-row strips;
 * K-iteration tiles of 256, 1024 and small 1024-thread work-groups for every K in [2, 16] that is
 * the smallest giving its number of launches per warp, ceil(iters / n) (50 iterations: K = 2, 3,
 * 4, 5, 6, 7, 8, 9, 10, 13; tiles shortened to fill one round of work-groups where a level needs
 * less); the wave-row tiles of 64 x 32 / 48 / 64 cells for the same K; a resident tile where the
 * level fits.  pDR: the three-pass iteration, K-iteration tiles (1024 / 512 threads, one or two
 * cells of each colour, wave-row tiles with a cell pair or one cell per lane) for K = 1, 2, 3, 4, a
 * resident tile; ALG1: tiles of 1024 / 512 threads and wave-row tiles of 64 x 48 / 64 x 32 cells for
 * the same launch-count K values in [1, 10], a resident tile (all with balanced tiles).  Every choice computes the same iteration (results agree to rounding).  Blocking;
 * uses the context's arena (contents are overwritten). */
flow_status flow_autotune(flow_ctx* ctx, int32_t H, int32_t W, const flow_params* p, void* stream);

/* JSON report of the context's last autotuning call into buf (host, cap bytes including the
 * terminating NUL); FLOW_E_INVAL if it does not fit.  After flow_autotune: the choice and every
 * measured candidate per level shape.  After flow_autotune_batched: {"stages": [...]}, one entry
 * per stage (level, pairs, order 0 table / 1 work queue, K, extended tile width ew, and the
 * measured microseconds of one warp's tile launches). */
flow_status flow_get_tuning(const flow_ctx* ctx, char* buf, size_t cap);

/* Set the iteration-kernel choice of one level shape (H x W, with or without the w / p block, iters
 * per warp) by hand, as flow_autotune would.  pdr_sweeps = 0: the ADMM family, mode 1 = one-pass
 * kernel with `rows` rows per strip (0 = built-in; 2, 4 or 8), 2 / 3 / 4 / 7 / 6 / 8 / 9 = K-iteration
 * tiles of 256 / 1024 threads / small tiles of 1024 / 512 / 256 threads / one-pixel tiles of 1024 /
 * 512 threads with K iterations per launch (K = 0:
 * resident if the level fits one tile, else the built-in K) and `rows` the target width of a tile's
 * extended region (0 = built-in, else 16..512); 12 / 13 / 14 = wave-row tiles of 64 x 32 / 64 x 48 /
 * 64 x 64 cells (a `rows` above 64 acts as 64).  pdr_sweeps = n >= 1: pDR with n sweeps, mode 1 =
 * three-pass iteration, 5 / 6 = K-iteration tiles of 1024 / 512 threads (K = 0: resident), 10 / 11 =
 * the same with two cells of each colour per thread (beta = 0 only), 12 / 13 = wave-row tiles of
 * 128 x 32 / 128 x 48 cells with a cell pair per lane (13: beta = 0 only), 14 / 15 = wave-row tiles
 * of 64 x 48 / 64 x 32 cells with one cell per lane (14: beta = 0 only); pdr_sweeps = -1: ALG1,
 * modes 5 / 6 as for pDR and 14 / 15 = its wave-row tiles of 64 x 48 (beta = 0 only) / 64 x 32
 * cells.  Other modes: FLOW_E_INVAL.  Lets a caller reuse a tuning measured in another process.
 * Drops the context's captured graphs. */
flow_status flow_tune_choice(flow_ctx* ctx, int32_t H, int32_t W, int32_t has_w, int32_t iters, int32_t pdr_sweeps,
                             int32_t mode, int32_t K, int32_t rows);

/* Enable (1) or disable (0) per-solve event timing; flow_get_stats returns the last solve's. */
flow_status flow_set_stats(flow_ctx* ctx, int32_t enable);
flow_status flow_get_stats(const flow_ctx* ctx, flow_stats* out);

/* Bytes of device memory the context currently holds. */
flow_status flow_memory_in_use(const flow_ctx* ctx, size_t* bytes);

/* Process-wide kernel tuning knobs (set by the autotuner; 0 restores the built-in heuristic):
 *   "admm_rows"   rows per wavefront strip of the fused one-pass ADMM iteration kernel: 2, 4 or 8.
 *   "tb_mode"     iteration kernel per level: 0 built-in choice (levels that fit one 1024-thread tile
 *                 stay resident for a whole warp, larger ones use the one-pass kernel), 1 one-pass
 *                 kernel only, 2 K-iteration tiles of 256 threads, 3 of 1024 threads, 4 / 7 / 6
 *                 small tiles (2 pixels per thread) of 1024 / 512 / 256 threads, 8 / 9 one-pixel
 *                 tiles of 1024 / 512 threads, 12 / 13 / 14 wave-row tiles of 1024 threads (extended
 *                 regions of at most 64 columns and 32 / 48 / 64 rows, every field in registers).
 *   "tb_k"        iterations per tile launch on levels that do not fit one tile (0 = 4).
 *   "pdr_mode"    pDR iteration kernel: 0 built-in (tiles; a level that fits one tile keeps the whole
 *                 warp resident), 1 three-pass iteration, 5 / 6 tiles of 1024 / 512 threads, 10 / 11
 *                 large tiles (1024 / 512 threads, two cells of each colour per thread; with
 *                 beta > 0: 5 / 6), 12 / 13 wave-row tiles of 128 x 32 / 128 x 48 cells with a cell
 *                 pair per lane (with beta > 0: 12), 14 / 15 wave-row tiles of 64 x 48 / 64 x 32
 *                 cells with one cell per lane (with beta > 0: 15).  12 to 15 also select the
 *                 wave-row tiles in flow_op_pdr_tb, 14 and 15 those of ALG1 in flow_op_alg1_tb
 *                 (ALG1 solves take their kernels from flow_autotune or flow_tune_choice).
 *   "pdr_k"       iterations per pDR tile launch (0 = built-in 2).
 *   "batch_order" batched tile launches: -1 tuned / built-in, 0 tile table in XCD order, 1 per-XCD
 *                 work queues.
 *   "batch_k"     iterations per batched tile launch (0 = tuned / built-in; lowered where a level's
 *                 tiles cannot hold the halo).
 *   "batch_ew"    extended tile width target of batched tiles (0 = tuned / built-in, else 16..512).
 *   "batch_nt"    ADMM tile kernel of every batched and served stage: 0 tuned / built-in, 1025 the
 *                 general small tiles, 2049 / 3073 / 4097 the wave-row tiles (table order; a stage
 *                 whose levels take none of them keeps the general tiles).
 *   "serve_graph" serving epochs: 1 (default) replay their tile launches from captured graphs, 0
 *                 launch them directly (the same kernels and results).
 * FLOW_E_INVAL for an unknown key or value.  Not thread-safe against concurrent solves. */
flow_status flow_tune_set(const char* key, int64_t value);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* flow_last_error(void);

/* ------------------------------------------------------------------------------------------------
 * Operator-level entry points: one step of the pipeline on caller-provided device planes, for
 * testing each stage in isolation.  All planes of one call share H, W and the pitch ld.  They are
 * stream-ordered and do not synchronise; errors are reported before any launch.
 * ----------------------------------------------------------------------------------------------*/

/* Next pyramid level: dst (ceil(H/2) x ceil(W/2), pitch ldd) = mean of 2x2 blocks of src with
 * rows / columns past the edge replicated. */
flow_status flow_op_downsample(const float* src, int32_t H, int32_t W, int64_t ld, float* dst, int64_t ldd,
                               void* stream);

/* Central differences of I with replicated neighbours: Dx = (I[j+1] - I[j-1]) / 2, Dy likewise. */
flow_status flow_op_derivatives(const float* I, int32_t H, int32_t W, int64_t ld, float* Dx, float* Dy,
                                void* stream);

/* Warp and linearise (Sec. 1: rho(d) = grad I^T d + I_t) around (u0, v0):
 *   I_x = kappa B(DxI1)(x + d0), I_y = kappa B(DyI1)(x + d0),
 *   I_t = kappa (B(I1)(x + d0) - I0) - I_x u0 - I_y v0,
 * with B bilinear sampling at clamped coordinates, and at_out (device, one float) receives
 * max_ij(beta^2 + I_x^2 + I_y^2) = ||M_s||, the a~ of Prop. 3.1 (the iteration floors it at 1e-12). */
flow_status flow_op_linearize(const float* I0, const float* I1, const float* DxI1, const float* DyI1,
                              const float* u0, const float* v0, int32_t H, int32_t W, int64_t ld,
                              double kappa, double beta, float* Ix, float* Iy, float* It, float* at_out,
                              void* stream);

/* fine (Hf x Wf, pitch ldf) = scale * B(coarse)(i/2 - 1/4, j/2 - 1/4); the coarse plane is
 * ceil(Hf/2) x ceil(Wf/2) with pitch ldc.  Flow components use scale 2, illumination scale 1. */
flow_status flow_op_upsample(const float* coarse, int64_t ldc, float* fine, int32_t Hf, int32_t Wf, int64_t ldf,
                             double scale, void* stream);

/* State planes of the ADMM family (device, H x W, pitch ld).  w, px, py are only read / written
 * when beta > 0 (they may be NULL otherwise).  u0, v0 (read only, may be NULL) select the
 * increment form the solver uses: the multipliers are u0 + u, v0 + v, and I_t passed with them is
 * relative to (u0, v0), i.e. kappa (I1(x + d0) - I0); with u0 = v0 = NULL, u and v are the flow
 * and I_t is absolute.  flow_op_energy ignores u0, v0. */
typedef struct flow_admm_state {
    float *w, *u, *v, *px, *py, *q1x, *q1y, *q2x, *q2y, *s;
    const float *u0, *v0;
} flow_admm_state;

/* One iteration of the scheme in p->scheme (FLOW_PADMM or FLOW_RPADMM2) from `in` to `out`
 * (distinct planes).  Ix, Iy, It are the linearisation and at (device, one float) is a~. */
flow_status flow_op_admm_iter(const flow_admm_state* in, const flow_admm_state* out, const float* Ix,
                              const float* Iy, const float* It, const float* at, int32_t H, int32_t W,
                              int64_t ld, const flow_params* p, void* stream);

/* `iters` iterations in ONE launch of the temporally blocked tile kernel (the solver's path for
 * levels that do not need the one-pass kernel), increment form only (in->u0, in->v0 set).
 * threads: 256 (6 pixels per thread, 4 with beta > 0), 1024 (4, 3 with beta > 0), the small-tile
 * codes 1025 / 513 / 257 (1024 / 512 / 256 threads, 2 pixels per thread) or the one-pixel codes
 * 1026 / 514 (1024 / 512 threads, 1 pixel per thread); codes 513, 257, 1026 and 514 with order 0
 * only.  tile_h x tile_w: output tile; each tile's extended region (halo iters + 1 above and to the
 * left, iters below and to the right) min(H, tile_h + 2 iters + 1) x min(W, tile_w + 2 iters + 1)
 * must fit that capacity, else FLOW_E_INVAL.
 * order: 0 = one work-group per tile (tile from the work-group index), 1 = persistent work-groups
 * pulling tiles from one counter, 2 = the same with 8 per-XCD sub-queues (the batched path's work
 * queue), 3 = one work-group per entry of a tile table in XCD order (the batched path's table
 * order).  Every order computes the same values.  Blocking (synchronises the stream). */
flow_status flow_op_admm_tb(const flow_admm_state* in, const flow_admm_state* out, const float* Ix, const float* Iy,
                            const float* It, const float* at, int32_t H, int32_t W, int64_t ld,
                            const flow_params* p, int32_t iters, int32_t threads, int32_t tile_h, int32_t tile_w,
                            int32_t use_queue, void* stream);

/* State planes of pDR: X = (w, u, v), X bar = (wb, ub, vb), y bar = (pbx, pby, qb1x, qb1y, qb2x,
 * qb2y); w, wb, pbx, pby only when beta > 0.  Updated in place.  work: 3 scratch planes (device,
 * same shape and pitch).  s_out (may be NULL) receives Theta, the data dual of the resolvent. */
typedef struct flow_pdr_state {
    float *w, *u, *v, *wb, *ub, *vb, *pbx, *pby, *qb1x, *qb1y, *qb2x, *qb2y;
} flow_pdr_state;

/* One pDR iteration in place (Sec. 3.1.2, eq:resolvent, eq. neumann:boudary). */
flow_status flow_op_pdr_iter(const flow_pdr_state* st, float* work0, float* work1, float* work2,
                             float* s_out, const float* Ix, const float* Iy, const float* It, int32_t H,
                             int32_t W, int64_t ld, const flow_params* p, void* stream);

/* `iters` pDR iterations in ONE launch of the temporally blocked pDR tile kernel (the solver's path
 * for pDR levels), from `in` to `out` (distinct planes; in is not modified), with I_t relative to
 * the linearisation point (u0, v0) as in the solver: rho = I_t + beta w + I_x (u - u0) + I_y (v - v0).
 * tile_h x tile_w: output tile; each tile's extended region
 * min(H, tile_h + (4 gs_sweeps + 2) iters + 1) x min(W, tile_w + (4 gs_sweeps + 2) iters + 1) must hold
 * at most 2048 pixels, or 4096 with beta = 0 (regions above 2048 run the large tiles: 1024 threads
 * with two cells of each colour), else FLOW_E_INVAL.  With the "pdr_mode" knob at 12 to 15 the
 * wave-row tiles run instead: the region must then be at most 128 columns wide (knobs 12, 13) or
 * 64 (knobs 14, 15) and 32 rows high (48 with beta = 0 and knob 13 or 14), else FLOW_E_INVAL.
 * Every tile kernel gives bitwise the same iterates.  s_out
 * receives Theta of the last iteration.  Blocking. */
flow_status flow_op_pdr_tb(const flow_pdr_state* in, const flow_pdr_state* out, float* s_out, const float* Ix,
                           const float* Iy, const float* It, const float* u0, const float* v0, int32_t H, int32_t W,
                           int64_t ld, const flow_params* p, int32_t iters, int32_t tile_h, int32_t tile_w,
                           void* stream);

/* `iters` ALG1 iterations in ONE launch of its tile kernel, as flow_op_pdr_tb (same state planes:
 * X, X bar = the extrapolated point, y in the y bar slots; steps p->alg1_tau, p->alg1_sigma); each
 * tile's extended region min(H, tile_h + 2 iters) x min(W, tile_w + 2 iters) must hold at most 2048
 * pixels, else FLOW_E_INVAL.  With the "pdr_mode" knob at 14 or 15 the ALG1 wave-row tiles run
 * instead: the region must then be at most 64 columns wide and 48 (knob 14, beta = 0) or 32 rows
 * high.  Every tile kernel gives bitwise the same iterates.  Blocking. */
flow_status flow_op_alg1_tb(const flow_pdr_state* in, const flow_pdr_state* out, float* s_out, const float* Ix,
                            const float* Iy, const float* It, const float* u0, const float* v0, int32_t H, int32_t W,
                            int64_t ld, const flow_params* p, int32_t iters, int32_t tile_h, int32_t tile_w,
                            void* stream);

/* FP64 energy / dual / gap / residual of an ADMM-family state (see flow_result), blocking:
 * res is host memory and the stream is synchronised. */
flow_status flow_op_energy(const flow_admm_state* st, const float* Ix, const float* Iy, const float* It,
                           int32_t H, int32_t W, int64_t ld, double lambda, double beta, flow_result* res,
                           void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FLOWMI_FLOW_H */
