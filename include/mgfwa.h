/*
 * mgfwa.h -- C ABI of the MI355X (gfx950) MGFWA hot path.
 *
 * The library runs the generation loop of GPU-MGFWA (the GPU multi-guiding spark
 * fireworks algorithm, Sec. 3 and Alg. 1 of the paper) on one GPU for black-box
 * optimisation of an MLP's weights (every spark is one weight vector of length
 * D, its fitness the MLP's loss over a fixed, shared sample set) or of a fixed
 * MLP's input (the paper's testbed, Sec. 4.1: the spark is the input, its
 * fitness the network's output; see mgfwa_problem).  Per
 * generation it generates the explosion sparks of all fireworks of all
 * populations at once, maps out-of-bounds coordinates back into the box,
 * evaluates every spark, builds the multi-guiding sparks from the top and
 * bottom sparks of each group, evaluates those, then selects each firework's
 * best individual, updates the dynamic amplitude and runs the loser-out
 * tournament (Alg. 1; Table 1 gives the batched B x N x D variables).
 *
 * Conventions shared by every entry point:
 *  - All functions return an mgfwa_status (0 = success) and never abort; on
 *    failure mgfwa_last_error() returns a thread-local message.
 *  - Device memory is owned by the caller: the workspace, the problem's sample,
 *    target and network-parameter buffers, and every buffer passed to
 *    ask/tell/evaluate.  The
 *    library never allocates device memory.  The context object itself is
 *    host memory owned by the library; release it with mgfwa_destroy.
 *  - All device work is enqueued on the caller's HIP stream given to
 *    mgfwa_init, in stream order; the library never uses the null stream
 *    (a NULL stream is rejected).  Only mgfwa_best, mgfwa_best_all,
 *    mgfwa_timing, mgfwa_autotune and the set-up of mgfwa_set_fit_plan
 *    synchronise with the host.
 *  - Determinism: the same (config, problem, seed, fitness plan) gives
 *    bit-identical state on any run.  The fitness plan is the launch shape of
 *    each fitness launch (mgfwa_plan_info); its FP32 summation order follows
 *    that shape.  Without autotuning the plan is a fixed function of the shape;
 *    mgfwa_autotune picks the fastest of the candidates by the clock, so two
 *    processes may pick different plans: every candidate meets the same
 *    fitness tolerance, and mgfwa_fit_candidates / mgfwa_set_fit_plan let a
 *    caller read the candidates and force one.
 */
#ifndef MGFWA_H
#define MGFWA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGFWA_API __attribute__((visibility("default")))

#define MGFWA_MAX_LAYERS 12       /* Linear layers of a problem's MLP */
#define MGFWA_MAX_TRAIN_LAYERS 4  /* ... when the spark is the MLP's weights */
#define MGFWA_MAX_WIDTH 256       /* largest layer output width (weights problems) */
#define MGFWA_MAX_NET_WIDTH 512   /* largest hidden width of a fixed network (input problems) */

typedef struct mgfwa_ctx mgfwa_ctx;

typedef enum {
    MGFWA_OK = 0,
    MGFWA_EINVAL = -1,       /* invalid argument or configuration */
    MGFWA_ENOMEM = -2,       /* workspace too small or misaligned */
    MGFWA_EHIP = -3,         /* a HIP runtime call failed (message has the HIP error) */
    MGFWA_ESTATE = -4,       /* call out of order (ask/tell protocol, step in tell mode) */
    MGFWA_EUNSUPPORTED = -5  /* valid MLP shape outside the compiled kernel set */
} mgfwa_status;

typedef enum { MGFWA_ACT_IDENTITY = 0, MGFWA_ACT_RELU = 1, MGFWA_ACT_TANH = 2,
               MGFWA_ACT_GELU = 3 } mgfwa_act;
typedef enum { MGFWA_LOSS_MSE = 0, MGFWA_LOSS_CE = 1 } mgfwa_loss;
typedef enum { MGFWA_FP32 = 0, MGFWA_BF16 = 1 } mgfwa_precision;
typedef enum { MGFWA_PROBLEM_WEIGHTS = 0, MGFWA_PROBLEM_INPUT = 1 } mgfwa_problem_kind;

/*
 * The black box f of Alg. 1, one of two kinds.
 *
 * kind = MGFWA_PROBLEM_WEIGHTS (0): the loss of an MLP whose weights are the spark.
 * Weight layout inside a spark (length D = sum_l in_l*out_l + out_l): for each
 * layer l in order, W_l as out_l x in_l row-major, then b_l (the nn.Linear
 * convention).  Hidden layers apply hidden_act[l]; the output layer is linear.
 *   MSE: mean over samples and outputs of (y_hat - y)^2.
 *   CE : mean over samples of logsumexp(z) - z[label].
 * x_dev    float32 [n_samples][widths[0]], row-major, device.
 * y_dev    float32 [n_samples][widths[n_layers]] (MSE only), device.
 * labels_dev int32 [n_samples], each in [0, widths[n_layers]) (CE only), device.
 * At most MGFWA_MAX_TRAIN_LAYERS layers, output widths <= MGFWA_MAX_WIDTH.
 *
 * kind = MGFWA_PROBLEM_INPUT (1): the paper's testbed (Sec. 4.1, eq. (1)): the
 * spark is the input x (D = widths[0]) of a fixed MLP and the fitness is its
 * scalar output f(x) (widths[n_layers] = 1).  net_dev holds the network's
 * float32 parameters in the weight layout above; hidden widths <= 512; loss,
 * n_samples, x_dev, y_dev and labels_dev are ignored.  FP32 only.
 *
 * The buffers are borrowed: mgfwa_init copies them into the workspace on the
 * stream, so they must stay valid until that work has run; afterwards the
 * library no longer reads them.
 */
typedef struct {
    int n_layers;                        /* 1..MGFWA_MAX_LAYERS */
    int widths[MGFWA_MAX_LAYERS + 1];    /* widths[0] = input dim ... widths[n_layers] = output */
    int hidden_act[MGFWA_MAX_LAYERS];    /* mgfwa_act per hidden layer (l < n_layers-1) */
    int loss;                            /* mgfwa_loss; CE needs widths[n_layers] >= 2 */
    int n_samples;                       /* >= 1 */
    const float *x_dev;
    const float *y_dev;
    const int32_t *labels_dev;
    int kind;                            /* mgfwa_problem_kind */
    const float *net_dev;                /* INPUT: the fixed network's parameters, device */
} mgfwa_problem;

/*
 * Algorithm parameters (Alg. 1; Sec. 2.1 names the operators).  B populations
 * of N fireworks each; every firework emits lambda explosion sparks, split into
 * G contiguous groups of m = lambda/G, and one guiding spark per group.
 *   sigma     fraction of a group in the top and the bottom set: k = max(1, floor(sigma*m)),
 *             sigma in (0, 0.5]
 *   boost     guiding spark = x + boost*delta (boosted guiding vector)
 *   amp_up, amp_down  dynamic amplitude factors on improvement / no improvement
 *   amp_init  initial and restart amplitude A0 (<= 0 selects ub - lb)
 *   lb, ub    search box [lb, ub]^D
 *   max_generations   T, the budget the loser-out prediction uses (>= 1)
 *   loser_out 1 enables the loser-out tournament
 *   precision fitness GEMMs in FP32, or BF16 operands with FP32 accumulation.
 *             With BF16 the candidates are ranked on their BF16 fitness (guiding
 *             groups, each firework's best candidate), and that best candidate is
 *             re-evaluated in FP32 before the selection compares it with its
 *             firework (Alg. 1, selection step), so the firework, initial and
 *             best-so-far fitness are FP32 values in every run
 *   external_fitness  1: no fitness kernels, the caller tells every fitness
 *   use_target, target_loss  stop once a population's best <= target_loss
 *   seed      key of the counter-based generator
 *   lag_guiding  1: Alg. 1's listing order taken literally -- each generation
 *             first builds its guiding sparks from the PREVIOUS generation's
 *             explosion sparks and their fitness (around the current fireworks;
 *             zero guiding vectors in the first generation), then explodes,
 *             then evaluates the explosion and guiding sparks in one fitness
 *             launch.  0 (the default) evaluates the explosion sparks first and
 *             builds the guiding sparks from them and their fitness (a guiding
 *             vector needs the fitness of the sparks it is built from: the
 *             guided-sparks scheme of GFWA that Sec. 2.1 credits).  Not
 *             available with external_fitness or with ask/tell.
 *   map_range 1: a coordinate that leaves [lb, ub] lands uniformly in the
 *             population's current range min..max of that dimension over its
 *             fireworks instead of uniformly in [lb, ub] (one reading of the
 *             "population-based random mapping" that Sec. 2.1 names as part of
 *             MGFWA; the paper does not define it)
 *   fit_path  0: the fitness kernel family follows from the problem's shape.
 *             A non-zero value forces a family, for tests and measurement:
 *             weights problems 1 = register-chain kernels (the MLP chained in
 *             registers, weights staged in LDS or read from L2), 2 = the
 *             K-streamed wide-first-layer kernel (two-layer nets with hidden
 *             width <= 256 and <= 16 outputs); input problems 1 = whole-network
 *             tiles, 2 = layer by layer, 3 = layer by layer with LDS-staged
 *             tiles.  EUNSUPPORTED when the family does not cover the shape.
 *   regen_sparks  1: the explosion sparks are not stored; the fitness kernel
 *             regenerates each spark from the counter-based generator as it
 *             stages the spark's weights in LDS, and the guiding, selection and
 *             best-so-far steps regenerate the sparks they read (the sparks are
 *             counter-based, so every step sees the same values).  Takes effect
 *             when the explosion-fitness plan stages its weights in LDS and the
 *             order is not lag_guiding; otherwise the sparks are stored as usual.
 *             The wide fitness kernel never stores the FP32 rows (its explosion
 *             writes the packed rows it reads).  mgfwa_state_info.se_written
 *             tells which applies.
 */
typedef struct {
    int n_populations;      /* B >= 1 */
    int n_fireworks;        /* N >= 1 */
    int n_sparks;           /* lambda >= 2, multiple of n_guiding, lambda/G >= 2 */
    int n_guiding;          /* G >= 1 */
    float sigma;
    float boost;
    float amp_up;
    float amp_down;
    float amp_init;
    float lb;
    float ub;
    int max_generations;
    int loser_out;
    int precision;          /* mgfwa_precision */
    int external_fitness;
    int use_target;
    float target_loss;
    uint64_t seed;
    int lag_guiding;
    int map_range;
    int fit_path;
    int regen_sparks;
} mgfwa_config;

/* Layout of the device state inside the workspace, for inspection: byte
 * offsets from the workspace base, plus the dimensions needed to read them.
 * Row-major arrays; "Dp" is D rounded up to 64 floats (padding is zero). */
typedef struct {
    int D, Dp, m, k, n_candidates;   /* n_candidates = lambda + G */
    int generation;                  /* host view of completed generations */
    size_t F;        /* float [B*N][Dp]   firework positions */
    size_t A;        /* float [B*N]       amplitudes */
    size_t Y;        /* float [B*N]       firework fitness */
    size_t Yprev;    /* float [B*N]       fitness before the last selection */
    size_t fresh;    /* int32 [B*N]       re-initialised in the previous generation */
    size_t SE;       /* float [B*N*lambda][Dp] explosion sparks */
    size_t SG;       /* float [B*N*G][Dp] guiding sparks */
    size_t Yc;       /* float [B*N][lambda+G] candidate fitness */
    size_t top;      /* int32 [B*N*G][k]  top members, ascending spark index */
    size_t bottom;   /* int32 [B*N*G][k]  bottom members, ascending spark index */
    size_t tie;      /* int32 [B*N*G]     group fitness all equal */
    size_t cstar;    /* int32 [B*N]       best candidate of the last selection */
    size_t improved; /* int32 [B*N] */
    size_t reinit;   /* int32 [B*N] */
    size_t best_x;   /* float [B][Dp] */
    size_t best_y;   /* float [B] */
    size_t best_f;   /* int32 [B] */
    size_t best_gen; /* int32 [B] */
    size_t gen;      /* int32 device generation counter */
    size_t done;     /* int32 device stop flag */
    int se_written;  /* 1: mgfwa_step writes every explosion spark to SE.  0: it does
                        not (the wide fitness kernel reads packed rows, and the guiding,
                        selection and best-so-far steps regenerate the sparks they need
                        from the counter-based generator); SE then holds sparks only
                        after mgfwa_ask */
} mgfwa_state_info;

/* Per-phase device time accumulated while timing is on (milliseconds). */
#define MGFWA_N_PHASES 5
typedef struct {
    double ms[MGFWA_N_PHASES];  /* 0 explosion sparks, 1 explosion fitness, 2 ranking + guiding
                                   sparks, 3 guiding fitness, 4 selection + loser-out; with
                                   lag_guiding, 0 also holds the ranking and guiding sparks,
                                   1 the fitness of both kinds and 2, 3 are empty */
    double gen_ms_p50, gen_ms_p99, gen_ms_mean; /* whole-generation device time */
    double fit_kernel_ms;       /* explosion-spark fitness GEMM kernel(s) alone (subset of
                                   ms[1]; the layer-by-layer launches of an input problem) */
    double check_fit_ms;        /* BF16 runs: the FP32 fitness launch of the selection
                                   re-check (subset of ms[4]); 0 otherwise */
    int generations;            /* generations measured since timing was switched on */
} mgfwa_timing_info;

/* Bytes of device workspace needed for (config, problem); 0 on invalid input. */
MGFWA_API size_t mgfwa_workspace_bytes(const mgfwa_config *config, const mgfwa_problem *problem);

/*
 * Create a context and run the initialisation of Alg. 1: fireworks uniform in
 * the box, amplitude A0, fitness of every firework (unless external_fitness),
 * best-so-far.  workspace_dev must be 256-byte aligned and hold at least
 * mgfwa_workspace_bytes bytes; it is owned by the caller and must outlive the
 * context.  hip_stream is a hipStream_t created by the caller (NULL -> EINVAL);
 * every later call on the context enqueues its work there.  The control words
 * are cleared by a kernel on that stream: mgfwa_init does not wait for the
 * device.
 * Errors: EINVAL (config/problem, NULL stream), ENOMEM (workspace),
 * EUNSUPPORTED (shape), EHIP (no device, launch failure).  *out is NULL on
 * failure.
 */
MGFWA_API mgfwa_status mgfwa_init(mgfwa_ctx **out, const mgfwa_config *config,
                                  const mgfwa_problem *problem, void *workspace_dev,
                                  size_t workspace_bytes, void *hip_stream);

/*
 * Enqueue n_generations generations (the repeat loop of Alg. 1) on the stream
 * and return without waiting.  Generations after the stop flag is raised are
 * no-ops on the device.  ESTATE when external_fitness is set or an ask/tell
 * exchange is in progress.
 */
MGFWA_API mgfwa_status mgfwa_step(mgfwa_ctx *ctx, int n_generations);

/*
 * The returned answer of Alg. 1: the best fitness found and its position, over
 * all populations (lowest fitness, lower population on ties).  Synchronises
 * the stream.  x_host: float[D] or NULL; f_host, generation: may be NULL;
 * *generation receives the number of completed generations.
 */
MGFWA_API mgfwa_status mgfwa_best(mgfwa_ctx *ctx, float *x_host, float *f_host, int *generation);

/* Per-population best: x_host float[B][D] (or NULL), f_host float[B], gen_host
 * int32[B] = generation at which each best was found (NULLs allowed). Syncs. */
MGFWA_API mgfwa_status mgfwa_best_all(mgfwa_ctx *ctx, float *x_host, float *f_host,
                                      int32_t *gen_host);

/*
 * Black-box form of Alg. 1 (the caller evaluates f).  The exchange is
 *   [after init, external_fitness only] ask -> B*N fireworks, tell -> their fitness;
 *   then per generation: ask -> B*N*lambda explosion sparks, tell;
 *                        ask -> B*N*G guiding sparks, tell (runs the selection).
 * ask returns a device pointer into the workspace (float, rows x ld, row-major,
 * valid until the next tell) and enqueues the work that produces it.  tell reads
 * fitness_dev (float[rows], device, caller-owned) in stream order; NaN counts as
 * +inf.  Any other order -> ESTATE.  In problem mode (external_fitness = 0)
 * ask/tell may replace the built-in fitness for any generation.  A context with
 * lag_guiding returns EUNSUPPORTED (its order has no ask/tell form).
 */
MGFWA_API mgfwa_status mgfwa_ask(mgfwa_ctx *ctx, const float **sparks_dev, int *rows, int *ld);
MGFWA_API mgfwa_status mgfwa_tell(mgfwa_ctx *ctx, const float *fitness_dev);

/*
 * Fitness of `rows` sparks (weight vectors, or network inputs for an input
 * problem; the evaluation step of Alg. 1 on its own):
 * w_dev float [rows][ld] device (16-byte aligned, ld >= D, ld % 4 == 0),
 * out_dev float [rows] device; both caller-owned, read/written in stream order.
 * Uses the context's problem and precision.  EINVAL without a problem.
 */
MGFWA_API mgfwa_status mgfwa_evaluate(mgfwa_ctx *ctx, const float *w_dev, int rows, int ld,
                                      float *out_dev);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops or harnesses that forbid allocation): the fitness of `rows`
 * sparks of a weights problem (kind = MGFWA_PROBLEM_WEIGHTS), with no context and
 * no workspace.  It runs the kernels and launch shapes of mgfwa_evaluate (no
 * autotuning) in the given precision, so its values equal those of mgfwa_evaluate
 * on a context of the same problem and precision whenever both take the rows in
 * one launch.
 * problem   the MLP loss problem as for mgfwa_init; its x/y/labels buffers are
 *           read in stream order by this call.
 * precision mgfwa_precision of the fitness GEMMs.
 * w_dev     float [rows][ld] device (16-byte aligned, ld >= D, ld % 4 == 0);
 * out_dev   float [rows] device; both caller-owned, in stream order.
 * hip_stream  a stream created by the caller (NULL -> EINVAL).
 * Scratch: the packed samples, targets and per-row partial sums live in a
 * library-held device array of MGFWA_NOALLOC_SCRATCH_BYTES (one per device, held
 * until the process ends); rows are taken in chunks that fit it.  EINVAL when
 * the packed problem plus one row does not fit.  The call allocates nothing
 * (no hipMalloc/hipFree, no library allocation) and does not wait for the device.
 * Every call on one device shares that device's array: calls that may overlap
 * on one device (different streams, or different host threads) race; order
 * them on one stream.  Errors: EINVAL (arguments, problem too large for the
 * scratch), EUNSUPPORTED (input problems, shapes outside the compiled kernels),
 * EHIP.
 */
#define MGFWA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
MGFWA_API mgfwa_status mgfwa_evaluate_noalloc(const mgfwa_problem *problem, int precision,
                                              const float *w_dev, int rows, int ld,
                                              float *out_dev, void *hip_stream);

/* Offsets and dimensions of the device state (no device work). */
MGFWA_API mgfwa_status mgfwa_state(const mgfwa_ctx *ctx, mgfwa_state_info *info);

/*
 * Timing: while on, generations are launched kernel by kernel with HIP events
 * around each phase (instead of one graph per generation); mgfwa_timing
 * synchronises and reports the accumulated per-phase device time.  Switching
 * on resets the totals.
 */
MGFWA_API mgfwa_status mgfwa_set_timing(mgfwa_ctx *ctx, int on);
MGFWA_API mgfwa_status mgfwa_timing(mgfwa_ctx *ctx, mgfwa_timing_info *info);

/* Release the context (waits for its pending work).  NULL is a no-op. */
MGFWA_API void mgfwa_destroy(mgfwa_ctx *ctx);

/* Thread-local message of the last failure in this thread ("" if none). */
MGFWA_API const char *mgfwa_last_error(void);

/* Library version string. */
MGFWA_API const char *mgfwa_version(void);

/* ------------------------------------------------------------------------ */
/* Tuning and batched generations.                                          */
/* ------------------------------------------------------------------------ */

/* The fitness launch shape of a context (the fitness step of Alg. 1 as a grouped
 * GEMM): which = 0 explosion sparks (with lag_guiding: the explosion and the
 * guiding sparks, one launch), 1 guiding sparks (unused with lag_guiding), 2 the
 * FP32 re-check of each firework's best candidate in a run with BF16 built-in
 * fitness (B*N rows; ESTATE for other contexts).  EINVAL for other values. */
typedef struct {
    int wide;               /* 1: the K-streamed wide-first-layer kernel (fixed tiles) */
    int rows;               /* sparks per launch */
    int wavefronts;         /* per block */
    int slabs;              /* 16-sample slabs per wavefront in flight */
    int lds_weights;        /* 1: the spark's weights are staged in LDS */
    int blocks_per_row;     /* blocks per spark (sample split) */
    int samples_per_block;
    int lds_bytes;
    int row_blocks[4];      /* 16-row MFMA blocks per layer (padded widths / 16) */
    int net_kernel;         /* input problems: 0..3 layer by layer with 64x128, 64x64, 32x32
                               or K-split 16x16 output tiles, 4 whole-network 16/32-row tiles,
                               5 / 6 layer by layer with LDS-staged 64x128 / 64x64 tiles,
                               -1 chosen per launch from the shape (before autotuning) */
} mgfwa_plan_info;

MGFWA_API mgfwa_status mgfwa_fit_plan(const mgfwa_ctx *ctx, int which, mgfwa_plan_info *info);

/*
 * Autotune the fitness launches of a context (which = 0, 1 and, with BF16
 * fitness, 2 of mgfwa_plan_info): every compiled kernel variant that
 * covers the MLP shape, with a few sample splits, is timed on the device (reps
 * launches each, on the context's stream, over its own spark buffers) and the
 * fastest is kept.  The choice is cached for the process per (shape, precision,
 * samples, sparks): any later context of the same shape takes it without timing,
 * so within a process a job's fitness values (whose summation order follows the
 * launch shape) depend only on its shape, alone or in a batch.  Another process
 * may time the candidates differently and keep another one: read the choice with
 * mgfwa_fit_plan and force it with mgfwa_set_fit_plan where bit-identical
 * results across processes are needed.  Call before the first generation
 * (ESTATE otherwise).  Contexts on the wide kernel keep their fixed tiles (OK,
 * nothing changes).  Input problems time their kernels' tile shapes (net_kernel
 * of mgfwa_plan_info).  Synchronises the stream.
 */
MGFWA_API mgfwa_status mgfwa_autotune(mgfwa_ctx *ctx, int reps);

/*
 * The candidate plans of one fitness launch of a context (which as in
 * mgfwa_fit_plan): the compiled kernel variants that cover the shape with their
 * sample splits (weights problems), the tile shapes (input problems), or the one
 * fixed plan of the wide kernel.  Writes up to max_out entries to out (may be
 * NULL) and their total count to *n.  No device work.
 */
MGFWA_API mgfwa_status mgfwa_fit_candidates(const mgfwa_ctx *ctx, int which, mgfwa_plan_info *out,
                                            int max_out, int *n);

/*
 * Force candidate `index` (of mgfwa_fit_candidates) as the plan of fitness launch
 * `which`, bypassing the shape rule and the autotuner's cache.  Call before the
 * first generation (ESTATE otherwise).  EINVAL for an index out of range.
 */
MGFWA_API mgfwa_status mgfwa_set_fit_plan(mgfwa_ctx *ctx, int which, int index);

/*
 * Batched generations: many independent jobs (contexts of any shapes, each its
 * own run of Alg. 1 over its own workspace) advanced together by one HIP graph
 * launch per generation.  The graph holds every job's generation as independent
 * branches, so the kernels of different jobs overlap on the device; each job's
 * kernels, launch shapes and results are exactly those of stepping it alone.
 * The contexts stay owned by the caller and must outlive the batch; while they
 * are in a batch they may still be read (best, state) and stepped alone.
 * hip_stream: the launch stream, created by the caller (NULL -> EINVAL);
 * mgfwa_batch_step orders itself after work already queued on each job's stream
 * and before later work there.  Errors: EINVAL (no jobs, NULL or repeated job,
 * NULL stream), ESTATE (a job uses
 * external fitness, is in an ask/tell exchange or has timing on), EHIP.
 */
typedef struct mgfwa_batch mgfwa_batch;
MGFWA_API mgfwa_status mgfwa_batch_create(mgfwa_batch **out, mgfwa_ctx *const *ctxs, int n_jobs,
                                          void *hip_stream);
/* Enqueue n_generations generations of every job (asynchronous). */
MGFWA_API mgfwa_status mgfwa_batch_step(mgfwa_batch *batch, int n_generations);
/* Release the batch (waits for its launch stream); the contexts are untouched. */
MGFWA_API void mgfwa_batch_destroy(mgfwa_batch *batch);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of many optimisation jobs on one device.     */
/* Each job is an independent run of Alg. 1 (its own population, problem and */
/* seed).  The server sub-allocates job workspaces from one caller-owned     */
/* device arena, admits queued jobs in arrival order as soon as their        */
/* workspace fits (first fit), advances every active job by one generation   */
/* per tick on a pool of HIP streams so that different jobs' kernels overlap */
/* on the device, and retires a job when it reaches its generation budget or */
/* its target loss, freeing its memory for the queue.  A job's state is      */
/* bit-identical whether it runs alone or in the mix.                        */
/* ------------------------------------------------------------------------ */
typedef struct mgfwa_server mgfwa_server;

typedef enum { MGFWA_JOB_QUEUED = 0, MGFWA_JOB_RUNNING = 1, MGFWA_JOB_DONE = 2,
               MGFWA_JOB_FAILED = 3 } mgfwa_job_state;

typedef struct {
    int state;              /* mgfwa_job_state */
    int generations;        /* completed generations */
    float best_fitness;     /* over the job's populations (valid once RUNNING) */
    size_t workspace_bytes; /* footprint in the arena */
    double submit_ms, admit_ms, finish_ms;  /* host clock since server creation */
} mgfwa_job_info;

typedef struct {
    int queued, running, done, failed;
    long generations;                 /* total generations completed */
    double gen_ms_p50, gen_ms_p99;    /* per-generation device latency of running jobs */
    double wall_ms;                   /* host clock since server creation */
    double spark_evals_per_s;         /* completed candidate evaluations / wall time */
    size_t arena_bytes, arena_used, arena_peak;
} mgfwa_server_stats;

/* Create a server over arena_dev (256-byte aligned, caller-owned, outlives the
 * server) with n_streams HIP streams (1..64, created by the server).  */
MGFWA_API mgfwa_status mgfwa_server_create(mgfwa_server **out, void *arena_dev,
                                           size_t arena_bytes, int n_streams);

/* Queue a job.  config->max_generations is the job's generation budget (and
 * the loser-out horizon); use_target/target_loss stop it early.  The problem's
 * device buffers are read when the job is admitted and must stay valid until
 * mgfwa_server_job reports it RUNNING or later.  EINVAL on an invalid job,
 * ENOMEM if its workspace exceeds the whole arena.  *job_id is the handle. */
MGFWA_API mgfwa_status mgfwa_server_submit(mgfwa_server *s, const mgfwa_config *config,
                                           const mgfwa_problem *problem, int64_t *job_id);

/* One scheduling tick: collect finished generations, retire finished jobs,
 * admit queued jobs that fit, enqueue one generation of every running job.
 * Does not wait for the device. */
MGFWA_API mgfwa_status mgfwa_server_tick(mgfwa_server *s);

/* Tick until every submitted job is DONE or FAILED (waits for the device). */
MGFWA_API mgfwa_status mgfwa_server_drain(mgfwa_server *s);

/* Status of a job; x_host (float[D], may be NULL) receives its best position
 * once DONE (the job's device memory is then already released: the best is
 * kept on the host when the job retires). */
MGFWA_API mgfwa_status mgfwa_server_job(mgfwa_server *s, int64_t job_id, mgfwa_job_info *info,
                                        float *x_host);

MGFWA_API mgfwa_status mgfwa_server_stats_get(mgfwa_server *s, mgfwa_server_stats *stats);

/* Waits for outstanding work, releases every job and the streams. */
MGFWA_API void mgfwa_server_destroy(mgfwa_server *s);

#ifdef __cplusplus
}
#endif
#endif /* MGFWA_H */
