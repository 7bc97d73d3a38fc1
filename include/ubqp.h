/*
 * ubqp.h -- C ABI of libubqp.so, an MI355X (gfx950) implementation of the
 * data-parallel hot path of the diversified multi-start method for the
 * Unconstrained Binary Quadratic Problem (Lewis, arXiv:1706.00037):
 *
 *     maximise f(x) = x^T Q x,  Q symmetric integer n x n,  x in {0,1}^n
 *                                                   (problem (P), Introduction)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers with suffix _d are device memory owned by the caller; the library
 *   never frees them.  Pointers with suffix _host are host memory.
 * - Solutions are bit-packed: W = ceil(n/64) uint64 words per solution, bit j in
 *   word j/64 at position j%64.  Bits at positions >= n must be 0 on input and
 *   are 0 on output.  A population of M solutions is M consecutive rows.
 * - Objective values are int64; everything on the path is exact integer
 *   arithmetic.  Coefficients must lie in [-32768, 32767] and n in [1, 8192]
 *   (the int32 accumulators of the int8 matrix-core contraction are exact in
 *   that range).
 * - Calls are asynchronous on the context's stream unless stated otherwise;
 *   device outputs are valid after the stream has been synchronised.
 * - Every call returns UBQP_OK (0) or a negative error code; no exception
 *   crosses the ABI.  ubqp_last_error() gives a message for the last failure
 *   on a context.  A context must not be used from two threads at once.
 */
#ifndef UBQP_H
#define UBQP_H

#include <stdint.h>

#if defined(__GNUC__)
#define UBQP_API __attribute__((visibility("default")))
#else
#define UBQP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define UBQP_OK 0
#define UBQP_EINVAL -1  /* null pointer, size or parameter out of its domain        */
#define UBQP_ERANGE -2  /* coefficient or n beyond the exactness bounds above       */
#define UBQP_EASYM -3   /* Q is not symmetric                                       */
#define UBQP_ENOMEM -4  /* device allocation failed                                 */
#define UBQP_EDEVICE -5 /* a HIP call or a kernel-side check failed (see last_error) */
#define UBQP_EBUSY -6   /* serving: the waiting queue is at its limit; submit later  */
#define UBQP_ELIMIT -7  /* an ascent to a local optimum reached the flip limit      */
                        /* (ubqp_problem_set_flip_limit) and stopped short of it     */

#define UBQP_MAX_N 8192
#define UBQP_MAX_M (1ll << 22)
#define UBQP_MAX_H 256

/* flags of ubqp_params */
#define UBQP_DERIV_START 1u /* generation-0 seed 0 is the first-derivative solution */
#define UBQP_TIMING 2u      /* record stream events around every phase of a generation */
#define UBQP_NO_GRAPH 4u    /* launch every kernel directly instead of replaying a captured generation */
#define UBQP_AUTOTUNE 8u    /* tune the evaluation's tiling for every instance first (ubqp_tune_eval) */
#define UBQP_BLEND 16u      /* diversify by blending pairs of seeds (ubqp_blend) instead of Glover's generator */

/* variants of the evaluation's matrix-core tiling (ubqp_tune_eval) */
#define UBQP_EVAL_VARIANTS 6

/* phases of a generation, in order (ubqp_result.phase_ms_host) */
#define UBQP_PHASE_DIVERSIFY 0
#define UBQP_PHASE_EVAL 1
#define UBQP_PHASE_SCREEN 2
#define UBQP_PHASE_ASCENT 3 /* Delta initialisation and ascent of all passers */
#define UBQP_PHASE_SELECT 4
#define UBQP_PHASE_ASCENT_KERNEL 5 /* the ascent kernels alone (a part of UBQP_PHASE_ASCENT) */
#define UBQP_PHASES 6

typedef struct ubqp_ctx ubqp_ctx;         /* library-owned: device, stream, workspace */
typedef struct ubqp_problem ubqp_problem; /* library-owned: Q resident on the device  */

/* Parameters of the multi-start loop (Fig. 2 of the paper, run one generation of
 * M candidates at a time). */
typedef struct {
    int64_t M;          /* candidates per generation, 1..UBQP_MAX_M                    */
    int32_t H;          /* diversification steps h = 1..H per seed (x' and x'' each);  */
                        /* S = ceil(M / 2H) seeds per generation                       */
    int32_t lam_num;    /* screening lambda = lam_num / lam_den, 0 <= lambda <= 1      */
    int32_t lam_den;
    int32_t G;          /* generations (iterations of the main loop), >= 1             */
    int32_t max_flips;  /* flips per ascent, 0 = until a 1-flip local optimum          */
    uint32_t flags;     /* UBQP_DERIV_START | UBQP_TIMING | UBQP_NO_GRAPH | UBQP_AUTOTUNE |   */
                        /* UBQP_BLEND; other bits are rejected (UBQP_EINVAL)             */
    uint64_t run_seed;  /* SplitMix64 seed of the random solutions                     */
} ubqp_params;

/* Result of a multi-start run.  Buffers are caller-owned; any may be NULL. */
typedef struct {
    int64_t best_f;         /* out: incumbent value (INT64_MIN if no candidate ever passed) */
    int32_t have_best;      /* out: 1 if an incumbent exists                               */
    int32_t generations;    /* out: generations completed so far                           */
    uint64_t *best_x_host;  /* out, W words: incumbent solution                            */
    int64_t *stats_host;    /* out, G x 5: per generation {Sum, Max, passers, flips,       */
                            /*   incumbent after the generation}                           */
    double *gen_ms_host;    /* out, G: milliseconds from the start of the run to the end   */
                            /*   of each generation, measured with stream events           */
    double *phase_ms_host;  /* out, G x UBQP_PHASES: milliseconds of each phase (runs      */
                            /*   created with UBQP_TIMING; left untouched otherwise); the  */
                            /*   first five partition the generation                       */
} ubqp_result;

typedef struct ubqp_run ubqp_run;      /* library-owned: the device state of one multi-start run */
typedef struct ubqp_batch ubqp_batch;  /* library-owned: several runs advanced together          */

/* Create a context on HIP device `device` that launches on `stream` (a
 * hipStream_t; 0 is the null stream).  *out receives the handle. */
UBQP_API int ubqp_create(ubqp_ctx **out, int device, void *stream);
/* Change the stream later calls launch on. */
UBQP_API int ubqp_set_stream(ubqp_ctx *ctx, void *stream);
/* Release the context and its workspace.  Problems, runs, batches and servers
 * created on it may still be alive: the context is then freed when the last of
 * them is destroyed (their destroy calls stay valid; no other call may take the
 * context after this one).  Call it once per context. */
UBQP_API int ubqp_destroy(ubqp_ctx *ctx);
/* Message describing the last error on ctx (never NULL; "" if none). */
UBQP_API const char *ubqp_last_error(const ubqp_ctx *ctx);
/* Block until all work issued on the context's stream has completed. */
UBQP_API int ubqp_sync(ubqp_ctx *ctx);

/*
 * Upload Q once and keep it resident (the paper copies Q to the GPU a single
 * time, Pseudocode section).  q_host: n x n int32, row-major, must be symmetric
 * with every entry in [-32768, 32767].  Entries all in [-128, 127] are stored
 * as one int8 plane; otherwise as two int8 planes hi = q >> 8 and
 * lo = (q & 255) - 128, so that q = 256 hi + lo + 128 exactly.  Synchronous.
 * Errors: UBQP_EINVAL (n out of [1, UBQP_MAX_N], null), UBQP_ERANGE, UBQP_EASYM,
 * UBQP_ENOMEM.
 */
UBQP_API int ubqp_problem_create(ubqp_ctx *ctx, int32_t n, const int32_t *q_host, ubqp_problem **out);
/* The same from coefficients of elem_bytes = 1 (int8), 2 (int16) or 4 (int32)
 * bytes each.  The checks and the conversion to the resident layout run on the
 * device; the host only copies the n x n coefficients. */
UBQP_API int ubqp_problem_create_typed(ubqp_ctx *ctx, int32_t n, const void *q_host, int32_t elem_bytes,
                                       ubqp_problem **out);
UBQP_API int ubqp_problem_destroy(ubqp_problem *prob);
/* n, padded size n_pad (a multiple of 128) and number of int8 planes (1 or 2). */
UBQP_API int ubqp_problem_info(const ubqp_problem *prob, int32_t *n, int32_t *n_pad, int32_t *planes);
/*
 * Flip limit of the steepest ascent to a local optimum (max_flips = 0) on prob:
 * `limit` >= 1 flips, or 0 for the default 64 n_pad + 4096.  In exact arithmetic
 * the ascent always ends (every flip raises the integer f, which lies within
 * +-sum |q_ij|), but that bound can exceed 10^9 flips, so a device-side limit
 * keeps a runaway ascent from holding the GPU.  An ascent that reaches the limit
 * stops there and the call that reports the device's checks -- ubqp_sync after
 * ubqp_ascent or ubqp_relink, ubqp_run_result, ubqp_multistart,
 * ubqp_batch_result, ubqp_sequential -- returns UBQP_ELIMIT, so a result cut
 * short is never reported as a success.  (Served requests use the default; their
 * status is UBQP_ELIMIT in that case.)  Capped ascents (max_flips > 0) stop at
 * their cap without error, as the ascent's definition says.  Takes effect for
 * ascents queued, and runs and batches created, after the call.
 * Errors: UBQP_EINVAL (null prob, limit < 0).
 */
UBQP_API int ubqp_problem_set_flip_limit(ubqp_problem *prob, int32_t limit);

/*
 * Glover diversification (Pseudocode section, "Diversify"; Glover 1998):
 * candidate c (0 <= c < M) is built from seed s = c / (2H) with step
 * h = (c mod 2H)/2 + 1: the seed with variables j = 0, h, 2h, ... flipped (x')
 * when c is even, the complement of x' (x'') when c is odd.
 * seeds_d: S x W, X_d: M x W (output).  Requires 1 <= H <= UBQP_MAX_H and
 * M <= 2 H S.
 */
UBQP_API int ubqp_diversify(ubqp_ctx *ctx, int32_t n, const uint64_t *seeds_d, int64_t S, int32_t H,
                   uint64_t *X_d, int64_t M);

/*
 * Blending diversification (Pseudocode section: new solutions bred from two
 * solutions; the paper gives no rule, this is a uniform crossover).  Candidates
 * come in pairs k = c / 2 (0 <= c < M); pair k of generation g has parents
 * a = k mod S and b = (a + 1 + k / S + g) mod S, and mask word w equal to
 * output 2^62 + (g ceil(M/2) + k) W + w of SplitMix64 seeded with run_seed.
 * Candidate 2k takes a's bits where the mask is 1 and b's where it is 0;
 * candidate 2k + 1 takes the opposite choice.  seeds_d: S x W (bits >= n zero),
 * X_d: M x W (output, bits >= n cleared).  Requires S >= 1 and 0 <= g < 2^31.
 * Multi-start runs use it in place of ubqp_diversify under UBQP_BLEND, with
 * g the generation index.
 */
UBQP_API int ubqp_blend(ubqp_ctx *ctx, int32_t n, const uint64_t *seeds_d, int64_t S, int64_t M, int64_t g,
                        uint64_t run_seed, uint64_t *X_d);

/*
 * Exact objective of M candidates (Introduction, problem (P); the evaluation
 * the paper moves to the GPU): f_d[c] = X_c^T Q X_c.  X_d: M x W, f_d: M int64
 * (output).  Computed as Y = X Q on int8 matrix cores with int32 accumulation,
 * fused with the row dot product sum_j x_j Y_j in int64.
 */
UBQP_API int ubqp_eval(ubqp_ctx *ctx, const ubqp_problem *prob, const uint64_t *X_d, int64_t M,
              int64_t *f_d);

/*
 * Autotuning of the evaluation (the contraction behind ubqp_eval and every
 * multi-start generation).  Variant v stages K 64, 128 or 256 deep (v / 2 = 0, 1,
 * 2) and orders workgroup tiles n-tile-major (v even) or m-tile-major (v odd);
 * all variants give identical results.  ubqp_tune_eval times each variant on
 * prob with M synthetic candidates (M rounded up to a power of two, at least
 * 256), remembers the fastest for (planes, n_pad, that M) for the life of the
 * process, and returns it in *variant (may be NULL) with the milliseconds of
 * every variant in ms_host[UBQP_EVAL_VARIANTS] (may be NULL).  Cached keys
 * return at once.  Later ubqp_eval calls, runs, batches and server generations
 * use the chosen variant.  Synchronous.
 * ubqp_eval_variant is ubqp_eval with an explicit variant.
 */
UBQP_API int ubqp_tune_eval(ubqp_ctx *ctx, const ubqp_problem *prob, int64_t M, int32_t *variant, double *ms_host);
/*
 * Work of one ubqp_eval of M candidates on prob with the variant in force:
 * *executed (may be NULL) receives the int8 matrix-core operations the launch
 * executes (2 per multiply-add; the lower triangle by column tiles, K padded to
 * the staging depth, whole row tiles), *dense (may be NULL) the dense definition
 * 2 n^2 M per plane.  Host arithmetic only.  Errors: UBQP_EINVAL.
 */
UBQP_API int ubqp_eval_ops(const ubqp_problem *prob, int64_t M, double *executed, double *dense);
UBQP_API int ubqp_eval_variant(ubqp_ctx *ctx, const ubqp_problem *prob, const uint64_t *X_d, int64_t M,
                               int64_t *f_d, int32_t variant);

/*
 * Measurement: the int8 matrix-core rate the device sustains (tera-ops per
 * second, 2 ops per multiply-add) on v_mfma_i32_32x32x32_i8, the instruction of
 * the evaluation, with operands in registers, 16 waves per compute unit, best of
 * three timed launches after a warm-up.  Synchronous.
 */
UBQP_API int ubqp_mfma_peak(ubqp_ctx *ctx, double *tops);

/*
 * Measurement: the read bandwidth (GB/s, 10^9 bytes) a streaming kernel sustains
 * from a device buffer of `bytes` (a multiple of 4 KiB in [1 MiB, 64 GiB]) that
 * the library allocates, fills and frees.  8 blocks of 256 threads per compute
 * unit; block b reads `per_block` bytes (a multiple of 32 KiB) cycling through
 * its window of `window` bytes (a multiple of 4 KiB dividing `bytes`) that starts
 * at byte (b * window) mod bytes, in coalesced 16-byte loads, 8 in flight per
 * thread.  window = bytes = a few MB: every block re-reads a buffer each XCD's L2
 * holds.  bytes of about 100 MB with small windows: the XCD's concurrently
 * running blocks cycle through more than its L2 holds, so the Infinity Cache
 * serves the reads.  window = per_block, blocks * per_block = bytes >> 256 MB:
 * every byte comes once from HBM.  Best of three timed launches after a warm-up.
 * Synchronous.
 */
UBQP_API int ubqp_read_peak(ubqp_ctx *ctx, int64_t bytes, int64_t window, int64_t per_block, double *gbs);


/*
 * Screening (Pseudocode section): T(lambda) = Mean + lambda (Max - Mean) over
 * the M values f_d, lambda = lam_num / lam_den; candidate c passes iff
 * f_d[c] > T, decided exactly as
 *     lam_den * M * f  >  (lam_den - lam_num) * Sum + lam_num * M * Max.
 * Outputs: pass_idx_d (M int32 capacity) gets the passer indices in ascending
 * order, n_pass_d (1 int64) their count, sum_max_d (2 int64) {Sum, Max}.
 */
UBQP_API int ubqp_screen(ubqp_ctx *ctx, const int64_t *f_d, int64_t M, int32_t lam_num, int32_t lam_den,
                int32_t *pass_idx_d, int64_t *n_pass_d, int64_t *sum_max_d);

/*
 * ubqp_screen for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, layout and results as ubqp_screen, but the block partials live in a
 * static device array of the library (48 KiB per GPU, held until the process
 * ends) instead of the context's growable workspace, so the call allocates
 * nothing.  M must be at most UBQP_SCREEN_NOALLOC_MAX_M (else UBQP_EINVAL, nothing
 * launched).  Every call on one GPU shares that GPU's array: calls that overlap on
 * one GPU (other streams, other contexts, other threads) race and give wrong
 * results; calls ordered on one stream are safe.
 */
#define UBQP_SCREEN_NOALLOC_MAX_M (1ll << 22)
UBQP_API int ubqp_screen_noalloc(ubqp_ctx *ctx, const int64_t *f_d, int64_t M, int32_t lam_num, int32_t lam_den,
                                 int32_t *pass_idx_d, int64_t *n_pass_d, int64_t *sum_max_d);

/*
 * Steepest 1-flip ascent (Pseudocode section; deltas of Glover et al. 2002) of
 * the candidates X_d[idx_d[p]], p < *n_idx_d (device count, at most max_idx);
 * X_d, f_d and flips_d have M rows:
 * repeatedly flip the variable with the largest
 *     Delta_i = (1 - 2 x_i) (q_ii + 2 sum_{j != i} q_ij x_j),
 * the lowest index among equal maxima, while that Delta is > 0 and fewer than
 * max_flips flips were made (max_flips == 0: no cap).  In place: rows of X_d,
 * f_d[c] (in: f of the row, out: f after ascent) and flips_d[c] (int32, out).
 * Rows not listed are untouched.  Listed indices outside [0, M) are skipped and
 * reported as UBQP_EDEVICE by the next ubqp_sync; an uncapped ascent that
 * reaches the problem's flip limit (ubqp_problem_set_flip_limit) is reported as
 * UBQP_ELIMIT by the next ubqp_sync.
 */
UBQP_API int ubqp_ascent(ubqp_ctx *ctx, const ubqp_problem *prob, uint64_t *X_d, int64_t M, const int32_t *idx_d,
                const int64_t *n_idx_d, int64_t max_idx, int64_t *f_d, int32_t max_flips,
                int32_t *flips_d);

/*
 * The multi-start loop (Fig. 2), one generation of M candidates at a time, on
 * the device with no host synchronisation inside a generation:
 *   seeds -> diversify -> evaluate -> screen -> ascent of the passers ->
 *   incumbent update (strict '>', earliest index wins) -> next seeds.
 * Generation-0 seeds are random: word w of seed s in generation g is output
 * (g S + s) W + w of SplitMix64 seeded with run_seed, bits >= n cleared
 * (seed 0 is the derivative start with UBQP_DERIV_START).  Next generation:
 * seed 0 = incumbent, then the ascended passers by (f desc, index asc), then
 * random solutions.
 *
 * ubqp_run_create allocates the run's device state (ubqp_run_footprint bytes)
 * and queues the generation-0 seeds; ubqp_run_step queues `generations` more
 * generations (at most params->G in total) and returns without waiting;
 * ubqp_run_result waits for them and fills *result.  f_dump_d (optional,
 * device, G x M int64) receives every candidate's f before ascent.
 */
UBQP_API int64_t ubqp_run_footprint(const ubqp_problem *prob, const ubqp_params *params);
UBQP_API int ubqp_run_create(ubqp_ctx *ctx, const ubqp_problem *prob, const ubqp_params *params,
                             int64_t *f_dump_d, ubqp_run **out);
UBQP_API int ubqp_run_step(ubqp_run *run, int32_t generations);
UBQP_API int ubqp_run_result(ubqp_run *run, ubqp_result *result);
UBQP_API int ubqp_run_destroy(ubqp_run *run);

/* The whole loop in one synchronous call: create, params->G steps, result, destroy. */
UBQP_API int ubqp_multistart(ubqp_ctx *ctx, const ubqp_problem *prob, const ubqp_params *params,
                             int64_t *f_dump_d, ubqp_result *result);

/*
 * The main loop of Fig. 2 as printed: one candidate per iteration.
 *   Mean: the average objective of `samples` random solutions
 *     (EvaluateRandomStarts; word w of sample s is SplitMix64 output s W + w of
 *     run_seed, bits >= n cleared);
 *   x0: the first-derivative starting solution; Max starts at f(x0);
 *   iteration 0 takes x0; iteration i >= 1 diversifies the incumbent (x0 while
 *     there is none) with Glover's generator, the step tied to the loop counter:
 *     with c = i - 1, variables j = 0, h, 2h, ... flip for h = (c / 2 mod H) + 1,
 *     and the result is complemented when c is odd;
 *   a candidate with f > T = Mean + lambda (Max - Mean) (decided exactly, as
 *     den * samples * f > (den - num) * Sum + num * samples * Max) is ascended
 *     (steepest 1-flip, at most max_flips); when its value beats the incumbent
 *     (strictly, or there is none) it becomes the incumbent and Max its value
 *     (UpdateBestAndT).
 * lambda is a fixed rational (the printed lambda = Max / Mean would put T above
 * Max).  The device works a window of up to `batch` iterations ahead: their
 * candidates are built from the current incumbent, evaluated together,
 * screened in order and every passer ascended; the first passer that replaces
 * the incumbent closes the window, and the iterations after it are built again
 * from the new incumbent in the next window.  The result therefore equals the
 * one-candidate-at-a-time loop for every window size.
 */
/*
 * Path relinking, the improvement phase the paper names to follow its initial
 * phase (Introduction, Pseudocode section, Conclusions) but does not build;
 * greedy relinking (Glover, Laguna & Marti 2000) is the rule taken.  Path p goes
 * from the initiating solution elite_d[pairs_d[2p]] toward the guiding one
 * elite_d[pairs_d[2p+1]]: the free variables are those where the two differ;
 * each step flips the free variable with the largest Delta (the lowest index on
 * ties), improving or not, and retires it, for |D| - 1 steps.  The intermediate
 * of largest f (the first on ties) is then ascended (steepest 1-flip, at most
 * max_flips, 0 = to a local optimum).
 * Outputs, P rows each: X_out_d (P x W) the ascended intermediate, f_mid_d its
 * value before and f_out_d after the ascent, steps_d its distance from the
 * initiating solution.  A path whose two solutions differ in at most one
 * variable has no intermediate: steps 0, f_mid = f_out = INT64_MIN, X_out the
 * initiating solution.  elite_d: E x W; pairs_d: P x 2 int32, each in [0, E)
 * (others are skipped and reported as UBQP_EDEVICE by the next ubqp_sync).
 * Asynchronous on the context's stream; uses a workspace of
 * planes x min(P, 4096) x n_pad x 4 bytes.
 */
UBQP_API int ubqp_relink(ubqp_ctx *ctx, const ubqp_problem *prob, const uint64_t *elite_d, int64_t E,
                         const int32_t *pairs_d, int64_t P, int32_t max_flips, uint64_t *X_out_d, int64_t *f_mid_d,
                         int64_t *f_out_d, int32_t *steps_d);

#define UBQP_SEQ_MAX_SAMPLES (1 << 20)
#define UBQP_SEQ_MAX_BATCH 8192

typedef struct {
    int64_t iterations;     /* I >= 1: iterations of the main loop                            */
    int32_t samples;        /* random solutions behind Mean, 1..UBQP_SEQ_MAX_SAMPLES           */
    int32_t H;              /* cycle of the diversification step, >= 1; 0 means n              */
    int32_t lam_num;        /* lambda = lam_num / lam_den, 0 <= lam_num <= lam_den              */
    int32_t lam_den;
    int32_t max_flips;      /* flips per ascent, 0 = until a 1-flip local optimum             */
    int32_t batch;          /* largest window, 1..UBQP_SEQ_MAX_BATCH, 0 = 1024 (speed only)    */
    uint32_t flags;         /* UBQP_NO_GRAPH, or 0                                             */
    int32_t pad_;
    uint64_t run_seed;      /* SplitMix64 seed of the samples                                  */
    double time_budget_ms;  /* > 0: stop launching windows once this much time has passed      */
} ubqp_seq_params;

typedef struct {
    uint64_t *best_x_host;   /* out, W words (may be NULL)                                      */
    int64_t *history_host;   /* out, history_cap x 2: (iteration, value) of the first           */
                             /*   history_cap replacements of the incumbent (may be NULL)        */
    double *history_ms_host; /* out, history_cap: ms from the start of the loop to the commit of */
                             /*   each replacement, device wall clock (may be NULL)             */
    int64_t history_cap;     /* entries of the history arrays                                    */
    int64_t *f_dump_d;       /* device, `iterations` int64: each iteration's f before ascent     */
                             /*   (may be NULL)                                                  */
    int64_t best_f;          /* out: incumbent value (INT64_MIN if none)                         */
    int32_t have_best;       /* out                                                              */
    int32_t pad_;
    int64_t iterations_done; /* out: I, or fewer when the time budget ended the loop             */
    int64_t sample_sum;      /* out: Sum of the samples' objectives (Mean = sample_sum / samples) */
    int64_t start_f;         /* out: f(x0)                                                       */
    int64_t passers;         /* out: iterations whose candidate passed the screen                */
    int64_t flips;           /* out: flips of their ascents                                      */
    int64_t improvements;    /* out: replacements of the incumbent                               */
    int64_t windows;         /* out: windows evaluated                                           */
    int64_t evaluated;       /* out: candidates evaluated, discarded look-ahead included         */
    double ms;               /* out: time of the loop after the set-up, from stream events        */
                             /*   (includes the windows queued after the last one, which idle)   */
    double ms_device;        /* out: device wall clock from the start of the loop to the commit  */
                             /*   of the last window                                             */
} ubqp_seq_result;

/* Synchronous.  Errors: UBQP_EINVAL (parameters, flags other than UBQP_NO_GRAPH),
 * UBQP_ENOMEM, UBQP_EDEVICE (the ascent's safety bound). */
UBQP_API int ubqp_sequential(ubqp_ctx *ctx, const ubqp_problem *prob, const ubqp_seq_params *params,
                             ubqp_seq_result *result);

/*
 * Batched form: `count` independent multi-start runs (instance i: probs[i],
 * params[i]; sizes, coefficient widths and parameters may all differ, the
 * generation count G must be equal) advanced together.  Each step of a
 * generation is one launch covering every instance: the grid is the
 * concatenation of the instances' work (candidate tiles, passer waves, seed
 * words), and a block finds its instance from a prefix table.  Unless
 * UBQP_NO_GRAPH or UBQP_TIMING is set in params[0].flags, the launches of a
 * generation are captured once as a HIP graph and replayed.  Every instance's
 * result equals the result of running it alone.
 * ubqp_batch_result(batch, i, result) waits and fills instance i's result.
 */
UBQP_API int64_t ubqp_batch_footprint(int32_t count, const ubqp_problem *const *probs, const ubqp_params *params);
UBQP_API int ubqp_batch_create(ubqp_ctx *ctx, int32_t count, const ubqp_problem *const *probs,
                               const ubqp_params *params, ubqp_batch **out);
UBQP_API int ubqp_batch_step(ubqp_batch *batch, int32_t generations);
UBQP_API int ubqp_batch_result(ubqp_batch *batch, int32_t i, ubqp_result *result);
UBQP_API int ubqp_batch_destroy(ubqp_batch *batch);
/* create, G steps, every result, destroy */
UBQP_API int ubqp_multistart_batched(ubqp_ctx *ctx, int32_t count, const ubqp_problem *const *probs,
                                     const ubqp_params *params, ubqp_result *results);

/*
 * Serving form: a request loop that runs multi-start solves as they arrive,
 * several at a time, on one device.  A request is a problem given as host
 * coefficients plus its parameters; its result equals the result of running it
 * alone (ubqp_problem_create_typed + ubqp_multistart).
 *
 * The server owns a device memory pool of pool_bytes and a worker thread.
 * Requests wait in FIFO order; the worker admits the oldest one when fewer than
 * max_active requests are admitted and the pool has room for its footprint
 * (ubqp_request_footprint: resident Q planes and ascent matrix, population,
 * objectives, Delta workspace, seeds).  An admitted request's coefficients are
 * copied and converted on a second stream while admitted requests compute.  At
 * every generation boundary the requests whose upload has finished join, and
 * one batched generation (the launches of the batched form) advances every
 * running request; a request leaves after its G generations and its memory
 * returns to the pool.  No request's work waits for another's to finish.
 *
 * Coefficients: elem_bytes = 1 (int8, one plane) or 2 (int16, hi/lo planes) or
 * 4 (int32 within [-32768, 32767], hi/lo planes).  q_host, best_x_host (W words)
 * and stats_host (G x 5, may be NULL) must stay valid until the request is
 * reported done; page-locked q_host makes the upload asynchronous.  params.flags
 * may hold UBQP_DERIV_START and UBQP_BLEND only.
 *
 * ubqp_server_wait blocks until at least one request has finished or timeout_us
 * (< 0: no limit) has passed, and moves up to `max` finished requests into
 * done[] (*count of them).  ubqp_server_destroy finishes every submitted request,
 * then releases the server.  Calls may come from any thread; the ubqp_ctx given
 * at creation belongs to the server until it is destroyed.
 */
typedef struct ubqp_server ubqp_server;
typedef struct {
    int64_t id;             /* as returned by ubqp_server_submit                          */
    int32_t status;         /* UBQP_OK, or the error that ended the request               */
    int32_t generations;    /* generations completed                                      */
    int64_t best_f;         /* incumbent value (INT64_MIN if none)                        */
    int32_t have_best;
    int32_t planes;         /* int8 planes the request's Q used (1 or 2)                  */
    int64_t t_submit_ns;    /* CLOCK_MONOTONIC times: submitted, admitted, first          */
    int64_t t_admit_ns;     /*   generation queued, results on the host                   */
    int64_t t_start_ns;
    int64_t t_done_ns;
} ubqp_request_info;

/* Pool bytes a request occupies while admitted (-1 if the arguments are invalid). */
UBQP_API int64_t ubqp_request_footprint(int32_t n, int32_t elem_bytes, const ubqp_params *params);
UBQP_API int ubqp_server_create(ubqp_ctx *ctx, int64_t pool_bytes, int32_t max_active, ubqp_server **out);
/* Errors: UBQP_EINVAL (arguments, or a footprint larger than the whole pool),
 * UBQP_EBUSY (the waiting queue is at the limit set by ubqp_server_set_queue_limit). */
UBQP_API int ubqp_server_submit(ubqp_server *server, int32_t n, const void *q_host, int32_t elem_bytes,
                                const ubqp_params *params, uint64_t *best_x_host, int64_t *stats_host,
                                int64_t *id);
/* Most requests that may wait for admission at once (0, the default: no limit).
 * While that many wait, ubqp_server_submit returns UBQP_EBUSY and takes nothing
 * (backpressure for callers that must not queue without bound).  Errors:
 * UBQP_EINVAL (null server, max_waiting < 0). */
UBQP_API int ubqp_server_set_queue_limit(ubqp_server *server, int64_t max_waiting);
UBQP_API int ubqp_server_wait(ubqp_server *server, int64_t timeout_us, ubqp_request_info *done, int32_t max,
                              int32_t *count);
/* Counters: {submitted, finished, failed, generations launched, most requests
 * running in one generation, pool high-water bytes, requests waiting, requests
 * admitted}. */
UBQP_API int ubqp_server_stats(ubqp_server *server, int64_t out[8]);
/* Message of the last server-level failure (never NULL; valid until the next
 * failing call on the server). */
UBQP_API const char *ubqp_server_error(ubqp_server *server);
UBQP_API int ubqp_server_destroy(ubqp_server *server);

/*
 * Benchmark files (Computational results section: the OR-Library bqp sets and
 * the Palubeckis instances are the paper's test problems).  Host code only: no
 * context and no device are needed.  Both formats are whitespace-separated
 * integers whose entries are 1-based (i, j, q) triples; each listed value fills
 * q_ij and q_ji (so an off-diagonal pair adds 2 q x_i x_j to f = x'Qx); a pair
 * listed twice must carry the same value both times (else UBQP_EASYM).
 */
#define UBQP_FMT_ORLIB 1    /* K, then K problems, each: n, nnz, nnz triples          */
#define UBQP_FMT_TRIPLETS 2 /* one problem: n, nnz, nnz triples                       */

/* Read problem `index` (0-based) of the file at `path`.  *count_out receives the
 * number of problems in the file and *n_out that problem's n.  With q_host NULL
 * only these two are returned (a size query); otherwise q_host (q_cap >= n * n
 * int32, caller-owned) receives the dense row-major matrix, zero where no entry
 * is listed, ready for ubqp_problem_create.  Returns UBQP_OK, UBQP_EINVAL (null
 * argument, unknown format, unreadable or malformed file, index out of range,
 * q_cap too small), UBQP_ERANGE (n > UBQP_MAX_N or a value outside int32) or
 * UBQP_EASYM; err (err_len bytes, may be NULL) receives the reason. */
UBQP_API int ubqp_read_instance(const char *path, int32_t format, int32_t index, int32_t *count_out,
                                int32_t *n_out, int32_t *q_host, int64_t q_cap, char *err, int32_t err_len);

#ifdef __cplusplus
}
#endif
#endif /* UBQP_H */
