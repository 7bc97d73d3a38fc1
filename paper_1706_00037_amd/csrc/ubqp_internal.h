// Internal declarations of libubqp: context, resident problem, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <string>

#include "../../include/ubqp.h"

// Tile geometry of the int8 matrix-core contraction Y = X Q (eval_mfma.hip).
#define UBQP_NPAD_ALIGN 128

// Team ascent: a launch with at most UBQP_TEAM_MAX_P passers (one per SIMD of the
// 256-CU chip; two planes: UBQP_TEAM_MAX_P_I16; a launch table of several instances:
// at most UBQP_TEAM_MAX_P_GROUP / c each, c the instances of the (planes, NB) group) ascends each with UBQP_TEAM waves when the
// one-wave lane range has at least UBQP_TEAM_MIN_NB blocks of 16 columns
// (n_pad > 3072).  Relinking walks at most UBQP_RELINK_TEAM_MAX_P paths in teams.
#define UBQP_TEAM 4
#define UBQP_TEAM_MAX_P 1024
#define UBQP_TEAM_MAX_P_I16 512
#define UBQP_TEAM_MAX_P_GROUP 512
#define UBQP_RELINK_TEAM_MAX_P 512
#define UBQP_TEAM_MIN_NB 4

// The step-level ubqp_ascent works through passers in chunks of at most this many.
#define UBQP_ASCENT_CHUNK 4096
// A multi-start instance's Delta workspace holds at most this many bytes: its
// passers are ascended in one chunk when planes * M * n_pad * 4 bytes fit, else in
// chunks of as many passers as fit (a multiple of 256).
#define UBQP_DELTA_WS_BYTES (1ll << 30)

struct ubqp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // Growable device workspace of the step-level entry points, one buffer per slot
    // (a multi-start run owns its own device state).
    enum Slot { WS_PARTIALS, WS_Y, WS_STAGE, WS_TUNE, WS_RELINK, WS_COUNT };
    void *ws[WS_COUNT] = {};
    size_t ws_bytes[WS_COUNT] = {};
    int32_t *err_flag = nullptr;  // device int32: kernel-side checks (bit 0: flip limit, bit 1: index skipped)
    // Twice the number of live problems, runs, batches and servers created on the
    // context, plus 1 once ubqp_destroy has been called: the context is freed when
    // the call has come and the last of them is gone, in whichever order.
    std::atomic<int64_t> hold{0};
};
// A problem, run, batch or server that keeps ctx alive (hold when it takes the
// context, drop when it is freed; the drop frees a released context).
void ubqp_ctx_hold(ubqp_ctx *ctx);
void ubqp_ctx_drop(ubqp_ctx *ctx);

struct ubqp_problem {
    ubqp_ctx *ctx = nullptr;
    void *mem = nullptr;       // owned device block holding the arrays below (null: a view into server memory)
    int32_t n = 0, n_pad = 0, W = 0, planes = 1;
    int8_t *q = nullptr;       // [planes][n_pad][n_pad]: plane 0 (hi or the only plane), plane 1 (lo)
    void *qa = nullptr;        // ascent matrix, zero diagonal: int8 (planes 1) or int16 (planes 2) [n_pad][ncol_a]
    int32_t ncol_a = 0;        // columns of the ascent matrix: 1024 * ceil(n_pad / 1024)
    int32_t *diag = nullptr;   // [n_pad] q_ii (0 in the padding)
    uint64_t *deriv_x = nullptr;  // [W] first-derivative starting solution
    int64_t weight0 = 1;       // weight of plane 0 (256 when split)
    int64_t bias = 0;          // 128 when split: f += bias * popcount(x)^2, y_i += bias * popcount(x)
    int32_t flip_limit = 0;    // flips an uncapped ascent may make before it stops with UBQP_ELIMIT (0: default)
};
// The flip limit in force for p: its own, or 64 n_pad + 4096.
int32_t ubqp_problem_flip_limit(const ubqp_problem *p);

// Small device scalars of a multistart run.
struct ubqp_scal {
    int64_t npass;
    int64_t sum_max[2];
    int64_t best_f;
    int32_t have_best;
    int32_t best_c;
    int32_t gen;       // generation being processed (advanced at the end of each generation)
    int32_t pad_;
};

// SplitMix64 (Steele, Lea & Flood 2014) as a counter generator: output i of the
// generator seeded with `seed`.
__device__ inline uint64_t ubqp_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---- error handling shared by abi.hip and plan.hip ----------------------------
int ubqp_fail(ubqp_ctx *ctx, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int ubqp_hip_fail(ubqp_ctx *ctx, hipError_t e, const char *what);
int ubqp_set_device(ubqp_ctx *ctx);
int ubqp_check_flag(ubqp_ctx *ctx);  // read and clear the kernel-side error flag (synchronises)
int ubqp_check_params(ubqp_ctx *ctx, const ubqp_problem *p, const ubqp_params *pr);
// Make ctx->ws[slot] hold at least `bytes` (synchronises the stream when it grows).
int ubqp_ws_ensure(ubqp_ctx *ctx, int slot, size_t bytes, void **out);

#define UBQP_HIP_TRY(ctx, expr)                                         \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess) return ubqp_hip_fail((ctx), e_, #expr);   \
    } while (0)
#define UBQP_TRY(expr)                 \
    do {                               \
        int r_ = (expr);               \
        if (r_ != UBQP_OK) return r_;  \
    } while (0)

// Loads through global-address-space pointers: pointers read from argument tables
// are generic, so plain dereferences become flat loads (slower to issue and also
// counted by the LDS/scalar wait counter); these become global loads.
typedef unsigned int ubqp_v4u __attribute__((ext_vector_type(4)));
__device__ inline uint4 ubqp_ldg16(const void *p)
{
    const ubqp_v4u v = *(const __attribute__((address_space(1))) ubqp_v4u *)p;
    return uint4{v.x, v.y, v.z, v.w};
}
__device__ inline int4 ubqp_ldg16i(const void *p)
{
    const ubqp_v4u v = *(const __attribute__((address_space(1))) ubqp_v4u *)p;
    return int4{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
}
__device__ inline uint64_t ubqp_ldg8(const uint64_t *p) { return *(const __attribute__((address_space(1))) uint64_t *)p; }
__device__ inline int8_t ubqp_ldg1(const int8_t *p) { return *(const __attribute__((address_space(1))) int8_t *)p; }
// Relaxed device-scope int64 add in global memory (a global atomic, not a flat one).
__device__ inline void ubqp_atomic_add_i64(int64_t *p, int64_t v)
{
    __hip_atomic_fetch_add((unsigned long long __attribute__((address_space(1))) *)p, (unsigned long long)v,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Batched launches: a kernel covering several instances gets, per instance, its
// argument struct and the number of blocks (or waves) it needs; block b of the
// grid belongs to the instance i with prefix[i] <= b < prefix[i + 1].
__device__ inline int ubqp_find_inst(const int64_t *prefix, int count, int64_t b)
{
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// ---- resident problem construction (problem.hip) ------------------------------
#define UBQP_CHECK_ASYM 1u   // some q_ij != q_ji
#define UBQP_CHECK_RANGE 2u  // some q_ij outside [-32768, 32767]
#define UBQP_CHECK_WIDE 4u   // some q_ij outside [-128, 127]
struct ubqp_check_flags {
    uint32_t bits;
    uint32_t pad_;
    unsigned long long first[2];  // smallest linear index of an asymmetric / out-of-range entry
};
// Sets n, n_pad, W, planes, weight0, bias, ncol_a (device pointers untouched).
void ubqp_problem_geometry(ubqp_problem *p, int32_t n, int32_t planes);
// Bytes of one block holding the planes, the ascent matrix, diag and deriv_x.
size_t ubqp_problem_bytes(const ubqp_problem *p);
// Points q, qa, diag and deriv_x into `mem` (ubqp_problem_bytes(p) bytes).
void ubqp_problem_bind(ubqp_problem *p, char *mem);
// Queue the check of the staged coefficients (elem bytes each, n x n) into *fl.
hipError_t ubqp_queue_problem_check(hipStream_t st, const void *stage, int elem, int32_t n, ubqp_check_flags *fl);
// Queue the build of p's resident arrays from the staged coefficients.
hipError_t ubqp_queue_problem_build(hipStream_t st, const void *stage, int elem, const ubqp_problem *p);
// Queue a fill of `words` 32-bit zeros.
hipError_t ubqp_queue_zero(hipStream_t st, void *p, int64_t words);
// UBQP_OK, or the error (with message) that the check flags report.
int ubqp_check_outcome(ubqp_ctx *ctx, const ubqp_check_flags &fl, int32_t n);

// ---- per-instance kernel arguments --------------------------------------------
// Every kernel body takes one of these for its instance; single-instance
// launches pass it by value, batched launches read it from a device array.

struct DivArgs {             // Glover diversification, or blending of pairs of seeds
    const uint64_t *seeds;
    int32_t n, W, H;
    uint64_t *X;
    int64_t total;           // M * W output words
    int32_t blend;           // 0: Glover's generator; 1: blending (the fields below)
    int64_t M, S;
    uint64_t run_seed;
    const ubqp_scal *scal;   // generation index from scal->gen, or the constant g when null
    int64_t g;
};

struct EvalArgs {            // int8 matrix-core contraction Y = X Q and its epilogues
    const int8_t *q;         // plane 0; plane p at q + p * plane_stride
    int64_t plane_stride;
    int32_t n_pad;
    int32_t planes;
    const uint64_t *X;
    int32_t W;
    int64_t M;               // rows (or capacity of the gather list)
    const int32_t *rows;     // gather list (Y / key epilogues), already offset to the chunk
    int64_t x_rows;          // rows of X (gather targets outside [0, x_rows) read as zero)
    const int64_t *nrows_d;  // device length of the whole list (Y / key epilogues); row dot: null,
                             // or a device count of the rows to evaluate (the rest are skipped)
    int64_t offset;          // first list entry of this chunk
    int64_t *f;              // row-dot output
    int32_t *Y;              // Y output [planes][M][n_pad] or keys [M][n_pad]
    int64_t weight0;         // weight of plane 0 in the row dot
    int32_t m_tiles, n_tiles;
    const int32_t *diag;     // keys: q_jj
    int64_t bias;            // eval_init: f starts at bias * popcount(x)^2
    int32_t order;           // tile order: 0 n-tile-major, 1 m-tile-major (an eval variant choice)
    int32_t split_target;    // Y / key epilogues: split K below this many workgroups (0: never)
    int64_t split_team_max;  // ... and only while the ascent takes the rows in teams (its team_max)
};

struct ScreenArgs {          // exact T(lambda) screening
    const int64_t *f;
    int64_t M;
    int32_t lam_num, lam_den;
    int32_t *idx;
    int64_t *npass, *sum_max;
    int64_t *psum, *pmax, *cnt;  // partials, nblk each
    int32_t nblk;
};

struct OrdArgs {             // the order in which the ascent takes the passers
    const int64_t *f;        // objectives before the ascent
    const int32_t *idx;      // passers, ascending
    const int64_t *npass;
    int32_t *oidx;           // out: the passers, lowest objective first (bucketed)
};

struct AscArgs {             // steepest 1-flip ascent
    const void *qa;          // zero diagonal: int8 or int16 [n_pad][ncol_a]
    int32_t ncol_a;          // columns of the ascent matrix (1024 NB)
    const int32_t *diag;
    int32_t n, n_pad, W, planes;
    int64_t weight0, bias;
    uint64_t *X;
    int64_t x_rows;
    const int32_t *idx;
    const int64_t *nidx_d;   // length of the whole list
    int64_t offset;          // first list entry of this chunk
    int64_t max_idx;         // chunk capacity
    const int32_t *Y;        // [planes][max_idx][n_pad] (keys for one plane), row r for entry offset + r
    int64_t *f;
    int32_t *flips;
    int32_t max_flips, safety_cap;
    int32_t *err;
    int64_t team_max;        // launches with at most this many passers ascend them in teams (0: never)
    int32_t split_target;    // the Delta initialisation's split target (ubqp_dinit_split)
    int32_t pad_;
};

// Split K of the Delta initialisation.  A launch with few passers has few row tiles
// of 256: fewer workgroups than the chip holds.  While the team ascent takes the
// passers (P <= team_max), S workgroups share each tile's K range (K steps of 128)
// and store raw partial rows of x Q, partial s of row r at row s R 256 + r of the Y
// workspace (R = ceil(P / 256) row tiles, per plane); the team kernels sum the S
// partials when they load a passer.  Both sides take S from this function of the
// device passer count.  S x (active tiles) stays near `target` workgroups, the
// partials inside the workspace's cap rows, and the tiles inside the launch's grid
// (cap / 256 rounded up, times the column tiles and planes).
#define UBQP_SPLIT_TARGET 512
#define UBQP_SPLIT_MAX 8
__host__ __device__ inline int ubqp_dinit_split(int64_t P, int64_t cap, int n_pad, int planes, int64_t team_max,
                                                int target)
{
    if (P <= 0 || P > cap || P > team_max || target <= 0) return 1;
    const int64_t R = (P + 255) / 256, nk = n_pad / 128;
    const int64_t A = R * nk * planes;  // active tiles: row tiles x column tiles of 128 x planes
    if (A >= target) return 1;
    int64_t S = (target + A - 1) / A;
    S = S < UBQP_SPLIT_MAX ? S : UBQP_SPLIT_MAX;
    S = S < nk ? S : nk;
    const int64_t fit = (cap - P) / (R * 256) + 1, grid = ((cap + 255) / 256) / R;
    S = S < fit ? S : fit;
    S = S < grid ? S : grid;
    return S < 1 ? 1 : (int)S;
}

struct RelArgs {             // greedy path relinking, one wave per path
    const void *qa;          // ascent matrix (zero diagonal), int8 or int16 [n_pad][ncol_a]
    int32_t ncol_a;
    const int32_t *diag;
    int32_t n, n_pad, W, planes;
    int64_t weight0, bias;
    const uint64_t *elite;   // [E][W]
    int64_t E;
    const int32_t *pairs;    // [P][2]: initiating, guiding (this chunk's first pair at index 0)
    int64_t P;
    uint64_t *X;             // [P][W]: the initiating rows; receive the best intermediates
    const int32_t *Y;        // keys (one plane) or Y planes (two) of the initiating rows, [planes][P][n_pad]
    const int64_t *f0;       // [P] f of the initiating rows
    int64_t *f_mid, *f_out;  // [P]
    int32_t *steps;          // [P]
    int32_t *err;
};

struct SelArgs {             // incumbent update, next seeds, statistics, generation counter
    int32_t n, W;
    int64_t M, S;
    uint64_t run_seed;
    const uint64_t *X;
    const int64_t *f;
    const int32_t *flips;
    const int32_t *idx;
    int32_t *rank;           // [M] scratch: rank of each passer
    ubqp_scal *scal;
    uint64_t *best_x, *seeds;
    int64_t *stats;
    const uint64_t *deriv_x; // seed init: generation-0 seed 0 (or null)
    int64_t *f_dump;         // optional: G x M objective dump
};

// ---- argument builders, grid sizes and launchers --------------------------------
// Single-instance launchers take the arguments by value; *_batch launchers take a
// device array of per-instance arguments and the block prefix (count + 1 entries).
// Launchers return hipGetLastError() of the launch.

#define UBQP_EPI_ROWDOT 0  // f += x . (x Q) (the batched objective)
#define UBQP_EPI_Y 1       // store rows of x Q per plane (Delta initialisation, two planes)
#define UBQP_EPI_KEYS 2    // store the ascent keys (Delta initialisation, one plane)

int64_t ubqp_div_blocks(const DivArgs &a);
hipError_t ubqp_launch_diversify(hipStream_t st, const DivArgs &a);
hipError_t ubqp_launch_diversify_batch(hipStream_t st, const DivArgs *args, const int64_t *prefix, int count,
                                       int64_t blocks);

EvalArgs ubqp_eval_args(const ubqp_problem *p, const uint64_t *X, int64_t M, int64_t *f);
// Chunk [offset, offset + cap) of a device-counted list: r < min(*nrows_d - offset, cap).
// Two planes: Y[plane][r][:] = X_{rows[offset + r]} Q_plane; Y is [planes][cap][n_pad] int32.
// One plane: Y[r][j] = the ascent key of column j (Delta_j * 256 + 2 (127 - j mod PL) + x_j).
// Rows outside [0, x_rows) read as zero.
EvalArgs ubqp_yrows_args(const ubqp_problem *p, const uint64_t *X, int64_t x_rows, const int32_t *rows,
                         const int64_t *nrows_d, int64_t offset, int64_t cap, int32_t *Y);
int64_t ubqp_eval_tiles(const EvalArgs &a);
int64_t ubqp_yrows_tiles(const EvalArgs &a);
int64_t ubqp_eval_init_blocks(const EvalArgs &a);
hipError_t ubqp_launch_yrows(hipStream_t st, const EvalArgs &a);
hipError_t ubqp_launch_eval_init_batch(hipStream_t st, const EvalArgs *args, const int64_t *prefix, int count,
                                       int64_t blocks);
hipError_t ubqp_launch_eval_batch(hipStream_t st, int epilogue, const EvalArgs *args, const int64_t *prefix,
                                  int count, int64_t tiles);

// Variants of the row-dot contraction (the autotuner's choices): variant v uses
// column tiles ubqp_eval_variant_bn(v) wide, stages K ubqp_eval_variant_kc(v) deep
// and orders the tiles n-tile-major (v even) or m-tile-major (v odd).
#define UBQP_EVAL_DEFAULT_VARIANT 2
int ubqp_eval_variant_kc(int variant);
// Column-tile width of a variant (128 for every variant in use).
int ubqp_eval_variant_bn(int variant);
// Set a's tile order and column-tile count for a variant (before ubqp_eval_tiles).
void ubqp_eval_set_variant(EvalArgs &a, int variant);
hipError_t ubqp_launch_eval_v(hipStream_t st, EvalArgs a, int variant);  // eval_init + contraction
// The contraction alone, batched; every args[i].order must equal variant & 1.
hipError_t ubqp_launch_eval_rowdot_batch(hipStream_t st, int variant, const EvalArgs *args, const int64_t *prefix,
                                         int count, int64_t tiles);
// Variant the autotuner chose for (p, M), or UBQP_EVAL_DEFAULT_VARIANT if it has not run.
int ubqp_eval_variant_for(const ubqp_problem *p, int64_t M);
// Tune (p, M) unless cached; synchronous on ctx->stream.
int ubqp_tune_eval_internal(ubqp_ctx *ctx, const ubqp_problem *p, int64_t M, int32_t *variant, double *ms);

int32_t ubqp_screen_blocks(int64_t M);
size_t ubqp_screen_partials_bytes(int64_t M);
// One block per instance (args[i] for block i).
hipError_t ubqp_launch_order_batch(hipStream_t st, const OrdArgs *args, int count);
ScreenArgs ubqp_screen_args(const int64_t *f, int64_t M, int32_t lam_num, int32_t lam_den, int32_t *idx,
                            int64_t *npass, int64_t *sum_max, void *partials);
hipError_t ubqp_launch_screen(hipStream_t st, const ScreenArgs &a);
// Look up (once per device, with ctx->device current) the device address of the
// static scratch behind ubqp_screen_noalloc.
int ubqp_screen_scratch_init(ubqp_ctx *ctx);
hipError_t ubqp_launch_screen_batch(hipStream_t st, const ScreenArgs *args, const int64_t *prefix, int count,
                                    int64_t blocks);

// err_flag |= 1: an uncapped ascent reached the flip limit; |= 2: an index outside [0, x_rows) was skipped.
// Ascends X[idx[offset + r]] for r < min(*nidx_d - offset, cap), starting from Y rows r.
AscArgs ubqp_ascent_args(const ubqp_problem *p, uint64_t *X, int64_t x_rows, const int32_t *idx, const int64_t *nidx_d,
                         int64_t offset, int64_t cap, const int32_t *Y, int64_t *f, int32_t max_flips, int32_t *flips,
                         int32_t *err_flag);
int ubqp_ascent_nb(const AscArgs &a);
int64_t ubqp_ascent_waves(const AscArgs &a);
// Let the Delta initialisation yr split K (ubqp_dinit_split) for the ascent as that
// consumes its rows: both take the split from the same device passer count, target
// and team bound (call after ubqp_ascent_share_team).
void ubqp_split_dinit(EvalArgs &yr, AscArgs &as, int target);
// A launch table of `instances` instances (a batch or the server's active requests),
// `group` of them in this ascent's (planes, NB) group: with more than one instance,
// teams only while each has at most UBQP_TEAM_MAX_P_GROUP / group passers.
void ubqp_ascent_share_team(AscArgs &a, int group, int instances);
// Workgroups of the team launch (0 when the launch never uses teams).
int64_t ubqp_ascent_team_blocks(const AscArgs &a);
// Team launch of a batched ascent group (one coefficient width); n_pad_max: the
// largest n_pad of the group (sets the lane range).
hipError_t ubqp_launch_ascent_team_batch(hipStream_t st, int planes, int n_pad_max, const AscArgs *args,
                                         const int64_t *prefix, int count, int64_t blocks);
hipError_t ubqp_launch_ascent(hipStream_t st, const AscArgs &a);
RelArgs ubqp_relink_args(const ubqp_problem *p, const uint64_t *elite, int64_t E, const int32_t *pairs, int64_t P,
                         uint64_t *X, const int32_t *Y, const int64_t *f0, int64_t *f_mid, int64_t *f_out,
                         int32_t *steps, int32_t *err);
hipError_t ubqp_launch_relink(hipStream_t st, const RelArgs &a);
hipError_t ubqp_launch_ascent_batch(hipStream_t st, int planes, int nb, const AscArgs *args, const int64_t *prefix,
                                    int count, int64_t waves);

SelArgs ubqp_sel_args(int32_t n, int64_t M, int64_t S, uint64_t run_seed, const uint64_t *X, const int64_t *f,
                      const int32_t *flips, const int32_t *idx, int32_t *rank, ubqp_scal *scal, uint64_t *best_x,
                      uint64_t *seeds, int64_t *stats, const uint64_t *deriv_x, int64_t *f_dump);
int64_t ubqp_seed_blocks(const SelArgs &a);
int64_t ubqp_cand_blocks(const SelArgs &a);
int64_t ubqp_rank_blocks(const SelArgs &a);
hipError_t ubqp_launch_seed_init(hipStream_t st, const SelArgs &a);
hipError_t ubqp_launch_seed_init_batch(hipStream_t st, const SelArgs *args, const int64_t *seed_prefix, int count,
                                       int64_t seed_blocks);
hipError_t ubqp_launch_dump_batch(hipStream_t st, const SelArgs *args, const int64_t *cand_prefix, int count,
                                  int64_t cand_blocks);
// incumbent update + statistics, ranking and placement into seeds 1.., seed 0 and random fill,
// generation counter
hipError_t ubqp_launch_select_batch(hipStream_t st, const SelArgs *args, const int64_t *cand_prefix,
                                    int64_t cand_blocks, const int64_t *rank_prefix, int64_t rank_blocks,
                                    const int64_t *seed_prefix, int64_t seed_blocks, int count);
