// Internal declarations of libubqp: context, resident problem, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ubqp.h"

// Tile geometry of the int8 matrix-core contraction Y = X Q (eval_mfma.hip).
#define UBQP_NPAD_ALIGN 128

// Passers are ascended in chunks of at most this many (bounds the Y workspace).
#define UBQP_ASCENT_CHUNK 4096

struct ubqp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // Growable device workspace of the step-level entry points, one buffer per slot
    // (a multi-start run owns its own device state).
    enum Slot { WS_PARTIALS, WS_Y, WS_COUNT };
    void *ws[WS_COUNT] = {};
    size_t ws_bytes[WS_COUNT] = {};
    int32_t *err_flag = nullptr;  // device int32: kernel-side checks (ascent safety cap)
};

struct ubqp_problem {
    ubqp_ctx *ctx = nullptr;
    int32_t n = 0, n_pad = 0, W = 0, planes = 1;
    int8_t *q = nullptr;       // [planes][n_pad][n_pad]: plane 0 (hi or the only plane), plane 1 (lo)
    void *qa = nullptr;        // ascent matrix, zero diagonal: int8 [n_pad][ncol_a] (planes 1) or int16 [n_pad][n_pad]
    int32_t ncol_a = 0;        // columns of the int8 ascent matrix: 1024 * ceil(n_pad / 1024)
    int32_t *diag = nullptr;   // [n_pad] q_ii (0 in the padding)
    uint64_t *deriv_x = nullptr;  // [W] first-derivative starting solution
    int64_t weight0 = 1;       // weight of plane 0 (256 when split)
    int64_t bias = 0;          // 128 when split: f += bias * popcount(x)^2, y_i += bias * popcount(x)
};

// Small device scalars of a multistart run (WS_SCAL).
struct ubqp_scal {
    int64_t npass;
    int64_t sum_max[2];
    int64_t best_f;
    int32_t have_best;
    int32_t best_c;
};

// ---- launchers (return hipGetLastError() of the launch) ----
hipError_t ubqp_launch_diversify(hipStream_t st, int32_t n, const uint64_t *seeds, int64_t S, int32_t H,
                                 uint64_t *X, int64_t M);
// f[c] = X_c^T Q X_c for c < M.
hipError_t ubqp_launch_eval(hipStream_t st, const ubqp_problem *p, const uint64_t *X, int64_t M, int64_t *f);
// Chunk [offset, offset + cap) of a device-counted list: r < min(*nrows_d - offset, cap).
// Two planes: Y[plane][r][:] = X_{rows[offset + r]} Q_plane; Y is [planes][cap][n_pad] int32.
// One plane: Y[r][j] = the ascent key of column j (Delta_j * 256 + 2 (127 - j mod PL) + x_j).
// Rows outside [0, x_rows) read as zero.
hipError_t ubqp_launch_yrows(hipStream_t st, const ubqp_problem *p, const uint64_t *X, int64_t x_rows,
                             const int32_t *rows, const int64_t *nrows_d, int64_t offset, int64_t cap, int32_t *Y);
size_t ubqp_screen_partials_bytes(int64_t M);
hipError_t ubqp_launch_screen(hipStream_t st, const int64_t *f, int64_t M, int32_t lam_num, int32_t lam_den,
                              int32_t *idx, int64_t *npass, int64_t *sum_max, void *partials);
// err_flag |= 1: safety cap reached; |= 2: an index outside [0, x_rows) was skipped.
// Ascends X[idx[offset + r]] for r < min(*nidx_d - offset, cap), starting from Y rows r.
hipError_t ubqp_launch_ascent(hipStream_t st, const ubqp_problem *p, uint64_t *X, int64_t x_rows, const int32_t *idx,
                              const int64_t *nidx_d, int64_t offset, int64_t cap, const int32_t *Y, int64_t *f,
                              int32_t max_flips, int32_t *flips, int32_t *err_flag);
// Multistart selection kernels (select.hip).
hipError_t ubqp_launch_seed_init(hipStream_t st, uint64_t *seeds, int64_t S, int32_t n, uint64_t run_seed,
                                 const uint64_t *deriv_x, ubqp_scal *scal);
hipError_t ubqp_launch_select(hipStream_t st, int32_t n, int64_t M, int64_t S, int32_t g, uint64_t run_seed,
                              const uint64_t *X, const int64_t *f, const int32_t *flips, const int32_t *idx,
                              ubqp_scal *scal, uint64_t *best_x, uint64_t *seeds, int64_t *stats);
