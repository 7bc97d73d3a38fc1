// C ABI of libubqp, part 1: contexts and the step-level entry points
// (diversify, eval, screen, ascent).  Resident problems are in problem.hip, the
// multi-start runs and batches in plan.hip, the request server in serve.hip.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "ubqp_internal.h"

int ubqp_fail(ubqp_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

int ubqp_hip_fail(ubqp_ctx *ctx, hipError_t e, const char *what)
{
    return ubqp_fail(ctx, e == hipErrorOutOfMemory ? UBQP_ENOMEM : UBQP_EDEVICE, "%s: %s", what,
                     hipGetErrorString(e));
}

int ubqp_set_device(ubqp_ctx *ctx)
{
    UBQP_HIP_TRY(ctx, hipSetDevice(ctx->device));
    return UBQP_OK;
}

// Make ctx->ws[slot] hold at least `bytes`.
int ubqp_ws_ensure(ubqp_ctx *ctx, int slot, size_t bytes, void **out)
{
    if (bytes == 0) bytes = 256;
    if (ctx->ws_bytes[slot] < bytes) {
        if (ctx->ws[slot]) {
            UBQP_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            UBQP_HIP_TRY(ctx, hipFree(ctx->ws[slot]));
            ctx->ws[slot] = nullptr;
            ctx->ws_bytes[slot] = 0;
        }
        UBQP_HIP_TRY(ctx, hipMalloc(&ctx->ws[slot], bytes));
        ctx->ws_bytes[slot] = bytes;
    }
    *out = ctx->ws[slot];
    return UBQP_OK;
}

namespace {

__global__ void zero_i32(int32_t *p) { *p = 0; }

int check_words(ubqp_ctx *ctx, int32_t n, int64_t M)
{
    if (n < 1 || n > UBQP_MAX_N) return ubqp_fail(ctx, UBQP_EINVAL, "n=%d outside [1, %d]", n, UBQP_MAX_N);
    if (M < 1 || M > UBQP_MAX_M)
        return ubqp_fail(ctx, UBQP_EINVAL, "M=%lld outside [1, %lld]", (long long)M, (long long)UBQP_MAX_M);
    return UBQP_OK;
}

}  // namespace

int ubqp_check_flag(ubqp_ctx *ctx)
{
    int32_t v = 0;
    UBQP_HIP_TRY(ctx, hipMemcpyAsync(&v, ctx->err_flag, 4, hipMemcpyDeviceToHost, ctx->stream));
    UBQP_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (v) {
        hipLaunchKernelGGL(zero_i32, dim3(1), dim3(1), 0, ctx->stream, ctx->err_flag);
        UBQP_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (v & 2)
            return ubqp_fail(ctx, UBQP_EDEVICE, "an index outside its range was skipped (an ascent candidate or a "
                                                "relinking pair)%s", (v & 1) ? "; an ascent also reached its flip limit" : "");
        return ubqp_fail(ctx, UBQP_ELIMIT, "an ascent to a local optimum reached the problem's flip limit and stopped "
                                           "short of it (ubqp_problem_set_flip_limit)");
    }
    return UBQP_OK;
}

int ubqp_check_params(ubqp_ctx *ctx, const ubqp_problem *p, const ubqp_params *pr)
{
    UBQP_TRY(check_words(ctx, p->n, pr->M));
    if (pr->H < 1 || pr->H > UBQP_MAX_H)
        return ubqp_fail(ctx, UBQP_EINVAL, "H=%d outside [1, %d]", pr->H, UBQP_MAX_H);
    if (pr->lam_den < 1 || pr->lam_num < 0 || pr->lam_num > pr->lam_den)
        return ubqp_fail(ctx, UBQP_EINVAL, "lambda=%d/%d outside [0, 1]", pr->lam_num, pr->lam_den);
    if (pr->G < 1) return ubqp_fail(ctx, UBQP_EINVAL, "G < 1");
    if (pr->max_flips < 0) return ubqp_fail(ctx, UBQP_EINVAL, "max_flips < 0");
    const uint32_t known = UBQP_DERIV_START | UBQP_TIMING | UBQP_NO_GRAPH | UBQP_AUTOTUNE | UBQP_BLEND;
    if (pr->flags & ~known) return ubqp_fail(ctx, UBQP_EINVAL, "unknown flags 0x%x", pr->flags & ~known);
    return UBQP_OK;
}

static void ctx_free(ubqp_ctx *ctx)
{
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < ubqp_ctx::WS_COUNT; i++)
        if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
    (void)hipFree(ctx->err_flag);
    delete ctx;
}

void ubqp_ctx_hold(ubqp_ctx *ctx) { ctx->hold.fetch_add(2); }

void ubqp_ctx_drop(ubqp_ctx *ctx)
{
    if (ctx->hold.fetch_sub(2) == 3) ctx_free(ctx);  // the last holder of a released context
}

extern "C" {

int ubqp_create(ubqp_ctx **out, int device, void *stream)
{
    if (!out) return UBQP_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return UBQP_EDEVICE;
    ubqp_ctx *ctx = new (std::nothrow) ubqp_ctx();
    if (!ctx) return UBQP_ENOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    if (hipSetDevice(device) != hipSuccess || hipMalloc(&ctx->err_flag, 256) != hipSuccess) {
        delete ctx;
        return UBQP_EDEVICE;
    }
    hipLaunchKernelGGL(zero_i32, dim3(1), dim3(1), 0, ctx->stream, ctx->err_flag);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess || ubqp_screen_scratch_init(ctx) != UBQP_OK) {
        (void)hipFree(ctx->err_flag);
        delete ctx;
        return UBQP_EDEVICE;
    }
    *out = ctx;
    return UBQP_OK;
}

int ubqp_set_stream(ubqp_ctx *ctx, void *stream)
{
    if (!ctx) return UBQP_EINVAL;
    ctx->stream = (hipStream_t)stream;
    return UBQP_OK;
}

int ubqp_destroy(ubqp_ctx *ctx)
{
    if (!ctx) return UBQP_EINVAL;
    const int64_t old = ctx->hold.fetch_or(1);
    if (old & 1) return UBQP_EINVAL;  // released before
    if (old == 0) ctx_free(ctx);      // else the last problem, run, batch or server frees it
    return UBQP_OK;
}

const char *ubqp_last_error(const ubqp_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ubqp_sync(ubqp_ctx *ctx)
{
    if (!ctx) return UBQP_EINVAL;
    UBQP_TRY(ubqp_set_device(ctx));
    UBQP_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return ubqp_check_flag(ctx);
}

int ubqp_diversify(ubqp_ctx *ctx, int32_t n, const uint64_t *seeds_d, int64_t S, int32_t H, uint64_t *X_d,
                   int64_t M)
{
    if (!ctx || !seeds_d || !X_d) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    UBQP_TRY(check_words(ctx, n, M));
    if (H < 1 || H > UBQP_MAX_H) return ubqp_fail(ctx, UBQP_EINVAL, "H=%d outside [1, %d]", H, UBQP_MAX_H);
    if (S < 1 || M > 2 * (int64_t)H * S) return ubqp_fail(ctx, UBQP_EINVAL, "M=%lld exceeds 2 H S", (long long)M);
    UBQP_TRY(ubqp_set_device(ctx));
    DivArgs a{};
    a.seeds = seeds_d;
    a.n = n;
    a.W = (n + 63) / 64;
    a.H = H;
    a.X = X_d;
    a.total = M * a.W;
    UBQP_HIP_TRY(ctx, ubqp_launch_diversify(ctx->stream, a));
    return UBQP_OK;
}

int ubqp_blend(ubqp_ctx *ctx, int32_t n, const uint64_t *seeds_d, int64_t S, int64_t M, int64_t g,
               uint64_t run_seed, uint64_t *X_d)
{
    if (!ctx || !seeds_d || !X_d) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    UBQP_TRY(check_words(ctx, n, M));
    if (S < 1) return ubqp_fail(ctx, UBQP_EINVAL, "S < 1");
    if (g < 0 || g > INT32_MAX) return ubqp_fail(ctx, UBQP_EINVAL, "g=%lld outside [0, 2^31)", (long long)g);
    UBQP_TRY(ubqp_set_device(ctx));
    DivArgs a{};
    a.seeds = seeds_d;
    a.n = n;
    a.W = (n + 63) / 64;
    a.H = 1;
    a.X = X_d;
    a.total = M * a.W;
    a.blend = 1;
    a.M = M;
    a.S = S;
    a.run_seed = run_seed;
    a.scal = nullptr;
    a.g = g;
    UBQP_HIP_TRY(ctx, ubqp_launch_diversify(ctx->stream, a));
    return UBQP_OK;
}

int ubqp_eval(ubqp_ctx *ctx, const ubqp_problem *p, const uint64_t *X_d, int64_t M, int64_t *f_d)
{
    if (!ctx || !p || !X_d || !f_d) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    UBQP_TRY(check_words(ctx, p->n, M));
    UBQP_TRY(ubqp_set_device(ctx));
    UBQP_HIP_TRY(ctx, ubqp_launch_eval_v(ctx->stream, ubqp_eval_args(p, X_d, M, f_d), ubqp_eval_variant_for(p, M)));
    return UBQP_OK;
}

int ubqp_screen(ubqp_ctx *ctx, const int64_t *f_d, int64_t M, int32_t lam_num, int32_t lam_den, int32_t *pass_idx_d,
                int64_t *n_pass_d, int64_t *sum_max_d)
{
    if (!ctx || !f_d || !pass_idx_d || !n_pass_d || !sum_max_d) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    if (M < 1 || M > UBQP_MAX_M) return ubqp_fail(ctx, UBQP_EINVAL, "M=%lld out of range", (long long)M);
    if (lam_den < 1 || lam_num < 0 || lam_num > lam_den)
        return ubqp_fail(ctx, UBQP_EINVAL, "lambda=%d/%d outside [0, 1]", lam_num, lam_den);
    UBQP_TRY(ubqp_set_device(ctx));
    void *part;
    UBQP_TRY(ubqp_ws_ensure(ctx, ubqp_ctx::WS_PARTIALS, ubqp_screen_partials_bytes(M), &part));
    UBQP_HIP_TRY(ctx, ubqp_launch_screen(ctx->stream, ubqp_screen_args(f_d, M, lam_num, lam_den, pass_idx_d, n_pass_d,
                                                                       sum_max_d, part)));
    return UBQP_OK;
}

int ubqp_ascent(ubqp_ctx *ctx, const ubqp_problem *p, uint64_t *X_d, int64_t M, const int32_t *idx_d,
                const int64_t *n_idx_d, int64_t max_idx, int64_t *f_d, int32_t max_flips, int32_t *flips_d)
{
    if (!ctx || !p || !X_d || !idx_d || !n_idx_d || !f_d || !flips_d)
        return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    if (max_idx < 1 || max_idx > UBQP_MAX_M)
        return ubqp_fail(ctx, UBQP_EINVAL, "max_idx=%lld out of range", (long long)max_idx);
    if (max_flips < 0) return ubqp_fail(ctx, UBQP_EINVAL, "max_flips < 0");
    if (M < 1 || M > UBQP_MAX_M) return ubqp_fail(ctx, UBQP_EINVAL, "M=%lld out of range", (long long)M);
    UBQP_TRY(ubqp_set_device(ctx));
    // Delta initialisation then ascent, in chunks of at most UBQP_ASCENT_CHUNK list
    // entries through the workspace Y; the list length is a device value, so every
    // chunk that could hold entries is queued and chunks past the end exit at once.
    const int64_t cap = max_idx < UBQP_ASCENT_CHUNK ? max_idx : UBQP_ASCENT_CHUNK;
    void *Y;
    UBQP_TRY(ubqp_ws_ensure(ctx, ubqp_ctx::WS_Y, (size_t)p->planes * cap * p->n_pad * sizeof(int32_t), &Y));
    for (int64_t off = 0; off < max_idx; off += cap) {
        const int64_t c = max_idx - off < cap ? max_idx - off : cap;
        EvalArgs yr = ubqp_yrows_args(p, X_d, M, idx_d, n_idx_d, off, c, (int32_t *)Y);
        AscArgs as = ubqp_ascent_args(p, X_d, M, idx_d, n_idx_d, off, c, (const int32_t *)Y, f_d, max_flips, flips_d,
                                      ctx->err_flag);
        ubqp_split_dinit(yr, as, UBQP_SPLIT_TARGET);
        UBQP_HIP_TRY(ctx, ubqp_launch_yrows(ctx->stream, yr));
        UBQP_HIP_TRY(ctx, ubqp_launch_ascent(ctx->stream, as));
    }
    return UBQP_OK;
}

}  // extern "C"
