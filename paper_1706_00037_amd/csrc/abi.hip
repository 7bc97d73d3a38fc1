// C ABI of libubqp: argument checks, resident problem upload, device workspace,
// and the generation loop of the multi-start method (Fig. 2), which issues
// every step on the context's stream without a host synchronisation inside.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "ubqp_internal.h"

namespace {

int fail(ubqp_ctx *ctx, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(ubqp_ctx *ctx, int code, const char *fmt, ...)
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

int hip_fail(ubqp_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? UBQP_ENOMEM : UBQP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                        \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);  \
    } while (0)

// Make ctx->ws[slot] hold at least `bytes`.
int ws_ensure(ubqp_ctx *ctx, int slot, size_t bytes, void **out)
{
    if (bytes == 0) bytes = 256;
    if (ctx->ws_bytes[slot] < bytes) {
        if (ctx->ws[slot]) {
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            HIP_TRY(ctx, hipFree(ctx->ws[slot]));
            ctx->ws[slot] = nullptr;
            ctx->ws_bytes[slot] = 0;
        }
        HIP_TRY(ctx, hipMalloc(&ctx->ws[slot], bytes));
        ctx->ws_bytes[slot] = bytes;
    }
    *out = ctx->ws[slot];
    return UBQP_OK;
}

#define TRY(expr)                      \
    do {                               \
        int r_ = (expr);               \
        if (r_ != UBQP_OK) return r_;  \
    } while (0)

int set_device(ubqp_ctx *ctx)
{
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    return UBQP_OK;
}

__global__ void zero_i32(int32_t *p) { *p = 0; }

// Read and clear the kernel-side error flag (synchronises the stream).
int check_flag(ubqp_ctx *ctx)
{
    int32_t v = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&v, ctx->err_flag, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (v) {
        hipLaunchKernelGGL(zero_i32, dim3(1), dim3(1), 0, ctx->stream, ctx->err_flag);
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        return fail(ctx, UBQP_EDEVICE, "%s", (v & 2) ? "ascent skipped a candidate index outside [0, M)"
                                                     : "ascent exceeded its safety bound of flips");
    }
    return UBQP_OK;
}

int check_words(ubqp_ctx *ctx, int32_t n, int64_t M)
{
    if (n < 1 || n > UBQP_MAX_N) return fail(ctx, UBQP_EINVAL, "n=%d outside [1, %d]", n, UBQP_MAX_N);
    if (M < 1 || M > UBQP_MAX_M) return fail(ctx, UBQP_EINVAL, "M=%lld outside [1, %lld]", (long long)M,
                                             (long long)UBQP_MAX_M);
    return UBQP_OK;
}

// Delta initialisation (Y = X Q on the listed rows) followed by the ascent, in
// chunks of `cap` list entries through the workspace Y ([planes][cap][n_pad]).
// The list length is a device value, so every chunk that could hold entries is
// queued; chunks past the end exit at once.
int queue_ascent(ubqp_ctx *ctx, const ubqp_problem *p, uint64_t *X, int64_t M, const int32_t *idx,
                 const int64_t *nidx_d, int64_t max_idx, int64_t *f, int32_t max_flips, int32_t *flips, int32_t *Y,
                 int64_t cap)
{
    for (int64_t off = 0; off < max_idx; off += cap) {
        const int64_t c = max_idx - off < cap ? max_idx - off : cap;
        HIP_TRY(ctx, ubqp_launch_yrows(ctx->stream, p, X, M, idx, nidx_d, off, c, Y));
        HIP_TRY(ctx, ubqp_launch_ascent(ctx->stream, p, X, M, idx, nidx_d, off, c, Y, f, max_flips, flips,
                                        ctx->err_flag));
    }
    return UBQP_OK;
}

int check_params(ubqp_ctx *ctx, const ubqp_problem *p, const ubqp_params *pr)
{
    TRY(check_words(ctx, p->n, pr->M));
    if (pr->H < 1 || pr->H > UBQP_MAX_H) return fail(ctx, UBQP_EINVAL, "H=%d outside [1, %d]", pr->H, UBQP_MAX_H);
    if (pr->lam_den < 1 || pr->lam_num < 0 || pr->lam_num > pr->lam_den)
        return fail(ctx, UBQP_EINVAL, "lambda=%d/%d outside [0, 1]", pr->lam_num, pr->lam_den);
    if (pr->G < 1) return fail(ctx, UBQP_EINVAL, "G < 1");
    if (pr->max_flips < 0) return fail(ctx, UBQP_EINVAL, "max_flips < 0");
    return UBQP_OK;
}

// Layout of a run's single device allocation.
struct RunLayout {
    size_t seeds, X, f, flips, idx, scal, bestx, stats, part, Y, total;
    int64_t S, cap;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

RunLayout run_layout(const ubqp_problem *p, const ubqp_params *pr)
{
    RunLayout L{};
    const int64_t M = pr->M, W = p->W;
    L.S = (M + 2 * pr->H - 1) / (2 * pr->H);
    L.cap = M < UBQP_ASCENT_CHUNK ? M : UBQP_ASCENT_CHUNK;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    L.seeds = take((size_t)(L.S * W * 8));
    L.X = take((size_t)(M * W * 8));
    L.f = take((size_t)M * 8);
    L.flips = take((size_t)M * 4);
    L.idx = take((size_t)M * 4);
    L.scal = take(sizeof(ubqp_scal));
    L.bestx = take((size_t)W * 8);
    L.stats = take((size_t)pr->G * 5 * 8);
    L.part = take(ubqp_screen_partials_bytes(M));
    L.Y = take((size_t)p->planes * L.cap * p->n_pad * 4);
    L.total = off;
    return L;
}

}  // namespace

struct ubqp_run {
    ubqp_ctx *ctx = nullptr;
    const ubqp_problem *prob = nullptr;
    ubqp_params pr{};
    RunLayout L{};
    char *mem = nullptr;
    int64_t *f_dump = nullptr;
    int32_t g = 0;
    hipEvent_t ev0 = nullptr;
    std::vector<hipEvent_t> ev;     // end of each generation
    std::vector<hipEvent_t> phase;  // UBQP_TIMING: G x (UBQP_PHASES + 1) phase boundaries
    template <typename T> T *at(size_t off) const { return (T *)(mem + off); }
};

extern "C" {}  // namespace

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
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
        hipFree(ctx->err_flag);
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
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < ubqp_ctx::WS_COUNT; i++)
        if (ctx->ws[i]) hipFree(ctx->ws[i]);
    hipFree(ctx->err_flag);
    delete ctx;
    return UBQP_OK;
}

const char *ubqp_last_error(const ubqp_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ubqp_sync(ubqp_ctx *ctx)
{
    if (!ctx) return UBQP_EINVAL;
    TRY(set_device(ctx));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return check_flag(ctx);
}

int ubqp_problem_create(ubqp_ctx *ctx, int32_t n, const int32_t *q, ubqp_problem **out)
{
    if (!ctx || !q || !out) return fail(ctx, UBQP_EINVAL, "null argument");
    *out = nullptr;
    if (n < 1 || n > UBQP_MAX_N) return fail(ctx, UBQP_EINVAL, "n=%d outside [1, %d]", n, UBQP_MAX_N);
    bool narrow = true;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < n; j++) {
            const int32_t v = q[i * n + j];
            if (v < -32768 || v > 32767)
                return fail(ctx, UBQP_ERANGE, "q[%lld][%lld]=%d outside [-32768, 32767]", (long long)i, (long long)j, v);
            if (j > i && v != q[j * n + i])
                return fail(ctx, UBQP_EASYM, "q[%lld][%lld]=%d != q[%lld][%lld]=%d", (long long)i, (long long)j, v,
                            (long long)j, (long long)i, q[j * n + i]);
            if (v < -128 || v > 127) narrow = false;
        }
    TRY(set_device(ctx));
    ubqp_problem *p = new (std::nothrow) ubqp_problem();
    if (!p) return fail(ctx, UBQP_ENOMEM, "host allocation");
    p->ctx = ctx;
    p->n = n;
    p->n_pad = (n + UBQP_NPAD_ALIGN - 1) / UBQP_NPAD_ALIGN * UBQP_NPAD_ALIGN;
    p->W = (n + 63) / 64;
    p->planes = narrow ? 1 : 2;
    p->weight0 = narrow ? 1 : 256;
    p->bias = narrow ? 0 : 128;
    const int64_t np = p->n_pad, NN = np * np;
    std::vector<int8_t> planes((size_t)(p->planes * NN), 0);
    std::vector<int32_t> diag((size_t)np, 0);
    std::vector<uint64_t> dx((size_t)p->W, 0);
    p->ncol_a = narrow ? (int32_t)((np + 1023) / 1024 * 1024) : (int32_t)np;
    const int64_t nca = p->ncol_a;
    const size_t qa_elem = narrow ? 1 : 2;
    std::vector<uint8_t> qa((size_t)(np * nca) * qa_elem, 0);
    for (int64_t i = 0; i < n; i++) {
        int64_t rs = 0;
        for (int64_t j = 0; j < n; j++) {
            const int32_t v = q[i * n + j];
            rs += v;
            if (narrow) {
                planes[i * np + j] = (int8_t)v;
                if (i != j) ((int8_t *)qa.data())[i * nca + j] = (int8_t)v;
            } else {
                planes[i * np + j] = (int8_t)(v >> 8);                    // hi, in [-128, 127]
                planes[NN + i * np + j] = (int8_t)((v & 255) - 128);      // lo, in [-128, 127]
                if (i != j) ((int16_t *)qa.data())[i * np + j] = (int16_t)v;
            }
        }
        diag[i] = q[i * n + i];
        if (rs > 0) dx[i >> 6] |= 1ull << (i & 63);
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&p->q, planes.size());
    if (e == hipSuccess) e = hipMalloc(&p->qa, qa.size());
    if (e == hipSuccess) e = hipMalloc(&p->diag, diag.size() * 4);
    if (e == hipSuccess) e = hipMalloc(&p->deriv_x, dx.size() * 8);
    if (e == hipSuccess) e = hipMemcpy(p->q, planes.data(), planes.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->qa, qa.data(), qa.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->diag, diag.data(), diag.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->deriv_x, dx.data(), dx.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ubqp_problem_destroy(p);
        return hip_fail(ctx, e, "problem upload");
    }
    *out = p;
    return UBQP_OK;
}

int ubqp_problem_destroy(ubqp_problem *p)
{
    if (!p) return UBQP_EINVAL;
    hipSetDevice(p->ctx->device);
    hipStreamSynchronize(p->ctx->stream);
    if (p->q) hipFree(p->q);
    if (p->qa) hipFree(p->qa);
    if (p->diag) hipFree(p->diag);
    if (p->deriv_x) hipFree(p->deriv_x);
    delete p;
    return UBQP_OK;
}

int ubqp_problem_info(const ubqp_problem *p, int32_t *n, int32_t *n_pad, int32_t *planes)
{
    if (!p) return UBQP_EINVAL;
    if (n) *n = p->n;
    if (n_pad) *n_pad = p->n_pad;
    if (planes) *planes = p->planes;
    return UBQP_OK;
}

int ubqp_diversify(ubqp_ctx *ctx, int32_t n, const uint64_t *seeds_d, int64_t S, int32_t H, uint64_t *X_d,
                   int64_t M)
{
    if (!ctx || !seeds_d || !X_d) return fail(ctx, UBQP_EINVAL, "null argument");
    TRY(check_words(ctx, n, M));
    if (H < 1 || H > UBQP_MAX_H) return fail(ctx, UBQP_EINVAL, "H=%d outside [1, %d]", H, UBQP_MAX_H);
    if (S < 1 || M > 2 * (int64_t)H * S) return fail(ctx, UBQP_EINVAL, "M=%lld exceeds 2 H S", (long long)M);
    TRY(set_device(ctx));
    HIP_TRY(ctx, ubqp_launch_diversify(ctx->stream, n, seeds_d, S, H, X_d, M));
    return UBQP_OK;
}

int ubqp_eval(ubqp_ctx *ctx, const ubqp_problem *p, const uint64_t *X_d, int64_t M, int64_t *f_d)
{
    if (!ctx || !p || !X_d || !f_d) return fail(ctx, UBQP_EINVAL, "null argument");
    TRY(check_words(ctx, p->n, M));
    TRY(set_device(ctx));
    HIP_TRY(ctx, ubqp_launch_eval(ctx->stream, p, X_d, M, f_d));
    return UBQP_OK;
}

int ubqp_screen(ubqp_ctx *ctx, const int64_t *f_d, int64_t M, int32_t lam_num, int32_t lam_den,
                int32_t *pass_idx_d, int64_t *n_pass_d, int64_t *sum_max_d)
{
    if (!ctx || !f_d || !pass_idx_d || !n_pass_d || !sum_max_d) return fail(ctx, UBQP_EINVAL, "null argument");
    if (M < 1 || M > UBQP_MAX_M) return fail(ctx, UBQP_EINVAL, "M=%lld out of range", (long long)M);
    if (lam_den < 1 || lam_num < 0 || lam_num > lam_den)
        return fail(ctx, UBQP_EINVAL, "lambda=%d/%d outside [0, 1]", lam_num, lam_den);
    TRY(set_device(ctx));
    void *part;
    TRY(ws_ensure(ctx, ubqp_ctx::WS_PARTIALS, ubqp_screen_partials_bytes(M), &part));
    HIP_TRY(ctx, ubqp_launch_screen(ctx->stream, f_d, M, lam_num, lam_den, pass_idx_d, n_pass_d, sum_max_d, part));
    return UBQP_OK;
}

int ubqp_ascent(ubqp_ctx *ctx, const ubqp_problem *p, uint64_t *X_d, int64_t M, const int32_t *idx_d,
                const int64_t *n_idx_d, int64_t max_idx, int64_t *f_d, int32_t max_flips, int32_t *flips_d)
{
    if (!ctx || !p || !X_d || !idx_d || !n_idx_d || !f_d || !flips_d) return fail(ctx, UBQP_EINVAL, "null argument");
    if (max_idx < 1 || max_idx > UBQP_MAX_M) return fail(ctx, UBQP_EINVAL, "max_idx=%lld out of range",
                                                         (long long)max_idx);
    if (max_flips < 0) return fail(ctx, UBQP_EINVAL, "max_flips < 0");
    if (M < 1 || M > UBQP_MAX_M) return fail(ctx, UBQP_EINVAL, "M=%lld out of range", (long long)M);
    TRY(set_device(ctx));
    const int64_t cap = max_idx < UBQP_ASCENT_CHUNK ? max_idx : UBQP_ASCENT_CHUNK;
    void *Y;
    TRY(ws_ensure(ctx, ubqp_ctx::WS_Y, (size_t)p->planes * cap * p->n_pad * sizeof(int32_t), &Y));
    return queue_ascent(ctx, p, X_d, M, idx_d, n_idx_d, max_idx, f_d, max_flips, flips_d, (int32_t *)Y, cap);
}

int64_t ubqp_run_footprint(const ubqp_problem *p, const ubqp_params *pr)
{
    if (!p || !pr || pr->M < 1 || pr->H < 1 || pr->G < 1) return -1;
    return (int64_t)run_layout(p, pr).total;
}

int ubqp_run_create(ubqp_ctx *ctx, const ubqp_problem *p, const ubqp_params *pr, int64_t *f_dump_d, ubqp_run **out)
{
    if (!ctx || !p || !pr || !out) return fail(ctx, UBQP_EINVAL, "null argument");
    *out = nullptr;
    TRY(check_params(ctx, p, pr));
    TRY(set_device(ctx));
    ubqp_run *r = new (std::nothrow) ubqp_run();
    if (!r) return fail(ctx, UBQP_ENOMEM, "host allocation");
    r->ctx = ctx;
    r->prob = p;
    r->pr = *pr;
    r->L = run_layout(p, pr);
    r->f_dump = f_dump_d;
    hipError_t e = hipMalloc(&r->mem, r->L.total);
    if (e == hipSuccess) e = hipEventCreate(&r->ev0);
    r->ev.assign((size_t)pr->G, nullptr);
    for (size_t i = 0; e == hipSuccess && i < r->ev.size(); i++) e = hipEventCreate(&r->ev[i]);
    if (pr->flags & UBQP_TIMING) r->phase.assign((size_t)pr->G * (UBQP_PHASES + 1), nullptr);
    for (size_t i = 0; e == hipSuccess && i < r->phase.size(); i++) e = hipEventCreate(&r->phase[i]);
    if (e == hipSuccess)
        e = ubqp_launch_seed_init(ctx->stream, r->at<uint64_t>(r->L.seeds), r->L.S, p->n, pr->run_seed,
                                  (pr->flags & UBQP_DERIV_START) ? p->deriv_x : nullptr, r->at<ubqp_scal>(r->L.scal));
    if (e == hipSuccess) e = hipEventRecord(r->ev0, ctx->stream);
    if (e != hipSuccess) {
        const int rc = hip_fail(ctx, e, "run setup");
        ubqp_run_destroy(r);
        return rc;
    }
    *out = r;
    return UBQP_OK;
}

int ubqp_run_step(ubqp_run *r, int32_t generations)
{
    if (!r) return UBQP_EINVAL;
    ubqp_ctx *ctx = r->ctx;
    if (generations < 0 || r->g + generations > r->pr.G)
        return fail(ctx, UBQP_EINVAL, "%d more generations exceed G=%d (done %d)", generations, r->pr.G, r->g);
    TRY(set_device(ctx));
    const ubqp_problem *p = r->prob;
    const ubqp_params &pr = r->pr;
    const RunLayout &L = r->L;
    const int64_t M = pr.M;
    hipStream_t st = ctx->stream;
    uint64_t *seeds = r->at<uint64_t>(L.seeds), *X = r->at<uint64_t>(L.X), *bestx = r->at<uint64_t>(L.bestx);
    int64_t *f = r->at<int64_t>(L.f), *stats = r->at<int64_t>(L.stats);
    int32_t *flips = r->at<int32_t>(L.flips), *idx = r->at<int32_t>(L.idx), *Y = r->at<int32_t>(L.Y);
    ubqp_scal *sc = r->at<ubqp_scal>(L.scal);
    const bool timing = !r->phase.empty();
    for (int32_t k = 0; k < generations; k++, r->g++) {
        const int32_t g = r->g;
        hipEvent_t *pe = timing ? &r->phase[(size_t)g * (UBQP_PHASES + 1)] : nullptr;
#define PHASE_MARK(i) \
    if (pe) HIP_TRY(ctx, hipEventRecord(pe[i], st))
        PHASE_MARK(0);
        HIP_TRY(ctx, ubqp_launch_diversify(st, p->n, seeds, L.S, pr.H, X, M));
        PHASE_MARK(1);
        HIP_TRY(ctx, ubqp_launch_eval(st, p, X, M, f));
        PHASE_MARK(2);
        if (r->f_dump)
            HIP_TRY(ctx, hipMemcpyAsync(r->f_dump + (int64_t)g * M, f, (size_t)M * 8, hipMemcpyDeviceToDevice, st));
        HIP_TRY(ctx, ubqp_launch_screen(st, f, M, pr.lam_num, pr.lam_den, idx, &sc->npass, sc->sum_max,
                                        r->at<void>(L.part)));
        PHASE_MARK(3);
        TRY(queue_ascent(ctx, p, X, M, idx, &sc->npass, M, f, pr.max_flips, flips, Y, L.cap));
        PHASE_MARK(4);
        HIP_TRY(ctx, ubqp_launch_select(st, p->n, M, L.S, g, pr.run_seed, X, f, flips, idx, sc, bestx, seeds, stats));
        PHASE_MARK(5);
#undef PHASE_MARK
        HIP_TRY(ctx, hipEventRecord(r->ev[(size_t)g], st));
    }
    return UBQP_OK;
}

int ubqp_run_result(ubqp_run *r, ubqp_result *res)
{
    if (!r || !res) return UBQP_EINVAL;
    ubqp_ctx *ctx = r->ctx;
    TRY(set_device(ctx));
    hipStream_t st = ctx->stream;
    ubqp_scal hs;
    HIP_TRY(ctx, hipMemcpyAsync(&hs, r->at<ubqp_scal>(r->L.scal), sizeof hs, hipMemcpyDeviceToHost, st));
    if (res->best_x_host)
        HIP_TRY(ctx, hipMemcpyAsync(res->best_x_host, r->at<uint64_t>(r->L.bestx), (size_t)r->prob->W * 8,
                                    hipMemcpyDeviceToHost, st));
    if (res->stats_host && r->g > 0)
        HIP_TRY(ctx, hipMemcpyAsync(res->stats_host, r->at<int64_t>(r->L.stats), (size_t)r->g * 5 * 8,
                                    hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    TRY(check_flag(ctx));
    if (res->gen_ms_host)
        for (int32_t g = 0; g < r->g; g++) {
            float ms = 0.f;
            HIP_TRY(ctx, hipEventElapsedTime(&ms, r->ev0, r->ev[(size_t)g]));
            res->gen_ms_host[g] = ms;
        }
    if (res->phase_ms_host && !r->phase.empty())
        for (int32_t g = 0; g < r->g; g++)
            for (int i = 0; i < UBQP_PHASES; i++) {
                float ms = 0.f;
                const size_t b = (size_t)g * (UBQP_PHASES + 1);
                HIP_TRY(ctx, hipEventElapsedTime(&ms, r->phase[b + i], r->phase[b + i + 1]));
                res->phase_ms_host[(size_t)g * UBQP_PHASES + i] = ms;
            }
    res->have_best = hs.have_best;
    res->best_f = hs.have_best ? hs.best_f : INT64_MIN;
    res->generations = r->g;
    return UBQP_OK;
}

int ubqp_run_destroy(ubqp_run *r)
{
    if (!r) return UBQP_EINVAL;
    hipSetDevice(r->ctx->device);
    hipStreamSynchronize(r->ctx->stream);
    for (hipEvent_t e : r->ev)
        if (e) hipEventDestroy(e);
    for (hipEvent_t e : r->phase)
        if (e) hipEventDestroy(e);
    if (r->ev0) hipEventDestroy(r->ev0);
    if (r->mem) hipFree(r->mem);
    delete r;
    return UBQP_OK;
}

int ubqp_multistart(ubqp_ctx *ctx, const ubqp_problem *p, const ubqp_params *pr, int64_t *f_dump_d, ubqp_result *res)
{
    if (!ctx || !p || !pr || !res) return fail(ctx, UBQP_EINVAL, "null argument");
    ubqp_run *r = nullptr;
    TRY(ubqp_run_create(ctx, p, pr, f_dump_d, &r));
    int rc = ubqp_run_step(r, pr->G);
    if (rc == UBQP_OK) rc = ubqp_run_result(r, res);
    ubqp_run_destroy(r);
    return rc;
}

}  // extern "C"
