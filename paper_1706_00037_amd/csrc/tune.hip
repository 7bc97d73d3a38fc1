// Autotuner of the batched objective's matrix-core tiling.
//
// The contraction Y = X Q has six variants (eval_mfma.hip): K staged 64, 128 or
// 256 deep per LDS step (two, two or one workgroups per CU) times two tile
// orders (n-tile-major: neighbouring workgroups share a Q column
// block in L2; m-tile-major: they share an X row block).  Which is fastest depends on n_pad,
// the number of candidates and the number of planes, so the tuner times every
// variant once per key (planes, n_pad, M rounded up to a power of two) on the
// problem itself and keeps the fastest for the process.  All variants compute
// the same exact integers; only the time differs.  Launch tables consult the
// cache, so a batch groups its instances by their variant.
#include <map>
#include <mutex>
#include <tuple>

#include "ubqp_internal.h"

namespace {

struct Tuned {
    int variant;
    double ms[UBQP_EVAL_VARIANTS];
};

std::mutex g_tune_m;
std::map<std::tuple<int, int, int64_t>, Tuned> g_tuned;

int64_t m_bucket(int64_t M)
{
    int64_t b = 256;
    while (b < M) b <<= 1;
    return b;
}

std::tuple<int, int, int64_t> key_of(const ubqp_problem *p, int64_t M) { return {p->planes, p->n_pad, m_bucket(M)}; }

// Candidate rows for timing: a fixed hash of (row, word), bits >= n cleared.
__global__ __launch_bounds__(256) void fill_rows(uint64_t *X, int64_t M, int32_t W, int32_t n)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= M * W) return;
    uint64_t z = (uint64_t)k * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 31)) * 0xD6E8FEB86659FD93ull;
    z ^= z >> 32;
    const int w = (int)(k % W);
    const int rem = n - 64 * w;
    if (rem < 64) z &= (1ull << rem) - 1;
    X[k] = z;
}

}  // namespace

int ubqp_eval_variant_for(const ubqp_problem *p, int64_t M)
{
    std::lock_guard<std::mutex> lk(g_tune_m);
    auto it = g_tuned.find(key_of(p, M));
    return it == g_tuned.end() ? UBQP_EVAL_DEFAULT_VARIANT : it->second.variant;
}

int ubqp_tune_eval_internal(ubqp_ctx *ctx, const ubqp_problem *p, int64_t M, int32_t *variant, double *ms)
{
    const auto key = key_of(p, M);
    {
        std::lock_guard<std::mutex> lk(g_tune_m);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            if (variant) *variant = it->second.variant;
            if (ms)
                for (int v = 0; v < UBQP_EVAL_VARIANTS; v++) ms[v] = it->second.ms[v];
            return UBQP_OK;
        }
    }
    UBQP_TRY(ubqp_set_device(ctx));
    hipStream_t st = ctx->stream;
    const int64_t Mt = std::get<2>(key);  // time the bucket's size
    const size_t xb = (size_t)(Mt * p->W * 8 + 255) / 256 * 256;
    void *ws = nullptr;
    UBQP_TRY(ubqp_ws_ensure(ctx, ubqp_ctx::WS_TUNE, xb + (size_t)Mt * 8, &ws));
    uint64_t *X = (uint64_t *)ws;
    int64_t *f = (int64_t *)((char *)ws + xb);
    hipLaunchKernelGGL(fill_rows, dim3((unsigned)((Mt * p->W + 255) / 256)), dim3(256), 0, st, X, Mt, p->W, p->n);
    UBQP_HIP_TRY(ctx, hipGetLastError());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    UBQP_HIP_TRY(ctx, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    Tuned t{};
    t.variant = UBQP_EVAL_DEFAULT_VARIANT;
    double best = 1e30;
    const EvalArgs a = ubqp_eval_args(p, X, Mt, f);
    for (int v = 0; e == hipSuccess && v < UBQP_EVAL_VARIANTS; v++) {
        e = ubqp_launch_eval_v(st, a, v);  // warm-up
        double vbest = 1e30;
        for (int r = 0; e == hipSuccess && r < 3; r++) {
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = ubqp_launch_eval_v(st, a, v);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float msr = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&msr, e0, e1);
            if (e == hipSuccess && msr < vbest) vbest = msr;
        }
        t.ms[v] = vbest;
        if (vbest < best) {
            best = vbest;
            t.variant = v;
        }
    }
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return ubqp_hip_fail(ctx, e, "eval autotuning");
    {
        std::lock_guard<std::mutex> lk(g_tune_m);
        g_tuned[key] = t;
    }
    if (variant) *variant = t.variant;
    if (ms)
        for (int v = 0; v < UBQP_EVAL_VARIANTS; v++) ms[v] = t.ms[v];
    return UBQP_OK;
}

extern "C" {

int ubqp_tune_eval(ubqp_ctx *ctx, const ubqp_problem *prob, int64_t M, int32_t *variant, double *ms_host)
{
    if (!ctx || !prob) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    if (M < 1 || M > UBQP_MAX_M) return ubqp_fail(ctx, UBQP_EINVAL, "M=%lld out of range", (long long)M);
    return ubqp_tune_eval_internal(ctx, prob, M, variant, ms_host);
}

int ubqp_eval_variant(ubqp_ctx *ctx, const ubqp_problem *prob, const uint64_t *X_d, int64_t M, int64_t *f_d,
                      int32_t variant)
{
    if (!ctx || !prob || !X_d || !f_d) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    if (M < 1 || M > UBQP_MAX_M) return ubqp_fail(ctx, UBQP_EINVAL, "M=%lld out of range", (long long)M);
    if (variant < 0 || variant >= UBQP_EVAL_VARIANTS)
        return ubqp_fail(ctx, UBQP_EINVAL, "variant %d outside [0, %d)", variant, UBQP_EVAL_VARIANTS);
    UBQP_TRY(ubqp_set_device(ctx));
    UBQP_HIP_TRY(ctx, ubqp_launch_eval_v(ctx->stream, ubqp_eval_args(prob, X_d, M, f_d), variant));
    return UBQP_OK;
}

}  // extern "C"
