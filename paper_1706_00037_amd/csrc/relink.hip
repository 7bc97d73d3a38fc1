// Path relinking of pairs of elite solutions, then the steepest ascent from
// each path's best intermediate (the improvement phase the paper names to
// follow its initial phase; greedy relinking, the rule stated in the header).
//
// Per chunk of at most UBQP_ASCENT_CHUNK paths: copy each path's initiating
// solution into its output row, evaluate those rows (matrix-core row dot),
// initialise their deltas (keys or Y rows, as for the ascent), walk every path
// (one wave each, relink_kernel), list the paths that have an intermediate, and
// ascend those rows in place.
#include "ubqp_internal.h"

namespace {

constexpr int THR = 256;

// Output rows = the initiating solutions; the identity list of the chunk.
__global__ __launch_bounds__(THR) void rl_setup(const uint64_t *elite, int64_t E, const int32_t *pairs, int64_t P,
                                                int32_t W, uint64_t *X, int32_t *list, int64_t *count,
                                                int32_t *err)
{
    const int64_t id = (int64_t)blockIdx.x * THR + threadIdx.x;
    if (id == 0) *count = P;
    if (id < P) list[id] = (int32_t)id;
    if (id >= P * W) return;
    const int64_t p = id / W;
    const int32_t w = (int32_t)(id - p * W);
    const int64_t ii = pairs[2 * p];
    uint64_t v = 0;
    if (ii >= 0 && ii < E) v = elite[ii * W + w];
    else if (w == 0) atomicOr(err, 2);
    X[id] = v;
}

// The paths with an intermediate, in order (one block).
__global__ __launch_bounds__(THR) void rl_list(const int32_t *steps, int64_t P, int32_t *list, int64_t *count)
{
    __shared__ int32_t wtot[THR / 64];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t base = 0; base < P; base += THR) {
        const int64_t p = base + threadIdx.x;
        const int mine = (p < P && steps[p] > 0) ? 1 : 0;
        int incl = mine;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wtot[wv] = incl;
        __syncthreads();
        int64_t pos = carry + incl - mine, total = 0;
        for (int i = 0; i < THR / 64; i++) {
            if (i < wv) pos += wtot[i];
            total += wtot[i];
        }
        if (mine) list[pos] = (int32_t)p;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

}  // namespace

extern "C" int ubqp_relink(ubqp_ctx *ctx, const ubqp_problem *p, const uint64_t *elite_d, int64_t E,
                           const int32_t *pairs_d, int64_t P, int32_t max_flips, uint64_t *X_out_d,
                           int64_t *f_mid_d, int64_t *f_out_d, int32_t *steps_d)
{
    if (!ctx || !p || !elite_d || !pairs_d || !X_out_d || !f_mid_d || !f_out_d || !steps_d)
        return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    if (E < 1 || E > UBQP_MAX_M) return ubqp_fail(ctx, UBQP_EINVAL, "E=%lld out of range", (long long)E);
    if (P < 1 || P > UBQP_MAX_M) return ubqp_fail(ctx, UBQP_EINVAL, "P=%lld out of range", (long long)P);
    if (max_flips < 0) return ubqp_fail(ctx, UBQP_EINVAL, "max_flips < 0");
    UBQP_TRY(ubqp_set_device(ctx));
    const int64_t C = P < UBQP_ASCENT_CHUNK ? P : UBQP_ASCENT_CHUNK;
    const int64_t W = p->W;
    void *Y = nullptr, *stage = nullptr;
    UBQP_TRY(ubqp_ws_ensure(ctx, ubqp_ctx::WS_Y, (size_t)p->planes * C * p->n_pad * sizeof(int32_t), &Y));
    // list (C int32), count (int64), flips (C int32), f0 (C int64)
    const size_t o_list = 0, o_cnt = ((size_t)C * 4 + 255) & ~(size_t)255, o_fl = o_cnt + 256,
                 o_f0 = o_fl + (((size_t)C * 4 + 255) & ~(size_t)255);
    UBQP_TRY(ubqp_ws_ensure(ctx, ubqp_ctx::WS_RELINK, o_f0 + (size_t)C * 8, &stage));
    int32_t *list = (int32_t *)((char *)stage + o_list);
    int64_t *count = (int64_t *)((char *)stage + o_cnt);
    int32_t *flips = (int32_t *)((char *)stage + o_fl);
    int64_t *f0 = (int64_t *)((char *)stage + o_f0);
    hipStream_t st = ctx->stream;
    for (int64_t off = 0; off < P; off += C) {
        const int64_t c = P - off < C ? P - off : C;
        uint64_t *X = X_out_d + off * W;
        const int32_t *pr = pairs_d + 2 * off;
        hipLaunchKernelGGL(rl_setup, dim3((unsigned)((c * W + THR - 1) / THR)), dim3(THR), 0, st, elite_d, E, pr, c,
                           (int32_t)W, X, list, count, ctx->err_flag);
        UBQP_HIP_TRY(ctx, hipGetLastError());
        UBQP_HIP_TRY(ctx, ubqp_launch_eval_v(st, ubqp_eval_args(p, X, c, f0), ubqp_eval_variant_for(p, c)));
        UBQP_HIP_TRY(ctx, ubqp_launch_yrows(st, ubqp_yrows_args(p, X, c, list, count, 0, c, (int32_t *)Y)));
        UBQP_HIP_TRY(ctx, ubqp_launch_relink(st, ubqp_relink_args(p, elite_d, E, pr, c, X, (const int32_t *)Y, f0,
                                                                  f_mid_d + off, f_out_d + off, steps_d + off,
                                                                  ctx->err_flag)));
        hipLaunchKernelGGL(rl_list, dim3(1), dim3(THR), 0, st, steps_d + off, c, list, count);
        UBQP_HIP_TRY(ctx, hipGetLastError());
        EvalArgs yr = ubqp_yrows_args(p, X, c, list, count, 0, c, (int32_t *)Y);
        AscArgs as = ubqp_ascent_args(p, X, c, list, count, 0, c, (const int32_t *)Y, f_out_d + off, max_flips,
                                      flips, ctx->err_flag);
        ubqp_split_dinit(yr, as, UBQP_SPLIT_TARGET);
        UBQP_HIP_TRY(ctx, ubqp_launch_yrows(st, yr));
        UBQP_HIP_TRY(ctx, ubqp_launch_ascent(st, as));
    }
    return UBQP_OK;
}
