// Exact T(lambda) screening (Pseudocode section): T = Mean + lambda (Max - Mean)
// over the generation's M objective values, pass iff f > T, decided in 128-bit
// integers as  den*M*f > (den - num)*Sum + num*M*Max  (lambda = num/den).
// Passer indices are compacted in ascending order.
//
// Three HBM-bound passes over f (8 B/candidate each): block partial Sum/Max,
// per-block passer counts, and an order-preserving scatter.  No atomics, so the
// output is the same on every run.
#include <mutex>

#include "ubqp_internal.h"

namespace {

constexpr int THR = 256;
constexpr int PER = 8;
constexpr int64_t CH = THR * PER;  // candidates per block

__device__ inline int64_t wave_sum(int64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline int64_t wave_max(int64_t v)
{
    for (int o = 32; o > 0; o >>= 1) {
        int64_t u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

// Block-wide sum and max; every thread gets the result.
__device__ void block_sum_max(int64_t &s, int64_t &m)
{
    __shared__ int64_t ss[THR / 64], sm[THR / 64];
    s = wave_sum(s);
    m = wave_max(m);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { ss[wv] = s; sm[wv] = m; }
    __syncthreads();
    s = ss[0];
    m = sm[0];
    for (int i = 1; i < THR / 64; i++) { s += ss[i]; m = sm[i] > m ? sm[i] : m; }
    __syncthreads();
}

__device__ inline bool passes(int64_t f, int64_t M, int32_t den, __int128 rhs) { return (__int128)den * M * f > rhs; }

__device__ void reduce_body(const ScreenArgs &a, int64_t bid)
{
    const int64_t base = bid * CH;
    int64_t s = 0, m = INT64_MIN;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const int64_t c = base + i * THR + threadIdx.x;
        if (c < a.M) { const int64_t v = a.f[c]; s += v; m = v > m ? v : m; }
    }
    block_sum_max(s, m);
    if (threadIdx.x == 0) { a.psum[bid] = s; a.pmax[bid] = m; }
}

// Sum and Max of the whole population from the block partials.
__device__ void total_sum_max(const ScreenArgs &a, int64_t &s, int64_t &m)
{
    s = 0;
    m = INT64_MIN;
    for (int b = threadIdx.x; b < a.nblk; b += THR) { s += a.psum[b]; m = a.pmax[b] > m ? a.pmax[b] : m; }
    block_sum_max(s, m);
}

__device__ void count_body(const ScreenArgs &a, int64_t bid)
{
    int64_t S, Mx;
    total_sum_max(a, S, Mx);
    const __int128 rhs = (__int128)(a.lam_den - a.lam_num) * S + (__int128)a.lam_num * a.M * Mx;
    const int64_t base = bid * CH;
    int64_t k = 0;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const int64_t c = base + i * THR + threadIdx.x;
        if (c < a.M && passes(a.f[c], a.M, a.lam_den, rhs)) k++;
    }
    int64_t dummy = 0;
    block_sum_max(k, dummy);
    if (threadIdx.x == 0) {
        a.cnt[bid] = k;
        if (bid == 0) { a.sum_max[0] = S; a.sum_max[1] = Mx; }
    }
}

__device__ void scatter_body(const ScreenArgs &a, int64_t bid)
{
    __shared__ int64_t wtot[THR / 64];
    // passers in earlier blocks
    int64_t off = 0, dummy = 0;
    for (int b = threadIdx.x; b < (int)bid; b += THR) off += a.cnt[b];
    block_sum_max(off, dummy);
    const __int128 rhs = (__int128)(a.lam_den - a.lam_num) * a.sum_max[0] + (__int128)a.lam_num * a.M * a.sum_max[1];
    // each thread owns PER consecutive candidates, so thread order is index order
    const int64_t c0 = bid * CH + (int64_t)threadIdx.x * PER;
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const int64_t c = c0 + i;
        if (c < a.M && passes(a.f[c], a.M, a.lam_den, rhs)) bits |= 1u << i;
    }
    const int mine = __popc(bits);
    // exclusive scan of `mine` over the block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = mine;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    int64_t pos = off + incl - mine;
    for (int i = 0; i < wv; i++) pos += wtot[i];
    for (int i = 0; i < PER; i++)
        if (bits & (1u << i)) a.idx[pos++] = (int32_t)(c0 + i);
    if (bid == a.nblk - 1 && threadIdx.x == THR - 1) *a.npass = pos;
}

__global__ __launch_bounds__(THR) void screen_reduce(ScreenArgs a) { reduce_body(a, blockIdx.x); }
__global__ __launch_bounds__(THR) void screen_count(ScreenArgs a) { count_body(a, blockIdx.x); }
__global__ __launch_bounds__(THR) void screen_scatter(ScreenArgs a) { scatter_body(a, blockIdx.x); }

__global__ __launch_bounds__(THR) void screen_reduce_b(const ScreenArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const ScreenArgs a = args[i];
    reduce_body(a, blockIdx.x - prefix[i]);
}
__global__ __launch_bounds__(THR) void screen_count_b(const ScreenArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const ScreenArgs a = args[i];
    count_body(a, blockIdx.x - prefix[i]);
}
__global__ __launch_bounds__(THR) void screen_scatter_b(const ScreenArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const ScreenArgs a = args[i];
    scatter_body(a, blockIdx.x - prefix[i]);
}

// Ascent order of the passers: lowest objective first, in power-of-two-wide
// buckets of the objective range, so that the candidates furthest below a local
// optimum (the longest flip chains) are taken first and short chains fill in
// behind them.  Only the order in which the ascent's waves take candidates
// changes; every candidate's result is the same in any order.
constexpr int ORD_THR = 1024;
constexpr int ORD_BUCKETS = 1024;
static_assert(ORD_THR == ORD_BUCKETS, "one bucket per thread: zeroing and the scan assume it");

__global__ __launch_bounds__(ORD_THR) void order_batched(const OrdArgs *args, int count)
{
    __shared__ int32_t start[ORD_BUCKETS];
    __shared__ int64_t lo_w[ORD_THR / 64], hi_w[ORD_THR / 64];
    __shared__ int32_t wsum[ORD_THR / 64];
    if ((int)blockIdx.x >= count) return;
    const OrdArgs a = args[blockIdx.x];
    const int64_t P = *a.npass;
    if (P <= 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int64_t p = threadIdx.x; p < P; p += ORD_THR) {
        const int64_t v = a.f[a.idx[p]];
        lo = v < lo ? v : lo;
        hi = v > hi ? v : hi;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t l2 = __shfl_xor(lo, o), h2 = __shfl_xor(hi, o);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    if (lane == 0) { lo_w[wv] = lo; hi_w[wv] = hi; }
    start[threadIdx.x] = 0;  // ORD_THR == ORD_BUCKETS
    __syncthreads();
    for (int i = 0; i < ORD_THR / 64; i++) {
        lo = lo_w[i] < lo ? lo_w[i] : lo;
        hi = hi_w[i] > hi ? hi_w[i] : hi;
    }
    // bucket = (v - lo) >> shift with (hi - lo) >> shift < ORD_BUCKETS
    const uint64_t span = (uint64_t)(hi - lo);
    int shift = 0;
    while ((span >> shift) >= (uint64_t)ORD_BUCKETS) shift++;
    for (int64_t p = threadIdx.x; p < P; p += ORD_THR)
        atomicAdd(&start[(int)((uint64_t)(a.f[a.idx[p]] - lo) >> shift)], 1);
    __syncthreads();
    // exclusive scan of the counts, one bucket per thread
    const int cnt = start[threadIdx.x];
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int before = 0;
    for (int i = 0; i < wv; i++) before += wsum[i];
    start[threadIdx.x] = before + incl - cnt;
    __syncthreads();
    for (int64_t p = threadIdx.x; p < P; p += ORD_THR) {
        const int32_t c = a.idx[p];
        const int pos = atomicAdd(&start[(int)((uint64_t)(a.f[c] - lo) >> shift)], 1);
        a.oidx[pos] = c;
    }
}

}  // namespace

hipError_t ubqp_launch_order_batch(hipStream_t st, const OrdArgs *args, int count)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(order_batched, dim3((unsigned)count), dim3(ORD_THR), 0, st, args, count);
    return hipGetLastError();
}

int32_t ubqp_screen_blocks(int64_t M) { return (int32_t)((M + CH - 1) / CH); }
size_t ubqp_screen_partials_bytes(int64_t M) { return (size_t)ubqp_screen_blocks(M) * 3 * sizeof(int64_t); }

ScreenArgs ubqp_screen_args(const int64_t *f, int64_t M, int32_t lam_num, int32_t lam_den, int32_t *idx,
                            int64_t *npass, int64_t *sum_max, void *partials)
{
    ScreenArgs a{};
    a.f = f;
    a.M = M;
    a.lam_num = lam_num;
    a.lam_den = lam_den;
    a.idx = idx;
    a.npass = npass;
    a.sum_max = sum_max;
    a.nblk = ubqp_screen_blocks(M);
    a.psum = (int64_t *)partials;
    a.pmax = a.psum + a.nblk;
    a.cnt = a.pmax + a.nblk;
    return a;
}

hipError_t ubqp_launch_screen(hipStream_t st, const ScreenArgs &a)
{
    hipLaunchKernelGGL(screen_reduce, dim3(a.nblk), dim3(THR), 0, st, a);
    hipLaunchKernelGGL(screen_count, dim3(a.nblk), dim3(THR), 0, st, a);
    hipLaunchKernelGGL(screen_scatter, dim3(a.nblk), dim3(THR), 0, st, a);
    return hipGetLastError();
}

hipError_t ubqp_launch_screen_batch(hipStream_t st, const ScreenArgs *args, const int64_t *prefix, int count,
                                    int64_t blocks)
{
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(screen_reduce_b, dim3((unsigned)blocks), dim3(THR), 0, st, args, prefix, count);
    hipLaunchKernelGGL(screen_count_b, dim3((unsigned)blocks), dim3(THR), 0, st, args, prefix, count);
    hipLaunchKernelGGL(screen_scatter_b, dim3((unsigned)blocks), dim3(THR), 0, st, args, prefix, count);
    return hipGetLastError();
}

// ---- screening without allocation ----------------------------------------------
// The block partials of ubqp_screen_noalloc live in one file-scope device array per
// GPU.  Host code never passes the array's name to a kernel (on the host it is only
// a stand-in): the device address of each GPU's copy is looked up once, with that
// GPU current, when the first context on it is created, and kept per device.
static constexpr int64_t STATIC_BLOCKS = (UBQP_SCREEN_NOALLOC_MAX_M + CH - 1) / CH;
static __device__ __align__(256) int64_t scratch[3 * STATIC_BLOCKS];  // psum, pmax, cnt: 48 KiB

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};

}  // namespace

int ubqp_screen_scratch_init(ubqp_ctx *ctx)
{
    if (ctx->device < 0 || ctx->device >= MAX_DEVICES)
        return ubqp_fail(ctx, UBQP_EDEVICE, "device %d beyond the %d the static screen scratch tracks", ctx->device,
                         MAX_DEVICES);
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_ptr[ctx->device]) return UBQP_OK;
    void *ptr = nullptr;
    UBQP_HIP_TRY(ctx, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return ubqp_fail(ctx, UBQP_EDEVICE, "hipGetSymbolAddress returned a null address for the screen scratch");
    scratch_ptr[ctx->device] = ptr;
    return UBQP_OK;
}

extern "C" int ubqp_screen_noalloc(ubqp_ctx *ctx, const int64_t *f_d, int64_t M, int32_t lam_num, int32_t lam_den,
                                   int32_t *pass_idx_d, int64_t *n_pass_d, int64_t *sum_max_d)
{
    if (!ctx || !f_d || !pass_idx_d || !n_pass_d || !sum_max_d) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    if (M < 1 || M > UBQP_SCREEN_NOALLOC_MAX_M)
        return ubqp_fail(ctx, UBQP_EINVAL, "M=%lld outside [1, %lld], the size of the static screen scratch",
                         (long long)M, (long long)UBQP_SCREEN_NOALLOC_MAX_M);
    if (lam_den < 1 || lam_num < 0 || lam_num > lam_den)
        return ubqp_fail(ctx, UBQP_EINVAL, "lambda=%d/%d outside [0, 1]", lam_num, lam_den);
    UBQP_TRY(ubqp_set_device(ctx));
    void *part = nullptr;
    {
        std::lock_guard<std::mutex> lk(scratch_mu);
        if (ctx->device >= 0 && ctx->device < MAX_DEVICES) part = scratch_ptr[ctx->device];
    }
    if (!part) return ubqp_fail(ctx, UBQP_EDEVICE, "the static screen scratch of device %d was not set up", ctx->device);
    // every partial is written (reduce: psum, pmax; count: cnt) before it is read
    UBQP_HIP_TRY(ctx, ubqp_launch_screen(ctx->stream, ubqp_screen_args(f_d, M, lam_num, lam_den, pass_idx_d, n_pass_d,
                                                                       sum_max_d, part)));
    return UBQP_OK;
}
