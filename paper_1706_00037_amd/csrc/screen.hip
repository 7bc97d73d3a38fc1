// Exact T(lambda) screening (Pseudocode section): T = Mean + lambda (Max - Mean)
// over the generation's M objective values, pass iff f > T, decided in 128-bit
// integers as  den*M*f > (den - num)*Sum + num*M*Max  (lambda = num/den).
// Passer indices are compacted in ascending order.
//
// Three HBM-bound passes over f (8 B/candidate each): block partial Sum/Max,
// per-block passer counts, and an order-preserving scatter.  No atomics, so the
// output is the same on every run.
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

__device__ inline bool passes(int64_t f, int64_t M, int32_t num, int32_t den, __int128 rhs)
{
    return (__int128)den * M * f > rhs;
}

__global__ __launch_bounds__(THR) void screen_reduce(const int64_t *__restrict__ f, int64_t M,
                                                     int64_t *__restrict__ psum, int64_t *__restrict__ pmax)
{
    const int64_t base = blockIdx.x * CH;
    int64_t s = 0, m = INT64_MIN;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const int64_t c = base + i * THR + threadIdx.x;
        if (c < M) { const int64_t v = f[c]; s += v; m = v > m ? v : m; }
    }
    block_sum_max(s, m);
    if (threadIdx.x == 0) { psum[blockIdx.x] = s; pmax[blockIdx.x] = m; }
}

// Sum and Max of the whole population from the block partials.
__device__ void total_sum_max(const int64_t *psum, const int64_t *pmax, int nblk, int64_t &s, int64_t &m)
{
    s = 0;
    m = INT64_MIN;
    for (int b = threadIdx.x; b < nblk; b += THR) { s += psum[b]; m = pmax[b] > m ? pmax[b] : m; }
    block_sum_max(s, m);
}

__global__ __launch_bounds__(THR) void screen_count(const int64_t *__restrict__ f, int64_t M, int32_t num,
                                                    int32_t den, const int64_t *__restrict__ psum,
                                                    const int64_t *__restrict__ pmax, int nblk,
                                                    int64_t *__restrict__ cnt, int64_t *__restrict__ sum_max)
{
    int64_t S, Mx;
    total_sum_max(psum, pmax, nblk, S, Mx);
    const __int128 rhs = (__int128)(den - num) * S + (__int128)num * M * Mx;
    const int64_t base = blockIdx.x * CH;
    int64_t k = 0;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const int64_t c = base + i * THR + threadIdx.x;
        if (c < M && passes(f[c], M, num, den, rhs)) k++;
    }
    int64_t dummy = 0;
    block_sum_max(k, dummy);
    if (threadIdx.x == 0) {
        cnt[blockIdx.x] = k;
        if (blockIdx.x == 0) { sum_max[0] = S; sum_max[1] = Mx; }
    }
}

__global__ __launch_bounds__(THR) void screen_scatter(const int64_t *__restrict__ f, int64_t M, int32_t num,
                                                      int32_t den, const int64_t *__restrict__ cnt, int nblk,
                                                      const int64_t *__restrict__ sum_max,
                                                      int32_t *__restrict__ idx, int64_t *__restrict__ npass)
{
    __shared__ int64_t wtot[THR / 64];
    // passers in earlier blocks
    int64_t off = 0, dummy = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += THR) off += cnt[b];
    block_sum_max(off, dummy);
    const __int128 rhs = (__int128)(den - num) * sum_max[0] + (__int128)num * M * sum_max[1];
    // each thread owns PER consecutive candidates, so thread order is index order
    const int64_t c0 = blockIdx.x * CH + (int64_t)threadIdx.x * PER;
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const int64_t c = c0 + i;
        if (c < M && passes(f[c], M, num, den, rhs)) bits |= 1u << i;
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
        if (bits & (1u << i)) idx[pos++] = (int32_t)(c0 + i);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == THR - 1) *npass = pos;
}

}  // namespace

size_t ubqp_screen_partials_bytes(int64_t M) { return (size_t)((M + CH - 1) / CH) * 3 * sizeof(int64_t); }

hipError_t ubqp_launch_screen(hipStream_t st, const int64_t *f, int64_t M, int32_t lam_num, int32_t lam_den,
                              int32_t *idx, int64_t *npass, int64_t *sum_max, void *partials)
{
    const int nblk = (int)((M + CH - 1) / CH);
    int64_t *psum = (int64_t *)partials, *pmax = psum + nblk, *cnt = pmax + nblk;
    hipLaunchKernelGGL(screen_reduce, dim3(nblk), dim3(THR), 0, st, f, M, psum, pmax);
    hipLaunchKernelGGL(screen_count, dim3(nblk), dim3(THR), 0, st, f, M, lam_num, lam_den, psum, pmax, nblk, cnt,
                       sum_max);
    hipLaunchKernelGGL(screen_scatter, dim3(nblk), dim3(THR), 0, st, f, M, lam_num, lam_den, cnt, nblk, sum_max,
                       idx, npass);
    return hipGetLastError();
}
