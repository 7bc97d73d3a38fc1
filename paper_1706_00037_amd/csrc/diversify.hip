// Glover diversification generator on bit-packed solutions (the paper's
// Diversify step, after Glover 1998): candidate c takes seed s = c / 2H and step
// h = (c mod 2H)/2 + 1, flips the variables j = 0, h, 2h, ... of the seed (x'),
// and is complemented when c is odd (x'').
//
// HBM-bound: one thread per output word; the seed word is read once per
// candidate row (L2 hits across the 2H candidates of a seed), the output is
// written once, fully coalesced.  The periodic flip pattern of step h is a
// 64-bit word P_h (bits 0, h, 2h, ...) shifted to the phase of the word.
#include "ubqp_internal.h"

namespace {

constexpr int THR = 256;

__device__ void diversify_body(const DivArgs &a, int64_t bid)
{
    __shared__ uint64_t pat[UBQP_MAX_H];
    for (int h = threadIdx.x + 1; h <= a.H; h += blockDim.x) {
        uint64_t m = 0;
        for (int b = 0; b < 64; b += h) m |= 1ull << b;
        pat[h - 1] = m;
    }
    __syncthreads();
    const int64_t id = bid * THR + threadIdx.x;
    if (id >= a.total) return;
    const int32_t W = a.W;
    const int64_t c = id / W;
    const int32_t w = (int32_t)(id - c * W);
    const int64_t twoH = 2 * (int64_t)a.H;
    const int64_t s = c / twoH;
    const int32_t r = (int32_t)(c - s * twoH);
    const int32_t h = r / 2 + 1;
    // first flipped bit inside word w: smallest b >= 0 with (64 w + b) % h == 0
    const int32_t ph = (int32_t)((64ll * w) % h);
    const int32_t b0 = ph == 0 ? 0 : h - ph;
    uint64_t v = a.seeds[s * W + w] ^ (b0 < 64 ? pat[h - 1] << b0 : 0ull);
    if (r & 1) v = ~v;
    const int32_t tail = a.n - 64 * w;  // valid bits in this word
    if (tail < 64) v &= (1ull << tail) - 1ull;
    a.X[id] = v;
}

__global__ __launch_bounds__(THR) void diversify_kernel(DivArgs a) { diversify_body(a, blockIdx.x); }

__global__ __launch_bounds__(THR) void diversify_batched(const DivArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const DivArgs a = args[i];  // a local copy: fields stay in registers across stores
    diversify_body(a, blockIdx.x - prefix[i]);
}

}  // namespace

int64_t ubqp_div_blocks(const DivArgs &a) { return (a.total + THR - 1) / THR; }

hipError_t ubqp_launch_diversify(hipStream_t st, const DivArgs &a)
{
    hipLaunchKernelGGL(diversify_kernel, dim3((unsigned)ubqp_div_blocks(a)), dim3(THR), 0, st, a);
    return hipGetLastError();
}

hipError_t ubqp_launch_diversify_batch(hipStream_t st, const DivArgs *args, const int64_t *prefix, int count,
                                       int64_t blocks)
{
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(diversify_batched, dim3((unsigned)blocks), dim3(THR), 0, st, args, prefix, count);
    return hipGetLastError();
}
