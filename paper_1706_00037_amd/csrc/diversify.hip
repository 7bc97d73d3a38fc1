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

__global__ __launch_bounds__(256) void diversify_kernel(const uint64_t *__restrict__ seeds, int32_t n, int32_t W,
                                                        int32_t H, uint64_t *__restrict__ X, int64_t total)
{
    __shared__ uint64_t pat[UBQP_MAX_H];
    for (int h = threadIdx.x + 1; h <= H; h += blockDim.x) {
        uint64_t m = 0;
        for (int b = 0; b < 64; b += h) m |= 1ull << b;
        pat[h - 1] = m;
    }
    __syncthreads();
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const int64_t c = id / W;
    const int32_t w = (int32_t)(id - c * W);
    const int64_t twoH = 2 * (int64_t)H;
    const int64_t s = c / twoH;
    const int32_t r = (int32_t)(c - s * twoH);
    const int32_t h = r / 2 + 1;
    // first flipped bit inside word w: smallest b >= 0 with (64 w + b) % h == 0
    const int32_t ph = (int32_t)((64ll * w) % h);
    const int32_t b0 = ph == 0 ? 0 : h - ph;
    uint64_t v = seeds[s * W + w] ^ (b0 < 64 ? pat[h - 1] << b0 : 0ull);
    if (r & 1) v = ~v;
    const int32_t tail = n - 64 * w;  // valid bits in this word
    if (tail < 64) v &= (1ull << tail) - 1ull;
    X[id] = v;
}

}  // namespace

hipError_t ubqp_launch_diversify(hipStream_t st, int32_t n, const uint64_t *seeds, int64_t S, int32_t H,
                                 uint64_t *X, int64_t M)
{
    (void)S;
    const int32_t W = (n + 63) / 64;
    const int64_t total = M * W;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(diversify_kernel, dim3((unsigned)blocks), dim3(256), 0, st, seeds, n, W, H, X, total);
    return hipGetLastError();
}
