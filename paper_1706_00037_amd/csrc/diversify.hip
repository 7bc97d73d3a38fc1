// Glover diversification generator on bit-packed solutions (the paper's
// Diversify step, after Glover 1998): candidate c takes seed s = c / 2H and step
// h = (c mod 2H)/2 + 1, flips the variables j = 0, h, 2h, ... of the seed (x'),
// and is complemented when c is odd (x'').
//
// Blending (the paper reports combining two solutions into new ones, with no
// rule; the rule here is a uniform crossover): candidates come in pairs
// k = c / 2 with parents a = k mod S and b = (a + 1 + k / S + g) mod S in
// generation g; mask word w of pair k is SplitMix64 output
// 2^62 + (g ceil(M/2) + k) W + w of run_seed; the even candidate takes a's bits
// where the mask is 1 and b's elsewhere, the odd one the opposite choice.
//
// HBM-bound: one thread per output word; the seed word is read once per
// candidate row (L2 hits across the 2H candidates of a seed), the output is
// written once, fully coalesced.  The periodic flip pattern of step h is a
// 64-bit word P_h (bits 0, h, 2h, ...) shifted to the phase of the word.
#include "ubqp_internal.h"

namespace {

constexpr int THR = 256;

__device__ void blend_body(const DivArgs &a, int64_t bid)
{
    const int64_t id = bid * THR + threadIdx.x;
    if (id >= a.total) return;
    const int32_t W = a.W;
    const int64_t c = id / W;
    const int32_t w = (int32_t)(id - c * W);
    const int64_t k = c >> 1;
    const int64_t lap = k / a.S;
    const int64_t pa = k - lap * a.S;
    const int64_t g = a.scal ? (int64_t)a.scal->gen : a.g;
    const int64_t pb = (pa + 1 + lap + g) % a.S;
    const int64_t pairs = (a.M + 1) >> 1;
    const uint64_t m = ubqp_splitmix64(a.run_seed, (1ull << 62) + (uint64_t)((g * pairs + k) * W + w));
    const uint64_t A = a.seeds[pa * W + w], B = a.seeds[pb * W + w];
    uint64_t v = (c & 1) ? (A & ~m) | (B & m) : (A & m) | (B & ~m);
    const int32_t tail = a.n - 64 * w;
    if (tail < 64) v &= (1ull << tail) - 1ull;
    a.X[id] = v;
}

__device__ void diversify_body(const DivArgs &a, int64_t bid)
{
    if (a.blend) {            // uniform over the block: a block serves one instance
        blend_body(a, bid);
        return;
    }
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
