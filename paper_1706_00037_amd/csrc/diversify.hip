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
// Word indices fit 32 bits (M W <= 2^22 * 128 = 2^29), so the index arithmetic
// is 32-bit: a 64-bit division costs several times a 32-bit one.
#include "ubqp_internal.h"

namespace {

constexpr int THR = 256;
constexpr int WPT = 4;  // output words per thread: fewer, longer blocks pay the start-up latency less often

__device__ void blend_word(const DivArgs &a, int64_t id)
{
    const uint32_t W = (uint32_t)a.W, S = (uint32_t)a.S;
    const uint32_t c = (uint32_t)id / W;
    const uint32_t w = (uint32_t)id - c * W;
    const uint32_t k = c >> 1;
    const uint32_t lap = k / S;
    const uint32_t pa = k - lap * S;
    const int64_t g = a.scal ? (int64_t)a.scal->gen : a.g;
    const uint32_t pb = (pa + 1 + lap + (uint32_t)((uint64_t)g % S)) % S;  // lap < 2^22, g any int64 >= 0
    const int64_t pairs = (a.M + 1) >> 1;
    const uint64_t m = ubqp_splitmix64(a.run_seed, (1ull << 62) + (uint64_t)((g * pairs + k) * W + w));
    const uint64_t A = a.seeds[(int64_t)pa * W + w], B = a.seeds[(int64_t)pb * W + w];
    uint64_t v = (c & 1) ? (A & ~m) | (B & m) : (A & m) | (B & ~m);
    const int32_t tail = a.n - 64 * (int32_t)w;
    if (tail < 64) v &= (1ull << tail) - 1ull;
    a.X[id] = v;
}

__device__ inline void glover_word(const DivArgs &a, const uint64_t *pat, int64_t id)
{
    const uint32_t W = (uint32_t)a.W;
    const uint32_t c = (uint32_t)id / W;
    const uint32_t w = (uint32_t)id - c * W;
    const uint32_t twoH = 2u * (uint32_t)a.H;
    const uint32_t s = c / twoH;
    const uint32_t r = c - s * twoH;
    const uint32_t h = r / 2 + 1;
    // first flipped bit inside word w: smallest b >= 0 with (64 w + b) % h == 0
    const uint32_t ph = (64u * w) % h;
    const uint32_t b0 = ph == 0 ? 0 : h - ph;
    uint64_t v = a.seeds[(int64_t)s * W + w] ^ (b0 < 64 ? pat[h - 1] << b0 : 0ull);
    if (r & 1) v = ~v;
    const int32_t tail = a.n - 64 * (int32_t)w;  // valid bits in this word
    if (tail < 64) v &= (1ull << tail) - 1ull;
    a.X[id] = v;
}

__device__ void diversify_body(const DivArgs &a, int64_t bid)
{
    if (a.blend) {            // uniform over the block: a block serves one instance
        for (int k = 0; k < WPT; k++) {
            const int64_t id = (bid * WPT + k) * THR + threadIdx.x;
            if (id < a.total) blend_word(a, id);
        }
        return;
    }
    __shared__ uint64_t pat[UBQP_MAX_H];
    for (int h = threadIdx.x + 1; h <= a.H; h += blockDim.x) {
        uint64_t m = 0;
        for (int b = 0; b < 64; b += h) m |= 1ull << b;
        pat[h - 1] = m;
    }
    __syncthreads();
    for (int k = 0; k < WPT; k++) {
        const int64_t id = (bid * WPT + k) * THR + threadIdx.x;
        if (id < a.total) glover_word(a, pat, id);
    }
}

__global__ __launch_bounds__(THR) void diversify_kernel(DivArgs a) { diversify_body(a, blockIdx.x); }

__global__ __launch_bounds__(THR) void diversify_batched(const DivArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const DivArgs a = args[i];  // a local copy: fields stay in registers across stores
    diversify_body(a, blockIdx.x - prefix[i]);
}

}  // namespace

int64_t ubqp_div_blocks(const DivArgs &a) { return (a.total + THR * WPT - 1) / (THR * WPT); }

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
