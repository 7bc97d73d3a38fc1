// Per-generation bookkeeping of the multi-start loop (Fig. 2):
//  - UpdateBestAndT: among the ascended passers, scanned by ascending index, the
//    incumbent is replaced when f > f* (strict), so the earliest maximiser wins;
//  - next seeds (the reading of Diversify(x, best, i) for a generation of many
//    candidates): seed 0 = incumbent, then the ascended passers ranked by
//    (f desc, index asc), then random solutions for the remaining slots;
//  - per-generation statistics {Sum, Max, passers, flips, f*}.
// Random solutions are SplitMix64 (Steele, Lea & Flood 2014) used as a counter
// generator: word w of seed slot s in generation g is output (g S + s) W + w of
// the generator seeded with run_seed.
#include "ubqp_internal.h"

namespace {

__device__ inline uint64_t splitmix_output(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline uint64_t random_word(uint64_t run_seed, int64_t g, int64_t S, int64_t s, int32_t W, int32_t w,
                                       int32_t n)
{
    uint64_t v = splitmix_output(run_seed, (uint64_t)((g * S + s) * W + w));
    const int32_t tail = n - 64 * w;
    if (tail < 64) v &= (1ull << tail) - 1ull;
    return v;
}

__global__ __launch_bounds__(256) void seed_init_kernel(uint64_t *seeds, int64_t S, int32_t n, int32_t W,
                                                        uint64_t run_seed, const uint64_t *deriv_x,
                                                        ubqp_scal *scal)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id == 0) {
        scal->have_best = 0;
        scal->best_f = INT64_MIN;
        scal->best_c = -1;
    }
    if (id >= S * W) return;
    const int64_t s = id / W;
    const int32_t w = (int32_t)(id - s * W);
    seeds[id] = (s == 0 && deriv_x) ? deriv_x[w] : random_word(run_seed, 0, S, s, W, w, n);
}

// One block: incumbent update and statistics of generation g.
__global__ __launch_bounds__(256) void incumbent_kernel(const uint64_t *X, int32_t W, const int64_t *f,
                                                        const int32_t *flips, const int32_t *idx, ubqp_scal *scal,
                                                        uint64_t *best_x, int64_t *stats, int32_t g)
{
    __shared__ int64_t sf[4], sfl[4];
    __shared__ int32_t sc[4];
    __shared__ int32_t winner;
    const int64_t P = scal->npass;
    int64_t bf = INT64_MIN, fl = 0;
    int32_t bc = 0x7FFFFFFF;
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
        const int32_t c = idx[p];
        const int64_t v = f[c];
        fl += flips[c];
        if (v > bf || (v == bf && c < bc)) { bf = v; bc = c; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t ov = __shfl_xor(bf, o);
        const int32_t oc = __shfl_xor(bc, o);
        fl += __shfl_xor(fl, o);
        if (ov > bf || (ov == bf && oc < bc)) { bf = ov; bc = oc; }
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sf[wv] = bf; sc[wv] = bc; sfl[wv] = fl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        bf = sf[0]; bc = sc[0]; fl = sfl[0];
        for (int i = 1; i < 4; i++) {
            fl += sfl[i];
            if (sf[i] > bf || (sf[i] == bf && sc[i] < bc)) { bf = sf[i]; bc = sc[i]; }
        }
        winner = -1;
        if (P > 0 && (!scal->have_best || bf > scal->best_f)) {
            scal->have_best = 1;
            scal->best_f = bf;
            scal->best_c = bc;
            winner = bc;
        }
        int64_t *st = stats + (int64_t)g * 5;
        st[0] = scal->sum_max[0];
        st[1] = scal->sum_max[1];
        st[2] = P;
        st[3] = fl;
        st[4] = scal->have_best ? scal->best_f : INT64_MIN;
    }
    __syncthreads();
    if (winner >= 0)
        for (int w = threadIdx.x; w < W; w += blockDim.x) best_x[w] = X[(int64_t)winner * W + w];
}

// Rank of each passer by (f desc, index asc); the top S-1 become seeds 1..S-1.
__global__ __launch_bounds__(256) void rank_kernel(const uint64_t *X, int32_t W, const int64_t *f,
                                                   const int32_t *idx, const ubqp_scal *scal, int64_t S,
                                                   uint64_t *seeds)
{
    __shared__ int64_t tf[256];
    const int64_t P = scal->npass;
    const int64_t p0 = (int64_t)blockIdx.x * blockDim.x;
    if (p0 >= P) return;
    const int64_t p = p0 + threadIdx.x;
    const int64_t fp = p < P ? f[idx[p]] : 0;
    int64_t r = 0;
    for (int64_t base = 0; base < P; base += 256) {
        __syncthreads();
        if (base + threadIdx.x < P) tf[threadIdx.x] = f[idx[base + threadIdx.x]];
        __syncthreads();
        const int64_t lim = P - base < 256 ? P - base : 256;
        for (int64_t q = 0; q < lim; q++) {
            const int64_t fq = tf[q];
            r += (fq > fp) || (fq == fp && base + q < p);
        }
    }
    if (p < P && r < S - 1) {
        const uint64_t *src = X + (int64_t)idx[p] * W;
        uint64_t *dst = seeds + (1 + r) * W;
        for (int w = 0; w < W; w++) dst[w] = src[w];
    }
}

// Seed 0 (incumbent, or random while none exists) and the random tail slots.
__global__ __launch_bounds__(256) void seed_fill_kernel(uint64_t *seeds, int64_t S, int32_t n, int32_t W,
                                                        uint64_t run_seed, int32_t g_next, const ubqp_scal *scal,
                                                        const uint64_t *best_x)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= S * W) return;
    const int64_t s = id / W;
    const int32_t w = (int32_t)(id - s * W);
    const int64_t P = scal->npass;
    const int64_t ranked = P < S - 1 ? P : S - 1;
    if (s == 0)
        seeds[id] = scal->have_best ? best_x[w] : random_word(run_seed, g_next, S, 0, W, w, n);
    else if (s >= 1 + ranked)
        seeds[id] = random_word(run_seed, g_next, S, s, W, w, n);
}

}  // namespace

hipError_t ubqp_launch_seed_init(hipStream_t st, uint64_t *seeds, int64_t S, int32_t n, uint64_t run_seed,
                                 const uint64_t *deriv_x, ubqp_scal *scal)
{
    const int32_t W = (n + 63) / 64;
    hipLaunchKernelGGL(seed_init_kernel, dim3((unsigned)((S * W + 255) / 256)), dim3(256), 0, st, seeds, S, n, W,
                       run_seed, deriv_x, scal);
    return hipGetLastError();
}

hipError_t ubqp_launch_select(hipStream_t st, int32_t n, int64_t M, int64_t S, int32_t g, uint64_t run_seed,
                              const uint64_t *X, const int64_t *f, const int32_t *flips, const int32_t *idx,
                              ubqp_scal *scal, uint64_t *best_x, uint64_t *seeds, int64_t *stats)
{
    const int32_t W = (n + 63) / 64;
    hipLaunchKernelGGL(incumbent_kernel, dim3(1), dim3(256), 0, st, X, W, f, flips, idx, scal, best_x, stats, g);
    hipLaunchKernelGGL(rank_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, X, W, f, idx, scal, S,
                       seeds);
    hipLaunchKernelGGL(seed_fill_kernel, dim3((unsigned)((S * W + 255) / 256)), dim3(256), 0, st, seeds, S, n, W,
                       run_seed, g + 1, scal, best_x);
    return hipGetLastError();
}
