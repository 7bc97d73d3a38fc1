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
//
// The generation index lives on the device (ubqp_scal::gen, advanced by the
// last kernel of a generation), so the launches of a generation do not depend
// on it and can be replayed as a graph.
#include "ubqp_internal.h"

namespace {

constexpr int THR = 256;
constexpr int RANK_SPLIT = 4;  // ranking blocks per 256 candidates

__device__ inline uint64_t random_word(uint64_t run_seed, int64_t g, int64_t S, int64_t s, int32_t W, int32_t w,
                                       int32_t n)
{
    uint64_t v = ubqp_splitmix64(run_seed, (uint64_t)((g * S + s) * W + w));
    const int32_t tail = n - 64 * w;
    if (tail < 64) v &= (1ull << tail) - 1ull;
    return v;
}

__device__ void seed_init_body(const SelArgs &a, int64_t bid)
{
    const int64_t id = bid * THR + threadIdx.x;
    if (id == 0) {
        a.scal->have_best = 0;
        a.scal->best_f = INT64_MIN;
        a.scal->best_c = -1;
        a.scal->gen = 0;
    }
    if (id >= a.S * a.W) return;
    const int64_t s = id / a.W;
    const int32_t w = (int32_t)(id - s * a.W);
    a.seeds[id] = (s == 0 && a.deriv_x) ? a.deriv_x[w] : random_word(a.run_seed, 0, a.S, s, a.W, w, a.n);
}

// f before ascent into row `gen` of the dump.
__device__ void dump_body(const SelArgs &a, int64_t bid)
{
    const int64_t c = bid * THR + threadIdx.x;
    if (a.f_dump && c < a.M) a.f_dump[(int64_t)a.scal->gen * a.M + c] = a.f[c];
}

// One block: incumbent update and statistics of the current generation.
__device__ void incumbent_body(const SelArgs &a)
{
    __shared__ int64_t sf[THR / 64], sfl[THR / 64];
    __shared__ int32_t sc[THR / 64];
    __shared__ int32_t winner;
    ubqp_scal *scal = a.scal;
    const int64_t P = scal->npass;
    int64_t bf = INT64_MIN, fl = 0;
    int32_t bc = 0x7FFFFFFF;
    for (int64_t p = threadIdx.x; p < P; p += THR) {
        const int32_t c = a.idx[p];
        const int64_t v = a.f[c];
        fl += a.flips[c];
        a.rank[p] = 0;
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
        for (int i = 1; i < THR / 64; i++) {
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
        int64_t *st = a.stats + (int64_t)scal->gen * 5;
        st[0] = scal->sum_max[0];
        st[1] = scal->sum_max[1];
        st[2] = P;
        st[3] = fl;
        st[4] = scal->have_best ? scal->best_f : INT64_MIN;
    }
    __syncthreads();
    if (winner >= 0)
        for (int w = threadIdx.x; w < a.W; w += THR) a.best_x[w] = a.X[(int64_t)winner * a.W + w];
}

// Rank of each passer by (f desc, index asc): the instance's RANK_SPLIT ceil(M / 256)
// blocks split into E = ceil(P / 256) passer chunks times as many slices of the
// comparison range as fit; each block adds its partial counts to rank[] (zeroed
// by the incumbent kernel).
__device__ void rank_body(const SelArgs &a, int64_t bid)
{
    __shared__ int64_t tf[THR];
    const int64_t P = a.scal->npass;
    const int64_t E = (P + THR - 1) / THR;
    if (E == 0) return;
    const int64_t nblk = RANK_SPLIT * ((a.M + THR - 1) / THR);
    const int64_t slices = nblk / E > 0 ? nblk / E : 1;
    if (bid >= E * slices) return;
    const int64_t p = (bid % E) * THR + threadIdx.x, slice = bid / E;
    const int64_t lo = P * slice / slices, hi = P * (slice + 1) / slices;
    const int64_t fp = p < P ? a.f[a.idx[p]] : 0;
    int32_t r = 0;
    for (int64_t base = lo; base < hi; base += THR) {
        __syncthreads();
        if (base + threadIdx.x < hi) tf[threadIdx.x] = a.f[a.idx[base + threadIdx.x]];
        __syncthreads();
        const int64_t lim = hi - base < THR ? hi - base : THR;
        for (int64_t q = 0; q < lim; q++) {
            const int64_t fq = tf[q];
            r += (fq > fp) || (fq == fp && base + q < p);
        }
    }
    if (p < P && r) atomicAdd(&a.rank[p], r);
}

// The top S-1 passers become seeds 1..S-1: the instance's blocks stride over the
// (passer, word) pairs, so consecutive threads copy consecutive words of a row.
__device__ void place_body(const SelArgs &a, int64_t bid)
{
    // indices fit 32 bits (P W <= M W <= 2^29): 32-bit division
    const uint32_t P = (uint32_t)a.scal->npass, W = (uint32_t)a.W;
    const uint32_t nblk = (uint32_t)((a.M + THR - 1) / THR);
    const uint32_t total = P * W;
    for (uint32_t k = (uint32_t)bid * THR + threadIdx.x; k < total; k += nblk * THR) {
        const uint32_t p = k / W, w = k - p * W;
        const int64_t r = a.rank[p];
        if (r < a.S - 1) a.seeds[(1 + r) * W + w] = a.X[(int64_t)a.idx[p] * W + w];
    }
}

// Seed 0 (incumbent, or random while none exists) and the random tail slots.
__device__ void seed_fill_body(const SelArgs &a, int64_t bid)
{
    const int64_t id = bid * THR + threadIdx.x;
    if (id >= a.S * a.W) return;
    const int64_t s = id / a.W;
    const int32_t w = (int32_t)(id - s * a.W);
    const int64_t P = a.scal->npass;
    const int64_t ranked = P < a.S - 1 ? P : a.S - 1;
    const int32_t g_next = a.scal->gen + 1;
    if (s == 0)
        a.seeds[id] = a.scal->have_best ? a.best_x[w] : random_word(a.run_seed, g_next, a.S, 0, a.W, w, a.n);
    else if (s >= 1 + ranked)
        a.seeds[id] = random_word(a.run_seed, g_next, a.S, s, a.W, w, a.n);
}

__global__ __launch_bounds__(THR) void seed_init_kernel(SelArgs a) { seed_init_body(a, blockIdx.x); }

#define BATCHED(NAME, BODY)                                                                               \
    __global__ __launch_bounds__(THR) void NAME(const SelArgs *args, const int64_t *prefix, int count)  \
    {                                                                                                     \
        const int i = ubqp_find_inst(prefix, count, blockIdx.x);                                         \
        const SelArgs a = args[i];                                                                        \
        BODY(a, blockIdx.x - prefix[i]);                                                                  \
    }
BATCHED(seed_init_b, seed_init_body)
BATCHED(dump_b, dump_body)
BATCHED(rank_b, rank_body)
BATCHED(place_b, place_body)
BATCHED(seed_fill_b, seed_fill_body)
#undef BATCHED

__global__ __launch_bounds__(THR) void incumbent_b(const SelArgs *args, int count)
{
    const SelArgs a = args[blockIdx.x];
    incumbent_body(a);
}

__global__ void advance_b(const SelArgs *args, int count)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i < count) args[i].scal->gen += 1;
}

}  // namespace

SelArgs ubqp_sel_args(int32_t n, int64_t M, int64_t S, uint64_t run_seed, const uint64_t *X, const int64_t *f,
                      const int32_t *flips, const int32_t *idx, int32_t *rank, ubqp_scal *scal, uint64_t *best_x,
                      uint64_t *seeds, int64_t *stats, const uint64_t *deriv_x, int64_t *f_dump)
{
    SelArgs a{};
    a.rank = rank;
    a.n = n;
    a.W = (n + 63) / 64;
    a.M = M;
    a.S = S;
    a.run_seed = run_seed;
    a.X = X;
    a.f = f;
    a.flips = flips;
    a.idx = idx;
    a.scal = scal;
    a.best_x = best_x;
    a.seeds = seeds;
    a.stats = stats;
    a.deriv_x = deriv_x;
    a.f_dump = f_dump;
    return a;
}

int64_t ubqp_seed_blocks(const SelArgs &a) { return (a.S * a.W + THR - 1) / THR; }
int64_t ubqp_cand_blocks(const SelArgs &a) { return (a.M + THR - 1) / THR; }
int64_t ubqp_rank_blocks(const SelArgs &a) { return RANK_SPLIT * ((a.M + THR - 1) / THR); }

hipError_t ubqp_launch_seed_init(hipStream_t st, const SelArgs &a)
{
    hipLaunchKernelGGL(seed_init_kernel, dim3((unsigned)ubqp_seed_blocks(a)), dim3(THR), 0, st, a);
    return hipGetLastError();
}

hipError_t ubqp_launch_seed_init_batch(hipStream_t st, const SelArgs *args, const int64_t *seed_prefix, int count,
                                       int64_t seed_blocks)
{
    hipLaunchKernelGGL(seed_init_b, dim3((unsigned)seed_blocks), dim3(THR), 0, st, args, seed_prefix, count);
    return hipGetLastError();
}

hipError_t ubqp_launch_dump_batch(hipStream_t st, const SelArgs *args, const int64_t *cand_prefix, int count,
                                  int64_t cand_blocks)
{
    hipLaunchKernelGGL(dump_b, dim3((unsigned)cand_blocks), dim3(THR), 0, st, args, cand_prefix, count);
    return hipGetLastError();
}

hipError_t ubqp_launch_select_batch(hipStream_t st, const SelArgs *args, const int64_t *cand_prefix,
                                    int64_t cand_blocks, const int64_t *rank_prefix, int64_t rank_blocks,
                                    const int64_t *seed_prefix, int64_t seed_blocks, int count)
{
    hipLaunchKernelGGL(incumbent_b, dim3(count), dim3(THR), 0, st, args, count);
    hipLaunchKernelGGL(rank_b, dim3((unsigned)rank_blocks), dim3(THR), 0, st, args, rank_prefix, count);
    hipLaunchKernelGGL(place_b, dim3((unsigned)cand_blocks), dim3(THR), 0, st, args, cand_prefix, count);
    hipLaunchKernelGGL(seed_fill_b, dim3((unsigned)seed_blocks), dim3(THR), 0, st, args, seed_prefix, count);
    hipLaunchKernelGGL(advance_b, dim3((count + 63) / 64), dim3(64), 0, st, args, count);
    return hipGetLastError();
}
