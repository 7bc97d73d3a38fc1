/*
 * ubqp_oracle.c -- plain, slow, obviously-correct CPU reference for the
 * diversified multi-start UBQP method (Lewis, "A Diversified Multi-Start
 * Algorithm for Unconstrained Binary Quadratic Problems Leveraging the
 * Graphics Processor Unit", arXiv:1706.00037).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which is
 * loaded by tests/, by __graft_entry__.smoke() and by the cpu_baseline leg of
 * bench.py, and by nothing else.  The GPU library shares no source, header,
 * table or helper with it.
 *
 * Every step is written from its definition in the paper, in the paper's
 * order, with scalar loops and int64 / __int128 integer arithmetic:
 *   objective        f(x) = x^T Q x                 (problem (P), Introduction)
 *   screening        T(lambda) = Mean + lambda (Max - Mean), pass iff f > T
 *                                                   (Pseudocode section, Fig. 2)
 *   1-flip ascent    Delta_i = f(x xor e_i) - f(x), steepest improving flip,
 *                    stop at a 1-flip local optimum or after max flips, no tabu
 *                    (Pseudocode section; Glover et al. 2002 for the deltas)
 *   diversification  Glover's generator: flip every h-th variable, plus the
 *                    complement (Pseudocode section, Glover 1998); or blending
 *                    two seeds (Pseudocode section, rule read here)
 *   main loop        diversify -> evaluate -> screen -> ascent -> update best
 *                    (Fig. 2), a generation of many candidates at a time, or
 *                    one candidate per iteration as printed (orc_sequential)
 *   path relinking   the polishing phase the paper names but does not build
 *                    (greedy relinking, rule read here; orc_relink_path)
 * The readings taken where the paper is silent are listed at each function.
 *
 * Pins that do not come from this file are in tests/test_oracle_*.py.  Parity
 * unpinned: beyond the properties those pins fix (brute force at small n, closed
 * forms, invariants, sign-definite Q), the full multi-generation trajectories of
 * orc_multistart, orc_sequential and orc_relink_many at large n are checked by
 * nothing but this file; the paper prints no per-instance trajectory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ---------------------------------------------------------------- helpers */

static int get_bit(const uint64_t *x, int64_t j) { return (int)((x[j >> 6] >> (j & 63)) & 1u); }
static void put_bit(uint64_t *x, int64_t j, int b)
{
    uint64_t m = 1ull << (j & 63);
    if (b) x[j >> 6] |= m; else x[j >> 6] &= ~m;
}
static int64_t words_for(int64_t n) { return (n + 63) / 64; }

/* ------------------------------------------------------- random solutions */

/*
 * SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the state advances by the golden-ratio gamma and
 * each output is the state passed through the variant-13 finaliser.  The i-th
 * output (i = 0, 1, ...) of a generator seeded with `seed` is returned, which
 * makes it usable as a counter-based generator.
 */
ORC_API uint64_t orc_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/*
 * A random Bernoulli(1/2) solution (the paper evaluates randomly generated x,
 * Pseudocode section; the generator is not named there).  Reading: word w of
 * seed slot s in generation g is output number (g*S + s)*W + w of SplitMix64
 * seeded with run_seed; bits at positions >= n are cleared.
 */
ORC_API void orc_random_solution(int32_t n, uint64_t run_seed, int64_t g, int64_t S, int64_t s,
                                 uint64_t *x)
{
    int64_t W = words_for(n);
    for (int64_t w = 0; w < W; w++)
        x[w] = orc_splitmix64(run_seed, (uint64_t)((g * S + s) * W + w));
    for (int64_t j = n; j < W * 64; j++) put_bit(x, j, 0);
}

/* ------------------------------------------------------------- objective */

/* f(x) = sum_i sum_j q_ij x_i x_j over the full symmetric Q (problem (P)). */
ORC_API int64_t orc_f(int32_t n, const int32_t *Q, const uint64_t *x)
{
    int64_t acc = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!get_bit(x, i)) continue;
        for (int64_t j = 0; j < n; j++)
            if (get_bit(x, j)) acc += Q[i * n + j];
    }
    return acc;
}

/* f for each of M candidates (rows of X, W words each).  `threads` only
 * partitions the candidates for timing; each value is orc_f. */
ORC_API void orc_eval(int32_t n, const int32_t *Q, const uint64_t *X, int64_t M, int64_t *f,
                      int32_t threads)
{
    int64_t W = words_for(n);
    if (threads < 1) threads = 1;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (int64_t c = 0; c < M; c++) f[c] = orc_f(n, Q, X + c * W);
}

/* ------------------------------------------------------- diversification */

/*
 * Glover's diversification generator (Glover 1998, used by the paper's
 * Diversify step).  For step h the variables j = 0, h, 2h, ... (the 1-based
 * "1 + kh" positions) of the seed are flipped, giving x'; the complement of x'
 * gives x''.  Reading: candidate c comes from seed s = c / (2H), step
 * h = (c mod 2H)/2 + 1, and is x' when c is even, x'' when c is odd.
 */
ORC_API void orc_diversify(int32_t n, const uint64_t *seeds, int64_t S, int32_t H, uint64_t *X,
                           int64_t M)
{
    int64_t W = words_for(n);
    (void)S;
    for (int64_t c = 0; c < M; c++) {
        int64_t s = c / (2 * H), r = c % (2 * H);
        int64_t h = r / 2 + 1;
        int comp = (int)(r % 2);
        const uint64_t *seed = seeds + s * W;
        uint64_t *x = X + c * W;
        memset(x, 0, (size_t)W * 8);
        for (int64_t j = 0; j < n; j++) {
            int b = get_bit(seed, j);
            if (j % h == 0) b ^= 1;
            if (comp) b ^= 1;
            put_bit(x, j, b);
        }
    }
}

/*
 * Blending (breeding) diversification.  The paper reports diversification by
 * blending two solutions into new ones (Pseudocode section) without a rule;
 * the reading taken here is a uniform crossover of two seeds with a random mask:
 *   candidates come in pairs k = c / 2 (k < ceil(M / 2));
 *   parents are seeds a = k mod S and b = (a + 1 + k / S + g) mod S;
 *   mask word w is output 2^62 + (g * ceil(M / 2) + k) * W + w of SplitMix64
 *   seeded with run_seed (a counter range apart from the random solutions');
 *   bit j of the child is the parent-a bit where the mask is 1 and the parent-b
 *   bit where it is 0 for even c, the other way round for odd c.
 * Positions >= n are 0 (the seeds' are).
 */
ORC_API void orc_blend(int32_t n, const uint64_t *seeds, int64_t S, int64_t M, int64_t g, uint64_t run_seed,
                       uint64_t *X)
{
    int64_t W = words_for(n);
    int64_t pairs = (M + 1) / 2;
    for (int64_t c = 0; c < M; c++) {
        int64_t k = c / 2;
        int64_t a = k % S;
        int64_t b = (a + 1 + k / S + g) % S;
        int odd = (int)(c % 2);
        uint64_t *x = X + c * W;
        memset(x, 0, (size_t)W * 8);
        for (int64_t j = 0; j < n; j++) {
            uint64_t mw = orc_splitmix64(run_seed, (1ull << 62) + (uint64_t)((g * pairs + k) * W + j / 64));
            int m = (int)((mw >> (j % 64)) & 1u);
            int from_a = odd ? !m : m;
            put_bit(x, j, get_bit(seeds + (from_a ? a : b) * W, j));
        }
    }
}

/* -------------------------------------------------------------- screening */

/*
 * T(lambda) = Mean + lambda (Max - Mean) with Mean = Sum / M over the current
 * population and lambda = p / q; a candidate passes iff f > T (strict, as in
 * Fig. 2).  Multiplying through by q*M > 0 keeps it exact:
 *     q*M*f  >  (q - p)*Sum + p*M*Max        (evaluated in __int128).
 * Passer indices are written in ascending order; returns their count.
 */
ORC_API int64_t orc_screen(const int64_t *f, int64_t M, int32_t p, int32_t q, int32_t *idx,
                           int64_t *sum_out, int64_t *max_out)
{
    int64_t sum = 0, mx = f[0];
    for (int64_t c = 0; c < M; c++) {
        sum += f[c];
        if (f[c] > mx) mx = f[c];
    }
    __int128 rhs = (__int128)(q - p) * sum + (__int128)p * M * mx;
    int64_t P = 0;
    for (int64_t c = 0; c < M; c++)
        if ((__int128)q * M * f[c] > rhs) idx[P++] = (int32_t)c;
    *sum_out = sum;
    *max_out = mx;
    return P;
}

/* ----------------------------------------------------------- 1-flip deltas */

/* Delta_i = f(x xor e_i) - f(x), each by a full re-evaluation. */
ORC_API void orc_delta_recompute(int32_t n, const int32_t *Q, const uint64_t *x, int64_t *delta)
{
    int64_t W = words_for(n);
    uint64_t *y = (uint64_t *)malloc((size_t)W * 8);
    int64_t f0 = orc_f(n, Q, x);
    for (int64_t i = 0; i < n; i++) {
        memcpy(y, x, (size_t)W * 8);
        put_bit(y, i, !get_bit(y, i));
        delta[i] = orc_f(n, Q, y) - f0;
    }
    free(y);
}

/* The 1-flip delta in closed form (Glover et al. 2002):
 *   Delta_i = (1 - 2 x_i) (q_ii + 2 sum_{j != i} q_ij x_j). */
ORC_API void orc_delta(int32_t n, const int32_t *Q, const uint64_t *x, int64_t *delta)
{
    for (int64_t i = 0; i < n; i++) {
        int64_t s = Q[i * n + i];
        for (int64_t j = 0; j < n; j++)
            if (j != i && get_bit(x, j)) s += 2 * (int64_t)Q[i * n + j];
        delta[i] = (1 - 2 * get_bit(x, i)) * s;
    }
}

/*
 * Steepest ascent with 1-bit flips (Pseudocode section): repeatedly flip the
 * variable with the largest Delta -- the lowest index among equal maxima -- as
 * long as that Delta is > 0, stopping at a 1-flip local optimum or once
 * max_flips flips were made (max_flips == 0: no cap).  No tabu list, no cycle
 * check.  *f enters as f(x) and leaves as f of the final x.
 * mode 0: after flipping k (old value x_k), Delta_i += 2 q_ik (1-2x_i)(1-2x_k^old)
 *         for i != k and Delta_k = -Delta_k (the one-column update).
 * mode 1: every Delta is recomputed from its definition after each flip.
 * Returns the number of flips made.
 */
ORC_API int64_t orc_ascent(int32_t n, const int32_t *Q, uint64_t *x, int64_t *f, int32_t max_flips,
                           int32_t mode)
{
    int64_t *d = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * 8);
    if (mode == 1) orc_delta_recompute(n, Q, x, d); else orc_delta(n, Q, x, d);
    int64_t flips = 0;
    for (;;) {
        if (max_flips > 0 && flips >= max_flips) break;
        int64_t k = 0;
        for (int64_t i = 1; i < n; i++)
            if (d[i] > d[k]) k = i;
        if (n == 0 || d[k] <= 0) break;
        int old = get_bit(x, k);
        put_bit(x, k, !old);
        *f += d[k];
        flips++;
        if (mode == 1) {
            orc_delta_recompute(n, Q, x, d);
        } else {
            for (int64_t i = 0; i < n; i++)
                if (i != k) d[i] += 2 * (int64_t)Q[i * n + k] * (1 - 2 * get_bit(x, i)) * (1 - 2 * old);
            d[k] = -d[k];
        }
    }
    free(d);
    return flips;
}

/* Ascent of several candidates (rows idx[0..P) of X, f indexed like X);
 * flips[c] receives the flip count.  `threads` only partitions the work. */
ORC_API void orc_ascent_many(int32_t n, const int32_t *Q, uint64_t *X, const int32_t *idx,
                             int64_t P, int64_t *f, int32_t max_flips, int64_t *flips,
                             int32_t threads)
{
    int64_t W = words_for(n);
    if (threads < 1) threads = 1;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (int64_t p = 0; p < P; p++) {
        int64_t c = idx[p];
        flips[c] = orc_ascent(n, Q, X + c * W, f + c, max_flips, 0);
    }
}

/* Starting solution from the partial first derivative (Pseudocode section):
 * x_i = 1 iff the i-th row sum of Q is > 0. */
ORC_API void orc_derivative_start(int32_t n, const int32_t *Q, uint64_t *x)
{
    memset(x, 0, (size_t)words_for(n) * 8);
    for (int64_t i = 0; i < n; i++) {
        int64_t s = 0;
        for (int64_t j = 0; j < n; j++) s += Q[i * n + j];
        put_bit(x, i, s > 0);
    }
}

/* ------------------------------------------------------------ main loop */

typedef struct {
    int64_t M;          /* candidates per generation                           */
    int32_t H;          /* diversification steps per seed (h = 1..H, x' and x'') */
    int32_t lam_num;    /* lambda = lam_num / lam_den                          */
    int32_t lam_den;
    int32_t G;          /* generations                                         */
    int32_t max_flips;  /* 0 = ascend to a 1-flip local optimum                */
    int32_t flags;      /* bit 0: generation-0 seed 0 is the derivative start; */
                        /* bit 1: blending diversification instead of Glover's  */
    uint64_t run_seed;
} orc_params;

typedef struct { int64_t f; int32_t c; } ranked;
static int rank_cmp(const void *a, const void *b)
{
    const ranked *u = (const ranked *)a, *v = (const ranked *)b;
    if (u->f != v->f) return u->f > v->f ? -1 : 1;   /* f descending */
    return u->c < v->c ? -1 : (u->c > v->c);         /* index ascending */
}

/*
 * The multi-start loop of Fig. 2, one generation at a time with M candidates:
 *   1. candidates: Glover diversification of the S = ceil(M / 2H) seeds
 *      (or blending of pairs of them, flags & 2);
 *   2. evaluate f for every candidate;
 *   3. screen with T(lambda) over this generation's Sum and Max;
 *   4. steepest ascent of every passer;
 *   5. UpdateBestAndT: scanning passers by ascending index, the incumbent is
 *      replaced when f_after > f* (strict);
 *   6. seeds of the next generation (reading of Diversify(x, best, i)):
 *      seed 0 = the incumbent, then the ascended passers ranked by f_after
 *      descending and index ascending, then random solutions for the rest.
 * Generation-0 seeds are random (seed 0 the derivative start when flags&1).
 * stats[g*5 + {0..4}] = {Sum, Max, passers, total flips, f* after g}; f* is
 * INT64_MIN while no incumbent exists.  Returns 1 if an incumbent exists.
 * Optional dumps (NULL to skip), per generation g:
 *   f[g*M + c]        f of every candidate before ascent
 *   fa[g*M + c]       f after ascent (passers; others keep f)
 *   pass[g*M + c]     1 iff candidate c passed the screen
 *   xa[(g*M + c)*W]   candidates after ascent
 *   seeds[(g*S)*W]    the S seeds generation g was diversified from
 */
typedef struct {
    int64_t *f, *fa;
    uint8_t *pass;
    uint64_t *xa, *seeds;
} orc_dump;

ORC_API int32_t orc_multistart(int32_t n, const int32_t *Q, const orc_params *pr, int64_t *best_f,
                               uint64_t *best_x, int64_t *stats, const orc_dump *dump,
                               int32_t threads)
{
    const int64_t M = pr->M, H = pr->H, W = words_for(n);
    const int64_t S = (M + 2 * H - 1) / (2 * H);
    uint64_t *seeds = (uint64_t *)calloc((size_t)(S * W), 8);
    uint64_t *X = (uint64_t *)calloc((size_t)(M * W), 8);
    int64_t *f = (int64_t *)calloc((size_t)M, 8);
    int64_t *flips = (int64_t *)calloc((size_t)M, 8);
    int32_t *idx = (int32_t *)calloc((size_t)M, 4);
    ranked *rk = (ranked *)calloc((size_t)M, sizeof(ranked));
    int have_best = 0;
    int64_t bf = INT64_MIN;

    for (int64_t s = 0; s < S; s++) orc_random_solution(n, pr->run_seed, 0, S, s, seeds + s * W);
    if (pr->flags & 1) orc_derivative_start(n, Q, seeds);

    for (int64_t g = 0; g < pr->G; g++) {
        if (dump && dump->seeds) memcpy(dump->seeds + g * S * W, seeds, (size_t)(S * W) * 8);
        if (pr->flags & 2) orc_blend(n, seeds, S, M, g, pr->run_seed, X);
        else orc_diversify(n, seeds, S, (int32_t)H, X, M);
        orc_eval(n, Q, X, M, f, threads);
        if (dump && dump->f) memcpy(dump->f + g * M, f, (size_t)M * 8);
        int64_t sum, mx;
        int64_t P = orc_screen(f, M, pr->lam_num, pr->lam_den, idx, &sum, &mx);
        orc_ascent_many(n, Q, X, idx, P, f, pr->max_flips, flips, threads);
        if (dump && dump->fa) memcpy(dump->fa + g * M, f, (size_t)M * 8);
        if (dump && dump->xa) memcpy(dump->xa + g * M * W, X, (size_t)(M * W) * 8);
        if (dump && dump->pass) {
            memset(dump->pass + g * M, 0, (size_t)M);
            for (int64_t p = 0; p < P; p++) dump->pass[g * M + idx[p]] = 1;
        }
        int64_t tot = 0;
        for (int64_t p = 0; p < P; p++) {
            int64_t c = idx[p];
            tot += flips[c];
            if (!have_best || f[c] > bf) {
                have_best = 1;
                bf = f[c];
                memcpy(best_x, X + c * W, (size_t)W * 8);
            }
            rk[p].f = f[c];
            rk[p].c = (int32_t)c;
        }
        qsort(rk, (size_t)P, sizeof(ranked), rank_cmp);
        stats[g * 5 + 0] = sum;
        stats[g * 5 + 1] = mx;
        stats[g * 5 + 2] = P;
        stats[g * 5 + 3] = tot;
        stats[g * 5 + 4] = bf;
        /* next generation's seeds */
        int64_t used = 0;
        if (have_best) memcpy(seeds, best_x, (size_t)W * 8);
        else orc_random_solution(n, pr->run_seed, g + 1, S, 0, seeds);
        for (int64_t s = 1; s < S; s++) {
            if (used < P) memcpy(seeds + s * W, X + (int64_t)rk[used++].c * W, (size_t)W * 8);
            else orc_random_solution(n, pr->run_seed, g + 1, S, s, seeds + s * W);
        }
    }
    *best_f = bf;
    free(seeds); free(X); free(f); free(flips); free(idx); free(rk);
    return have_best;
}

/* -------------------------------------------------- sequential main loop */

typedef struct {
    int64_t iterations; /* I: iterations of the main loop                      */
    int64_t samples;    /* random solutions whose mean objective is Mean       */
    int64_t H;          /* cycle of the diversification step                   */
    int32_t lam_num;    /* lambda = lam_num / lam_den                          */
    int32_t lam_den;
    int32_t max_flips;  /* 0 = ascend to a 1-flip local optimum                */
    int32_t pad_;
    uint64_t run_seed;
} orc_seq_params;

typedef struct {
    int64_t best_f;
    int32_t have_best;
    int32_t pad_;
    int64_t sample_sum;   /* Sum over the samples (Mean = sample_sum / samples) */
    int64_t start_f;      /* f of the derivative start                          */
    int64_t passers;      /* iterations whose candidate passed the screen       */
    int64_t flips;        /* flips of all ascents                               */
    int64_t improvements; /* times the incumbent was replaced                   */
} orc_seq_out;

/*
 * The main loop of Fig. 2 as printed: one candidate per iteration.
 *   Mean: average objective of `samples` random solutions (EvaluateRandomStarts;
 *         sample s is orc_random_solution(run_seed, g = 0, S = samples, s));
 *   starting solution x0: the first-derivative solution; Max starts at f(x0)
 *         (CalculateFirstDerivativeSolution, CalculateT);
 *   iteration 0 takes x0 itself; iteration i >= 1 diversifies the incumbent
 *         (x0 while there is none) with Glover's generator, the step tied to
 *         the loop counter: c = i - 1, h = (c / 2 mod H) + 1, variables
 *         j = 0, h, 2h, ... flipped, and the result complemented when c is odd;
 *   screen: f > T = Mean + lambda (Max - Mean), decided exactly as
 *         den * samples * f > (den - num) * Sum + num * samples * Max;
 *   a passer is ascended (steepest 1-flip, max_flips) and replaces the
 *         incumbent when its f is larger (strictly) or there is none; then
 *         Max = the new incumbent value (UpdateBestAndT).
 * The readings: lambda is a fixed rational (the printed lambda = Max / Mean
 * would put T above Max); the incumbent is the solution diversified.
 * f_dump (I entries, may be NULL) receives each iteration's f before ascent;
 * history (history_cap pairs, may be NULL) the (iteration, value) of each
 * replacement of the incumbent, the first history_cap of them.
 */
ORC_API void orc_sequential(int32_t n, const int32_t *Q, const orc_seq_params *pr, orc_seq_out *out,
                            uint64_t *best_x, int64_t *f_dump, int64_t *history, int64_t history_cap,
                            int32_t threads)
{
    const int64_t W = words_for(n), Ms = pr->samples;
    uint64_t *X = (uint64_t *)calloc((size_t)(Ms * W), 8);
    int64_t *fs = (int64_t *)calloc((size_t)Ms, 8);
    uint64_t *x0 = (uint64_t *)calloc((size_t)W, 8);
    uint64_t *x = (uint64_t *)calloc((size_t)W, 8);
    memset(out, 0, sizeof(*out));

    /* Mean from random solutions */
    for (int64_t s = 0; s < Ms; s++) orc_random_solution(n, pr->run_seed, 0, Ms, s, X + s * W);
    orc_eval(n, Q, X, Ms, fs, threads);
    int64_t sum = 0;
    for (int64_t s = 0; s < Ms; s++) sum += fs[s];
    /* starting solution and the initial Max */
    orc_derivative_start(n, Q, x0);
    const int64_t f0 = orc_f(n, Q, x0);
    int64_t mx = f0, bf = INT64_MIN;
    int have_best = 0;

    for (int64_t i = 0; i < pr->iterations; i++) {
        const uint64_t *seed = have_best ? best_x : x0;
        memcpy(x, seed, (size_t)W * 8);
        if (i > 0) {
            const int64_t c = i - 1;
            const int64_t h = (c / 2) % pr->H + 1;
            for (int64_t j = 0; j < n; j += h) put_bit(x, j, !get_bit(x, j));
            if (c % 2)
                for (int64_t j = 0; j < n; j++) put_bit(x, j, !get_bit(x, j));
        }
        int64_t fx = orc_f(n, Q, x);
        if (f_dump) f_dump[i] = fx;
        const __int128 lhs = (__int128)pr->lam_den * Ms * fx;
        const __int128 rhs = (__int128)(pr->lam_den - pr->lam_num) * sum + (__int128)pr->lam_num * Ms * mx;
        if (!(lhs > rhs)) continue;
        out->passers++;
        out->flips += orc_ascent(n, Q, x, &fx, pr->max_flips, 0);
        if (!have_best || fx > bf) {
            have_best = 1;
            bf = fx;
            memcpy(best_x, x, (size_t)W * 8);
            mx = bf;
            if (history && out->improvements < history_cap) {
                history[2 * out->improvements] = i;
                history[2 * out->improvements + 1] = fx;
            }
            out->improvements++;
        }
    }
    out->best_f = bf;
    out->have_best = have_best;
    out->sample_sum = sum;
    out->start_f = f0;
    free(X); free(fs); free(x0); free(x);
}

/* ------------------------------------------------------- path relinking */

/*
 * Path relinking, the improvement phase the paper names as the one to follow
 * its initial phase (Introduction, Pseudocode section, Conclusions; Glover,
 * Laguna & Marti 2000), which the paper does not implement.  The rule read
 * here is greedy relinking:
 *   D = the variables where the initiating solution x and the guiding one
 *       differ; from x, repeatedly flip the k in D with the largest
 *       Delta_k = f(x xor e_k) - f(x) (the lowest k on ties), improving or
 *       not, and remove k from D, for |D| - 1 steps (the last flip would reach
 *       the guiding solution, which is not an intermediate);
 *   the result is the intermediate of largest f, the earliest on ties (strict
 *       comparison), and the number of steps to it; none when |D| <= 1.
 * mode 0 keeps the deltas by the one-column update of orc_ascent, mode 1
 * recomputes them from their definition after every flip.
 * Returns the steps to the best intermediate (0: none); x_mid and f_mid
 * receive it.
 */
ORC_API int64_t orc_relink_path(int32_t n, const int32_t *Q, const uint64_t *x_init, const uint64_t *x_guide,
                                int32_t mode, uint64_t *x_mid, int64_t *f_mid)
{
    const int64_t W = words_for(n);
    uint64_t *x = (uint64_t *)malloc((size_t)W * 8);
    uint8_t *free_ = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t *d = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * 8);
    memcpy(x, x_init, (size_t)W * 8);
    int64_t nd = 0;
    for (int64_t j = 0; j < n; j++) {
        free_[j] = get_bit(x_init, j) != get_bit(x_guide, j);
        nd += free_[j];
    }
    if (mode == 1) orc_delta_recompute(n, Q, x, d); else orc_delta(n, Q, x, d);
    int64_t fx = orc_f(n, Q, x), best = INT64_MIN, best_step = 0;
    for (int64_t s = 1; s < nd; s++) {
        int64_t k = -1;
        for (int64_t i = 0; i < n; i++)
            if (free_[i] && (k < 0 || d[i] > d[k])) k = i;
        const int old = get_bit(x, k);
        put_bit(x, k, !old);
        free_[k] = 0;
        fx += d[k];
        if (fx > best) {
            best = fx;
            best_step = s;
            memcpy(x_mid, x, (size_t)W * 8);
        }
        if (mode == 1) {
            orc_delta_recompute(n, Q, x, d);
        } else {
            for (int64_t i = 0; i < n; i++)
                if (i != k) d[i] += 2 * (int64_t)Q[i * n + k] * (1 - 2 * get_bit(x, i)) * (1 - 2 * old);
            d[k] = -d[k];
        }
    }
    if (best_step == 0) memcpy(x_mid, x_init, (size_t)W * 8);
    *f_mid = best;
    free(x); free(free_); free(d);
    return best_step;
}

/*
 * Relinking of P pairs (initiating, guiding) = (elite[pairs[2p]], elite[pairs[2p+1]]):
 * X_out row p, f_mid[p], steps[p] from orc_relink_path; then the steepest ascent
 * (orc_ascent, max_flips) from the intermediate gives f_out[p] and the final
 * row.  Paths without an intermediate keep the initiating row, and
 * f_mid = f_out = INT64_MIN.  `threads` only partitions the paths.
 */
ORC_API void orc_relink_many(int32_t n, const int32_t *Q, const uint64_t *elite, const int32_t *pairs, int64_t P,
                             int32_t max_flips, uint64_t *X_out, int64_t *f_mid, int64_t *f_out, int64_t *steps,
                             int32_t threads)
{
    const int64_t W = words_for(n);
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
    for (int64_t p = 0; p < P; p++) {
        uint64_t *xo = X_out + p * W;
        steps[p] = orc_relink_path(n, Q, elite + (int64_t)pairs[2 * p] * W, elite + (int64_t)pairs[2 * p + 1] * W, 0,
                                   xo, &f_mid[p]);
        f_out[p] = f_mid[p];
        if (steps[p] > 0) orc_ascent(n, Q, xo, &f_out[p], max_flips, 0);
    }
}
