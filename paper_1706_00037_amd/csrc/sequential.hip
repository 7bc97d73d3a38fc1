// The main loop of Fig. 2 as printed: one candidate per iteration (Pseudocode
// section).  Mean comes from random solutions, Max starts at the value of the
// first-derivative solution x0, iteration 0 takes x0 and iteration i >= 1
// diversifies the incumbent (x0 while there is none) with Glover's generator,
// step h = ((i-1)/2 mod H) + 1, complemented for odd i-1; a candidate above
// T = Mean + lambda (Max - Mean) is ascended and, if it beats the incumbent,
// replaces it and becomes Max.
//
// The chain is sequential only through the incumbent: every candidate up to the
// next replacement is built from the same seed.  The device therefore works a
// window of iterations at once: build their candidates from the current
// incumbent (seq_gen), evaluate them with the matrix-core row dot, screen them
// in order (seq_screen), initialise and ascend every passer in parallel, and
// commit (seq_commit) the iterations up to and including the first passer that
// replaces the incumbent; the look-ahead past it is discarded and rebuilt from
// the new incumbent in the next window.  What is committed is exactly what the
// one-at-a-time loop does, for every window size.  The window restarts at one
// evaluation tile (256 candidates) after a replacement and doubles, up to the
// caller's batch, while none occurs.
//
// Every launch of a window reads its sizes from device state, so a group of
// windows is captured once as a HIP graph and replayed; windows after the last
// iteration do nothing.  The host reads the state back one group behind.  The
// commit stamps each replacement of the incumbent with the device's
// constant-rate wall clock, so times to target have the resolution of a window.
#include <chrono>
#include <new>
#include <vector>

#include "plan.h"

namespace {

constexpr int GEN_THR = 256;
constexpr int SCR_THR = 1024;
constexpr int SCR_PER = 8;
constexpr int COM_THR = 256;
constexpr int64_t MIN_WINDOW = 256;   // one evaluation tile of candidates
constexpr int WINDOWS_PER_GROUP = 8;  // windows per graph launch
constexpr int64_t DEFAULT_BATCH = 1024;  // measured best of 512..8192 at n = 2500 and 7000

struct SeqState {
    int64_t sum;        // Sum of the samples' objectives
    int64_t start_f;    // f(x0)
    int64_t max;        // Max of T: f(x0), then the incumbent's value
    int64_t best_f;
    int64_t next;       // first iteration of the next window
    int64_t valid;      // iterations in the next window (0 once the loop is done)
    int64_t window;     // size allowed for the next window
    int64_t npass;      // passers of the current window
    int64_t passers, flips, improvements, windows, evaluated;
    uint64_t t0, t_last;  // device wall clock at the start of the loop and at the last commit
    int32_t have_best, done;
};

struct SeqArgs {
    SeqState *st;
    int32_t n, W;
    int64_t I, B, H, Ms;
    int32_t lam_num, lam_den;
    uint64_t run_seed;
    const uint64_t *x0;   // [W] first-derivative solution
    uint64_t *X;          // [rows][W]: samples then x0 at set-up; the window's candidates
    int64_t *f;           // [rows] objectives (passers: after ascent)
    int64_t *f0;          // [B] the window's objectives before ascent
    int32_t *idx;         // [B] the window's passers, ascending
    int32_t *flips;       // [B] flips per window row
    uint64_t *best_x;     // [W]
    int64_t *hist;        // [hist_cap][3]: iteration, value, device wall clock
    int64_t hist_cap;
    int64_t *f_dump;      // [I] or null
};

template <int THR>
__device__ int64_t block_sum(int64_t v)
{
    __shared__ int64_t part[THR / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();  // earlier readers of part are done
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t s = 0;
    for (int i = 0; i < THR / 64; i++) s += part[i];
    return s;
}

__device__ inline uint64_t tail_mask(int32_t n, int32_t w, uint64_t v)
{
    const int32_t tail = n - 64 * w;
    return tail < 64 ? v & ((1ull << tail) - 1ull) : v;
}

// Rows 0..Ms-1: the samples (word w of sample s is SplitMix64 output s W + w);
// row Ms: x0.
__global__ __launch_bounds__(GEN_THR) void seq_samples(SeqArgs a)
{
    const int64_t id = (int64_t)blockIdx.x * GEN_THR + threadIdx.x;
    if (id >= (a.Ms + 1) * a.W) return;
    const int64_t s = id / a.W;
    const int32_t w = (int32_t)(id - s * a.W);
    a.X[id] = s < a.Ms ? tail_mask(a.n, w, ubqp_splitmix64(a.run_seed, (uint64_t)id)) : a.x0[w];
}

__global__ __launch_bounds__(COM_THR) void seq_setup(SeqArgs a)
{
    int64_t s = 0;
    for (int64_t i = threadIdx.x; i < a.Ms; i += COM_THR) s += a.f[i];
    s = block_sum<COM_THR>(s);
    if (threadIdx.x == 0) {
        SeqState *st = a.st;
        st->sum = s;
        st->start_f = a.f[a.Ms];
        st->max = st->start_f;
        st->best_f = INT64_MIN;
        st->have_best = 0;
        st->next = 0;
        st->window = MIN_WINDOW < a.B ? MIN_WINDOW : a.B;
        st->valid = st->window < a.I ? st->window : a.I;
        st->npass = 0;
        st->passers = st->flips = st->improvements = st->windows = st->evaluated = 0;
        st->done = 0;
    }
}

// Start of the loop on the device wall clock.
__global__ void seq_stamp(SeqState *st)
{
    if (threadIdx.x == 0) st->t0 = st->t_last = wall_clock64();
}

// Row b of the window: the candidate of iteration next + b.
__global__ __launch_bounds__(GEN_THR) void seq_gen(SeqArgs a)
{
    const SeqState *st = a.st;
    const int64_t id = (int64_t)blockIdx.x * GEN_THR + threadIdx.x;
    if (id >= st->valid * a.W) return;
    const int64_t b = id / a.W;
    const int32_t w = (int32_t)(id - b * a.W);
    const int64_t it = st->next + b;
    uint64_t v = (st->have_best ? a.best_x : a.x0)[w];
    if (it > 0) {
        const int64_t c = it - 1;
        const int64_t h = (c >> 1) % a.H + 1;
        // variables j = 0, h, 2h, ... inside word w: bits k >= k0 in steps of h
        const int64_t ph = (64 * (int64_t)w) % h;
        uint64_t m = 0;
        for (int64_t k = ph == 0 ? 0 : h - ph; k < 64; k += h) m |= 1ull << k;
        v ^= m;
        if (c & 1) v = ~v;
        v = tail_mask(a.n, w, v);
    }
    a.X[id] = v;
}

// Passers of the window in ascending order: f > T, decided as
// den * samples * f > (den - num) * Sum + num * samples * Max.  Keeps each
// row's objective before the ascent in f0.
__global__ __launch_bounds__(SCR_THR) void seq_screen(SeqArgs a)
{
    __shared__ int32_t wtot[SCR_THR / 64];
    __shared__ int64_t carry;
    SeqState *st = a.st;
    const int64_t valid = st->valid;
    const __int128 rhs = (__int128)(a.lam_den - a.lam_num) * st->sum + (__int128)a.lam_num * a.Ms * st->max;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t base = 0; base < valid; base += SCR_THR * SCR_PER) {
        const int64_t c0 = base + (int64_t)threadIdx.x * SCR_PER;
        uint32_t bits = 0;
        for (int i = 0; i < SCR_PER; i++) {
            const int64_t c = c0 + i;
            if (c < valid) {
                const int64_t fv = a.f[c];
                a.f0[c] = fv;
                if ((__int128)a.lam_den * a.Ms * fv > rhs) bits |= 1u << i;
            }
        }
        const int mine = __popc(bits);
        int incl = mine;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wtot[wv] = incl;
        __syncthreads();
        int64_t pos = carry + incl - mine;
        int64_t total = 0;
        for (int i = 0; i < SCR_THR / 64; i++) {
            if (i < wv) pos += wtot[i];
            total += wtot[i];
        }
        for (int i = 0; i < SCR_PER; i++)
            if (bits & (1u << i)) a.idx[pos++] = (int32_t)(c0 + i);
        __syncthreads();  // carry and wtot read by every thread
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) st->npass = carry;
}

// Commit the window up to its first passer that replaces the incumbent (or the
// whole window), and size the next one.
__global__ __launch_bounds__(COM_THR) void seq_commit(SeqArgs a)
{
    __shared__ int32_t first;
    SeqState *st = a.st;
    const int64_t valid = st->valid;
    if (valid == 0) return;
    const int64_t np = st->npass;
    const int32_t have = st->have_best;
    const int64_t bf = st->best_f;
    const int64_t next = st->next;
    if (threadIdx.x == 0) first = (int32_t)np;
    __syncthreads();
    for (int64_t p = threadIdx.x; p < np; p += COM_THR)
        if (!have || a.f[a.idx[p]] > bf) atomicMin(&first, (int32_t)p);
    __syncthreads();
    const int64_t pf = first;
    const bool found = pf < np;
    const int64_t cf = found ? a.idx[pf] : -1;
    const int64_t committed = found ? cf + 1 : valid;
    const int64_t npassed = found ? pf + 1 : np;
    int64_t fl = 0;
    for (int64_t p = threadIdx.x; p < npassed; p += COM_THR) fl += a.flips[a.idx[p]];
    fl = block_sum<COM_THR>(fl);
    if (a.f_dump)
        for (int64_t b = threadIdx.x; b < committed; b += COM_THR) a.f_dump[next + b] = a.f0[b];
    if (found)
        for (int32_t w = threadIdx.x; w < a.W; w += COM_THR) a.best_x[w] = a.X[cf * a.W + w];
    if (threadIdx.x == 0) {
        const uint64_t now = wall_clock64();
        st->passers += npassed;
        st->flips += fl;
        st->windows += 1;
        st->t_last = now;
        st->evaluated += valid;
        int64_t win = st->window;
        if (found) {
            const int64_t v = a.f[cf];
            st->best_f = v;
            st->have_best = 1;
            st->max = v;
            const int64_t k = st->improvements;
            if (k < a.hist_cap) {
                a.hist[3 * k] = next + cf;
                a.hist[3 * k + 1] = v;
                a.hist[3 * k + 2] = (int64_t)now;
            }
            st->improvements = k + 1;
            win = MIN_WINDOW < a.B ? MIN_WINDOW : a.B;
        } else {
            win = 2 * win < a.B ? 2 * win : a.B;
        }
        st->window = win;
        const int64_t nx = next + committed;
        const int64_t left = a.I - nx;
        st->next = nx;
        st->valid = left <= 0 ? 0 : (left < win ? left : win);
        st->done = left <= 0 ? 1 : 0;
    }
}

// Device memory of one call: state, rows, window buffers, the Delta workspace,
// history.
struct SeqRun {
    ubqp_ctx *ctx = nullptr;
    char *mem = nullptr;
    SeqState *pin = nullptr;  // two page-locked copies of the state
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t start = nullptr, end = nullptr, copied[2] = {};

    ~SeqRun()
    {
        (void)hipStreamSynchronize(ctx->stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        for (hipEvent_t e : {start, end, copied[0], copied[1]})
            if (e) (void)hipEventDestroy(e);
        if (pin) (void)hipHostFree(pin);
        if (mem) (void)hipFree(mem);
    }
};

hipError_t queue_window(hipStream_t s, const SeqArgs &a, const EvalArgs &ev, int variant, const EvalArgs &yr,
                        const AscArgs &as)
{
    hipError_t e;
    hipLaunchKernelGGL(seq_gen, dim3((unsigned)((a.B * a.W + GEN_THR - 1) / GEN_THR)), dim3(GEN_THR), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = ubqp_launch_eval_v(s, ev, variant)) != hipSuccess) return e;
    hipLaunchKernelGGL(seq_screen, dim3(1), dim3(SCR_THR), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = ubqp_launch_yrows(s, yr)) != hipSuccess) return e;
    if ((e = ubqp_launch_ascent(s, as)) != hipSuccess) return e;
    hipLaunchKernelGGL(seq_commit, dim3(1), dim3(COM_THR), 0, s, a);
    return hipGetLastError();
}

}  // namespace

extern "C" int ubqp_sequential(ubqp_ctx *ctx, const ubqp_problem *p, const ubqp_seq_params *sp,
                               ubqp_seq_result *r)
{
    if (!ctx || !p || !sp || !r) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    if (sp->iterations < 1) return ubqp_fail(ctx, UBQP_EINVAL, "iterations < 1");
    if (sp->samples < 1 || sp->samples > UBQP_SEQ_MAX_SAMPLES)
        return ubqp_fail(ctx, UBQP_EINVAL, "samples=%d outside [1, %d]", sp->samples, UBQP_SEQ_MAX_SAMPLES);
    if (sp->H < 0) return ubqp_fail(ctx, UBQP_EINVAL, "H < 0");
    if (sp->lam_den < 1 || sp->lam_num < 0 || sp->lam_num > sp->lam_den)
        return ubqp_fail(ctx, UBQP_EINVAL, "lambda=%d/%d outside [0, 1]", sp->lam_num, sp->lam_den);
    if (sp->max_flips < 0) return ubqp_fail(ctx, UBQP_EINVAL, "max_flips < 0");
    if (sp->batch < 0 || sp->batch > UBQP_SEQ_MAX_BATCH)
        return ubqp_fail(ctx, UBQP_EINVAL, "batch=%d outside [0, %d]", sp->batch, UBQP_SEQ_MAX_BATCH);
    if (sp->flags & ~UBQP_NO_GRAPH) return ubqp_fail(ctx, UBQP_EINVAL, "flags other than UBQP_NO_GRAPH");
    if (!(sp->time_budget_ms >= 0.0)) return ubqp_fail(ctx, UBQP_EINVAL, "time_budget_ms < 0");
    if (r->history_cap < 0) return ubqp_fail(ctx, UBQP_EINVAL, "history_cap < 0");
    UBQP_TRY(ubqp_set_device(ctx));

    const int64_t I = sp->iterations, Ms = sp->samples, W = p->W;
    const int64_t B = sp->batch ? sp->batch : DEFAULT_BATCH;
    const int64_t rows = Ms + 1 > B ? Ms + 1 : B;
    const bool want_hist = r->history_host || r->history_ms_host;
    const int64_t hist_cap = want_hist ? (r->history_cap < I ? r->history_cap : I) : 0;

    SeqRun run;
    run.ctx = ctx;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += ubqp_align256(bytes); return o; };
    const size_t o_st = take(sizeof(SeqState)), o_X = take((size_t)(rows * W * 8)), o_f = take((size_t)rows * 8);
    const size_t o_f0 = take((size_t)B * 8), o_idx = take((size_t)B * 4), o_fl = take((size_t)B * 4);
    const size_t o_bx = take((size_t)W * 8), o_h = take((size_t)(hist_cap > 0 ? hist_cap : 1) * 24);
    const size_t o_Y = take((size_t)p->planes * B * p->n_pad * 4);
    if (hipMalloc(&run.mem, off) != hipSuccess) {
        (void)hipGetLastError();
        run.mem = nullptr;
        return ubqp_fail(ctx, UBQP_ENOMEM, "sequential run: %zu bytes of device memory", off);
    }
    UBQP_HIP_TRY(ctx, hipHostMalloc((void **)&run.pin, 2 * sizeof(SeqState), hipHostMallocDefault));
    for (hipEvent_t *e : {&run.start, &run.end, &run.copied[0], &run.copied[1]})
        UBQP_HIP_TRY(ctx, hipEventCreate(e));

    SeqArgs a{};
    a.st = (SeqState *)(run.mem + o_st);
    a.n = p->n;
    a.W = (int32_t)W;
    a.I = I;
    a.B = B;
    a.H = sp->H ? sp->H : p->n;
    a.Ms = Ms;
    a.lam_num = sp->lam_num;
    a.lam_den = sp->lam_den;
    a.run_seed = sp->run_seed;
    a.x0 = p->deriv_x;
    a.X = (uint64_t *)(run.mem + o_X);
    a.f = (int64_t *)(run.mem + o_f);
    a.f0 = (int64_t *)(run.mem + o_f0);
    a.idx = (int32_t *)(run.mem + o_idx);
    a.flips = (int32_t *)(run.mem + o_fl);
    a.best_x = (uint64_t *)(run.mem + o_bx);
    a.hist = (int64_t *)(run.mem + o_h);
    a.hist_cap = hist_cap;
    a.f_dump = r->f_dump_d;
    int32_t *Y = (int32_t *)(run.mem + o_Y);
    hipStream_t st = ctx->stream;

    // set-up: Mean over the samples and f(x0) in one evaluation
    hipLaunchKernelGGL(seq_samples, dim3((unsigned)(((Ms + 1) * W + GEN_THR - 1) / GEN_THR)), dim3(GEN_THR), 0, st,
                       a);
    UBQP_HIP_TRY(ctx, hipGetLastError());
    UBQP_HIP_TRY(ctx, ubqp_launch_eval_v(st, ubqp_eval_args(p, a.X, Ms + 1, a.f), ubqp_eval_variant_for(p, Ms + 1)));
    hipLaunchKernelGGL(seq_setup, dim3(1), dim3(COM_THR), 0, st, a);
    UBQP_HIP_TRY(ctx, hipGetLastError());

    // one window: the row dot over the window's rows, then Delta init and ascent of its passers
    EvalArgs ev = ubqp_eval_args(p, a.X, B, a.f);
    ev.nrows_d = &a.st->valid;
    const int variant = ubqp_eval_variant_for(p, B);
    EvalArgs yr = ubqp_yrows_args(p, a.X, B, a.idx, &a.st->npass, 0, B, Y);
    AscArgs as = ubqp_ascent_args(p, a.X, B, a.idx, &a.st->npass, 0, B, Y, a.f, sp->max_flips, a.flips,
                                  ctx->err_flag);
    ubqp_split_dinit(yr, as, UBQP_SPLIT_TARGET);
    const bool use_graph = !(sp->flags & UBQP_NO_GRAPH);
    if (use_graph) {
        UBQP_HIP_TRY(ctx, hipStreamCreateWithFlags(&run.cap, hipStreamNonBlocking));
        UBQP_HIP_TRY(ctx, hipStreamBeginCapture(run.cap, hipStreamCaptureModeThreadLocal));
        hipError_t qe = hipSuccess;
        for (int k = 0; k < WINDOWS_PER_GROUP && qe == hipSuccess; k++) qe = queue_window(run.cap, a, ev, variant, yr, as);
        const hipError_t ce = hipStreamEndCapture(run.cap, &run.graph);
        UBQP_HIP_TRY(ctx, qe);
        UBQP_HIP_TRY(ctx, ce);
        UBQP_HIP_TRY(ctx, hipGraphInstantiateWithFlags(&run.exec, run.graph, 0));
    }

    UBQP_HIP_TRY(ctx, hipEventRecord(run.start, st));
    hipLaunchKernelGGL(seq_stamp, dim3(1), dim3(64), 0, st, a.st);
    UBQP_HIP_TRY(ctx, hipGetLastError());
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t max_groups = I / WINDOWS_PER_GROUP + 3;  // every window commits at least one iteration
    for (int64_t g = 0;; g++) {
        if (g > max_groups) return ubqp_fail(ctx, UBQP_EDEVICE, "sequential loop did not finish");
        if (use_graph) {
            UBQP_HIP_TRY(ctx, hipGraphLaunch(run.exec, st));
        } else {
            for (int k = 0; k < WINDOWS_PER_GROUP; k++) UBQP_HIP_TRY(ctx, queue_window(st, a, ev, variant, yr, as));
        }
        UBQP_HIP_TRY(ctx, hipMemcpyAsync(run.pin + (g & 1), a.st, sizeof(SeqState), hipMemcpyDeviceToHost, st));
        UBQP_HIP_TRY(ctx, hipEventRecord(run.copied[g & 1], st));
        if (g == 0) continue;
        // the state after the previous group (this group is already queued behind it)
        UBQP_HIP_TRY(ctx, hipEventSynchronize(run.copied[(g - 1) & 1]));
        if (run.pin[(g - 1) & 1].done) break;
        if (sp->time_budget_ms > 0.0 &&
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() >=
                sp->time_budget_ms)
            break;
    }
    UBQP_HIP_TRY(ctx, hipEventRecord(run.end, st));
    UBQP_HIP_TRY(ctx, hipStreamSynchronize(st));
    UBQP_TRY(ubqp_check_flag(ctx));

    SeqState hs;
    UBQP_HIP_TRY(ctx, hipMemcpy(&hs, a.st, sizeof(SeqState), hipMemcpyDeviceToHost));
    r->best_f = hs.best_f;
    r->have_best = hs.have_best;
    r->iterations_done = hs.next;
    r->sample_sum = hs.sum;
    r->start_f = hs.start_f;
    r->passers = hs.passers;
    r->flips = hs.flips;
    r->improvements = hs.improvements;
    r->windows = hs.windows;
    r->evaluated = hs.evaluated;
    float ms = 0.f;
    UBQP_HIP_TRY(ctx, hipEventElapsedTime(&ms, run.start, run.end));
    r->ms = ms;
    int clock_khz = 0;
    UBQP_HIP_TRY(ctx, hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, ctx->device));
    if (clock_khz <= 0) return ubqp_fail(ctx, UBQP_EDEVICE, "device wall clock rate unknown");
    r->ms_device = (double)(hs.t_last - hs.t0) / clock_khz;
    if (r->best_x_host) UBQP_HIP_TRY(ctx, hipMemcpy(r->best_x_host, a.best_x, (size_t)W * 8, hipMemcpyDeviceToHost));
    const int64_t kept = hs.improvements < hist_cap ? hs.improvements : hist_cap;
    if (kept > 0) {
        std::vector<int64_t> h((size_t)(3 * kept));
        UBQP_HIP_TRY(ctx, hipMemcpy(h.data(), a.hist, h.size() * 8, hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < kept; k++) {
            if (r->history_host) {
                r->history_host[2 * k] = h[3 * k];
                r->history_host[2 * k + 1] = h[3 * k + 1];
            }
            if (r->history_ms_host) r->history_ms_host[k] = (double)((uint64_t)h[3 * k + 2] - hs.t0) / clock_khz;
        }
    }
    return UBQP_OK;
}
