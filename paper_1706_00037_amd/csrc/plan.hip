// C ABI of libubqp, part 2: the multi-start loop of Fig. 2 for one instance (a
// run) or many instances advanced together (a batch).
//
// A generation plan owns the device state of a fixed set of instances and the
// launch tables of one generation (plan.h).  Nothing in a generation's launch
// sequence depends on host values that change between generations (the
// generation index and passer counts live on the device), so the sequence is
// captured once as a HIP graph and replayed.  A run is a plan of one instance:
// the batched and the single path execute the same kernels.
#include <algorithm>
#include <map>
#include <new>
#include <utility>

#include "plan.h"

InstLayout ubqp_inst_layout(const ubqp_problem *p, const ubqp_params *pr)
{
    InstLayout L{};
    const int64_t M = pr->M, W = p->W;
    L.S = (M + 2 * pr->H - 1) / (2 * pr->H);
    const int64_t row_bytes = (int64_t)p->planes * p->n_pad * 4;
    const int64_t fit = UBQP_DELTA_WS_BYTES / row_bytes / 256 * 256;
    L.cap = M <= fit ? M : (fit > 256 ? fit : 256);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += ubqp_align256(bytes); return o; };
    L.seeds = take((size_t)(L.S * W * 8));
    L.X = take((size_t)(M * W * 8));
    L.f = take((size_t)M * 8);
    L.flips = take((size_t)M * 4);
    L.idx = take((size_t)M * 4);
    L.oidx = take((size_t)M * 4);
    L.rank = take((size_t)M * 4);
    L.scal = take(sizeof(ubqp_scal));
    L.bestx = take((size_t)W * 8);
    L.stats = take((size_t)pr->G * 5 * 8);
    L.part = take(ubqp_screen_partials_bytes(M));
    L.err = take(sizeof(int32_t));
    L.Y = take((size_t)p->planes * L.cap * p->n_pad * 4);
    L.total = off;
    return L;
}

void GenTables::build(const std::vector<InstRef> &inst, const std::vector<char> *join)
{
    count = (int)inst.size();
    for (const InstRef &r : inst) {
        const ubqp_problem *p = r.p;
        const ubqp_params &pr = r.pr;
        const InstLayout &L = r.L;
        uint64_t *seeds = r.at<uint64_t>(L.seeds), *X = r.at<uint64_t>(L.X);
        int64_t *f = r.at<int64_t>(L.f);
        int32_t *idx = r.at<int32_t>(L.idx), *flips = r.at<int32_t>(L.flips);
        ubqp_scal *sc = r.at<ubqp_scal>(L.scal);
        DivArgs d{};
        d.seeds = seeds;
        d.n = p->n;
        d.W = p->W;
        d.H = pr.H;
        d.X = X;
        d.total = pr.M * p->W;
        d.blend = (pr.flags & UBQP_BLEND) ? 1 : 0;
        d.M = pr.M;
        d.S = L.S;
        d.run_seed = pr.run_seed;
        d.scal = sc;
        div.add(d, ubqp_div_blocks(d));
        EvalArgs ea = ubqp_eval_args(p, X, pr.M, f);
        einit.add(ea, ubqp_eval_init_blocks(ea));
        const int variant = ubqp_eval_variant_for(p, pr.M);
        ubqp_eval_set_variant(ea, variant);
        size_t gi = 0;
        while (gi < ev.size() && ev[gi].variant != variant) gi++;
        if (gi == ev.size()) ev.push_back(EvalGroup{variant, {}});
        ev[gi].t.add(ea, ubqp_eval_tiles(ea));
        const ScreenArgs sa = ubqp_screen_args(f, pr.M, pr.lam_num, pr.lam_den, idx, &sc->npass, sc->sum_max,
                                               r.at<void>(L.part));
        scr.add(sa, sa.nblk);
        ord.add(OrdArgs{f, idx, &sc->npass, r.at<int32_t>(L.oidx)}, 1);
        if (r.dump) has_dump = true;
        const SelArgs sl = ubqp_sel_args(p->n, pr.M, L.S, pr.run_seed, X, f, flips, idx, r.at<int32_t>(L.rank), sc,
                                         r.at<uint64_t>(L.bestx), seeds, r.at<int64_t>(L.stats),
                                         (pr.flags & UBQP_DERIV_START) ? p->deriv_x : nullptr, r.dump);
        sel_cand.add(sl, ubqp_cand_blocks(sl));
        sel_rank.add(sl, ubqp_rank_blocks(sl));
        sel_seed.add(sl, ubqp_seed_blocks(sl));
        if (!join || (*join)[(size_t)(&r - inst.data())]) init.add(sl, ubqp_seed_blocks(sl));
    }
    std::map<std::pair<int, int>, int> group_lane;
    int64_t max_chunks = 0;
    for (const InstRef &r : inst) max_chunks = std::max(max_chunks, (r.pr.M + r.L.cap - 1) / r.L.cap);
    for (int64_t j = 0; j < max_chunks; j++) {
        std::map<std::pair<int, int>, Chunk> groups;
        // instances per (planes, nb) group of this chunk offset
        std::map<std::pair<int, int>, int> members;
        for (const InstRef &r : inst)
            if (r.pr.M > j * r.L.cap) members[{r.p->planes, (int)((r.p->n_pad + 1023) / 1024)}]++;
        for (const InstRef &r : inst) {
            const ubqp_problem *p = r.p;
            const ubqp_params &pr = r.pr;
            const InstLayout &L = r.L;
            const int64_t off = j * L.cap;
            if (pr.M <= off) continue;
            const int64_t cap = std::min<int64_t>(pr.M - off, L.cap);
            uint64_t *X = r.at<uint64_t>(L.X);
            // the ascent takes the passers in the order list (lowest objective first)
            int32_t *idx = r.at<int32_t>(L.oidx), *Y = r.at<int32_t>(L.Y);
            ubqp_scal *sc = r.at<ubqp_scal>(L.scal);
            EvalArgs yr = ubqp_yrows_args(p, X, pr.M, idx, &sc->npass, off, cap, Y);
            AscArgs as = ubqp_ascent_args(p, X, pr.M, idx, &sc->npass, off, cap, Y, r.at<int64_t>(L.f),
                                          pr.max_flips, r.at<int32_t>(L.flips), r.err);
            const int nb = ubqp_ascent_nb(as);
            ubqp_ascent_share_team(as, members[{p->planes, nb}], (int)inst.size());
            ubqp_split_dinit(yr, as, UBQP_SPLIT_TARGET / members[{p->planes, nb}]);
            Chunk &ch = groups[{p->planes, nb}];
            ch.planes = p->planes;
            ch.nb = nb;
            ch.yr.add(yr, ubqp_yrows_tiles(yr));
            ch.asc.add(as, ubqp_ascent_waves(as));
            if (ubqp_ascent_team_blocks(as) > 0) ch.team.add(as, ubqp_ascent_team_blocks(as));
            ch.n_pad_max = std::max(ch.n_pad_max, (int)p->n_pad);
        }
        for (auto &kv : groups) {
            // the same (planes, nb) group keeps its side stream across chunk offsets
            int lane = 0;
            auto it = group_lane.find(kv.first);
            if (it != group_lane.end()) {
                lane = it->second;
            } else {
                lane = (int)(group_lane.size() % UBQP_SIDE_STREAMS);
                group_lane[kv.first] = lane;
            }
            kv.second.lane = lane;
            chunks.push_back(std::move(kv.second));
        }
    }
    host.clear();
    div.stage(host);
    einit.stage(host);
    for (EvalGroup &g : ev) g.t.stage(host);
    scr.stage(host);
    ord.stage(host);
    sel_cand.stage(host);
    sel_rank.stage(host);
    sel_seed.stage(host);
    init.stage(host);
    for (Chunk &ch : chunks) {
        ch.yr.stage(host);
        ch.asc.stage(host);
        ch.team.stage(host);
    }
}

void GenTables::bind(char *dev)
{
    div.bind(dev);
    einit.bind(dev);
    for (EvalGroup &g : ev) g.t.bind(dev);
    scr.bind(dev);
    ord.bind(dev);
    sel_cand.bind(dev);
    sel_rank.bind(dev);
    sel_seed.bind(dev);
    init.bind(dev);
    for (Chunk &ch : chunks) {
        ch.yr.bind(dev);
        ch.asc.bind(dev);
        ch.team.bind(dev);
    }
}

hipError_t ubqp_queue_seed_init(const GenTables &t, hipStream_t st)
{
    if (t.init.count() == 0) return hipSuccess;
    return ubqp_launch_seed_init_batch(st, t.init.d_args, t.init.d_pre, t.init.count(), t.init.total());
}

hipError_t SideStreams::create()
{
    hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    for (int i = 0; e == hipSuccess && i < UBQP_SIDE_STREAMS; i++) {
        e = hipStreamCreateWithFlags(&s[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
    }
    return e;
}

void SideStreams::destroy()
{
    for (int i = 0; i < UBQP_SIDE_STREAMS; i++) {
        if (s[i]) (void)hipStreamSynchronize(s[i]);
        if (s[i]) (void)hipStreamDestroy(s[i]);
        if (join[i]) (void)hipEventDestroy(join[i]);
        s[i] = nullptr;
        join[i] = nullptr;
    }
    if (fork) (void)hipEventDestroy(fork);
    fork = nullptr;
}

hipError_t ubqp_queue_generation(const GenTables &t, hipStream_t st, hipEvent_t *pe, hipEvent_t *ae,
                                 const SideStreams *side)
{
    hipError_t e = hipSuccess;
#define Q(expr)                                   \
    do {                                          \
        if ((e = (expr)) != hipSuccess) return e; \
    } while (0)
#define MARK(i) \
    if (pe) Q(hipEventRecord(pe[i], st))
    const int n = t.count;
    MARK(0);
    Q(ubqp_launch_diversify_batch(st, t.div.d_args, t.div.d_pre, n, t.div.total()));
    MARK(1);
    Q(ubqp_launch_eval_init_batch(st, t.einit.d_args, t.einit.d_pre, n, t.einit.total()));
    for (const EvalGroup &g : t.ev)
        Q(ubqp_launch_eval_rowdot_batch(st, g.variant, g.t.d_args, g.t.d_pre, g.t.count(), g.t.total()));
    MARK(2);
    if (t.has_dump) Q(ubqp_launch_dump_batch(st, t.sel_cand.d_args, t.sel_cand.d_pre, n, t.sel_cand.total()));
    Q(ubqp_launch_screen_batch(st, t.scr.d_args, t.scr.d_pre, n, t.scr.total()));
    Q(ubqp_launch_order_batch(st, t.ord.d_args, t.ord.count()));
    MARK(3);
    int lanes = 0;
    for (const Chunk &ch : t.chunks) lanes = ch.lane + 1 > lanes ? ch.lane + 1 : lanes;
    const bool fork = side && !pe && lanes > 1;
    if (fork) {
        Q(hipEventRecord(side->fork, st));
        for (int l = 0; l < lanes; l++) Q(hipStreamWaitEvent(side->s[l], side->fork, 0));
    }
    for (size_t c = 0; c < t.chunks.size(); c++) {
        const Chunk &ch = t.chunks[c];
        hipStream_t cs = fork ? side->s[ch.lane] : st;
        Q(ubqp_launch_eval_batch(cs, ch.planes == 1 ? UBQP_EPI_KEYS : UBQP_EPI_Y, ch.yr.d_args, ch.yr.d_pre,
                                 ch.yr.count(), ch.yr.total()));
        if (ae) Q(hipEventRecord(ae[2 * c], cs));
        if (ch.team.count() > 0)
            Q(ubqp_launch_ascent_team_batch(cs, ch.planes, ch.n_pad_max, ch.team.d_args, ch.team.d_pre, ch.team.count(),
                                            ch.team.total()));
        Q(ubqp_launch_ascent_batch(cs, ch.planes, ch.nb, ch.asc.d_args, ch.asc.d_pre, ch.asc.count(),
                                   ch.asc.total()));
        if (ae) Q(hipEventRecord(ae[2 * c + 1], cs));
    }
    if (fork) {
        for (int l = 0; l < lanes; l++) {
            Q(hipEventRecord(side->join[l], side->s[l]));
            Q(hipStreamWaitEvent(st, side->join[l], 0));
        }
    }
    MARK(4);
    Q(ubqp_launch_select_batch(st, t.sel_cand.d_args, t.sel_cand.d_pre, t.sel_cand.total(), t.sel_rank.d_pre,
                               t.sel_rank.total(), t.sel_seed.d_pre, t.sel_seed.total(), n));
    MARK(5);
#undef MARK
#undef Q
    return e;
}

struct ubqp_plan {
    ubqp_ctx *ctx = nullptr;
    int count = 0;
    int32_t G = 0, g = 0;
    std::vector<InstRef> inst;
    char *state = nullptr;
    char *tables = nullptr;
    GenTables t;
    bool timing = false, use_graph = true;
    hipStream_t cap_stream = nullptr;
    SideStreams side;                // forked to by the (planes, NB) groups of a generation
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr;
    std::vector<hipEvent_t> gen_ev; // end of each generation
    std::vector<hipEvent_t> phase;  // UBQP_TIMING: G x (UBQP_PHASE_ASCENT_KERNEL + 1)
    std::vector<hipEvent_t> asc_ev; // UBQP_TIMING: G x chunk groups x 2
};

namespace {

void plan_free(ubqp_plan *pl)
{
    if (!pl) return;
    ubqp_ctx *ctx = pl->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    pl->side.destroy();
    for (hipEvent_t e : pl->gen_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : pl->phase)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : pl->asc_ev)
        if (e) (void)hipEventDestroy(e);
    if (pl->ev0) (void)hipEventDestroy(pl->ev0);
    if (pl->state) (void)hipFree(pl->state);
    if (pl->tables) (void)hipFree(pl->tables);
    delete pl;
    ubqp_ctx_drop(ctx);
}

int plan_create(ubqp_ctx *ctx, int count, const ubqp_problem *const *probs, const ubqp_params *params,
                int64_t *const *dumps, ubqp_plan **out)
{
    *out = nullptr;
    if (count < 1) return ubqp_fail(ctx, UBQP_EINVAL, "count=%d < 1", count);
    for (int i = 0; i < count; i++) {
        if (!probs[i]) return ubqp_fail(ctx, UBQP_EINVAL, "null problem %d", i);
        UBQP_TRY(ubqp_check_params(ctx, probs[i], &params[i]));
        if (params[i].G != params[0].G)
            return ubqp_fail(ctx, UBQP_EINVAL, "G differs between instances (%d vs %d)", params[i].G, params[0].G);
    }
    UBQP_TRY(ubqp_set_device(ctx));
    for (int i = 0; i < count; i++)
        if (params[i].flags & UBQP_AUTOTUNE) UBQP_TRY(ubqp_tune_eval_internal(ctx, probs[i], params[i].M, nullptr, nullptr));
    ubqp_plan *pl = new (std::nothrow) ubqp_plan();
    if (!pl) return ubqp_fail(ctx, UBQP_ENOMEM, "host allocation");
    pl->ctx = ctx;
    ubqp_ctx_hold(ctx);
    pl->count = count;
    pl->G = params[0].G;
    pl->timing = (params[0].flags & UBQP_TIMING) != 0;
    pl->use_graph = !pl->timing && !(params[0].flags & UBQP_NO_GRAPH);
    size_t total = 0;
    std::vector<size_t> base;
    for (int i = 0; i < count; i++) {
        InstRef r{};
        r.p = probs[i];
        r.pr = params[i];
        r.L = ubqp_inst_layout(probs[i], &params[i]);
        r.dump = dumps ? dumps[i] : nullptr;
        pl->inst.push_back(r);
        base.push_back(total);
        total += r.L.total;
    }
    hipError_t e = hipMalloc(&pl->state, total);
    if (e != hipSuccess) {
        plan_free(pl);
        return ubqp_hip_fail(ctx, e, "multistart state");
    }
    for (int i = 0; i < count; i++) {
        // each instance reports its ascent's checks to a flag of its own, so a result
        // names the instance whose ascent failed
        InstRef &r = pl->inst[(size_t)i];
        r.base = pl->state + base[(size_t)i];
        r.err = r.at<int32_t>(r.L.err);
        if (e == hipSuccess) e = ubqp_queue_zero(ctx->stream, r.err, 1);
    }
    if (e != hipSuccess) {
        plan_free(pl);
        return ubqp_hip_fail(ctx, e, "error flags");
    }
    pl->t.build(pl->inst);
    e = hipMalloc(&pl->tables, std::max<size_t>(pl->t.host.size(), 256));
    if (e == hipSuccess) e = hipMemcpy(pl->tables, pl->t.host.data(), pl->t.host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreate(&pl->ev0);
    pl->gen_ev.assign((size_t)pl->G, nullptr);
    for (size_t k = 0; e == hipSuccess && k < pl->gen_ev.size(); k++) e = hipEventCreate(&pl->gen_ev[k]);
    if (pl->timing) {
        pl->phase.assign((size_t)pl->G * (UBQP_PHASE_ASCENT_KERNEL + 1), nullptr);
        pl->asc_ev.assign((size_t)pl->G * pl->t.chunks.size() * 2, nullptr);
    }
    for (size_t k = 0; e == hipSuccess && k < pl->phase.size(); k++) e = hipEventCreate(&pl->phase[k]);
    for (size_t k = 0; e == hipSuccess && k < pl->asc_ev.size(); k++) e = hipEventCreate(&pl->asc_ev[k]);
    if (e != hipSuccess) {
        plan_free(pl);
        return ubqp_hip_fail(ctx, e, "plan setup");
    }
    pl->t.bind(pl->tables);
    e = pl->side.create();
    if (e != hipSuccess) {
        plan_free(pl);
        return ubqp_hip_fail(ctx, e, "side streams");
    }
    // generation-0 seeds and scalars, then the start event
    e = ubqp_queue_seed_init(pl->t, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(pl->ev0, ctx->stream);
    if (e != hipSuccess) {
        plan_free(pl);
        return ubqp_hip_fail(ctx, e, "seed init");
    }
    *out = pl;
    return UBQP_OK;
}

int plan_step(ubqp_plan *pl, int32_t generations)
{
    ubqp_ctx *ctx = pl->ctx;
    if (generations < 0 || pl->g + generations > pl->G)
        return ubqp_fail(ctx, UBQP_EINVAL, "%d more generations exceed G=%d (done %d)", generations, pl->G, pl->g);
    UBQP_TRY(ubqp_set_device(ctx));
    hipStream_t st = ctx->stream;
    if (pl->use_graph && generations > 0 && !pl->exec) {
        // capture one generation on a private stream (the caller's may be the null stream)
        UBQP_HIP_TRY(ctx, hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
        UBQP_HIP_TRY(ctx, hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
        const hipError_t qe = ubqp_queue_generation(pl->t, pl->cap_stream, nullptr, nullptr, &pl->side);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(pl->cap_stream, &g);
        if (qe != hipSuccess) return ubqp_hip_fail(ctx, qe, "generation capture");
        UBQP_HIP_TRY(ctx, ce);
        pl->graph = g;
        UBQP_HIP_TRY(ctx, hipGraphInstantiateWithFlags(&pl->exec, pl->graph, 0));
    }
    for (int32_t k = 0; k < generations; k++, pl->g++) {
        if (pl->exec) {
            UBQP_HIP_TRY(ctx, hipGraphLaunch(pl->exec, st));
        } else {
            hipEvent_t *pe = pl->timing ? &pl->phase[(size_t)pl->g * (UBQP_PHASE_ASCENT_KERNEL + 1)] : nullptr;
            hipEvent_t *ae = pl->timing && !pl->t.chunks.empty()
                                 ? &pl->asc_ev[(size_t)pl->g * pl->t.chunks.size() * 2]
                                 : nullptr;
            UBQP_HIP_TRY(ctx, ubqp_queue_generation(pl->t, st, pe, ae, &pl->side));
        }
        UBQP_HIP_TRY(ctx, hipEventRecord(pl->gen_ev[(size_t)pl->g], st));
    }
    return UBQP_OK;
}

int plan_result(ubqp_plan *pl, int i, ubqp_result *res)
{
    ubqp_ctx *ctx = pl->ctx;
    if (i < 0 || i >= pl->count) return ubqp_fail(ctx, UBQP_EINVAL, "instance %d outside [0, %d)", i, pl->count);
    UBQP_TRY(ubqp_set_device(ctx));
    hipStream_t st = ctx->stream;
    const InstRef &r = pl->inst[(size_t)i];
    ubqp_scal hs;
    int32_t errv = 0;
    UBQP_HIP_TRY(ctx, hipMemcpyAsync(&hs, r.at<ubqp_scal>(r.L.scal), sizeof hs, hipMemcpyDeviceToHost, st));
    UBQP_HIP_TRY(ctx, hipMemcpyAsync(&errv, r.err, sizeof errv, hipMemcpyDeviceToHost, st));
    if (res->best_x_host)
        UBQP_HIP_TRY(ctx, hipMemcpyAsync(res->best_x_host, r.at<uint64_t>(r.L.bestx), (size_t)r.p->W * 8,
                                         hipMemcpyDeviceToHost, st));
    if (res->stats_host && pl->g > 0)
        UBQP_HIP_TRY(ctx, hipMemcpyAsync(res->stats_host, r.at<int64_t>(r.L.stats), (size_t)pl->g * 5 * 8,
                                         hipMemcpyDeviceToHost, st));
    UBQP_HIP_TRY(ctx, hipStreamSynchronize(st));
    // the flag stays set: every later generation builds on the cut-short ascent
    if (errv & 2) return ubqp_fail(ctx, UBQP_EDEVICE, "instance %d: an ascent candidate index was out of range", i);
    if (errv & 1)
        return ubqp_fail(ctx, UBQP_ELIMIT, "instance %d: an ascent to a local optimum reached the problem's flip "
                                           "limit of %d flips and stopped short of it", i,
                         ubqp_problem_flip_limit(r.p));
    if (res->gen_ms_host)
        for (int32_t g = 0; g < pl->g; g++) {
            float ms = 0.f;
            UBQP_HIP_TRY(ctx, hipEventElapsedTime(&ms, pl->ev0, pl->gen_ev[(size_t)g]));
            res->gen_ms_host[g] = ms;
        }
    if (res->phase_ms_host && !pl->phase.empty())
        for (int32_t g = 0; g < pl->g; g++) {
            for (int k = 0; k < UBQP_PHASE_ASCENT_KERNEL; k++) {
                float ms = 0.f;
                const size_t b = (size_t)g * (UBQP_PHASE_ASCENT_KERNEL + 1);
                UBQP_HIP_TRY(ctx, hipEventElapsedTime(&ms, pl->phase[b + k], pl->phase[b + k + 1]));
                res->phase_ms_host[(size_t)g * UBQP_PHASES + k] = ms;
            }
            double asc = 0.0;
            const size_t nc = pl->t.chunks.size(), b = (size_t)g * nc * 2;
            for (size_t c = 0; c < nc; c++) {
                float ms = 0.f;
                UBQP_HIP_TRY(ctx, hipEventElapsedTime(&ms, pl->asc_ev[b + 2 * c], pl->asc_ev[b + 2 * c + 1]));
                asc += ms;
            }
            res->phase_ms_host[(size_t)g * UBQP_PHASES + UBQP_PHASE_ASCENT_KERNEL] = asc;
        }
    res->have_best = hs.have_best;
    res->best_f = hs.have_best ? hs.best_f : INT64_MIN;
    res->generations = pl->g;
    return UBQP_OK;
}

}  // namespace

struct ubqp_run {
    ubqp_plan *plan = nullptr;
};
struct ubqp_batch {
    ubqp_plan *plan = nullptr;
};

extern "C" {

int64_t ubqp_run_footprint(const ubqp_problem *p, const ubqp_params *pr)
{
    if (!p || !pr || pr->M < 1 || pr->H < 1 || pr->G < 1) return -1;
    return (int64_t)ubqp_inst_layout(p, pr).total;
}

int ubqp_run_create(ubqp_ctx *ctx, const ubqp_problem *p, const ubqp_params *pr, int64_t *f_dump_d, ubqp_run **out)
{
    if (!ctx || !p || !pr || !out) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    *out = nullptr;
    ubqp_run *r = new (std::nothrow) ubqp_run();
    if (!r) return ubqp_fail(ctx, UBQP_ENOMEM, "host allocation");
    int64_t *dumps[1] = {f_dump_d};
    const int rc = plan_create(ctx, 1, &p, pr, dumps, &r->plan);
    if (rc != UBQP_OK) {
        delete r;
        return rc;
    }
    *out = r;
    return UBQP_OK;
}

int ubqp_run_step(ubqp_run *r, int32_t generations) { return r ? plan_step(r->plan, generations) : UBQP_EINVAL; }

int ubqp_run_result(ubqp_run *r, ubqp_result *res) { return (r && res) ? plan_result(r->plan, 0, res) : UBQP_EINVAL; }

int ubqp_run_destroy(ubqp_run *r)
{
    if (!r) return UBQP_EINVAL;
    plan_free(r->plan);
    delete r;
    return UBQP_OK;
}

int ubqp_multistart(ubqp_ctx *ctx, const ubqp_problem *p, const ubqp_params *pr, int64_t *f_dump_d, ubqp_result *res)
{
    if (!ctx || !p || !pr || !res) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    ubqp_run *r = nullptr;
    UBQP_TRY(ubqp_run_create(ctx, p, pr, f_dump_d, &r));
    int rc = ubqp_run_step(r, pr->G);
    if (rc == UBQP_OK) rc = ubqp_run_result(r, res);
    ubqp_run_destroy(r);
    return rc;
}

int64_t ubqp_batch_footprint(int32_t count, const ubqp_problem *const *probs, const ubqp_params *params)
{
    if (count < 1 || !probs || !params) return -1;
    int64_t t = 0;
    for (int i = 0; i < count; i++) {
        const int64_t f = ubqp_run_footprint(probs[i], &params[i]);
        if (f < 0) return -1;
        t += f;
    }
    return t;
}

int ubqp_batch_create(ubqp_ctx *ctx, int32_t count, const ubqp_problem *const *probs, const ubqp_params *params,
                      ubqp_batch **out)
{
    if (!ctx || !probs || !params || !out) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    *out = nullptr;
    ubqp_batch *b = new (std::nothrow) ubqp_batch();
    if (!b) return ubqp_fail(ctx, UBQP_ENOMEM, "host allocation");
    const int rc = plan_create(ctx, count, probs, params, nullptr, &b->plan);
    if (rc != UBQP_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return UBQP_OK;
}

int ubqp_batch_step(ubqp_batch *b, int32_t generations) { return b ? plan_step(b->plan, generations) : UBQP_EINVAL; }

int ubqp_batch_result(ubqp_batch *b, int32_t i, ubqp_result *res)
{
    return (b && res) ? plan_result(b->plan, i, res) : UBQP_EINVAL;
}

int ubqp_batch_destroy(ubqp_batch *b)
{
    if (!b) return UBQP_EINVAL;
    plan_free(b->plan);
    delete b;
    return UBQP_OK;
}

int ubqp_multistart_batched(ubqp_ctx *ctx, int32_t count, const ubqp_problem *const *probs,
                            const ubqp_params *params, ubqp_result *results)
{
    if (!ctx || !probs || !params || !results) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    ubqp_batch *b = nullptr;
    UBQP_TRY(ubqp_batch_create(ctx, count, probs, params, &b));
    int rc = ubqp_batch_step(b, params[0].G);
    for (int i = 0; rc == UBQP_OK && i < count; i++) rc = ubqp_batch_result(b, i, &results[i]);
    ubqp_batch_destroy(b);
    return rc;
}

}  // extern "C"
