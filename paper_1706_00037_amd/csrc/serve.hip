// C ABI of libubqp, part 3: the request server (serving form).
//
// A worker thread owns the device work, on two non-blocking streams of the
// server's own: one computes, one uploads.  Requests wait in a FIFO queue; the
// oldest is admitted when a slot is free and the first-fit pool (one device
// allocation made at creation) has room for its footprint.  Admission queues
// the request's upload on a second stream: the copy of its coefficients, the
// device-side check and the build of its resident Q (problem.hip), while the
// running requests compute on the main stream.  At each generation boundary the
// worker
//   1. retires requests whose results have reached the host (memory back to
//      the pool, slot freed),
//   2. turns finished uploads into joining requests (or failures),
//   3. admits more requests,
//   4. rebuilds the launch tables when the running set changed (into the table
//      buffer the previous generation did not use), queues the joiners'
//      generation-0 seeds, and queues one batched generation for every running
//      request (plan.h),
//   5. queues the result copies of requests that have done their G generations.
// At most two generations are in flight, so a new request waits for at most
// one generation boundary after its upload before it joins.  Each request's
// results depend only on its own problem, parameters and seed, so they equal
// those of a solve run alone.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>

#include "plan.h"

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over [0, size) with 256-byte granules; coalesces on release.
struct Pool {
    size_t size = 0, used = 0, high = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
    void init(size_t s)
    {
        size = s;
        free_.clear();
        if (s) free_[0] = s;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = ubqp_align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o2 = it->first + bytes;
            free_.erase(it);
            if (rest) free_[o2] = rest;
            used += bytes;
            high = std::max(high, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = ubqp_align256(bytes);
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Where a request's pieces sit inside its pool block.
struct ReqLayout {
    ubqp_problem geom;  // geometry only
    InstLayout L;
    size_t prob, state, stage, flags, total;
};

bool req_layout(int32_t n, int32_t elem, const ubqp_params *pr, ReqLayout *out)
{
    if (n < 1 || n > UBQP_MAX_N || (elem != 1 && elem != 2 && elem != 4) || !pr) return false;
    ReqLayout R{};
    ubqp_problem_geometry(&R.geom, n, elem == 1 ? 1 : 2);
    if (ubqp_check_params(nullptr, &R.geom, pr) != UBQP_OK) return false;
    R.L = ubqp_inst_layout(&R.geom, pr);
    R.prob = 0;
    R.state = ubqp_align256(ubqp_problem_bytes(&R.geom));
    // The staged coefficients share the Delta workspace: the upload has
    // finished before the request's first generation writes it.
    const size_t stage_bytes = ubqp_align256((size_t)n * n * elem);
    const size_t state_bytes = std::max(R.L.total, R.L.Y + stage_bytes);
    R.stage = R.state + R.L.Y;
    R.flags = R.state + ubqp_align256(state_bytes);
    R.total = R.flags + 256;
    *out = R;
    return true;
}

// Host layout of a slot's page-locked buffer.
constexpr size_t PIN_FLAGS = 0, PIN_SCAL = 64, PIN_ERR = 128, PIN_BESTX = 192;
size_t pin_bytes(int32_t W, int32_t G) { return PIN_BESTX + (size_t)W * 8 + (size_t)G * 5 * 8; }

enum ReqState { QUEUED, UPLOADING, READY, RUNNING, FINISHING };

struct Req {
    int64_t id = 0;
    int32_t n = 0, elem = 1;
    const void *q_host = nullptr;
    ubqp_params pr{};
    uint64_t *bestx_host = nullptr;
    int64_t *stats_host = nullptr;
    ReqState st = QUEUED;
    ReqLayout R{};
    ubqp_problem prob{};
    size_t off = 0;
    int slot = -1;
    int32_t gens = 0;
    int64_t t_submit = 0, t_admit = 0, t_start = 0;
    InstRef ref() const
    {
        InstRef r{};
        r.p = &prob;
        r.pr = pr;
        r.L = R.L;
        r.base = nullptr;  // set by the server
        r.dump = nullptr;
        r.err = nullptr;
        return r;
    }
};

struct Slot {
    hipEvent_t up_ev = nullptr, res_ev = nullptr;
    char *pin = nullptr;
    size_t pin_bytes = 0;
};

struct TableBuf {
    char *dev = nullptr, *pin = nullptr;
    size_t dev_bytes = 0, pin_bytes = 0;
    hipEvent_t last = nullptr;  // end of the last generation that read it
    bool used = false;
};

}  // namespace

struct ubqp_server {
    ubqp_ctx *ctx = nullptr;
    hipStream_t cs = nullptr, up = nullptr;  // compute and upload streams, both the server's own
    SideStreams side;                        // the generation's (planes, NB) groups fork to these
    char *pool_mem = nullptr;
    Pool pool;
    int max_active = 0;
    std::vector<Slot> slots;
    std::vector<int> free_slots;
    TableBuf tb[2];
    int cur_tb = 0;
    GenTables tables;
    bool tables_valid = false;
    std::deque<hipEvent_t> inflight;  // ends of queued generations, oldest first
    std::vector<hipEvent_t> spare_ev;

    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> queue;               // guarded by m
    int64_t queue_limit = 0;               // guarded by m: most requests waiting (0: no limit)
    std::deque<ubqp_request_info> done;    // guarded by m
    bool stop = false;                     // guarded by m
    bool dead = false;                     // guarded by m: a device failure ended the worker
    std::string err;                       // guarded by m
    int64_t next_id = 1;                   // guarded by m
    std::atomic<int64_t> cnt[8];

    // worker-owned
    std::vector<Req *> uploading, ready, running, finishing;
    bool dirty = false;
    std::thread worker;

    char *base_of(const Req *r) const { return pool_mem + r->off; }
};

namespace {

enum { C_SUBMITTED, C_FINISHED, C_FAILED, C_GENERATIONS, C_MAX_RUNNING, C_POOL_HIGH, C_WAITING, C_ADMITTED };

void set_err(ubqp_server *s, const std::string &msg)
{
    std::lock_guard<std::mutex> lk(s->m);
    s->err = msg;
}

void release(ubqp_server *s, Req *r)
{
    s->pool.release(r->off, r->R.total);
    if (r->slot >= 0) s->free_slots.push_back(r->slot);
    r->slot = -1;
}

void publish(ubqp_server *s, Req *r, int status, const int64_t *scal_best, int32_t have_best)
{
    ubqp_request_info info{};
    info.id = r->id;
    info.status = status;
    info.generations = r->gens;
    info.have_best = have_best;
    info.best_f = have_best ? *scal_best : INT64_MIN;
    info.planes = r->prob.planes;
    info.t_submit_ns = r->t_submit;
    info.t_admit_ns = r->t_admit;
    info.t_start_ns = r->t_start;
    info.t_done_ns = now_ns();
    s->cnt[status == UBQP_OK ? C_FINISHED : C_FAILED]++;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->done.push_back(info);
    }
    s->cv_done.notify_all();
    delete r;
}

hipError_t grow_pin(Slot &sl, size_t bytes)
{
    if (sl.pin_bytes >= bytes) return hipSuccess;
    if (sl.pin) (void)hipHostFree(sl.pin);
    sl.pin = nullptr;
    sl.pin_bytes = 0;
    hipError_t e = hipHostMalloc((void **)&sl.pin, bytes, hipHostMallocDefault);
    if (e == hipSuccess) sl.pin_bytes = bytes;
    return e;
}

// Queue the upload of r on the upload stream.
hipError_t start_upload(ubqp_server *s, Req *r)
{
    Slot &sl = s->slots[(size_t)r->slot];
    hipError_t e = grow_pin(sl, pin_bytes(r->prob.W, r->pr.G));
    if (e != hipSuccess) return e;
    char *b = s->base_of(r);
    ubqp_problem_bind(&r->prob, b + r->R.prob);
    char *stage = b + r->R.stage;
    ubqp_check_flags *fl = (ubqp_check_flags *)(b + r->R.flags);
    e = hipMemcpyAsync(stage, r->q_host, (size_t)r->n * r->n * r->elem, hipMemcpyHostToDevice, s->up);
    if (e == hipSuccess) e = ubqp_queue_problem_check(s->up, stage, r->elem, r->n, fl);
    if (e == hipSuccess) e = ubqp_queue_problem_build(s->up, stage, r->elem, &r->prob);
    if (e == hipSuccess) e = ubqp_queue_zero(s->up, b + r->R.state + r->R.L.err, 1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.pin + PIN_FLAGS, fl, sizeof(ubqp_check_flags), hipMemcpyDeviceToHost, s->up);
    if (e == hipSuccess) e = hipEventRecord(sl.up_ev, s->up);
    return e;
}

hipError_t admit(ubqp_server *s)
{
    for (;;) {
        Req *r = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->m);
            if (s->queue.empty() || s->free_slots.empty()) return hipSuccess;
            size_t off = 0;
            if (!s->pool.alloc(s->queue.front()->R.total, &off)) return hipSuccess;
            r = s->queue.front();
            s->queue.pop_front();
            r->off = off;
            r->slot = s->free_slots.back();
            s->free_slots.pop_back();
            s->cnt[C_WAITING]--;
            s->cnt[C_POOL_HIGH] = (int64_t)s->pool.high;
        }
        s->cnt[C_ADMITTED]++;
        r->t_admit = now_ns();
        r->st = UPLOADING;
        s->uploading.push_back(r);
        const hipError_t e = start_upload(s, r);
        if (e != hipSuccess) return e;
    }
}

hipError_t poll_uploads(ubqp_server *s)
{
    for (size_t i = 0; i < s->uploading.size();) {
        Req *r = s->uploading[i];
        const hipError_t q = hipEventQuery(s->slots[(size_t)r->slot].up_ev);
        if (q == hipErrorNotReady) {
            i++;
            continue;
        }
        if (q != hipSuccess) return q;
        s->uploading.erase(s->uploading.begin() + (ptrdiff_t)i);
        const ubqp_check_flags fl = *(const ubqp_check_flags *)(s->slots[(size_t)r->slot].pin + PIN_FLAGS);
        const int v = ubqp_check_outcome(nullptr, fl, r->n);
        if (v != UBQP_OK) {
            {
                std::lock_guard<std::mutex> lk(s->m);
                release(s, r);
            }
            publish(s, r, v, nullptr, 0);
            continue;
        }
        r->st = READY;
        s->ready.push_back(r);
    }
    return hipSuccess;
}

hipError_t poll_finishing(ubqp_server *s)
{
    for (size_t i = 0; i < s->finishing.size();) {
        Req *r = s->finishing[i];
        Slot &sl = s->slots[(size_t)r->slot];
        const hipError_t q = hipEventQuery(sl.res_ev);
        if (q == hipErrorNotReady) {
            i++;
            continue;
        }
        if (q != hipSuccess) return q;
        s->finishing.erase(s->finishing.begin() + (ptrdiff_t)i);
        const ubqp_scal sc = *(const ubqp_scal *)(sl.pin + PIN_SCAL);
        const int32_t errv = *(const int32_t *)(sl.pin + PIN_ERR);
        memcpy(r->bestx_host, sl.pin + PIN_BESTX, (size_t)r->prob.W * 8);
        if (r->stats_host) memcpy(r->stats_host, sl.pin + PIN_BESTX + (size_t)r->prob.W * 8, (size_t)r->gens * 40);
        {
            std::lock_guard<std::mutex> lk(s->m);
            release(s, r);
        }
        publish(s, r, (errv & 2) ? UBQP_EDEVICE : (errv & 1) ? UBQP_ELIMIT : UBQP_OK, &sc.best_f, sc.have_best);
    }
    return hipSuccess;
}

hipError_t take_event(ubqp_server *s, hipEvent_t *ev)
{
    if (!s->spare_ev.empty()) {
        *ev = s->spare_ev.back();
        s->spare_ev.pop_back();
        return hipSuccess;
    }
    return hipEventCreateWithFlags(ev, hipEventDisableTiming);
}

// Rebuild the tables for running + ready (the ready ones join) and queue the
// joiners' seed initialisation.
hipError_t rebuild(ubqp_server *s)
{
    hipStream_t st = s->cs;
    std::vector<InstRef> inst;
    std::vector<char> join;
    for (Req *r : s->running) {
        InstRef x = r->ref();
        x.base = s->base_of(r) + r->R.state;
        x.err = (int32_t *)(x.base + r->R.L.err);
        inst.push_back(x);
        join.push_back(0);
    }
    for (Req *r : s->ready) {
        InstRef x = r->ref();
        x.base = s->base_of(r) + r->R.state;
        x.err = (int32_t *)(x.base + r->R.L.err);
        inst.push_back(x);
        join.push_back(1);
    }
    s->tables = GenTables();
    s->tables_valid = false;
    s->dirty = false;
    if (inst.empty()) return hipSuccess;
    s->tables.build(inst, &join);
    const size_t bytes = std::max<size_t>(s->tables.host.size(), 256);
    s->cur_tb ^= 1;
    TableBuf &tb = s->tb[s->cur_tb];
    hipError_t e = hipSuccess;
    if (tb.used) e = hipEventSynchronize(tb.last);
    if (e == hipSuccess && tb.dev_bytes < bytes) {
        if (tb.dev) e = hipFree(tb.dev);
        tb.dev = nullptr;
        tb.dev_bytes = 0;
        if (e == hipSuccess) e = hipMalloc(&tb.dev, bytes * 2);
        if (e == hipSuccess) tb.dev_bytes = bytes * 2;
    }
    if (e == hipSuccess && tb.pin_bytes < bytes) {
        if (tb.pin) e = hipHostFree(tb.pin);
        tb.pin = nullptr;
        tb.pin_bytes = 0;
        if (e == hipSuccess) e = hipHostMalloc((void **)&tb.pin, bytes * 2, hipHostMallocDefault);
        if (e == hipSuccess) tb.pin_bytes = bytes * 2;
    }
    if (e != hipSuccess) return e;
    memcpy(tb.pin, s->tables.host.data(), s->tables.host.size());
    e = hipMemcpyAsync(tb.dev, tb.pin, s->tables.host.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    s->tables.bind(tb.dev);
    s->tables_valid = true;
    e = ubqp_queue_seed_init(s->tables, st);
    if (e != hipSuccess) return e;
    const int64_t t = now_ns();
    for (Req *r : s->ready) {
        r->st = RUNNING;
        r->t_start = t;
        s->running.push_back(r);
    }
    s->ready.clear();
    return hipSuccess;
}

hipError_t step(ubqp_server *s)
{
    hipStream_t st = s->cs;
    hipError_t e = hipSuccess;
    if (s->dirty || !s->ready.empty()) e = rebuild(s);
    if (e != hipSuccess || s->running.empty()) return e;
    while (s->inflight.size() >= 2) {
        e = hipEventSynchronize(s->inflight.front());
        if (e != hipSuccess) return e;
        s->spare_ev.push_back(s->inflight.front());
        s->inflight.pop_front();
    }
    e = ubqp_queue_generation(s->tables, st, nullptr, nullptr, &s->side);
    hipEvent_t ev = nullptr;
    if (e == hipSuccess) e = take_event(s, &ev);
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    if (e != hipSuccess) return e;
    s->inflight.push_back(ev);
    TableBuf &tb = s->tb[s->cur_tb];
    if (!tb.last) e = hipEventCreateWithFlags(&tb.last, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(tb.last, st);
    if (e != hipSuccess) return e;
    tb.used = true;
    s->cnt[C_GENERATIONS]++;
    if ((int64_t)s->running.size() > s->cnt[C_MAX_RUNNING]) s->cnt[C_MAX_RUNNING] = (int64_t)s->running.size();
    for (size_t i = 0; i < s->running.size();) {
        Req *r = s->running[i];
        r->gens++;
        if (r->gens < r->pr.G) {
            i++;
            continue;
        }
        // results of a finished request, in order after its last generation
        Slot &sl = s->slots[(size_t)r->slot];
        char *b = s->base_of(r) + r->R.state;
        e = hipMemcpyAsync(sl.pin + PIN_SCAL, b + r->R.L.scal, sizeof(ubqp_scal), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(sl.pin + PIN_ERR, b + r->R.L.err, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.pin + PIN_BESTX, b + r->R.L.bestx, (size_t)r->prob.W * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && r->stats_host)
            e = hipMemcpyAsync(sl.pin + PIN_BESTX + (size_t)r->prob.W * 8, b + r->R.L.stats, (size_t)r->gens * 40,
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(sl.res_ev, st);
        if (e != hipSuccess) return e;
        r->st = FINISHING;
        s->finishing.push_back(r);
        s->running.erase(s->running.begin() + (ptrdiff_t)i);
        s->dirty = true;
    }
    return hipSuccess;
}

// Block until something the worker waits for may have happened.
hipError_t wait_any(ubqp_server *s)
{
    if (!s->inflight.empty()) {
        const hipError_t e = hipEventSynchronize(s->inflight.front());
        s->spare_ev.push_back(s->inflight.front());
        s->inflight.pop_front();
        return e;
    }
    if (!s->uploading.empty()) return hipEventSynchronize(s->slots[(size_t)s->uploading.front()->slot].up_ev);
    if (!s->finishing.empty()) return hipEventSynchronize(s->slots[(size_t)s->finishing.front()->slot].res_ev);
    std::unique_lock<std::mutex> lk(s->m);
    s->cv_work.wait_for(lk, std::chrono::milliseconds(50), [&] { return s->stop || !s->queue.empty(); });
    return hipSuccess;
}

void fail_all(ubqp_server *s, hipError_t e)
{
    (void)hipDeviceSynchronize();
    std::vector<Req *> all;
    for (auto *v : {&s->uploading, &s->ready, &s->running, &s->finishing}) {
        all.insert(all.end(), v->begin(), v->end());
        v->clear();
    }
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->dead = true;
        s->err = std::string("device failure in the request loop: ") + hipGetErrorString(e);
        for (Req *r : s->queue) all.push_back(r);
        s->queue.clear();
        for (Req *r : all)
            if (r->slot >= 0) release(s, r);
    }
    for (Req *r : all) publish(s, r, UBQP_EDEVICE, nullptr, 0);
}

void worker_main(ubqp_server *s)
{
    if (hipSetDevice(s->ctx->device) != hipSuccess) {
        fail_all(s, hipErrorInvalidDevice);
        return;
    }
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->m);
            const bool idle = s->uploading.empty() && s->ready.empty() && s->running.empty() &&
                              s->finishing.empty() && s->inflight.empty();
            if (idle && s->queue.empty()) {
                if (s->stop) break;
                s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
                continue;
            }
        }
        hipError_t e = poll_finishing(s);
        if (e == hipSuccess) e = poll_uploads(s);
        if (e == hipSuccess) e = admit(s);
        if (e == hipSuccess && (!s->running.empty() || !s->ready.empty() || s->dirty)) {
            e = step(s);
            if (e == hipSuccess && s->running.empty()) e = wait_any(s);
        } else if (e == hipSuccess) {
            e = wait_any(s);
        }
        if (e != hipSuccess) {
            fail_all(s, e);
            return;
        }
    }
}

void server_free(ubqp_server *s)
{
    ubqp_ctx *ctx = s->ctx;
    (void)hipSetDevice(ctx->device);
    if (s->cs) (void)hipStreamSynchronize(s->cs);
    if (s->up) (void)hipStreamSynchronize(s->up);
    s->side.destroy();
    for (Slot &sl : s->slots) {
        if (sl.up_ev) (void)hipEventDestroy(sl.up_ev);
        if (sl.res_ev) (void)hipEventDestroy(sl.res_ev);
        if (sl.pin) (void)hipHostFree(sl.pin);
    }
    for (TableBuf &tb : s->tb) {
        if (tb.dev) (void)hipFree(tb.dev);
        if (tb.pin) (void)hipHostFree(tb.pin);
        if (tb.last) (void)hipEventDestroy(tb.last);
    }
    for (hipEvent_t e : s->inflight) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->spare_ev) (void)hipEventDestroy(e);
    if (s->pool_mem) (void)hipFree(s->pool_mem);
    if (s->up) (void)hipStreamDestroy(s->up);
    if (s->cs) (void)hipStreamDestroy(s->cs);
    delete s;
    ubqp_ctx_drop(ctx);
}

}  // namespace

extern "C" {

int64_t ubqp_request_footprint(int32_t n, int32_t elem_bytes, const ubqp_params *params)
{
    ReqLayout R;
    if (!req_layout(n, elem_bytes, params, &R)) return -1;
    return (int64_t)R.total;
}

int ubqp_server_create(ubqp_ctx *ctx, int64_t pool_bytes, int32_t max_active, ubqp_server **out)
{
    if (!ctx || !out) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    *out = nullptr;
    if (pool_bytes < 256 || max_active < 1 || max_active > 4096)
        return ubqp_fail(ctx, UBQP_EINVAL, "pool_bytes=%lld or max_active=%d out of range", (long long)pool_bytes,
                         max_active);
    UBQP_TRY(ubqp_set_device(ctx));
    ubqp_server *s = new (std::nothrow) ubqp_server();
    if (!s) return ubqp_fail(ctx, UBQP_ENOMEM, "host allocation");
    s->ctx = ctx;
    ubqp_ctx_hold(ctx);
    s->max_active = max_active;
    for (auto &c : s->cnt) c = 0;
    const size_t pb = ubqp_align256((size_t)pool_bytes);
    hipError_t e = hipMalloc(&s->pool_mem, pb);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking);
    if (e == hipSuccess) e = s->side.create();
    s->slots.resize((size_t)max_active);
    for (int i = 0; e == hipSuccess && i < max_active; i++) {
        e = hipEventCreateWithFlags(&s->slots[(size_t)i].up_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->slots[(size_t)i].res_ev, hipEventDisableTiming);
        s->free_slots.push_back(max_active - 1 - i);
    }
    if (e != hipSuccess) {
        server_free(s);
        return ubqp_hip_fail(ctx, e, "server setup");
    }
    s->pool.init(pb);
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        server_free(s);
        return ubqp_fail(ctx, UBQP_ENOMEM, "worker thread");
    }
    *out = s;
    return UBQP_OK;
}

int ubqp_server_submit(ubqp_server *s, int32_t n, const void *q_host, int32_t elem_bytes, const ubqp_params *params,
                       uint64_t *best_x_host, int64_t *stats_host, int64_t *id)
{
    if (!s) return UBQP_EINVAL;
    if (!q_host || !params || !best_x_host || !id) {
        set_err(s, "null argument");
        return UBQP_EINVAL;
    }
    if (params->flags & ~(UBQP_DERIV_START | UBQP_BLEND)) {
        set_err(s, "request flags other than UBQP_DERIV_START and UBQP_BLEND");
        return UBQP_EINVAL;
    }
    Req *r = new (std::nothrow) Req();
    if (!r) return UBQP_ENOMEM;
    if (!req_layout(n, elem_bytes, params, &r->R)) {
        delete r;
        set_err(s, "invalid n, element size or parameters");
        return UBQP_EINVAL;
    }
    r->n = n;
    r->elem = elem_bytes;
    r->q_host = q_host;
    r->pr = *params;
    r->bestx_host = best_x_host;
    r->stats_host = stats_host;
    r->prob = r->R.geom;
    r->prob.ctx = s->ctx;
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(s->m);
        if (s->dead || s->stop) {
            delete r;
            return UBQP_EDEVICE;
        }
        if (r->R.total > s->pool.size) {
            s->err = "request footprint exceeds the pool";
            delete r;
            return UBQP_EINVAL;
        }
        if (s->queue_limit > 0 && (int64_t)s->queue.size() >= s->queue_limit) {
            s->err = "the waiting queue is at its limit";
            delete r;
            return UBQP_EBUSY;
        }
        r->id = s->next_id++;
        *id = r->id;
        s->queue.push_back(r);
        s->cnt[C_SUBMITTED]++;
        s->cnt[C_WAITING]++;
    }
    s->cv_work.notify_one();
    return UBQP_OK;
}

int ubqp_server_set_queue_limit(ubqp_server *s, int64_t max_waiting)
{
    if (!s) return UBQP_EINVAL;
    if (max_waiting < 0) {
        set_err(s, "negative queue limit");
        return UBQP_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->m);
    s->queue_limit = max_waiting;
    return UBQP_OK;
}

int ubqp_server_wait(ubqp_server *s, int64_t timeout_us, ubqp_request_info *done, int32_t max, int32_t *count)
{
    if (!s || !done || !count || max < 1) return UBQP_EINVAL;
    std::unique_lock<std::mutex> lk(s->m);
    auto ready = [&] { return !s->done.empty() || s->dead; };
    if (timeout_us < 0)
        s->cv_done.wait(lk, ready);
    else
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        done[k++] = s->done.front();
        s->done.pop_front();
    }
    *count = k;
    return (k == 0 && s->dead) ? UBQP_EDEVICE : UBQP_OK;
}

int ubqp_server_stats(ubqp_server *s, int64_t out[8])
{
    if (!s || !out) return UBQP_EINVAL;
    for (int i = 0; i < 8; i++) out[i] = s->cnt[i];
    return UBQP_OK;
}

const char *ubqp_server_error(ubqp_server *s)
{
    if (!s) return "null server";
    std::lock_guard<std::mutex> lk(s->m);
    return s->err.c_str();
}

int ubqp_server_destroy(ubqp_server *s)
{
    if (!s) return UBQP_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    {
        std::lock_guard<std::mutex> lk(s->m);
        for (Req *r : s->queue) delete r;
        s->queue.clear();
    }
    server_free(s);
    return UBQP_OK;
}

}  // extern "C"
