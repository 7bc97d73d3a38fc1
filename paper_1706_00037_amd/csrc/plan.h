// Generation launch tables shared by the multi-start run/batch (plan.hip) and
// the request server (serve.hip).
//
// One generation of the multi-start loop of Fig. 2 is a fixed sequence of
// launches, each covering every instance of a set:
//   diversify -> eval_init + eval (row dot) -> [f dump] -> screen -> ascent order ->
//   per passer chunk and (planes, 16-column blocks) group: Delta init + ascent ->
//   incumbent, ranking, seed fill, generation counter.
// A launch table holds, for one step, each instance's kernel arguments and the
// prefix of the blocks (or waves) each instance needs.  Instances are independent:
// each one's results depend only on its own problem, parameters and state.
#pragma once

#include <string.h>

#include <vector>

#include "ubqp_internal.h"

inline size_t ubqp_align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Offsets of one instance's device state inside its allocation.
struct InstLayout {
    size_t seeds, X, f, flips, idx, oidx, rank, scal, bestx, stats, part, err, Y, total;
    int64_t S, cap;
};
InstLayout ubqp_inst_layout(const ubqp_problem *p, const ubqp_params *pr);

// One instance as the launch tables see it.
struct InstRef {
    const ubqp_problem *p;
    ubqp_params pr;
    InstLayout L;
    char *base;      // device state, L.total bytes
    int64_t *dump;   // optional G x M objective dump (device)
    int32_t *err;    // device error flag the instance's ascent reports to
    template <typename T> T *at(size_t off) const { return (T *)(base + off); }
};

template <typename A> struct Table {
    std::vector<A> args;
    std::vector<int64_t> prefix{0};
    size_t args_off = 0, pre_off = 0;
    const A *d_args = nullptr;
    const int64_t *d_pre = nullptr;
    void add(const A &a, int64_t blocks)
    {
        args.push_back(a);
        prefix.push_back(prefix.back() + blocks);
    }
    int count() const { return (int)args.size(); }
    int64_t total() const { return prefix.back(); }
    void stage(std::vector<char> &host)
    {
        args_off = ubqp_align256(host.size());
        host.resize(args_off + args.size() * sizeof(A));
        if (!args.empty()) memcpy(host.data() + args_off, args.data(), args.size() * sizeof(A));
        pre_off = ubqp_align256(host.size());
        host.resize(pre_off + prefix.size() * sizeof(int64_t));
        memcpy(host.data() + pre_off, prefix.data(), prefix.size() * sizeof(int64_t));
    }
    void bind(char *dev)
    {
        d_args = (const A *)(dev + args_off);
        d_pre = (const int64_t *)(dev + pre_off);
    }
};

struct Chunk {
    int planes, nb;
    int lane;  // side stream of its (planes, nb) group: chunks of one group stay in order
    Table<EvalArgs> yr;
    Table<AscArgs> asc;
    Table<AscArgs> team;  // the same ascents' team launch (few passers), empty when the group never uses teams
    int n_pad_max = 0;
};

// Side streams on which the (planes, NB) groups of the Delta initialisation and
// ascent run concurrently (they touch different instances); the generation's
// stream forks to them after the screen and joins them before the selection.
#define UBQP_SIDE_STREAMS 3
struct SideStreams {
    hipStream_t s[UBQP_SIDE_STREAMS] = {};
    hipEvent_t fork = nullptr, join[UBQP_SIDE_STREAMS] = {};
    hipError_t create();
    void destroy();
};

struct EvalGroup {         // instances whose row-dot contraction uses one variant
    int variant;
    Table<EvalArgs> t;
};

struct GenTables {
    int count = 0;
    Table<DivArgs> div;
    Table<EvalArgs> einit;
    std::vector<EvalGroup> ev;
    Table<ScreenArgs> scr;
    Table<OrdArgs> ord;                 // one block per instance
    Table<SelArgs> sel_cand, sel_rank, sel_seed;  // same arguments, three prefixes
    Table<SelArgs> init;                // generation-0 seeds of the joining instances
    std::vector<Chunk> chunks;
    bool has_dump = false;
    std::vector<char> host;             // staged image of every table

    // Builds every table for the instances and stages them into `host`; the
    // init table covers the instances with join[i] != 0 (all when join is null).
    void build(const std::vector<InstRef> &inst, const std::vector<char> *join = nullptr);
    // Points the tables at the device copy of `host`.
    void bind(char *dev);
};

// Generation-0 seeds and scalars of the instances in the init table.
hipError_t ubqp_queue_seed_init(const GenTables &t, hipStream_t st);
// All launches of one generation.  When pe != null, events pe[0..5] bound the five
// sequential phases and ae[2c], ae[2c + 1] the ascent launch of chunk group c; the
// groups then run in order on st.  Otherwise, with side != null and more than one
// group, the groups run concurrently on the side streams.
hipError_t ubqp_queue_generation(const GenTables &t, hipStream_t st, hipEvent_t *pe, hipEvent_t *ae = nullptr,
                                 const SideStreams *side = nullptr);
