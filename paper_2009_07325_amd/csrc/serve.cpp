// Serving loop: continuous batching of IMM queries over one resident graph.
//
// The graph and one RR pool per model stay resident in HBM.  Queries (k, eps, ell, model)
// are queued by imm_server_submit and admitted while fewer than max_active are in flight
// and the device-memory estimate stays inside the budget.  A worker thread runs ticks:
//   1. every active query names its next selection (ImmPlan::next): an RR range and how
//      far its pool must reach;
//   2. each pool is extended once, to the largest demand of its active queries, so RR
//      sets are generated once and shared by every query that reads them;
//   3. the selections of all active queries run as one multi-instance cooperative launch
//      (their argmax/cover rounds overlap on the device);
//   4. each query applies its covered count (ImmPlan::complete); finished queries leave,
//      and queries that arrived meanwhile are admitted for the next tick.
// A query reads only RR sets [0, theta) of its pool (or its fresh range), so its result is
// a pure function of (graph, model, pool seed, k, eps, ell): the same alone or in any mix,
// and the same as imm_solve with that seed.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.hpp"

using namespace imm;

namespace {

struct Query {
    uint64_t ticket = 0;
    int32_t k = 0;
    double eps = 0, ell = 0;
    imm_model model = IMM_IC;
    int32_t fresh = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    ImmPlan plan;
    int slot = -1;
    // current selection
    int64_t gen_upto = 0, sel_first = 0, sel_count = 0;
    double t_gen = 0, t_sel = 0;
};

struct Result {
    imm_status status = IMM_OK;
    std::string error;
    std::vector<int32_t> seeds;
    imm_info info{};
};

}  // namespace

struct imm_server {
    const imm_graph* g = nullptr;
    imm_pool* pools[2] = {nullptr, nullptr};   // IC, LT (worker thread only after creation)
    uint64_t seeds[2] = {0, 0};
    int64_t budget = 0;
    int32_t max_active = 0;
    hipStream_t stream = nullptr;

    std::vector<SelectWs> slots;
    std::vector<int> free_slots;
    SelectLaunch launch;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Query> queue;
    std::vector<Query> active;
    std::unordered_map<uint64_t, Result> results;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    // statistics (under mu)
    int64_t submitted = 0, completed = 0, rejected = 0, ticks = 0;
    std::atomic<int64_t> pool_resets{0};
    double t_first_submit = -1.0, t_last_done = 0.0;
    std::vector<double> latencies;
    imm_status worker_status = IMM_OK;
    std::string worker_error;
    std::atomic<int64_t> n_active{0};
    std::atomic<int64_t> bytes_snapshot{0};                      // device_bytes() after a tick
    std::atomic<double> mean_members[2] = {{16.0}, {16.0}};   // per pool, after each generation
    std::atomic<int64_t> pool_sets[2] = {{0}, {0}};
    bool trace = false;                                        // IMM_SERVE_TRACE=1: a line per tick
    bool frugal = false;       // IMM_SERVE_FRUGAL=1: drop every pool no query reads after each tick
    // coverage seen per pool (worker thread only): for recent selections, the fraction of
    // their sets covered after each greedy round they ran, and their number of sets
    struct Seen {
        std::vector<double> cum;
        int64_t sets;
    };
    std::vector<Seen> cov_seen[2];

    int64_t device_bytes() const {
        int64_t b = 0;
        for (imm_pool* p : pools)
            if (p) b += p->bytes();
        for (const SelectWs& w : slots) b += w.bytes();
        return b;
    }
};

namespace {

// Device bytes of a query's selection workspace (counters, inverted index over the prefix
// it reads, covered flags).  The prefix is at least the first estimation phase,
// ceil(lambda' / (n/2)), and at most theta <= lambda*; for admission we take the larger of
// the first phase and the pool's current size (queries mostly read what is already there),
// for rejection at submission only the first phase.
int64_t query_bytes(const imm_server* S, const Query& q, bool minimal) {
    const int64_t n = S->g->n;
    const double mean = S->mean_members[q.model].load();
    const double first_phase = std::ceil(q.plan.lam1 / ((double)n / 2.0));
    double sets = minimal ? first_phase
                          : std::min(q.plan.lam2, std::max(first_phase, (double)S->pool_sets[q.model].load()));
    sets = std::min(sets, (double)kMaxSets);
    const double members = std::min(sets * mean, 4e9);
    return n * 20 + (int64_t)(members * 4.0) + (int64_t)(sets * 4.0);
}

// Device bytes that one query's next step needs on its own: the pool grown to the sets the
// step reads (offsets, lengths and members at the pool's measured mean size; the member
// buffer grows by doubling, so up to twice that) plus the step's selection workspace.  A
// query whose step needs more than the whole budget can never run and is rejected with
// IMM_ECAPACITY before its pool grows (gIM Alg. 2 / Alg. 1 sample sizes grow without
// bound as eps shrinks, while device memory does not).  The final selection reads at least
// theta = lambda* / LB >= lambda* / n sets (LB = n F_R(S) / (1 + eps') never exceeds n),
// so every step is charged for at least that many: a query that cannot reach its final
// selection is rejected at its first step instead of after its estimation phases.
double bytes_for(const imm_server* S, const Query& q, double sets, double sel) {
    const double n = (double)S->g->n;
    const double mean = S->mean_members[q.model].load();
    const imm_pool* p = S->pools[q.model];
    // generation scratch: what the pool's context holds, and the heavy scratch its first
    // heavy launch allocates
    const double gen = (double)p->gen.bytes() + (double)p->gen.heavy_bytes(S->g->n);
    const double pool = sets * 12.0 + 2.0 * sets * mean * 4.0 + n * 4.0 + gen;
    const double ws = n * 20.0 + sel * mean * 4.0 + sel * 4.0;
    return pool + ws;
}

// Upper bound on the coverage fraction that a query's k greedy seeds reach in its passing
// estimation phase, from the selections already run on its pool.  A selection that ran r
// rounds gives the coverage after each j <= r seeds; past r, greedy gains never increase,
// so k seeds cover at most the coverage after r plus (k - r) times round r's gain.  The
// fraction greedy reaches shrinks, if anything, as the sample grows (it fits a small sample
// better), so only selections over no more sets than the query's first phase reads are
// used.  The bound carries a 25 % allowance for sampling noise (1 when no such selection
// was seen).
double cover_bound(const imm_server* S, const Query& q) {
    const double first_phase = std::ceil(q.plan.lam1 / ((double)S->g->n / 2.0));
    double c = 1.0;
    for (const imm_server::Seen& o : S->cov_seen[q.model]) {
        const size_t r = o.cum.size();
        if (r == 0 || (double)o.sets > first_phase) continue;
        const size_t k = (size_t)q.k;
        const double at = k <= r ? o.cum[k - 1]
                                 : o.cum[r - 1] + (double)(k - r) * (o.cum[r - 1] - (r >= 2 ? o.cum[r - 2] : 0.0));
        c = std::min(c, 1.25 * at);
    }
    return std::max(c, 1e-12);
}

double step_bytes(const imm_server* S, const Query& q) {
    // theta = lambda* / LB with LB = n c / (1 + eps') for the passing phase's coverage c
    const double final_min = std::ceil(q.plan.lam2 * (1.0 + q.plan.ep) / ((double)S->g->n * cover_bound(S, q)));
    return bytes_for(S, q, std::max((double)q.gen_upto, final_min),
                     std::max((double)q.sel_count, final_min));
}

// After a failed estimation phase (coverage fraction c of its k seeds): the phase that
// passes has x <= n c' / (1 + eps') with c' its own coverage fraction, about c (greedy on
// the smaller sample tends to overstate it), so it reads about lambda' (1 + eps') / (n c)
// sets.  Bytes of that phase (lambda* when the seeds covered nothing).
double predicted_pass_bytes(const imm_server* S, const Query& q, int64_t cov, int64_t count) {
    const double n = (double)S->g->n;
    const ImmPlan& P = q.plan;
    const double sets = cov > 0 ? P.lam1 * (1.0 + P.ep) / (n * ((double)cov / (double)count)) : P.lam2;
    return bytes_for(S, q, sets, sets);
}

void finish(imm_server* S, Query& q, imm_status st, const std::string& err);

bool pool_in_use(const imm_server* S, int m, const std::vector<Query>* also = nullptr) {
    for (const Query& q : S->active)
        if (q.model == m) return true;
    if (also)
        for (const Query& q : *also)
            if (q.model == m) return true;
    return false;
}

// Device bytes held by the pools of the other model while queries read them.
double pinned_bytes(const imm_server* S, int m, const std::vector<Query>* also = nullptr) {
    const int o = 1 - m;
    return S->pools[o] && pool_in_use(S, o, also) ? (double)S->pools[o]->bytes() : 0.0;
}

// Drops the sets of a pool that no active query reads, to give its memory to queries that
// need it (a pool's sets are a pure function of its seed: a later query that reads them
// draws them again, identically).  Returns the device bytes given back.
double reset_idle_pool(imm_server* S, int m, const std::vector<Query>* also = nullptr) {
    imm_pool* p = S->pools[m];
    if (!p || p->count == 0 || pool_in_use(S, m, also)) return 0.0;
    imm_pool* fresh = nullptr;
    if (imm_pool_create(S->g, (imm_model)m, S->seeds[m], &fresh) != IMM_OK) return 0.0;
    const double freed = (double)p->bytes() - (double)fresh->bytes();
    for (SelectWs& w : S->slots)
        if (w.ix_pool == p) {
            w.ix_pool = nullptr;
            w.snap_valid = false;
        }
    imm_pool_destroy(p);
    S->pools[m] = fresh;
    S->pool_sets[m].store(0);
    S->pool_resets += 1;
    return freed;
}

void reject_budget(imm_server* S, Query& q, double need) {
    char msg[200];
    snprintf(msg, sizeof msg,
             "query needs about %.3g bytes of device memory (its final selection reads at least "
             "%.3g RR sets), more than the server budget of %lld",
             need, std::ceil(q.plan.lam2 * (1.0 + q.plan.ep) / ((double)S->g->n * cover_bound(S, q))),
             (long long)S->budget);
    finish(S, q, IMM_ECAPACITY, msg);
}

// Sets generated first on an empty pool, to measure its mean set size before any query's
// demand is checked against the budget.
constexpr int64_t kPilotSets = 1024;

void finish(imm_server* S, Query& q, imm_status st, const std::string& err) {
    S->n_active.fetch_sub(1);
    Result r;
    r.status = st;
    r.error = err;
    q.t_done = now_s();
    if (st == IMM_OK) {
        const ImmPlan& P = q.plan;
        imm_pool* p = S->pools[q.model];
        r.seeds.assign(S->slots[q.slot].host_seeds, S->slots[q.slot].host_seeds + q.k);
        imm_info& info = r.info;
        info.theta = P.theta;
        info.num_rr = P.upto;
        info.covered = P.covered;
        info.edges_examined = (int64_t)(p->sum.edges + p->sum.hedges);
        info.edges_heavy = (int64_t)p->sum.hedges;
        info.pool_ids = (int64_t)p->sum.placed;
        info.phases = P.phases;
        info.lb = P.lb;
        info.spread_est = P.spread_est();
        info.lambda_prime = P.lam1;
        info.lambda_star = P.lam2;
        info.t_generate_s = q.t_gen;
        info.t_select_s = q.t_sel;
        info.t_total_s = q.t_done - q.t_submit;   // latency: submission to completion
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->results[q.ticket] = std::move(r);
    if (q.slot >= 0) S->free_slots.push_back(q.slot);
    q.slot = -1;
    if (st == IMM_OK) {
        S->completed += 1;
        S->latencies.push_back(q.t_done - q.t_submit);
        S->t_last_done = q.t_done;
    } else {
        S->rejected += 1;
    }
    S->cv_done.notify_all();
}

// One scheduler iteration; returns false when there was nothing to do.
bool tick(imm_server* S) {
    // admission (continuous batching: new queries join at every tick)
    {
        std::lock_guard<std::mutex> lk(S->mu);
        while (!S->queue.empty() && !S->free_slots.empty()) {
            Query& q = S->queue.front();
            const int64_t need = query_bytes(S, q, false);
            const int64_t used = S->device_bytes();
            if (!S->active.empty() && used + need > S->budget) {
                // the memory of a pool no active query reads goes to the waiting query;
                // otherwise it waits for memory
                if (reset_idle_pool(S, 1 - q.model) > 0.0 || reset_idle_pool(S, q.model) > 0.0) continue;
                break;
            }
            q.slot = S->free_slots.back();
            S->free_slots.pop_back();
            q.t_admit = now_s();
            S->active.push_back(std::move(q));
            S->queue.pop_front();
            S->n_active.store((int64_t)S->active.size());
        }
        if (S->active.empty()) return false;
    }
    S->ticks += 1;
    S->bytes_snapshot.store(S->device_bytes());
    std::vector<Query>& act = S->active;
    const double t_tick = now_s();
    double tr_gen[2] = {0.0, 0.0};
    int64_t tr_sets = 0;
    // 1. next selection of every active query
    for (size_t i = 0; i < act.size();) {
        Query& q = act[i];
        imm_status st = q.plan.next(&q.gen_upto, &q.sel_first, &q.sel_count);
        if (st != IMM_OK) {
            finish(S, q, st, imm_last_error());
            act.erase(act.begin() + (long)i);
            continue;
        }
        // once its pool's set size is measured, a query whose final selection cannot fit the
        // budget leaves before any work on it (the same test as before a pool grows)
        const imm_pool* p = S->pools[q.model];
        if (p && p->count >= kPilotSets && !q.plan.reuses_last()) {
            const double need = step_bytes(S, q) + pinned_bytes(S, q.model);
            if (need > (double)S->budget) {
                reject_budget(S, q, need);
                act.erase(act.begin() + (long)i);
                continue;
            }
        }
        ++i;
    }
    if (act.empty()) return true;
    // 1b. the tick's added demand (pools grown to the largest step, every step's selection
    //     workspace) must fit what the budget and the device have left: the most recently
    //     admitted queries sit this tick out (their workspace memory given back) until it
    //     does, the oldest one always runs.  Without this, queries admitted together could
    //     each fit alone and run out of device memory together as their estimation phases
    //     grow.
    //     A query whose final selection repeats its last one (no selection, no memory)
    //     is never held: its result sits in its workspace.
    std::vector<Query> held;
    struct Restore {             // held queries rejoin the active list however the tick ends
        std::vector<Query>& act;
        std::vector<Query>& held;
        ~Restore() {             // newest was held first: rejoin oldest first
            for (auto it = held.rbegin(); it != held.rend(); ++it) act.push_back(std::move(*it));
        }
    } restore{act, held};
    {
        // room: what the budget leaves and what the device has (free plus the allocator's
        // cache, which is given back when an allocation fails), less a margin
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            free_b = 0;
        }
        const double margin = (double)((int64_t)2 << 30);
        double room = std::min((double)S->budget - (double)S->device_bytes(),
                               (double)free_b + (double)dev_cached_bytes() - margin);
        const double n = (double)S->g->n;
        auto ws_growth = [&](const Query& q) {
            if (q.plan.reuses_last()) return 0.0;
            const double need = n * 20.0 + (double)q.sel_count * (S->mean_members[q.model].load() * 4.0 + 4.0);
            return std::max(0.0, need - (double)S->slots[q.slot].bytes());
        };
        // transient bytes of growing a pool to `target` sets: new offset / length arrays
        // and a new id buffer (capacities double; old and new coexist during the copy),
        // plus the heavy-kernel scratch of a pool that has none yet
        auto pool_growth = [&](int m, int64_t target) {
            const imm_pool* p = S->pools[m];
            if (!p || target <= p->count) return 0.0;
            double b = 0.0;
            auto grown = [](int64_t cap, double need) {
                double c = cap > 0 ? (double)cap : 1024.0;
                while (c < need) c *= 2.0;
                return c;
            };
            if (target > p->cap_sets) b += grown(p->cap_sets, (double)target) * 12.0;
            const double ids = (double)p->sum.placed +
                               (double)(target - p->count) * S->mean_members[m].load() * 1.3 + (1 << 24);
            if (ids > (double)p->cap_ids) b += grown(p->cap_ids, ids) * 4.0;
            b += (double)p->gen.heavy_bytes(S->g->n);
            return b;
        };
        for (;;) {
            double need = 0.0;
            int64_t target[2] = {0, 0};
            for (const Query& q : act) {
                target[q.model] = std::max(target[q.model], q.gen_upto);
                need += ws_growth(q);
            }
            need += pool_growth(0, target[0]) + pool_growth(1, target[1]);
            if (need <= room) break;
            // first the memory of pools no query of this tick reads
            const double freed = reset_idle_pool(S, 0, &held) + reset_idle_pool(S, 1, &held);
            if (freed > 0.0) {
                room += freed;
                continue;
            }
            size_t at = act.size();              // the newest query that may sit out
            while (at > 1 && act[at - 1].plan.reuses_last()) --at;
            if (at <= 1) break;                  // the oldest query always runs
            Query& q = act[at - 1];
            room += (double)S->slots[q.slot].bytes();
            S->slots[q.slot].release();
            held.push_back(std::move(q));
            act.erase(act.begin() + (long)(at - 1));
        }
    }
    // 2. one generation per pool, to the largest demand.  An empty pool first gets a pilot
    //    of kPilotSets sets (the same sets any query reads first) so that the mean set size
    //    is measured; then queries whose step cannot fit the budget are rejected, and the
    //    pool is extended for the rest.
    auto fail_model = [&](int m, imm_status st, const std::string& err) {
        for (size_t i = 0; i < act.size();) {
            if (act[i].model != m) {
                ++i;
                continue;
            }
            finish(S, act[i], st, err);
            act.erase(act.begin() + (long)i);
        }
    };
    for (int m = 0; m < 2; ++m) {
        imm_pool* p = S->pools[m];
        if (!p) continue;
        int64_t target = 0;
        for (const Query& q : act)
            if (q.model == m) target = std::max(target, q.gen_upto);
        if (target <= p->count) continue;
        double t_pilot = 0.0;
        if (p->count < kPilotSets) {
            const double t0 = now_s();
            imm_status st = pool_generate(p, std::min(target, kPilotSets), S->stream);
            t_pilot = now_s() - t0;
            if (st != IMM_OK) {
                fail_model(m, st, imm_last_error());
                continue;
            }
            S->mean_members[m].store((double)p->sum.placed / (double)p->count);
            S->pool_sets[m].store(p->count);
        }
        target = 0;
        for (size_t i = 0; i < act.size();) {
            Query& q = act[i];
            if (q.model != m) {
                ++i;
                continue;
            }
            q.t_gen += t_pilot;
            const double need = step_bytes(S, q) + pinned_bytes(S, m, &held);
            if (need > (double)S->budget) {
                reject_budget(S, q, need);
                act.erase(act.begin() + (long)i);
                continue;
            }
            target = std::max(target, q.gen_upto);
            ++i;
        }
        if (target <= p->count) continue;
        const double t0 = now_s();
        imm_status st = pool_generate(p, target, S->stream);
        const double dt = now_s() - t0;
        tr_gen[m] += dt + t_pilot;
        if (st == IMM_OK && p->count > 0)
            S->mean_members[m].store((double)p->sum.placed / (double)p->count);
        S->pool_sets[m].store(p->count);
        for (Query& q : act)
            if (q.model == m) q.t_gen += dt;
        if (st != IMM_OK) fail_model(m, st, imm_last_error());
    }
    // 3. all selections in one cooperative launch
    //    (a query whose final selection repeats its last one keeps that one's result)
    const double t0 = now_s();
    std::vector<SelInst> inst;
    std::vector<SelectWs*> ws;
    // A launch of several instances reads every counter of every instance in each round; a
    // single instance keeps exact counts for its most frequent vertices only (hot set).  On
    // graphs large enough for a hot set, the tick's selections therefore run one launch
    // each, with their hot sets; otherwise together in one launch.
    size_t nsel = 0;
    bool hot_all = true;
    for (const Query& q : act) {
        if (q.plan.reuses_last()) continue;
        ++nsel;
        if (select_hot_max(S->pools[q.model]->g->n) == 0) hot_all = false;
    }
    const bool each = nsel == 1 || hot_all;
    imm_status st = IMM_OK;
    for (size_t i = 0; i < act.size();) {
        Query& q = act[i];
        if (q.plan.reuses_last()) {
            ++i;
            continue;
        }
        SelInst si{};
        const imm_status ps = select_prepare(S->pools[q.model], &S->slots[q.slot], q.sel_first, q.sel_count,
                                             q.k, S->stream, &si, false, each);
        if (ps != IMM_OK) {
            // this query's workspace did not fit: it alone fails, and its slot's memory is
            // given back for the others
            const std::string err = imm_last_error();
            S->slots[q.slot].release();
            finish(S, q, ps, err);
            act.erase(act.begin() + (long)i);
            continue;
        }
        si.need = q.plan.need_cov();
        tr_sets += q.sel_count;
        if (each) {
            SelectWs* w = &S->slots[q.slot];
            st = select_run(&S->launch, &w, &si, 1, S->stream);
            if (st != IMM_OK) break;
        } else {
            ws.push_back(&S->slots[q.slot]);
            inst.push_back(si);
        }
        ++i;
    }
    if (st == IMM_OK && !inst.empty())
        st = select_run(&S->launch, ws.data(), inst.data(), (int32_t)inst.size(), S->stream);
    const double dt = now_s() - t0;
    if (st != IMM_OK) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->worker_status = st;
        S->worker_error = imm_last_error();
        return false;
    }
    // 4. advance every query
    const size_t tr_ran = act.size();
    for (size_t i = 0; i < act.size();) {
        Query& q = act[i];
        q.t_sel += dt;
        const bool estimating = !q.plan.final_phase;
        const int64_t cov = (int64_t)*S->slots[q.slot].host_cov;
        if (!q.plan.reuses_last() && q.sel_count > 0) {
            // gains of the rounds run (a stopped phase ends early)
            imm_server::Seen o{{}, q.sel_count};
            const unsigned long long* keys = S->slots[q.slot].host_keys;
            double acc = 0.0;
            for (int32_t j = 0; j < q.k && keys[j] != 0; ++j) {
                acc += (double)((keys[j] >> 32) - 1);
                o.cum.push_back(acc / (double)q.sel_count);
            }
            auto& seen = S->cov_seen[q.model];
            if (seen.size() >= 32) seen.erase(seen.begin());
            if (!o.cum.empty()) seen.push_back(std::move(o));
        }
        imm_status cs = q.plan.complete(cov);
        if (cs != IMM_OK || q.plan.done) {
            finish(S, q, cs, cs == IMM_OK ? "" : imm_last_error());
            act.erase(act.begin() + (long)i);
            continue;
        }
        if (estimating && !q.plan.final_phase) {
            // the phase failed: a query whose passing phase cannot fit the budget leaves now
            // rather than after the phases in between
            const double need = predicted_pass_bytes(S, q, cov, q.sel_count) + pinned_bytes(S, q.model, &held);
            if (need > (double)S->budget) {
                char msg[200];
                snprintf(msg, sizeof msg,
                         "query's estimation would need about %.3g bytes of device memory (its "
                         "seeds covered %lld of %lld RR sets), more than the server budget of %lld",
                         need, (long long)cov, (long long)q.sel_count, (long long)S->budget);
                finish(S, q, IMM_ECAPACITY, msg);
                act.erase(act.begin() + (long)i);
                continue;
            }
        }
        ++i;
    }
    if (S->trace) {
        fprintf(stderr,
                "[imm serve] tick %lld: %zu ran, %zu held; generation IC %.3f s (%lld sets), LT "
                "%.3f s (%lld sets); %zu selections over %lld sets %.3f s; tick %.3f s; %.1f GB\n",
                (long long)S->ticks, tr_ran, held.size(), tr_gen[0],
                S->pools[0] ? (long long)S->pools[0]->count : 0ll, tr_gen[1],
                S->pools[1] ? (long long)S->pools[1]->count : 0ll, inst.size(), (long long)tr_sets, dt,
                now_s() - t_tick, (double)S->device_bytes() * 1e-9);
    }
    if (S->frugal) {
        reset_idle_pool(S, IMM_IC, &held);
        reset_idle_pool(S, IMM_LT, &held);
    }
    return true;
}

void worker_main(imm_server* S) {
    (void)hipSetDevice(S->g->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty() || !S->active.empty(); });
            if (S->stop) return;
            if (S->worker_status != IMM_OK) return;
        }
        if (!tick(S)) {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->worker_status != IMM_OK) {
                // fail every query still pending, then stop serving
                for (Query& q : S->active) {
                    Result r;
                    r.status = S->worker_status;
                    r.error = S->worker_error;
                    S->results[q.ticket] = std::move(r);
                }
                for (Query& q : S->queue) {
                    Result r;
                    r.status = S->worker_status;
                    r.error = S->worker_error;
                    S->results[q.ticket] = std::move(r);
                }
                S->active.clear();
                S->queue.clear();
                S->n_active.store(0);
                S->cv_done.notify_all();
                return;
            }
        }
    }
}

}  // namespace

extern "C" imm_status imm_server_create(const imm_graph* g, uint64_t seed_ic, uint64_t seed_lt,
                                        int64_t hbm_budget_bytes, int32_t max_active,
                                        imm_server** out) {
    if (!out) return fail(IMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(IMM_EINVAL, "graph is NULL");
    if (max_active < 1 || max_active > 1024) return fail(IMM_EINVAL, "max_active %d outside [1, 1024]", max_active);
    if (hbm_budget_bytes <= 0) return fail(IMM_EINVAL, "hbm budget must be positive");
    imm_server* S = new imm_server();
    S->g = g;
    S->budget = hbm_budget_bytes;
    S->max_active = max_active;
    S->seeds[IMM_IC] = seed_ic;
    S->seeds[IMM_LT] = seed_lt;
    if (const char* e = getenv("IMM_SERVE_TRACE")) S->trace = atoi(e) != 0;
    if (const char* e = getenv("IMM_SERVE_FRUGAL")) S->frugal = atoi(e) != 0;
    imm_status st = IMM_OK;
    if (g->has_ic) st = imm_pool_create(g, IMM_IC, seed_ic, &S->pools[IMM_IC]);
    if (st == IMM_OK && g->has_lt) st = imm_pool_create(g, IMM_LT, seed_lt, &S->pools[IMM_LT]);
    if (st == IMM_OK && hipStreamCreate(&S->stream) != hipSuccess)
        st = fail(IMM_EDEVICE, "hipStreamCreate failed");
    if (st != IMM_OK) {
        imm_pool_destroy(S->pools[0]);
        imm_pool_destroy(S->pools[1]);
        delete S;
        return st;
    }
    S->slots.resize((size_t)max_active);
    for (int i = max_active - 1; i >= 0; --i) S->free_slots.push_back(i);
    S->worker = std::thread(worker_main, S);
    *out = S;
    return IMM_OK;
}

extern "C" imm_status imm_server_submit(imm_server* S, int32_t k, double eps, double ell,
                                        imm_model model, int32_t fresh_final, uint64_t* ticket) {
    if (!S || !ticket) return fail(IMM_EINVAL, "NULL argument");
    if (model != IMM_IC && model != IMM_LT) return fail(IMM_EINVAL, "unknown model %d", (int)model);
    if (!(model == IMM_IC ? S->g->has_ic : S->g->has_lt))
        return fail(IMM_EINVAL, "graph has no encoding for model %d", (int)model);
    Query q;
    IMM_TRY(q.plan.init(S->g->n, k, eps, ell, fresh_final));
    q.k = k;
    q.eps = eps;
    q.ell = ell;
    q.model = model;
    q.fresh = fresh_final;
    q.t_submit = now_s();
    if (query_bytes(S, q, true) > S->budget)
        return fail(IMM_ECAPACITY, "query needs more device memory than the server budget");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->worker_status != IMM_OK) return fail(S->worker_status, "server stopped: %s", S->worker_error.c_str());
    q.ticket = S->next_ticket++;
    *ticket = q.ticket;
    S->submitted += 1;
    if (S->t_first_submit < 0) S->t_first_submit = q.t_submit;
    S->queue.push_back(std::move(q));
    S->cv_work.notify_one();
    return IMM_OK;
}

static imm_status take_result(imm_server* S, uint64_t ticket, int32_t* seeds_out, imm_info* info,
                              int32_t* done) {
    auto it = S->results.find(ticket);
    if (it == S->results.end()) {
        if (done) *done = 0;
        return IMM_OK;
    }
    if (done) *done = 1;
    const Result& r = it->second;
    if (r.status != IMM_OK) return fail(r.status, "query %llu failed: %s", (unsigned long long)ticket, r.error.c_str());
    if (seeds_out) memcpy(seeds_out, r.seeds.data(), sizeof(int32_t) * r.seeds.size());
    if (info) *info = r.info;
    return IMM_OK;
}

extern "C" imm_status imm_server_poll(imm_server* S, uint64_t ticket, int32_t* seeds_out,
                                      imm_info* info, int32_t* done) {
    if (!S) return fail(IMM_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    if (ticket == 0 || ticket >= S->next_ticket) return fail(IMM_EINVAL, "unknown ticket");
    return take_result(S, ticket, seeds_out, info, done);
}

extern "C" imm_status imm_server_wait(imm_server* S, uint64_t ticket, double timeout_s,
                                      int32_t* seeds_out, imm_info* info) {
    if (!S) return fail(IMM_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    if (ticket == 0 || ticket >= S->next_ticket) return fail(IMM_EINVAL, "unknown ticket");
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 1e9));
    if (!S->cv_done.wait_until(lk, deadline, [&] { return S->results.count(ticket) > 0; }))
        return fail(IMM_EBUSY, "query %llu not finished within %g s", (unsigned long long)ticket, timeout_s);
    int32_t done = 0;
    return take_result(S, ticket, seeds_out, info, &done);
}

extern "C" imm_status imm_server_stats_get(imm_server* S, imm_server_stats* out) {
    if (!S || !out) return fail(IMM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    memset(out, 0, sizeof *out);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->active = S->n_active.load();
    out->queued = (int64_t)S->queue.size();
    out->ticks = S->ticks;
    std::vector<double> lat = S->latencies;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            size_t i = (size_t)std::ceil(p * (double)lat.size()) - 1;
            return lat[std::min(i, lat.size() - 1)];
        };
        out->p50_latency_s = pct(0.50);
        out->p99_latency_s = pct(0.99);
        double sum = 0;
        for (double v : lat) sum += v;
        out->mean_latency_s = sum / (double)lat.size();
        out->max_latency_s = lat.back();
        const double span = S->t_last_done - S->t_first_submit;
        out->throughput_qps = span > 0 ? (double)S->completed / span : 0.0;
    }
    out->pool_sets_ic = S->pool_sets[IMM_IC].load();
    out->pool_sets_lt = S->pool_sets[IMM_LT].load();
    out->device_bytes = S->bytes_snapshot.load();
    out->pool_resets = S->pool_resets.load();
    return IMM_OK;
}

extern "C" imm_status imm_server_destroy(imm_server* S) {
    if (!S) return IMM_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (SelectWs& w : S->slots) w.release();
    S->launch.release();
    imm_pool_destroy(S->pools[0]);
    imm_pool_destroy(S->pools[1]);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return IMM_OK;
}
