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
    imm_pool* pools[2] = {nullptr, nullptr};   // IC, LT
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
    double t_first_submit = -1.0, t_last_done = 0.0;
    std::vector<double> latencies;
    imm_status worker_status = IMM_OK;
    std::string worker_error;
    std::atomic<int64_t> n_active{0};
    std::atomic<int64_t> bytes_snapshot{0};                      // device_bytes() after a tick
    std::atomic<double> mean_members[2] = {{16.0}, {16.0}};   // per pool, after each generation
    std::atomic<int64_t> pool_sets[2] = {{0}, {0}};

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
// bound as eps shrinks, while device memory does not).
double step_bytes(const imm_server* S, const Query& q) {
    const double n = (double)S->g->n;
    const double mean = S->mean_members[q.model].load();
    const double sets = (double)q.gen_upto;
    const double pool = sets * 12.0 + 2.0 * sets * mean * 4.0;
    const double sel = (double)q.sel_count;
    const double ws = n * 20.0 + sel * mean * 4.0 + sel * 4.0;
    return pool + ws;
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
            if (!S->active.empty() && used + need > S->budget) break;   // wait for memory
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
    // 1. next selection of every active query
    for (size_t i = 0; i < act.size();) {
        Query& q = act[i];
        imm_status st = q.plan.next(&q.gen_upto, &q.sel_first, &q.sel_count);
        if (st != IMM_OK) {
            finish(S, q, st, imm_last_error());
            act.erase(act.begin() + (long)i);
            continue;
        }
        ++i;
    }
    if (act.empty()) return true;
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
            const double need = step_bytes(S, q);
            if (need > (double)S->budget) {
                char msg[160];
                snprintf(msg, sizeof msg,
                         "query needs about %.3g bytes of device memory for %lld RR sets, more than "
                         "the server budget of %lld",
                         need, (long long)q.gen_upto, (long long)S->budget);
                finish(S, q, IMM_ECAPACITY, msg);
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
    for (size_t i = 0; i < act.size();) {
        Query& q = act[i];
        if (q.plan.reuses_last()) {
            ++i;
            continue;
        }
        SelInst si{};
        imm_status st = select_prepare(S->pools[q.model], &S->slots[q.slot], q.sel_first, q.sel_count,
                                       q.k, S->stream, &si);
        if (st != IMM_OK) {
            // this query's workspace did not fit: it alone fails, and its slot's memory is
            // given back for the others
            const std::string err = imm_last_error();
            S->slots[q.slot].release();
            finish(S, q, st, err);
            act.erase(act.begin() + (long)i);
            continue;
        }
        si.need = q.plan.need_cov();
        ws.push_back(&S->slots[q.slot]);
        inst.push_back(si);
        ++i;
    }
    imm_status st = inst.empty() ? IMM_OK
                                 : select_run(&S->launch, ws.data(), inst.data(), (int32_t)inst.size(),
                                              S->stream);
    const double dt = now_s() - t0;
    if (st != IMM_OK) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->worker_status = st;
        S->worker_error = imm_last_error();
        return false;
    }
    // 4. advance every query
    for (size_t i = 0; i < act.size();) {
        Query& q = act[i];
        q.t_sel += dt;
        imm_status cs = q.plan.complete((int64_t)*S->slots[q.slot].host_cov);
        if (cs != IMM_OK || q.plan.done) {
            finish(S, q, cs, cs == IMM_OK ? "" : imm_last_error());
            act.erase(act.begin() + (long)i);
            continue;
        }
        ++i;
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
    if (!S->pools[model]) return fail(IMM_EINVAL, "graph has no encoding for model %d", (int)model);
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
