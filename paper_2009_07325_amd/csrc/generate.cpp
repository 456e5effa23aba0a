// Host side of RR-set generation: one light launch (and, when sets overflow the light
// path, one heavy launch) per call extends any number of pools at once.
//
// A pool's RR index space only grows (gIM Alg. 2 reuses R across estimation rounds, and
// Alg. 1 tops it up to theta), so each call covers [count, upto) of every pool it extends.
// Sets that find a pool's id buffer full are listed by the kernels; the buffer is grown
// and only those sets are run again, so the result never depends on the first guess of
// the buffer size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host.hpp"

using namespace imm;

// ------------------------------------------------------------------------------------
// GenCtx
// ------------------------------------------------------------------------------------
imm_status GenCtx::init(int device_, imm_model model_, int cus_, const GenTuning* tuning) {
    device = device_;
    model = model_;
    cus = cus_;
    grid = cus * gen_blocks_per_cu(model == IMM_LT ? 2 : 0);
    IMM_TRY(dalloc(&lc, 1));
    HIP_TRY(hipHostMalloc((void**)&host_lc, sizeof(LaunchCounters), hipHostMallocDefault));
    memset(host_lc, 0, sizeof(LaunchCounters));
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    HIP_TRY(hipEventCreate(&ev2));
    if (tuning && tuning->budget > 0) budget = tuning->budget;
    if (tuning && tuning->heavy_block > 0) heavy_block = tuning->heavy_block;
    if (const char* b = getenv("IMM_LIGHT_BUDGET")) budget = std::max(1ll, atoll(b));
    if (const char* b = getenv("IMM_HEAVY_SCRATCH_GIB"))
        heavy_scratch = std::max(1ll, atoll(b)) << 30;
    if (const char* b = getenv("IMM_HEAVY_BLOCK")) {
        const int v = atoi(b);
        if (v == 64 || v == 128 || v == 256 || v == 1024) heavy_block = v;
    }
    return IMM_OK;
}

int64_t GenCtx::bytes() const {
    return (int64_t)grid * 4 * vis_words * 4 + hslots * (vis_words * 4 + vis_n * 4) +
           cap_queue * (handoff ? 12 : 8) + (arena ? kArenaWords * 4 : 0) +
           cap_inst * (int64_t)(sizeof(GenInst) + 8 + sizeof(PoolSummary));
}

void GenCtx::release() {
    dfree(visited);
    dfree(hvisited);
    dfree(hlist);
    dfree(lc);
    hfree(host_lc);
    dfree(queue);
    dfree(handoff);
    dfree(arena);
    dfree(d_inst);
    hfree(host_inst);
    dfree(d_work_off);
    hfree(host_work_off);
    dfree(d_sum);
    hfree(host_sum);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (ev2) (void)hipEventDestroy(ev2);
    ev0 = ev1 = ev2 = nullptr;
    vis_n = vis_words = hslots = cap_queue = cap_inst = 0;
}

namespace {

// Light bitmaps for graphs of up to n vertices: at most ~4 GiB (fewer resident blocks on
// huge graphs).
imm_status ensure_light(GenCtx* c, int64_t n) {
    if (n <= c->vis_n && c->visited) return IMM_OK;
    dfree(c->visited);
    dfree(c->hvisited);     // the heavy scratch is sized by the same n; rebuilt on demand
    dfree(c->hlist);
    c->hslots = 0;
    c->vis_n = n;
    c->vis_words = (n + 31) / 32;
    c->grid = c->cus * gen_blocks_per_cu(c->model == IMM_LT ? 2 : 0);
    const int64_t per_block = 4 * c->vis_words * 4;
    const int64_t max_blocks = std::max<int64_t>(c->cus, ((int64_t)4 << 30) / per_block);
    if (c->grid > max_blocks) c->grid = (int)max_blocks;
    const int64_t words = (int64_t)c->grid * 4 * c->vis_words;
    IMM_TRY(dalloc(&c->visited, words));
    HIP_TRY(hipMemset(c->visited, 0, sizeof(uint32_t) * (size_t)words));
    return IMM_OK;
}

// Heavy scratch: slots (IC one per workgroup, LT one per wave) each with a bitmap and a
// member list of vis_n entries, bounded to c->heavy_scratch bytes (fewer concurrent heavy
// sets on huge graphs).
imm_status ensure_heavy(GenCtx* c) {
    if (c->hlist) return IMM_OK;
    const bool lt = c->model == IMM_LT;
    const int64_t n = c->vis_n;
    int64_t want = lt ? (int64_t)c->cus * gen_blocks_per_cu(3) * 4
                      : (int64_t)c->cus * gen_blocks_per_cu(c->heavy_block == 1024 ? 1
                                                            : c->heavy_block == 256  ? 4
                                                            : c->heavy_block == 128  ? 5
                                                                                     : 6);
    int64_t cap = std::max<int64_t>(4, c->heavy_scratch / (4 * n + 4 * c->vis_words));
    int64_t slots = std::min(want, cap);
    if (lt) slots = std::max<int64_t>(4, (slots / 4) * 4);
    IMM_TRY(dalloc(&c->hlist, slots * n));
    IMM_TRY(dalloc(&c->hvisited, slots * c->vis_words));
    HIP_TRY(hipMemset(c->hvisited, 0, sizeof(uint32_t) * (size_t)(slots * c->vis_words)));
    c->hslots = slots;
    return IMM_OK;
}

imm_status ensure_inst(GenCtx* c, int64_t ninst, int64_t queue) {
    if (ninst > c->cap_inst) {
        dfree(c->d_inst);
        hfree(c->host_inst);
        dfree(c->d_work_off);
        hfree(c->host_work_off);
        dfree(c->d_sum);
        hfree(c->host_sum);
        c->cap_inst = 0;
        IMM_TRY(dalloc(&c->d_inst, ninst));
        IMM_TRY(dalloc(&c->d_work_off, ninst + 1));
        IMM_TRY(dalloc(&c->d_sum, ninst));
        HIP_TRY(hipHostMalloc((void**)&c->host_inst, sizeof(GenInst) * (size_t)ninst,
                              hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&c->host_work_off, sizeof(int64_t) * (size_t)(ninst + 1),
                              hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&c->host_sum, sizeof(PoolSummary) * (size_t)ninst,
                              hipHostMallocDefault));
        c->cap_inst = ninst;
    }
    if (queue > c->cap_queue) {
        dfree(c->queue);
        dfree(c->handoff);
        c->cap_queue = 0;
        IMM_TRY(dalloc(&c->queue, queue));
        if (c->model == IMM_IC) IMM_TRY(dalloc(&c->handoff, queue));
        c->cap_queue = queue;
    }
    if (c->model == IMM_IC && !c->arena) IMM_TRY(dalloc(&c->arena, kArenaWords));
    return IMM_OK;
}

double elapsed_s(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms * 1e-3;
}

GenInst inst_of(const imm_pool* p) {
    const imm_graph* g = p->g;
    GenInst a{};
    a.vrec = g->vrec;
    a.src = g->src;
    a.thr = g->thr;
    a.cum = g->cum;
    a.n = g->n;
    a.k0 = (uint32_t)p->seed;
    a.k1 = (uint32_t)(p->seed >> 32);
    a.ids = p->ids;
    a.cap_ids = p->cap_ids;
    a.rr_start = p->rr_start;
    a.rr_len = p->rr_len;
    a.hist = p->hist;
    a.ctr = p->ctr;
    a.cap_list = p->cap_list;
    return a;
}

// Id-buffer entries a launch over `cnt` sets of a pool may leave reserved but unused: each
// light wave holds at most one partly used chunk per pool, and a pool's sets reach at most
// one wave per fetch.
int64_t chunk_slack(const GenCtx* c, int64_t cnt) {
    const int64_t waves = (int64_t)c->grid * 4 + (int64_t)c->hslots;
    return std::min(waves, cnt / kGenFetch + 2) * (int64_t)kGenIdChunk;
}

}  // namespace

// ------------------------------------------------------------------------------------
// gen_run
// ------------------------------------------------------------------------------------
imm_status imm::gen_run(GenCtx* c, imm_pool* const* pools, const int64_t* upto, int32_t count,
                        hipStream_t s) {
    struct Item {
        imm_pool* p;
        int64_t upto;
        int64_t first, cnt;       // this launch's work: first + j, or list[j]
        const uint32_t* list;
        double mean;
    };
    std::vector<Item> items;
    int64_t max_n = 0, total_cnt = 0;
    for (int32_t i = 0; i < count; ++i) {
        imm_pool* p = pools[i];
        if (p->model != c->model) return fail(IMM_EINVAL, "pool model differs from the launch's");
        if (upto[i] <= p->count) continue;
        if (upto[i] > kMaxSets)
            return fail(IMM_ECAPACITY, "RR index %lld exceeds 2^31-1", (long long)upto[i]);
        const int64_t first = p->count, cnt = upto[i] - first;
        int64_t cap_sets = p->cap_sets;
        IMM_TRY(dgrow(&p->rr_start, &cap_sets, upto[i], p->count, s));
        cap_sets = p->cap_sets;
        IMM_TRY(dgrow(&p->rr_len, &cap_sets, upto[i], p->count, s));
        p->cap_sets = cap_sets;
        if (cnt > p->cap_lists) {
            dfree(p->cap_list);
            dfree(p->retry_list);
            p->cap_lists = 0;
            IMM_TRY(dalloc(&p->cap_list, cnt));
            IMM_TRY(dalloc(&p->retry_list, cnt));
            p->cap_lists = cnt;
        }
        const double mean = p->count > 0 ? (double)p->sum.placed / (double)p->count : 16.0;
        items.push_back(Item{p, upto[i], first, cnt, nullptr, mean});
        max_n = std::max<int64_t>(max_n, p->g->n);
        total_cnt += cnt;
    }
    if (items.empty()) return IMM_OK;
    IMM_TRY(ensure_light(c, max_n));
    IMM_TRY(ensure_inst(c, (int64_t)items.size(), total_cnt));
    // id buffers sized from the mean set size seen so far plus the chunk slack
    for (Item& it : items) {
        imm_pool* p = it.p;
        const int64_t need = (int64_t)p->sum.tail + (int64_t)(it.mean * 1.3 * (double)it.cnt) +
                             chunk_slack(c, it.cnt);
        IMM_TRY(dgrow(&p->ids, &p->cap_ids, need, (int64_t)p->sum.tail, s));
    }

    std::vector<int32_t> live;   // items of this launch
    for (int guard = 0; guard < 64; ++guard) {
        live.clear();
        int64_t off = 0;
        for (int32_t i = 0; i < (int32_t)items.size(); ++i) {
            const Item& it = items[i];
            if (it.cnt == 0) continue;
            GenInst a = inst_of(it.p);
            a.first = it.first;
            a.list = it.list;
            c->host_inst[live.size()] = a;
            c->host_work_off[live.size()] = off;
            off += it.cnt;
            live.push_back(i);
        }
        const int32_t ninst = (int32_t)live.size();
        c->host_work_off[ninst] = off;
        HIP_TRY(hipMemcpyAsync(c->d_inst, c->host_inst, sizeof(GenInst) * (size_t)ninst,
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(c->d_work_off, c->host_work_off, sizeof(int64_t) * (size_t)(ninst + 1),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(c->lc),
                                (int64_t)(sizeof(LaunchCounters) / 8), 0ull, s));

        GenLaunch L{};
        L.inst = c->d_inst;
        L.ninst = ninst;
        L.work_off = c->d_work_off;
        L.total = off;
        L.budget = c->budget;
        L.lc = c->lc;
        L.heavy_list = c->queue;
        L.handoff = c->handoff;
        L.arena = c->arena;
        L.arena_cap = c->arena ? kArenaWords : 0;
        L.visited = c->visited;
        L.vis_words = c->vis_words;
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(c->grid, (off + 3) / 4));
        HIP_TRY(hipEventRecord(c->ev0, s));
        if (c->model == IMM_IC) HIP_TRY(launch_ic_light(L, (int)grid, s));
        else HIP_TRY(launch_lt(L, false, (int)grid, s));
        HIP_TRY(hipEventRecord(c->ev1, s));
        HIP_TRY(hipMemcpyAsync(c->host_lc, c->lc, sizeof(LaunchCounters), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        c->kernel_s += elapsed_s(c->ev0, c->ev1);
        c->kernel_launches += 1;

        const uint32_t n_queue = c->host_lc->n_heavy;
        if (n_queue > 0) {
            IMM_TRY(ensure_heavy(c));
            L.hvisited = c->hvisited;
            L.hlist = c->hlist;
            L.list_stride = c->vis_n;
            L.n_queue = n_queue;
            HIP_TRY(hipEventRecord(c->ev1, s));
            if (c->model == IMM_IC) {
                const int64_t hg = std::min<int64_t>(c->hslots, n_queue);
                HIP_TRY(launch_ic_heavy(L, c->heavy_block, (int)std::max<int64_t>(hg, 1), s));
            } else {
                // LT: walks too long for the on-chip list, with their lists in HBM
                HIP_TRY(launch_fill_u64(&c->lc->work, 1, 0ull, s));
                L.heavy_in = c->queue;
                L.total = n_queue;
                const int64_t hg = std::min<int64_t>(c->hslots / 4, ((int64_t)n_queue + 3) / 4);
                HIP_TRY(launch_lt(L, true, (int)std::max<int64_t>(hg, 1), s));
            }
            HIP_TRY(hipEventRecord(c->ev2, s));
        }
        HIP_TRY(launch_pool_summary(c->d_inst, ninst, c->d_sum, s));
        HIP_TRY(hipMemcpyAsync(c->host_sum, c->d_sum, sizeof(PoolSummary) * (size_t)ninst,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (n_queue > 0) {
            c->heavy_s += elapsed_s(c->ev1, c->ev2);
            c->heavy_launches += 1;
        }

        bool again = false;
        for (int32_t j = 0; j < ninst; ++j) {
            Item& it = items[live[j]];
            imm_pool* p = it.p;
            p->sum = c->host_sum[j];
            const unsigned int n_cap = p->sum.n_capacity;
            p->sum.n_capacity = 0;
            if (n_cap == 0) {
                p->count = it.upto;
                it.cnt = 0;
                continue;
            }
            // grow the id buffer and rerun the sets that did not fit
            const int64_t tail = (int64_t)p->sum.tail;
            const int64_t want = tail + (int64_t)(std::max(it.mean, 64.0) * 2.0 * (double)n_cap) +
                                 chunk_slack(c, n_cap);
            IMM_TRY(dgrow(&p->ids, &p->cap_ids, std::max(want, 2 * p->cap_ids), tail, s));
            HIP_TRY(hipMemcpyAsync(p->retry_list, p->cap_list, sizeof(uint32_t) * n_cap,
                                   hipMemcpyDeviceToDevice, s));
            it.first = 0;
            it.cnt = n_cap;
            it.list = p->retry_list;
            again = true;
        }
        if (!again) return IMM_OK;
    }
    return fail(IMM_EDEVICE, "RR placement did not converge");
}

imm_status imm::pool_generate(imm_pool* p, int64_t upto, hipStream_t s) {
    return gen_run(&p->gen, &p, &upto, 1, s);
}
