// Host side of the forward Monte-Carlo spread (gIM Sec. II-C): out-edge lists built once
// per graph, per-simulation scratch from the caching allocator, one persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "host.hpp"

using namespace imm;

namespace {

imm_status ensure_out_lists(imm_graph* g, hipStream_t s) {
    if (g->out_off) return IMM_OK;
    const int64_t n = g->n, m = g->m;
    uint32_t* deg = nullptr;
    uint32_t* cursor = nullptr;
    int64_t* tmp = nullptr;
    int64_t* off = nullptr;
    int32_t* dst = nullptr;
    uint32_t* eid = nullptr;
    auto cleanup = [&](imm_status st) {
        dfree(deg);
        dfree(cursor);
        dfree(tmp);
        if (st != IMM_OK) {
            dfree(off);
            dfree(dst);
            dfree(eid);
        }
        return st;
    };
    imm_status st = dalloc(&deg, n);
    if (st == IMM_OK) st = dalloc(&cursor, n);
    if (st == IMM_OK) st = dalloc(&tmp, scan_tmp_elems(n));
    if (st == IMM_OK) st = dalloc(&off, n + 1);
    if (st == IMM_OK) st = dalloc(&dst, m);
    if (st == IMM_OK) st = dalloc(&eid, m);
    if (st != IMM_OK) return cleanup(st);
    hipError_t e = launch_fill_u32(deg, n, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(cursor, n, 0u, s);
    if (e == hipSuccess) e = launch_out_degree(m, g->src, deg, s);
    if (e == hipSuccess) e = launch_scan_u32(deg, n, off, tmp, s);
    if (e == hipSuccess) e = launch_out_scatter((int32_t)n, g->vrec, g->src, off, cursor, dst, eid, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup(fail(IMM_EDEVICE, "out-edge lists: %s", hipGetErrorString(e)));
    g->out_off = off;
    g->out_dst = dst;
    g->out_eid = eid;
    return cleanup(IMM_OK);
}

}  // namespace

extern "C" imm_status imm_spread_mc(const imm_graph* gc, imm_model model, int32_t rounds,
                                    const int32_t* seeds, int32_t nseeds, int64_t sims,
                                    uint64_t seed, uint32_t* per_sim_out, int64_t* total_out,
                                    double* mean_out, double* stderr_out, void* stream) {
    if (!gc) return fail(IMM_EINVAL, "graph is NULL");
    imm_graph* g = const_cast<imm_graph*>(gc);
    if (model == IMM_IC && !g->has_ic) return fail(IMM_EINVAL, "graph has no IC probabilities");
    if (model == IMM_LT && !g->has_lt) return fail(IMM_EINVAL, "graph has no LT encoding");
    if (model != IMM_IC && model != IMM_LT) return fail(IMM_EINVAL, "unknown model %d", (int)model);
    if (rounds < 1 || rounds > kMaxRounds) return fail(IMM_EINVAL, "rounds = %d outside [1, %d]", rounds, kMaxRounds);
    const int64_t n_elem = (int64_t)g->n * rounds;
    if (n_elem > (int64_t)INT32_MAX) return fail(IMM_ECAPACITY, "rounds * n exceeds 2^31 - 1");
    if (sims < 0 || sims > (int64_t)UINT32_MAX) return fail(IMM_EINVAL, "sims = %lld outside [0, 2^32)", (long long)sims);
    if (nseeds < 0 || (nseeds > 0 && !seeds)) return fail(IMM_EINVAL, "seeds missing");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> el((size_t)nseeds);
    if (nseeds > 0)
        HIP_TRY(hipMemcpy(el.data(), seeds, sizeof(int32_t) * (size_t)nseeds, hipMemcpyDefault));
    for (int32_t i = 0; i < nseeds; ++i)
        if (el[i] < 0 || el[i] >= n_elem)
            return fail(IMM_EINVAL, "seed element %d (index %d) outside [0, %lld)", el[i], i, (long long)n_elem);
    IMM_TRY(ensure_out_lists(g, s));      // also with sims = 0: prepares the graph
    if (sims == 0) {
        if (total_out) *total_out = 0;
        if (mean_out) *mean_out = 0.0;
        if (stderr_out) *stderr_out = 0.0;
        return IMM_OK;
    }

    // scratch per slot: a bitmap and a list of n entries (two of each with several rounds);
    // slots are bounded by the simulations and by 4 GiB of scratch
    const int64_t vis_words = ((int64_t)g->n + 31) / 32;
    const int64_t per_slot = (vis_words * 4 + (int64_t)g->n * 4) * (rounds > 1 ? 2 : 1);
    int64_t slots = std::min<int64_t>(sims, (int64_t)g->cus * 8);
    slots = std::max<int64_t>(1, std::min<int64_t>(slots, ((int64_t)4 << 30) / per_slot));
    uint32_t* vis = nullptr;
    uint32_t* uvis = nullptr;
    int32_t* list = nullptr;
    int32_t* ulist = nullptr;
    int32_t* d_el = nullptr;
    uint32_t* counts = nullptr;
    unsigned int* work = nullptr;
    auto cleanup = [&](imm_status st) {
        dfree(vis);
        dfree(uvis);
        dfree(list);
        dfree(ulist);
        dfree(d_el);
        dfree(counts);
        dfree(work);
        return st;
    };
    imm_status st = dalloc(&vis, slots * vis_words);
    if (st == IMM_OK) st = dalloc(&list, slots * (int64_t)g->n);
    if (st == IMM_OK && rounds > 1) st = dalloc(&uvis, slots * vis_words);
    if (st == IMM_OK && rounds > 1) st = dalloc(&ulist, slots * (int64_t)g->n);
    if (st == IMM_OK) st = dalloc(&d_el, nseeds);
    if (st == IMM_OK) st = dalloc(&counts, sims);
    if (st == IMM_OK) st = dalloc(&work, 1);
    if (st != IMM_OK) return cleanup(st);
    hipError_t e = launch_fill_u32(vis, slots * vis_words, 0u, s);
    if (e == hipSuccess && uvis) e = launch_fill_u32(uvis, slots * vis_words, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(work, 1, 0u, s);
    if (e == hipSuccess && nseeds > 0)
        e = hipMemcpyAsync(d_el, el.data(), sizeof(int32_t) * (size_t)nseeds, hipMemcpyHostToDevice, s);
    FwdLaunch L{};
    L.vrec = g->vrec;
    L.w = model == IMM_IC ? g->thr : g->cum;
    L.out_off = g->out_off;
    L.out_dst = g->out_dst;
    L.out_eid = g->out_eid;
    L.n = g->n;
    L.model = model == IMM_IC ? 0 : 1;
    L.rounds = rounds;
    L.k0 = (uint32_t)seed;
    L.k1 = (uint32_t)(seed >> 32);
    L.elems = d_el;
    L.nelem = nseeds;
    L.sims = sims;
    L.work = work;
    L.counts = counts;
    L.vis = vis;
    L.uvis = uvis;
    L.list = list;
    L.ulist = ulist;
    L.vis_words = vis_words;
    L.list_stride = g->n;
    if (e == hipSuccess) e = launch_spread_fwd(L, (int)slots, s);
    std::vector<uint32_t> host((size_t)sims);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host.data(), counts, sizeof(uint32_t) * (size_t)sims, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup(fail(IMM_EDEVICE, "spread simulations: %s", hipGetErrorString(e)));
    int64_t total = 0;
    for (uint32_t c : host) total += c;
    const double mean = (double)total / (double)sims;
    double ss = 0.0;
    for (uint32_t c : host) ss += ((double)c - mean) * ((double)c - mean);
    const double sd = sims > 1 ? std::sqrt(ss / (double)(sims - 1)) : 0.0;
    if (per_sim_out) std::copy(host.begin(), host.end(), per_sim_out);
    if (total_out) *total_out = total;
    if (mean_out) *mean_out = mean;
    if (stderr_out) *stderr_out = sd / std::sqrt((double)sims);
    return cleanup(IMM_OK);
}
