// Autotuning of the RR-generation launch configuration for one graph and model.
//
// Two knobs shape the generation launches: the light-wave budget (4-edge groups a set may
// examine before it is handed to the heavy kernel) and the threads per heavy set.  The
// best values depend on the graph's degree distribution and probabilities (how many sets
// overflow, how large they get).  imm_autotune times the generation of the same pilot sets
// under each candidate and keeps the fastest for later pools of that graph and model.  RR
// sets never depend on the configuration (each draw is keyed by (seed, r, edge)), so
// tuning changes speed only.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "host.hpp"

using namespace imm;

namespace {

// Seconds to generate sets [0, count) of a fresh pool under `t`.
imm_status time_generation(imm_graph* g, imm_model model, uint64_t seed, int64_t count,
                           const GenTuning& t, double* seconds) {
    imm_pool* p = nullptr;
    const GenTuning saved = g->tuned[model];
    g->tuned[model] = t;
    imm_status st = imm_pool_create(g, model, seed, &p);
    g->tuned[model] = saved;
    if (st != IMM_OK) return st;
    const double t0 = now_s();
    st = pool_generate(p, count, nullptr);
    *seconds = now_s() - t0;
    imm_pool_destroy(p);
    return st;
}

}  // namespace

extern "C" imm_status imm_autotune(imm_graph* g, imm_model model, uint64_t seed,
                                   int64_t pilot_sets, imm_tune_info* out) {
    if (!g) return fail(IMM_EINVAL, "graph is NULL");
    if (model != IMM_IC && model != IMM_LT) return fail(IMM_EINVAL, "unknown model %d", (int)model);
    if ((model == IMM_IC && !g->has_ic) || (model == IMM_LT && !g->has_lt))
        return fail(IMM_EINVAL, "graph has no encoding for model %d", (int)model);
    if (pilot_sets < 1 || pilot_sets > kMaxSets) return fail(IMM_EINVAL, "pilot_sets out of range");
    std::vector<GenTuning> cand;
    for (int64_t b : {1024, 2048, 4096, 8192, 16384})
        for (int hb : {128, 256}) cand.push_back(GenTuning{b, hb});
    if (model == IMM_LT) {   // LT has no budget or heavy block size: one measurement
        cand.assign(1, GenTuning{4096, 256});
    }
    double warm = 0.0;
    IMM_TRY(time_generation(g, model, seed, pilot_sets, cand[0], &warm));   // first-use costs
    double best = 0.0, def = 0.0;
    size_t best_i = 0;
    for (size_t i = 0; i < cand.size(); ++i) {
        double t = 0.0;
        IMM_TRY(time_generation(g, model, seed, pilot_sets, cand[i], &t));
        if (cand[i].budget == 4096 && cand[i].heavy_block == 256) def = t;
        if (i == 0 || t < best) {
            best = t;
            best_i = i;
        }
    }
    g->tuned[model] = cand[best_i];
    if (out) {
        memset(out, 0, sizeof *out);
        out->light_budget = cand[best_i].budget;
        out->heavy_block = cand[best_i].heavy_block;
        out->candidates = (int32_t)cand.size();
        out->best_sets_per_s = best > 0 ? (double)pilot_sets / best : 0.0;
        out->default_sets_per_s = def > 0 ? (double)pilot_sets / def : 0.0;
    }
    return IMM_OK;
}
