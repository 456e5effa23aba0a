// Autotuning of the RR-generation launch configuration for one graph and model.
//
// Four knobs shape the generation launches: the light-wave budget (4-edge groups a set may
// examine before it is handed to the heavy kernel), the threads per heavy set, the on-chip
// list capacity of a light set or LT walk (frontier capacity: beyond it the set moves to
// the heavy kernel / the walk to its extension list), and the RR indices a wave takes per
// fetch from the launch's work counter (queue depth).  The best values depend on the
// graph's degree distribution and probabilities (how many sets overflow, how large they
// get).  imm_autotune times the generation of the same pilot sets
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
    // The library defaults, then one knob group at a time (coordinate descent): IC light
    // budget x heavy block size, then the light list capacity, then the fetch depth; LT
    // the walk list capacity, then the fetch depth.
    const GenTuning dflt{4096, 256, 1024, kLtLdsCap, kGenFetch};
    GenTuning best = dflt;
    double warm = 0.0;
    IMM_TRY(time_generation(g, model, seed, pilot_sets, dflt, &warm));   // first-use costs
    double t_best = 0.0, t_def = 0.0;
    IMM_TRY(time_generation(g, model, seed, pilot_sets, dflt, &t_def));
    t_best = t_def;
    int32_t timed = 1;
    auto consider = [&](const GenTuning& c) -> imm_status {
        double t = 0.0;
        IMM_TRY(time_generation(g, model, seed, pilot_sets, c, &t));
        ++timed;
        if (t < t_best) {
            t_best = t;
            best = c;
        }
        return IMM_OK;
    };
    if (model == IMM_IC) {
        const GenTuning base = best;
        for (int64_t b : {1024, 2048, 4096, 8192, 16384})
            for (int hb : {128, 256}) {
                GenTuning c = base;
                c.budget = b;
                c.heavy_block = hb;
                if (b == dflt.budget && hb == dflt.heavy_block) continue;
                IMM_TRY(consider(c));
            }
        const GenTuning b2 = best;
        for (int cap : {256, 512}) {
            GenTuning c = b2;
            c.light_cap = cap;
            IMM_TRY(consider(c));
        }
    } else {
        const GenTuning b2 = best;
        for (int cap : {64, 128}) {
            GenTuning c = b2;
            c.lt_cap = cap;
            IMM_TRY(consider(c));
        }
    }
    const GenTuning b3 = best;
    for (int f : {4, 16, 32}) {
        GenTuning c = b3;
        c.fetch = f;
        IMM_TRY(consider(c));
    }
    g->tuned[model] = best;
    if (out) {
        memset(out, 0, sizeof *out);
        out->light_budget = best.budget;
        out->heavy_block = best.heavy_block;
        out->candidates = timed;
        out->best_sets_per_s = t_best > 0 ? (double)pilot_sets / t_best : 0.0;
        out->default_sets_per_s = t_def > 0 ? (double)pilot_sets / t_def : 0.0;
        out->light_cap = best.light_cap;
        out->lt_cap = best.lt_cap;
        out->fetch = best.fetch;
    }
    return IMM_OK;
}
