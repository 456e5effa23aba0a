// Batched IMM: many independent instances (each its own graph, model, pool seed, k, eps,
// ell) solved together.
//
// Each instance runs the same state machine as imm_solve (gIM Alg. 2, then Alg. 1), so its
// result is bit-identical to solving it alone.  The batch advances in ticks: every
// unfinished instance names its next selection; one light (+ heavy) generation launch per
// model extends every instance's pool to what that selection reads; then the greedy rounds
// of all instances run in one cooperative launch.  Instances with small graphs or loose
// eps finish after a few ticks and leave; the others continue.  The device is shared by
// all instances at each step, so small instances no longer leave most of it idle, and
// host round trips are paid per tick instead of per instance and step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host.hpp"

using namespace imm;

namespace {

struct Inst {
    imm_batch_item* item = nullptr;
    imm_pool* pool = nullptr;
    ImmPlan plan;
    bool active = false;
    int64_t gen_upto = 0, sel_first = 0, sel_count = 0;
    double t_gen = 0, t_sel = 0;
};

// The selection setup of every instance of a tick (counts, index, clears), enqueued on s;
// fills si / ws with the instances that select (an instance whose final selection repeats
// its last one keeps that one's seeds and coverage).
imm_status prepare_tick(std::vector<Inst>& inst, const std::vector<int32_t>& act,
                        std::vector<SelInst>& si, std::vector<SelectWs*>& ws, hipStream_t s) {
    si.clear();
    ws.clear();
    for (size_t j = 0; j < act.size(); ++j) {
        Inst& x = inst[(size_t)act[j]];
        if (x.plan.reuses_last()) continue;
        ws.push_back(&x.pool->sel);
        si.emplace_back();
        IMM_TRY(select_prepare(x.pool, ws.back(), x.sel_first, x.sel_count, x.item->k, s, &si.back()));
        si.back().need = x.plan.need_cov();
    }
    return IMM_OK;
}

// IMM_BATCH_GRAPH=1 captures every tick's selection half into a graph.  Off by default:
// on the 256-instance R-MAT mix, capturing and instantiating ~2000 nodes per tick cost more
// than the launches it saves (batch 1.10 s with capture, 1.02 s without).
bool batch_graph_enabled() {
    const char* e = getenv("IMM_BATCH_GRAPH");
    return e && e[0] == '1';
}

void release(std::vector<Inst>& v) {
    for (Inst& x : v) {
        if (x.pool) imm_pool_destroy(x.pool);
        x.pool = nullptr;
    }
}

}  // namespace

extern "C" imm_status imm_batch_solve(imm_batch_item* items, int32_t count, void* stream,
                                      imm_batch_stats* stats) {
    if (stats) memset(stats, 0, sizeof *stats);
    if (count < 0) return fail(IMM_EINVAL, "count < 0");
    if (count == 0) return IMM_OK;
    if (!items) return fail(IMM_EINVAL, "items is NULL");
    hipStream_t s = (hipStream_t)stream;
    const double t0 = now_s();

    // validate everything before any work
    int device = -1;
    for (int32_t i = 0; i < count; ++i) {
        imm_batch_item& it = items[i];
        it.status = IMM_OK;
        const imm_graph* g = it.graph;
        if (!g) return fail(IMM_EINVAL, "item %d: graph is NULL", i);
        if (!it.seeds_out) return fail(IMM_EINVAL, "item %d: seeds_out is NULL", i);
        if (it.model != IMM_IC && it.model != IMM_LT)
            return fail(IMM_EINVAL, "item %d: unknown model %d", i, (int)it.model);
        if ((it.model == IMM_IC && !g->has_ic) || (it.model == IMM_LT && !g->has_lt))
            return fail(IMM_EINVAL, "item %d: graph has no encoding for model %d", i, (int)it.model);
        if (device < 0) device = g->device;
        if (g->device != device) return fail(IMM_EINVAL, "item %d: graph on another device", i);
        ImmPlan probe;
        imm_status st = probe.init(g->n, it.k, it.eps, it.ell, it.fresh_final);
        if (st != IMM_OK) return fail(st, "item %d: %s", i, imm_last_error());
    }
    HIP_TRY(hipSetDevice(device));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));

    std::vector<Inst> inst((size_t)count);
    GenCtx gen[2];
    SelectLaunch launch;
    imm_status st = IMM_OK;
    for (int m = 0; m < 2 && st == IMM_OK; ++m) st = gen[m].init(device, (imm_model)m, cus);
    for (int32_t i = 0; i < count && st == IMM_OK; ++i) {
        imm_batch_item& it = items[i];
        Inst& x = inst[(size_t)i];
        x.item = &it;
        st = imm_pool_create(it.graph, it.model, it.seed, &x.pool);
        if (st == IMM_OK) st = x.plan.init(it.graph->n, it.k, it.eps, it.ell, it.fresh_final);
        x.active = true;
    }

    imm_batch_stats bs{};
    // a private stream to capture on (the caller's may be the null stream), default
    // priority
    const bool use_graph = batch_graph_enabled();
    hipStream_t cs = nullptr;
    if (use_graph && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        cs = nullptr;
    }
    std::vector<imm_pool*> gp;
    std::vector<int64_t> gu;
    std::vector<int32_t> act;
    std::vector<SelInst> si;
    std::vector<SelectWs*> ws;
    while (st == IMM_OK) {
        act.clear();
        for (int32_t i = 0; i < count; ++i)
            if (inst[(size_t)i].active) act.push_back(i);
        if (act.empty()) break;
        bs.ticks += 1;
        // 1. next selection of every unfinished instance
        for (int32_t i : act) {
            Inst& x = inst[(size_t)i];
            st = x.plan.next(&x.gen_upto, &x.sel_first, &x.sel_count);
            if (st != IMM_OK) break;
        }
        if (st != IMM_OK) break;
        // 2. one generation launch (light + heavy) per model over all instances
        const double ta = now_s();
        for (int m = 0; m < 2 && st == IMM_OK; ++m) {
            gp.clear();
            gu.clear();
            for (int32_t i : act) {
                Inst& x = inst[(size_t)i];
                if (x.item->model != m) continue;
                gp.push_back(x.pool);
                gu.push_back(x.gen_upto);
            }
            if (!gp.empty()) st = gen_run(&gen[m], gp.data(), gu.data(), (int32_t)gp.size(), s);
        }
        if (st != IMM_OK) break;
        const double tb = now_s();
        // 3. all greedy selections in one cooperative launch (an instance whose final
        //    selection repeats its last one keeps that one's seeds and coverage).  The
        //    shape of this half is fixed once the tick's instances are known, so its
        //    setup kernels (a handful per instance) and the greedy launch can be captured
        //    into one graph and launched at once (IMM_BATCH_GRAPH=1); if capture fails the
        //    tick runs them directly.
        bool graphed = false;
        if (use_graph && cs) {
            imm_status cst = IMM_OK;
            hipGraph_t graph = nullptr;
            if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) == hipSuccess) {
                cst = prepare_tick(inst, act, si, ws, cs);
                if (cst == IMM_OK && !si.empty())
                    cst = select_enqueue(&launch, ws.data(), si.data(), (int32_t)si.size(), cs, true);
                const hipError_t ee = hipStreamEndCapture(cs, &graph);
                if (cst == IMM_OK && ee == hipSuccess && graph) {
                    hipGraphExec_t exec = nullptr;
                    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
                        graphed = hipGraphLaunch(exec, s) == hipSuccess;
                        if (graphed && !si.empty()) st = select_wait(&launch, s);
                        else if (graphed) st = hipStreamSynchronize(s) == hipSuccess ? IMM_OK : IMM_EDEVICE;
                        (void)hipGraphExecDestroy(exec);
                    }
                }
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
            }
            if (graphed) bs.graph_ticks += 1;
        }
        if (!graphed && st == IMM_OK) {
            st = prepare_tick(inst, act, si, ws, s);
            if (st == IMM_OK && !si.empty())
                st = select_run(&launch, ws.data(), si.data(), (int32_t)si.size(), s);
        }
        if (st != IMM_OK) break;
        const double tc = now_s();
        bs.t_generate_s += tb - ta;
        bs.t_select_s += tc - tb;
        // 4. advance; finished instances hand back their seeds and leave
        for (size_t j = 0; j < act.size() && st == IMM_OK; ++j) {
            Inst& x = inst[(size_t)act[j]];
            x.t_gen += tb - ta;
            x.t_sel += tc - tb;
            st = x.plan.complete((int64_t)*x.pool->sel.host_cov);
            if (st != IMM_OK || !x.plan.done) continue;
            imm_batch_item& it = *x.item;
            memcpy(it.seeds_out, x.pool->sel.host_seeds, sizeof(int32_t) * (size_t)it.k);
            imm_info& info = it.info;
            memset(&info, 0, sizeof info);
            const ImmPlan& P = x.plan;
            info.theta = P.theta;
            info.num_rr = P.upto;
            info.covered = P.covered;
            info.edges_examined = (int64_t)(x.pool->sum.edges + x.pool->sum.hedges);
            info.edges_heavy = (int64_t)x.pool->sum.hedges;
            info.pool_ids = (int64_t)x.pool->sum.placed;
            info.phases = P.phases;
            info.lb = P.lb;
            info.spread_est = P.spread_est();
            info.lambda_prime = P.lam1;
            info.lambda_star = P.lam2;
            info.t_generate_s = x.t_gen;
            info.t_select_s = x.t_sel;
            info.t_total_s = now_s() - t0;      // completion time within the batch
            bs.rr_sets += P.upto;
            bs.edges_examined += info.edges_examined;
            bs.edges_heavy += info.edges_heavy;
            x.active = false;
            imm_pool_destroy(x.pool);           // free its RR sets for the others
            x.pool = nullptr;
        }
    }
    if (st != IMM_OK) {
        const std::string err = imm_last_error();
        for (Inst& x : inst)
            if (x.active && x.item) x.item->status = st;
        release(inst);
        for (GenCtx& c : gen) c.release();
        launch.release();
        if (cs) (void)hipStreamDestroy(cs);
        return fail(st, "%s", err.c_str());
    }
    bs.t_total_s = now_s() - t0;
    for (const GenCtx& c : gen) {
        bs.t_rr_kernel_s += c.kernel_s;
        bs.rr_kernel_launches += c.kernel_launches;
        bs.t_rr_heavy_s += c.heavy_s;
        bs.rr_heavy_launches += c.heavy_launches;
    }
    if (stats) *stats = bs;
    release(inst);
    for (GenCtx& c : gen) c.release();
    launch.release();
    if (cs) (void)hipStreamDestroy(cs);
    return IMM_OK;
}
