// Host side of multi-round influence maximisation (gIM Sec. IV-H, Table 3; CR-NAIMM of
// Sun et al., KDD'18): multi-round pools and the CR-NAIMM solve.
//
// A multi-round pool of T rounds holds T round pools, round t drawing its live edges with
// t in the third counter word (one root per index, shared by the rounds, since the root
// draw has no round word).  Generation extends all round pools in one launch (one
// instance per round, the batching path of gen_run) and then lays each index's T sets out
// side by side as one set of elements t * n + u (mr_sets.hip).  Histogram, inverted index
// and greedy then run over the element space of T * n counters; the greedy adds the
// partition-matroid constraint (at most k elements per round).  The IMM loop is the plain
// one with the multi-round sample sizes.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "host.hpp"

using namespace imm;

imm_status imm::mr_merge(imm_pool* p, int64_t upto, hipStream_t s) {
    const int64_t first = p->count, count = upto - first;
    if (count <= 0) return IMM_OK;
    const int32_t T = p->rounds;
    MrSrc src{};
    src.rounds = T;
    src.n_base = p->n_base;
    unsigned long long placed = 0, edges = 0, hedges = 0;
    for (int32_t t = 0; t < T; ++t) {
        const imm_pool* q = p->sub[t];
        if (q->count < upto) return fail(IMM_EDEVICE, "round pool %d holds %lld of %lld sets", t,
                                         (long long)q->count, (long long)upto);
        src.start[t] = q->rr_start;
        src.len[t] = q->rr_len;
        src.ids[t] = q->ids;
        placed += q->sum.placed;
        edges += q->sum.edges;
        hedges += q->sum.hedges;
    }
    // the round pools' member counts give the new elements exactly, so the id buffer is
    // grown before the copy without reading anything back
    const int64_t base = (int64_t)p->sum.tail;
    const int64_t add = (int64_t)placed - base;
    int64_t cap_sets = p->cap_sets;
    IMM_TRY(dgrow(&p->rr_start, &cap_sets, upto, p->count, s));
    cap_sets = p->cap_sets;
    IMM_TRY(dgrow(&p->rr_len, &cap_sets, upto, p->count, s));
    p->cap_sets = cap_sets;
    IMM_TRY(dgrow(&p->ids, &p->cap_ids, base + add, base, s));
    int64_t* sizes = nullptr;
    int64_t* off = nullptr;
    int64_t* tmp = nullptr;
    imm_status st = dalloc(&sizes, count);
    if (st == IMM_OK) st = dalloc(&off, count + 1);
    if (st == IMM_OK) st = dalloc(&tmp, scan_tmp_elems(count));
    hipError_t e = hipSuccess;
    if (st == IMM_OK) {
        e = launch_mr_sizes(src, first, count, sizes, s);
        if (e == hipSuccess) e = launch_scan_i64(sizes, count, off, tmp, s);
        if (e == hipSuccess)
            e = launch_mr_copy(src, first, count, off, base, p->rr_start, p->rr_len, p->ids, s);
        // element (u, t) occurs in as many multi-round sets as u in round t's sets
        for (int32_t t = 0; t < T && e == hipSuccess; ++t)
            e = hipMemcpyAsync(p->hist + (int64_t)t * p->n_base, p->sub[t]->hist,
                               sizeof(uint32_t) * (size_t)p->n_base, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    dfree(sizes);
    dfree(off);
    dfree(tmp);
    if (st != IMM_OK) return st;
    if (e != hipSuccess) return fail(IMM_EDEVICE, "multi-round layout: %s", hipGetErrorString(e));
    p->sum.tail = placed;
    p->sum.placed = placed;
    p->sum.edges = edges;
    p->sum.hedges = hedges;
    p->count = upto;
    return IMM_OK;
}

extern "C" imm_status imm_mr_pool_create(const imm_graph* g, imm_model model, uint64_t seed,
                                         int32_t rounds, imm_pool** out) {
    if (!out) return fail(IMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(IMM_EINVAL, "graph is NULL");
    if (rounds < 1 || rounds > kMaxRounds)
        return fail(IMM_EINVAL, "rounds = %d outside [1, %d]", rounds, kMaxRounds);
    if (rounds == 1) return imm_pool_create(g, model, seed, out);
    if ((int64_t)g->n * rounds > (int64_t)INT32_MAX)
        return fail(IMM_ECAPACITY, "%d rounds of %d vertices exceed 2^31 - 1 elements", rounds, g->n);
    imm_pool* p = new imm_pool();
    p->model = model;
    p->seed = seed;
    p->rounds = rounds;
    p->n_base = g->n;
    imm_status st = IMM_OK;
    for (int32_t t = 0; t < rounds && st == IMM_OK; ++t) {
        st = imm_pool_create(g, model, seed, &p->sub[t]);
        if (st == IMM_OK) p->sub[t]->round = (uint32_t)t;
    }
    if (st == IMM_OK) {
        // the element space: a graph record with rounds * n vertices and no arrays
        p->view = new imm_graph();
        p->view->tuned[0] = g->tuned[0];
        p->view->tuned[1] = g->tuned[1];
        p->view->device = g->device;
        p->view->n = g->n * rounds;
        p->view->m = g->m;
        p->view->has_ic = g->has_ic;
        p->view->has_lt = g->has_lt;
        p->view->ic_uniform = g->ic_uniform;
        p->view->cus = g->cus;
        p->g = p->view;
        st = pool_init(p);
    }
    if (st != IMM_OK) {
        imm_pool_destroy(p);
        return st;
    }
    *out = p;
    return IMM_OK;
}

extern "C" imm_status imm_mrim_solve(const imm_graph* g, int32_t k, int32_t rounds, double eps,
                                     double ell, imm_model model, const imm_options* opt,
                                     int32_t* seeds_out, imm_info* info) {
    if (!g) return fail(IMM_EINVAL, "graph is NULL");
    imm_options o{};
    if (opt) o = *opt;
    if (rounds > 1 && o.fresh_final) return fail(IMM_EINVAL, "multi-round solves reuse the estimation sets");
    imm_pool* p = nullptr;
    IMM_TRY(imm_mr_pool_create(g, model, o.seed, rounds, &p));
    imm_status st = run_imm(p, k, eps, ell, o.fresh_final, (hipStream_t)o.stream, seeds_out, info);
    imm_pool_destroy(p);
    return st;
}

extern "C" double imm_mr_lambda_prime(int64_t n, int64_t k, int32_t rounds, double eps, double ell) {
    return lambda_prime(n, k, eps, ell_prime(n, ell), rounds);
}

extern "C" double imm_mr_lambda_star(int64_t n, int64_t k, int32_t rounds, double eps, double ell) {
    return lambda_star(n, k, eps, ell_prime(n, ell), rounds);
}
