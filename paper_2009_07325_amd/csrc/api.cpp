// Host side of libimm: the C ABI declared in include/imm.h.
//
// Owns device memory for graphs and RR pools, launches the kernels of graph.hip,
// rr_gen.hip and select.hip, and runs IMM's estimation loop (gIM Alg. 2) and final
// sample/selection (gIM Alg. 1) on the host in IEEE double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "host.hpp"

using namespace imm;

namespace {
thread_local std::string g_err;
}

imm_status imm::fail(imm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

double imm::now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------------------------
// IMM sample sizes (Tang, Shi, Xiao 2015; gIM Alg. 2 defers f(n, eps, k) and theta to
// it).  All IEEE double; logarithms are run-time libm calls so that no compiler folds
// them differently; ln C(n, k) is summed term by term in ascending i.
// ------------------------------------------------------------------------------------
namespace {
double rt_log(double x) {
    volatile double v = x;
    return std::log(v);
}
constexpr double kE = 2.718281828459045;
}  // namespace

namespace imm {

double log_binom(int64_t n, int64_t k) {
    double acc = 0.0;
    for (int64_t i = 0; i < k; ++i) acc += rt_log((double)(n - i)) - rt_log((double)(i + 1));
    return acc;
}
double ell_prime(int64_t n, double ell) { return ell * (1.0 + rt_log(2.0) / rt_log((double)n)); }
double lambda_prime(int64_t n, int64_t k, double eps, double lp, int32_t rounds) {
    const double ep = std::sqrt(2.0) * eps;
    const double lnc = (double)rounds * log_binom(n, k);
    volatile double lg2n = std::log2((double)n);
    return (2.0 + 2.0 / 3.0 * ep) * (lnc + lp * rt_log((double)n) + rt_log(lg2n)) * (double)n /
           (ep * ep);
}
// The greedy's approximation ratio enters lambda*: 1 - 1/e for one round (IMM); for
// several rounds the seeds form a partition matroid (at most k per round), where greedy
// guarantees 1/2.  Both the union bound's ln C(n,k) (per round) and the ratio are the only
// places the multi-round problem differs.
double lambda_star(int64_t n, int64_t k, double eps, double lp, int32_t rounds) {
    const double g = rounds == 1 ? 1.0 - 1.0 / kE : 0.5;
    const double lnc = (double)rounds * log_binom(n, k);
    const double alpha = std::sqrt(lp * rt_log((double)n) + rt_log(2.0));
    const double beta = std::sqrt(g * (lnc + lp * rt_log((double)n) + rt_log(2.0)));
    return 2.0 * (double)n * (g * alpha + beta) * (g * alpha + beta) / (eps * eps);
}
// gIM Alg. 2 runs i = 1 .. log2(n) - 1; we read the bound as floor(log2 n) - 1.
int32_t estimation_rounds(int64_t n) {
    int32_t b = 0;
    while (b < 63 && ((int64_t)1 << b) <= n) ++b;
    return b - 2;
}

// ---- ImmPlan ---------------------------------------------------------------------------
imm_status ImmPlan::init(int64_t n_, int32_t k_, double eps_, double ell_, int32_t fresh_,
                         int32_t mr_) {
    if (k_ < 1 || k_ > n_) return fail(IMM_EINVAL, "k = %d outside [1, n]", k_);
    if (mr_ < 1 || mr_ > kMaxRounds) return fail(IMM_EINVAL, "rounds = %d outside [1, %d]", mr_, kMaxRounds);
    if (!(eps_ > 0.0 && eps_ < 1.0)) return fail(IMM_EINVAL, "eps = %g outside (0, 1)", eps_);
    if (!(ell_ > 0.0)) return fail(IMM_EINVAL, "ell = %g must be > 0", ell_);
    *this = ImmPlan();
    n = n_;
    k = k_;
    eps = eps_;
    ell = ell_;
    fresh = fresh_;
    mr = mr_;
    lp = ell_prime(n, ell);
    ep = std::sqrt(2.0) * eps;
    lam1 = lambda_prime(n, k, eps, lp, mr);
    lam2 = lambda_star(n, k, eps, lp, mr);
    rounds = estimation_rounds(n);
    if (rounds < 1) return enter_final();
    return IMM_OK;
}

imm_status ImmPlan::enter_final() {
    final_phase = true;
    const double want = std::ceil(lam2 / lb);
    if (want > (double)kMaxSets) return fail(IMM_ECAPACITY, "theta = %g too large", want);
    theta = (int64_t)want;
    first = fresh ? used : 0;
    upto = fresh ? used + theta : (theta > used ? theta : used);
    if (upto > kMaxSets) return fail(IMM_ECAPACITY, "sample end %lld too large", (long long)upto);
    return IMM_OK;
}

imm_status ImmPlan::next(int64_t* gen_upto, int64_t* sel_first, int64_t* sel_count) {
    if (!final_phase) {
        x = (double)n / (double)((int64_t)1 << i);
        const double want = std::ceil(lam1 / x);
        if (want > (double)kMaxSets) return fail(IMM_ECAPACITY, "theta_%d = %g too large", i, want);
        const int64_t th = (int64_t)want;
        if (th > used) used = th;
        *gen_upto = used;
        *sel_first = 0;
        *sel_count = used;
        return IMM_OK;
    }
    *gen_upto = upto;
    *sel_first = first;
    *sel_count = upto - first;
    return IMM_OK;
}

int64_t ImmPlan::need_cov() const {
    if (final_phase) return 0;
    // the test below, as a function of the coverage; it is monotone (each operation rounds
    // monotonically), so the threshold is found by bisection
    auto pass = [&](int64_t c) { return (double)n * (double)c / (double)used >= (1.0 + ep) * x; };
    if (!pass(used)) return used + 1;
    if (pass(0)) return 0;
    int64_t lo = 0, hi = used;     // !pass(lo), pass(hi)
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (pass(mid)) hi = mid; else lo = mid;
    }
    return hi;
}

imm_status ImmPlan::complete(int64_t cov) {
    ++phases;
    covered = cov;
    if (final_phase) {
        done = true;
        return IMM_OK;
    }
    if ((double)n * (double)cov / (double)used >= (1.0 + ep) * x) {
        lb = (double)n * (double)cov / (double)used / (1.0 + ep);
        IMM_TRY(enter_final());
        // a passing phase ran all (mr * k) greedy rounds over [0, used)
        reuse = first == 0 && upto == used;
        return IMM_OK;
    }
    if (++i > rounds) return enter_final();
    return IMM_OK;
}

}  // namespace imm



extern "C" double imm_log_binom(int64_t n, int64_t k) { return log_binom(n, k); }
extern "C" double imm_lambda_prime(int64_t n, int64_t k, double eps, double ell) {
    return lambda_prime(n, k, eps, ell_prime(n, ell));
}
extern "C" double imm_lambda_star(int64_t n, int64_t k, double eps, double ell) {
    return lambda_star(n, k, eps, ell_prime(n, ell));
}

// ------------------------------------------------------------------------------------
// init / errors
// ------------------------------------------------------------------------------------
extern "C" imm_status imm_init(int32_t device) {
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(IMM_EINVAL, "device %d of %d", device, count);
    HIP_TRY(hipSetDevice(device));
    return noalloc_setup(device);
}

extern "C" const char* imm_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------------------------
// graph
// ------------------------------------------------------------------------------------
extern "C" imm_status imm_graph_destroy(imm_graph* g) {
    if (!g) return IMM_OK;
    dfree(g->vrec);
    dfree(g->src);
    dfree(g->thr);
    dfree(g->cum);
    dfree(g->lrec);
    dfree(g->grec);
    dfree(g->gidx);
    dfree(g->out_off);
    dfree(g->out_dst);
    dfree(g->out_eid);
    delete g;
    return IMM_OK;
}

static imm_status graph_create_impl(imm_graph* g, const int64_t* in_off, const int32_t* in_src,
                                    const float* ic_p, const uint32_t* lt_w, uint32_t flags) {
    const int32_t n = g->n;
    const int64_t m = g->m;
    hipStream_t s = nullptr;
    int64_t* d_off = nullptr;
    float* d_p = nullptr;
    uint32_t* d_w = nullptr;
    uint32_t* d_err = nullptr;
    unsigned int* d_mixed = nullptr;
    imm_status st = IMM_OK;
    const int64_t m_pad = ((m + 3) / 4) * 4 + 4;
    auto cleanup = [&]() {
        dfree(d_off);
        dfree(d_p);
        dfree(d_w);
        dfree(d_err);
        dfree(d_mixed);
    };
#define G_TRY(expr)                  \
    do {                             \
        st = (expr);                 \
        if (st != IMM_OK) {          \
            cleanup();               \
            return st;               \
        }                            \
    } while (0)
#define G_HIP(expr) G_TRY(([&]() -> imm_status { HIP_TRY(expr); return IMM_OK; })())

    G_TRY(dalloc(&d_off, n + 1));
    G_TRY(dalloc(&g->src, m_pad));
    G_TRY(dalloc(&g->vrec, n + 1));
    G_TRY(dalloc(&d_err, 1));
    G_TRY(dalloc(&d_mixed, 1));
    G_HIP(hipMemcpy(d_off, in_off, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDefault));
    G_HIP(hipMemset(g->src, 0, sizeof(int32_t) * (size_t)m_pad));
    if (m > 0) G_HIP(hipMemcpy(g->src, in_src, sizeof(int32_t) * (size_t)m, hipMemcpyDefault));
    if (ic_p) {
        G_TRY(dalloc(&d_p, m));
        if (m > 0) G_HIP(hipMemcpy(d_p, ic_p, sizeof(float) * (size_t)m, hipMemcpyDefault));
    }
    if ((flags & IMM_GRAPH_LT) && lt_w) {
        G_TRY(dalloc(&d_w, m));
        if (m > 0) G_HIP(hipMemcpy(d_w, lt_w, sizeof(uint32_t) * (size_t)m, hipMemcpyDefault));
    }
    G_HIP(hipMemset(d_err, 0, sizeof(uint32_t)));
    G_HIP(hipMemset(d_mixed, 0, sizeof(unsigned int)));
    G_HIP(launch_validate(n, m, d_off, g->src, d_p, d_w, d_err, s));
    uint32_t err = 0;
    G_HIP(hipMemcpy(&err, d_err, sizeof err, hipMemcpyDeviceToHost));
    if (err) {
        cleanup();
        return fail(IMM_EINVAL, "graph arrays rejected:%s%s%s%s", (err & 1) ? " in_off" : "",
                    (err & 2) ? " in_src" : "", (err & 4) ? " ic_p" : "", (err & 8) ? " lt_w" : "");
    }
    if (ic_p) {
        G_TRY(dalloc(&g->thr, m_pad));
        G_HIP(hipMemset(g->thr, 0, sizeof(uint32_t) * (size_t)m_pad));
        G_HIP(launch_encode_ic(m, d_p, g->thr, s));
        g->has_ic = true;
    }
    G_HIP(launch_build_vrec(n, d_off, g->thr, g->vrec, d_mixed, s));
    unsigned int mixed = 0;
    G_HIP(hipMemcpy(&mixed, d_mixed, sizeof mixed, hipMemcpyDeviceToHost));
    g->ic_uniform = g->has_ic && mixed == 0;
    if (flags & IMM_GRAPH_LT) {
        G_TRY(dalloc(&g->cum, m_pad));
        G_HIP(hipMemset(g->cum, 0, sizeof(uint32_t) * (size_t)m_pad));
        G_HIP(launch_encode_lt(n, d_off, d_w, g->cum, s));
        G_TRY(dalloc(&g->lrec, m));
        G_TRY(dalloc(&g->grec, 4 * m));
        G_TRY(dalloc(&g->gidx, 2 * m));
        G_HIP(launch_build_lt_tables(n, m, g->cum, g->src, g->vrec, g->lrec, g->grec, g->gidx, s));
        g->has_lt = true;
    }
    G_HIP(hipDeviceSynchronize());
    cleanup();
    return IMM_OK;
#undef G_TRY
#undef G_HIP
}

extern "C" imm_status imm_graph_create(int32_t n, int64_t m, const int64_t* in_off,
                                       const int32_t* in_src, const float* ic_p,
                                       const uint32_t* lt_w, uint32_t flags, imm_graph** out) {
    if (!out) return fail(IMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 2) return fail(IMM_EINVAL, "n = %d; need n >= 2", n);
    if (m < 0 || m > (int64_t)INT32_MAX) return fail(IMM_EINVAL, "m = %lld out of range", (long long)m);
    if (!in_off || (m > 0 && !in_src)) return fail(IMM_EINVAL, "in_off/in_src missing");
    if (!ic_p && !(flags & IMM_GRAPH_LT)) return fail(IMM_EINVAL, "no IC probabilities and no LT flag");
    if (flags & ~IMM_GRAPH_LT) return fail(IMM_EINVAL, "unknown flags 0x%x", flags);
    imm_graph* g = new imm_graph();
    g->n = n;
    g->m = m;
    if (hipGetDevice(&g->device) != hipSuccess) g->device = 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) != hipSuccess) {
        delete g;
        return fail(IMM_EDEVICE, "hipGetDeviceProperties failed");
    }
    g->cus = prop.multiProcessorCount;
    imm_status st = graph_create_impl(g, in_off, in_src, ic_p, lt_w, flags);
    if (st != IMM_OK) {
        imm_graph_destroy(g);
        return st;
    }
    *out = g;
    return IMM_OK;
}

extern "C" imm_status imm_graph_info(const imm_graph* g, int32_t* n, int64_t* m, int32_t* has_ic,
                                     int32_t* has_lt) {
    if (!g) return fail(IMM_EINVAL, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (has_ic) *has_ic = g->has_ic;
    if (has_lt) *has_lt = g->has_lt;
    return IMM_OK;
}

extern "C" imm_status imm_graph_export_encoding(const imm_graph* g, uint32_t* thr_out,
                                                uint32_t* cum_out) {
    if (!g) return fail(IMM_EINVAL, "graph is NULL");
    if (thr_out) {
        if (!g->has_ic) return fail(IMM_EINVAL, "graph has no IC encoding");
        if (g->m) HIP_TRY(hipMemcpy(thr_out, g->thr, sizeof(uint32_t) * (size_t)g->m, hipMemcpyDeviceToHost));
    }
    if (cum_out) {
        if (!g->has_lt) return fail(IMM_EINVAL, "graph has no LT encoding");
        if (g->m) HIP_TRY(hipMemcpy(cum_out, g->cum, sizeof(uint32_t) * (size_t)g->m, hipMemcpyDeviceToHost));
    }
    return IMM_OK;
}

// ------------------------------------------------------------------------------------
// pool
// ------------------------------------------------------------------------------------
extern "C" imm_status imm_pool_destroy(imm_pool* p) {
    if (!p) return IMM_OK;
    dfree(p->rr_start);
    dfree(p->rr_len);
    dfree(p->ids);
    dfree(p->hist);
    dfree(p->ctr);
    dfree(p->cap_list);
    dfree(p->retry_list);
    p->gen.release();
    p->sel.release();
    p->launch.release();
    for (imm_pool*& q : p->sub) {
        if (q) imm_pool_destroy(q);
        q = nullptr;
    }
    delete p->view;
    delete p;
    return IMM_OK;
}

imm_status imm::pool_init(imm_pool* p) {
    const imm_graph* g = p->g;
    IMM_TRY(dalloc(&p->hist, g->n));
    IMM_TRY(dalloc(&p->ctr, 1));
    HIP_TRY(hipMemset(p->hist, 0, sizeof(uint32_t) * (size_t)g->n));
    HIP_TRY(hipMemset(p->ctr, 0, sizeof(PoolCounters)));
    return p->gen.init(g->device, p->model, g->cus, &g->tuned[p->model]);
}

extern "C" imm_status imm_pool_create(const imm_graph* g, imm_model model, uint64_t seed,
                                      imm_pool** out) {
    if (!out) return fail(IMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(IMM_EINVAL, "graph is NULL");
    if (model != IMM_IC && model != IMM_LT) return fail(IMM_EINVAL, "unknown model %d", (int)model);
    if (model == IMM_IC && !g->has_ic) return fail(IMM_EINVAL, "graph has no IC probabilities");
    if (model == IMM_LT && !g->has_lt) return fail(IMM_EINVAL, "graph has no LT encoding");
    imm_pool* p = new imm_pool();
    p->g = g;
    p->model = model;
    p->seed = seed;
    imm_status st = pool_init(p);
    if (st != IMM_OK) {
        imm_pool_destroy(p);
        return st;
    }
    *out = p;
    return IMM_OK;
}

extern "C" imm_status imm_pool_size(const imm_pool* p, int64_t* num_sets, int64_t* num_ids,
                                    int64_t* edges_examined) {
    if (!p) return fail(IMM_EINVAL, "pool is NULL");
    if (num_sets) *num_sets = p->count;
    if (num_ids) *num_ids = (int64_t)p->sum.placed;
    if (edges_examined) *edges_examined = (int64_t)(p->sum.edges + p->sum.hedges);
    return IMM_OK;
}

extern "C" imm_status imm_generate_rr(imm_pool* p, int64_t upto, void* stream) {
    if (!p) return fail(IMM_EINVAL, "pool is NULL");
    if (upto < 0) return fail(IMM_EINVAL, "upto < 0");
    return pool_generate(p, upto, (hipStream_t)stream);
}

imm_status imm::check_range(const imm_pool* p, int64_t first, int64_t count) {
    if (first < 0 || count < 0 || first + count > p->count)
        return fail(IMM_EINVAL, "range [%lld, %lld) outside pool of %lld sets", (long long)first,
                    (long long)(first + count), (long long)p->count);
    return IMM_OK;
}

extern "C" imm_status imm_rr_export(const imm_pool* pc, int64_t first, int64_t count,
                                    int64_t* off_out, int32_t* ids_out, int64_t ids_cap,
                                    int64_t* ids_needed) {
    if (!pc) return fail(IMM_EINVAL, "pool is NULL");
    imm_pool* p = const_cast<imm_pool*>(pc);
    IMM_TRY(check_range(p, first, count));
    if (!off_out) return fail(IMM_EINVAL, "off_out is NULL");
    hipStream_t s = nullptr;
    int64_t* sizes = nullptr;
    int64_t* off = nullptr;
    int64_t* tmp = nullptr;
    int32_t* out = nullptr;
    imm_status st = IMM_OK;
    auto done = [&](imm_status r) {
        dfree(sizes);
        dfree(off);
        dfree(tmp);
        dfree(out);
        return r;
    };
    if ((st = dalloc(&sizes, count)) != IMM_OK) return done(st);
    if ((st = dalloc(&off, count + 1)) != IMM_OK) return done(st);
    if ((st = dalloc(&tmp, scan_tmp_elems(count))) != IMM_OK) return done(st);
    hipError_t e = launch_set_sizes(p->rr_len, first, count, sizes, s);
    if (e == hipSuccess) e = launch_scan_i64(sizes, count, off, tmp, s);
    if (e == hipSuccess) e = hipMemcpy(off_out, off, sizeof(int64_t) * (size_t)(count + 1), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return done(fail(IMM_EDEVICE, "export: %s", hipGetErrorString(e)));
    const int64_t total = off_out[count];
    if (ids_needed) *ids_needed = total;
    if (!ids_out) return done(IMM_OK);
    if (ids_cap < total) return done(fail(IMM_ECAPACITY, "ids_cap %lld < %lld", (long long)ids_cap, (long long)total));
    if ((st = dalloc(&out, total)) != IMM_OK) return done(st);
    e = launch_gather_sets(p->rr_start, p->rr_len, first, count, off, p->ids, out, s);
    if (e == hipSuccess && total > 0)
        e = hipMemcpy(ids_out, out, sizeof(int32_t) * (size_t)total, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return done(fail(IMM_EDEVICE, "export: %s", hipGetErrorString(e)));
    return done(IMM_OK);
}

static imm_status range_hist(imm_pool* p, SelectWs* w, int64_t first, int64_t count,
                             const uint32_t** out, hipStream_t s) {
    if (first == 0 && count == p->count) {
        *out = p->hist;
        return IMM_OK;
    }
    if (!w->hist_tmp) IMM_TRY(dalloc(&w->hist_tmp, p->g->n));
    HIP_TRY(launch_fill_u32(w->hist_tmp, p->g->n, 0u, s));
    HIP_TRY(launch_hist_range(p->rr_start, p->rr_len, p->ids, first, count, w->hist_tmp, s));
    *out = w->hist_tmp;
    return IMM_OK;
}

extern "C" imm_status imm_rr_histogram(const imm_pool* pc, int64_t first, int64_t count,
                                       uint32_t* hist_out) {
    if (!pc || !hist_out) return fail(IMM_EINVAL, "NULL argument");
    imm_pool* p = const_cast<imm_pool*>(pc);
    IMM_TRY(check_range(p, first, count));
    const uint32_t* h = nullptr;
    IMM_TRY(range_hist(p, &p->sel, first, count, &h, nullptr));
    HIP_TRY(hipMemcpy(hist_out, h, sizeof(uint32_t) * (size_t)p->g->n, hipMemcpyDeviceToHost));
    return IMM_OK;
}

// ------------------------------------------------------------------------------------
// selection
// ------------------------------------------------------------------------------------
int64_t SelectWs::bytes() const {
    int64_t b = (hot_words ? (n + 31) / 32 * 8 + hot_list_blocks(n) * 4 + kSelectHotBuckets * 4 + 8 : 0) +
                hot_cap * 4 + part_cap * 4 + pair_cap * 8 + (bcur ? kInvBuckets * 8 : 0);
    if (h) b += n * (4 + 4 + 8 + 4) + 8;
    for (const IndexSeg& x : seg) b += x.off ? (n + 1) * 8 + x.cap * 4 : 0;
    if (snap) b += n * 4;
    b += cap_cov * 4 + cap_k * 12;
    return b;
}

void SelectWs::release() {
    dfree(h);
    dfree(hist_tmp);
    for (IndexSeg& x : seg) {
        dfree(x.off);
        dfree(x.inv);
        x.cap = 0;
    }
    nseg = 0;
    ix_pool = nullptr;
    snap_valid = false;
    dfree(snap);
    dfree(scan_tmp);
    dfree(cursor);
    dfree(covered);
    dfree(taken);
    dfree(keys);
    dfree(seeds);
    dfree(n_covered);
    hfree(host_seeds);
    hfree(host_keys);
    hfree(host_cov);
    dfree(hot_words);
    dfree(bcur);
    dfree(pairs);
    dfree(hot_blk);
    dfree(cnt_hist);
    dfree(hot_n);
    dfree(hot_ids);
    dfree(hot_part);
    cap_cov = cap_k = hot_cap = part_cap = pair_cap = 0;
}

void SelectLaunch::release() {
    dfree(d_inst);
    dfree(bar);
    hfree(host_bar);
    hfree(host_inst);
    cap = 0;
}

int64_t imm_pool::bytes() const {
    int64_t b = cap_sets * 12 + cap_ids * 4 + (int64_t)g->n * 4 + cap_lists * 8;
    b += gen.bytes();
    return b + sel.bytes();
}

static imm_status ensure_select(imm_pool* p, SelectWs* w, int64_t count, int32_t k) {
    const int64_t n = p->g->n;
    if (!w->h) {
        w->n = n;
        IMM_TRY(dalloc(&w->h, n));
        IMM_TRY(dalloc(&w->scan_tmp, scan_tmp_elems(n)));
        IMM_TRY(dalloc(&w->cursor, n));
        IMM_TRY(dalloc(&w->n_covered, 1));
        IMM_TRY(dalloc(&w->taken, kMaxRounds));
        IMM_TRY(halloc(&w->host_cov, 1));
    }
    if (count > w->cap_cov) {
        dfree(w->covered);
        int64_t c = count + count / 4 + 1024;
        IMM_TRY(dalloc(&w->covered, c));
        w->cap_cov = c;
    }
    if (k > w->cap_k) {
        dfree(w->keys);
        dfree(w->seeds);
        hfree(w->host_seeds);
        hfree(w->host_keys);
        IMM_TRY(dalloc(&w->keys, k));
        IMM_TRY(dalloc(&w->seeds, k));
        IMM_TRY(halloc(&w->host_seeds, k));
        IMM_TRY(halloc(&w->host_keys, k));
        w->cap_k = k;
    }
    return IMM_OK;
}

// Indexes sets [set_lo, set_lo + set_n) with counts cnt (n entries) as segment w->nseg,
// entries holding rel0 + (set - set_lo); members is an upper bound on their total.
static imm_status index_segment(imm_pool* p, SelectWs* w, const uint32_t* cnt, int64_t set_lo,
                                int64_t set_n, uint32_t rel0, int64_t members, hipStream_t s) {
    const int64_t n = p->g->n;
    SelectWs::IndexSeg& x = w->seg[w->nseg];
    if (!x.off) IMM_TRY(dalloc(&x.off, n + 1));
    if (members > x.cap) {
        dfree(x.inv);
        const int64_t c = members + members / 4 + 1024;
        IMM_TRY(dalloc(&x.inv, c));
        x.cap = c;
    }
    HIP_TRY(launch_scan_u32(cnt, n, x.off, w->scan_tmp, s));
    // bucketed build (IMM_INV_BUCKETED=0 selects the per-entry atomic scatter)
    const char* e = getenv("IMM_INV_BUCKETED");
    if ((!e || atoi(e) != 0) && inv_bucket_shift(n) != 0 && !no_alloc_active()) {
        if (!w->bcur) IMM_TRY(dalloc(&w->bcur, kInvBuckets));
        if (members > w->pair_cap) {
            dfree(w->pairs);
            const int64_t c = members + members / 4 + 1024;
            IMM_TRY(dalloc(&w->pairs, c));
            w->pair_cap = c;
        }
        HIP_TRY(launch_inv_bucketed(p->rr_start, p->rr_len, p->ids, set_lo, set_n, rel0, x.off, n, w->bcur,
                                    w->pairs, w->pair_cap, x.inv, s));
    } else {
        HIP_TRY(launch_fill_u32(w->cursor, n, 0u, s));
        HIP_TRY(launch_inv_scatter(p->rr_start, p->rr_len, p->ids, set_lo, set_n, rel0, x.off, w->cursor,
                                   x.inv, s));
    }
    ++w->nseg;
    return IMM_OK;
}

// Smallest gain of a dense selection round (IMM_SELECT_DENSE overrides, read at each
// selection; 0 turns them off).
int32_t imm::select_dense_gain() {
    const char* e = getenv("IMM_SELECT_DENSE");
    return e ? (int32_t)std::min(std::max(0ll, atoll(e)), 0x7FFFFFFFll) : (int32_t)2048;
}

int32_t imm::select_hot_max(int64_t n) {
    int64_t t = 16384;
    bool forced = false;
    if (const char* e = getenv("IMM_SELECT_HOT")) {
        t = std::max(0ll, atoll(e));
        forced = true;
    }
    t = std::min<int64_t>(t, (int64_t)kSelectHotPerBlock * select_coop_grid());
    if (t <= 0 || n <= (forced ? t : 2 * t)) return 0;
    return (int32_t)t;
}

imm_status imm::select_prepare(imm_pool* p, SelectWs* w, int64_t first, int64_t count, int32_t kr,
                               hipStream_t s, SelInst* out, bool segments, bool hot) {
    const int32_t n = p->g->n;
    const int32_t k = kr * p->rounds;        // multi-round: kr seeds per round
    IMM_TRY(ensure_select(p, w, count, k));
    const int32_t hot_max = hot ? select_hot_max(n) : 0;
    if (hot_max > 0) {
        if (!w->hot_words) {
            IMM_TRY(dalloc(&w->hot_words, (n + 31) / 32));
            IMM_TRY(dalloc(&w->hot_blk, hot_list_blocks(n)));
            IMM_TRY(dalloc(&w->cnt_hist, kSelectHotBuckets));
            IMM_TRY(dalloc(&w->hot_n, 2));
        }
        if (hot_max > w->hot_cap) {
            dfree(w->hot_ids);
            IMM_TRY(dalloc(&w->hot_ids, hot_max));
            w->hot_cap = hot_max;
        }
        const int64_t part = (int64_t)select_coop_grid() * hot_max;
        if (select_dense_gain() > 0 && hot_max <= kSelectDenseHot && part > w->part_cap &&
            !no_alloc_active()) {
            dfree(w->hot_part);
            IMM_TRY(dalloc(&w->hot_part, part));
            w->part_cap = part;
        }
    }
    const uint32_t* hsrc = nullptr;
    IMM_TRY(range_hist(p, w, first, count, &hsrc, s));
    if (hot_max == 0) HIP_TRY(launch_copy_hist(hsrc, w->h, n, s));
    const bool prefix = first == 0 && count == p->count;      // hsrc is the pool histogram
    const int64_t placed = (int64_t)p->sum.placed;
    if (segments && prefix && w->ix_pool == p && w->snap_valid && w->ix_first == 0 &&
        w->nseg > 0 && w->ix_end <= count && (w->ix_end == count || w->nseg < kMaxSegs)) {
        if (w->ix_end < count) {
            // a longer prefix of the same pool: index only the sets drawn since
            if (!w->hist_tmp) IMM_TRY(dalloc(&w->hist_tmp, n));
            HIP_TRY(launch_sub_u32(p->hist, w->snap, w->hist_tmp, n, s));
            IMM_TRY(index_segment(p, w, w->hist_tmp, w->ix_end, count - w->ix_end,
                                  (uint32_t)w->ix_end, placed - w->ix_members, s));
            HIP_TRY(hipMemcpyAsync(w->snap, p->hist, sizeof(uint32_t) * (size_t)n,
                                   hipMemcpyDeviceToDevice, s));
            w->ix_end = count;
            w->ix_members = placed;
        }
    } else {
        w->nseg = 0;
        IMM_TRY(index_segment(p, w, hsrc, first, count, 0u, placed, s));
        w->ix_pool = p;
        w->ix_first = first;
        w->ix_end = first + count;
        w->snap_valid = segments && prefix;
        if (w->snap_valid) {
            if (!w->snap) IMM_TRY(dalloc(&w->snap, n));
            HIP_TRY(hipMemcpyAsync(w->snap, p->hist, sizeof(uint32_t) * (size_t)n,
                                   hipMemcpyDeviceToDevice, s));
            w->ix_members = placed;
        }
    }
    HIP_TRY(launch_fill_u32(w->covered, count, 0u, s));
    if (hot_max > 0) {
        HIP_TRY(launch_fill_u32(w->cnt_hist, kSelectHotBuckets, 0u, s));
        HIP_TRY(launch_fill_u32(w->hot_n, 2, 0u, s));
        HIP_TRY(launch_hot_prepare(hsrc, w->h, n, hot_max, w->cnt_hist, w->hot_blk, w->hot_words,
                                   w->hot_ids, w->hot_n, s));
    }
    HIP_TRY(launch_fill_u64(w->keys, k, 0ull, s));
    HIP_TRY(launch_fill_u64(w->n_covered, 1, 0ull, s));
    if (p->rounds > 1) HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(w->taken), kMaxRounds, 0u, s));
    w->k = k;
    SelInst si{};
    si.n = n;
    si.k = k;
    si.part_n = p->rounds > 1 ? p->n_base : 0;
    si.part_k = kr;
    si.taken = w->taken;
    si.first = first;
    si.count = count;
    si.h = w->h;
    si.inv_off = w->seg[0].off;
    si.inv = w->seg[0].inv;
    si.nseg = w->nseg;
    for (int32_t j = 0; j < w->nseg; ++j) {
        si.seg_off[j] = w->seg[j].off;
        si.seg_inv[j] = w->seg[j].inv;
    }
    si.rr_start = p->rr_start;
    si.rr_len = p->rr_len;
    si.ids = p->ids;
    si.covered = w->covered;
    si.keys = w->keys;
    si.seeds = w->seeds;
    si.n_covered = w->n_covered;
    si.h0 = hsrc;
    si.hot_max = hot_max;
    si.hot_words = w->hot_words;
    si.hot_n = w->hot_n;
    si.hot_ids = w->hot_ids;
    if (hot_max > 0 && hot_max <= kSelectDenseHot &&
        w->part_cap >= (int64_t)select_coop_grid() * hot_max) {
        si.hot_part = w->hot_part;
        si.dense_gain = select_dense_gain();
    }
    *out = si;
    return IMM_OK;
}

imm_status imm::select_run(SelectLaunch* L, SelectWs* const* ws, const SelInst* inst, int32_t ninst,
                           hipStream_t s) {
    IMM_TRY(select_enqueue(L, ws, inst, ninst, s));
    return select_wait(L, s);
}

imm_status imm::select_enqueue(SelectLaunch* L, SelectWs* const* ws, const SelInst* inst,
                               int32_t ninst, hipStream_t s, bool captured) {
    if (ninst > L->cap) {
        L->release();
        IMM_TRY(dalloc(&L->d_inst, ninst));
        IMM_TRY(dalloc(&L->bar, 1));
        IMM_TRY(halloc(&L->host_bar, 1));
        IMM_TRY(halloc(&L->host_inst, ninst));
        L->cap = ninst;
    }
    // a captured copy reads its source when the graph runs: stage the descriptors in
    // pinned memory owned by the launch
    const SelInst* src = inst;
    if (L->host_inst) {
        memcpy(L->host_inst, inst, sizeof(SelInst) * (size_t)ninst);
        src = L->host_inst;
    }
    HIP_TRY(hipMemcpyAsync(L->d_inst, src, sizeof(SelInst) * (size_t)ninst, hipMemcpyHostToDevice, s));
    // one cooperative launch per group of at most select_max_inst() instances; the barrier
    // counters start from zero for each launch, and its error flag is collected at the end
    const int32_t per = select_max_inst();
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(L->bar), sizeof(GridBarrier) / 4, 0u, s));
    for (int32_t a = 0; a < ninst; a += per) {
        const int32_t cnt = std::min(per, ninst - a);
        int32_t maxk = 0;
        for (int32_t i = a; i < a + cnt; ++i) maxk = std::max(maxk, inst[i].k);
        if (a > 0) HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(L->bar), 16 * 16 + 1, 0u, s));
        HIP_TRY(launch_select_coop(L->d_inst + a, cnt, maxk, L->bar, s, captured));
    }
    HIP_TRY(hipMemcpyAsync(L->host_bar, L->bar, sizeof(GridBarrier), hipMemcpyDeviceToHost, s));
    for (int32_t i = 0; i < ninst; ++i) {
        SelectWs* w = ws[i];
        HIP_TRY(hipMemcpyAsync(w->host_seeds, w->seeds, sizeof(int32_t) * (size_t)w->k,
                               hipMemcpyDeviceToHost, s));
        if (w->host_keys)
            HIP_TRY(hipMemcpyAsync(w->host_keys, w->keys, sizeof(unsigned long long) * (size_t)w->k,
                                   hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(w->host_cov, w->n_covered, sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s));
    }
    return IMM_OK;
}

imm_status imm::select_wait(SelectLaunch* L, hipStream_t s) {
    HIP_TRY(hipStreamSynchronize(s));
    if (L->host_bar->err) return fail(IMM_EDEVICE, "selection grid barrier timed out");
    return IMM_OK;
}

static imm_status pool_select(imm_pool* p, int64_t first, int64_t count, int32_t k,
                              int32_t* seeds_out, int64_t* covered_out, hipStream_t s,
                              int64_t need = 0) {
    SelInst si;
    IMM_TRY(select_prepare(p, &p->sel, first, count, k, s, &si, true, true));
    si.need = need;
    SelectWs* w = &p->sel;
    IMM_TRY(select_run(&p->launch, &w, &si, 1, s));
    if (seeds_out) memcpy(seeds_out, w->host_seeds, sizeof(int32_t) * (size_t)w->k);
    if (covered_out) *covered_out = (int64_t)*w->host_cov;
    return IMM_OK;
}

extern "C" imm_status imm_select_seeds(imm_pool* p, int64_t first, int64_t count, int32_t k,
                                       int32_t* seeds_out, int64_t* covered_out, void* stream) {
    if (!p) return fail(IMM_EINVAL, "pool is NULL");
    IMM_TRY(check_range(p, first, count));
    if (k < 1 || k > pool_vertices(p)) return fail(IMM_EINVAL, "k = %d outside [1, n]", k);
    return pool_select(p, first, count, k, seeds_out, covered_out, (hipStream_t)stream);
}

// ------------------------------------------------------------------------------------
// IMM driver
// ------------------------------------------------------------------------------------
imm_status imm::run_imm(imm_pool* p, int32_t k, double eps, double ell, int32_t fresh,
                        hipStream_t s, int32_t* seeds_out, imm_info* info) {
    if (!seeds_out) return fail(IMM_EINVAL, "seeds_out is NULL");
    const double t0 = now_s();
    double t_gen = 0.0, t_sel = 0.0;
    const double kernel_s0 = p->gen.kernel_s, heavy_s0 = p->gen.heavy_s;
    const int64_t launches0 = p->gen.kernel_launches, heavy0 = p->gen.heavy_launches;
    const int64_t redrawn0 = p->gen.heavy_overflow;
    if (p->rounds > 1 && fresh) return fail(IMM_EINVAL, "multi-round solves reuse the estimation sets");
    ImmPlan plan;
    IMM_TRY(plan.init(pool_vertices(p), k, eps, ell, fresh, p->rounds));
    while (!plan.done) {
        if (plan.reuses_last()) {          // seeds_out holds that phase's seeds
            IMM_TRY(plan.complete(plan.covered));
            continue;
        }
        int64_t upto, first, count, cov = 0;
        IMM_TRY(plan.next(&upto, &first, &count));
        const double ta = now_s();
        IMM_TRY(pool_generate(p, upto, s));
        const double tb = now_s();
        IMM_TRY(pool_select(p, first, count, k, seeds_out, &cov, s, plan.need_cov()));
        t_gen += tb - ta;
        t_sel += now_s() - tb;
        IMM_TRY(plan.complete(cov));
    }
    if (info) {
        memset(info, 0, sizeof *info);
        info->theta = plan.theta;
        info->num_rr = plan.upto;
        info->covered = plan.covered;
        info->edges_examined = (int64_t)(p->sum.edges + p->sum.hedges);
        info->edges_heavy = (int64_t)p->sum.hedges;
        info->heavy_redrawn = (int32_t)std::min<int64_t>(p->gen.heavy_overflow - redrawn0, INT32_MAX);
        info->pool_ids = (int64_t)p->sum.placed;
        info->phases = plan.phases;
        info->lb = plan.lb;
        info->spread_est = plan.spread_est();
        info->lambda_prime = plan.lam1;
        info->lambda_star = plan.lam2;
        info->t_generate_s = t_gen;
        info->t_select_s = t_sel;
        info->t_total_s = now_s() - t0;
        info->t_rr_kernel_s = p->gen.kernel_s - kernel_s0;
        info->rr_kernel_launches = p->gen.kernel_launches - launches0;
        info->t_rr_heavy_s = p->gen.heavy_s - heavy_s0;
        info->rr_heavy_launches = p->gen.heavy_launches - heavy0;
    }
    return IMM_OK;
}

extern "C" imm_status imm_solve_pool(imm_pool* p, int32_t k, double eps, double ell,
                                     int32_t fresh_final, void* stream, int32_t* seeds_out,
                                     imm_info* info) {
    if (!p) return fail(IMM_EINVAL, "pool is NULL");
    return run_imm(p, k, eps, ell, fresh_final, (hipStream_t)stream, seeds_out, info);
}

extern "C" imm_status imm_solve(const imm_graph* g, int32_t k, double eps, double ell,
                                imm_model model, const imm_options* opt, int32_t* seeds_out,
                                imm_info* info) {
    if (!g) return fail(IMM_EINVAL, "graph is NULL");
    imm_options o{};
    if (opt) o = *opt;
    imm_pool* p = nullptr;
    IMM_TRY(imm_pool_create(g, model, o.seed, &p));
    imm_status st = run_imm(p, k, eps, ell, o.fresh_final, (hipStream_t)o.stream, seeds_out, info);
    imm_pool_destroy(p);
    return st;
}
