// Host side of libimm: the C ABI declared in include/imm.h.
//
// Owns device memory for graphs and RR pools, launches the kernels of graph.hip,
// rr_gen.hip and select.hip, and runs IMM's estimation loop (gIM Alg. 2) and final
// sample/selection (gIM Alg. 1) on the host in IEEE double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/imm.h"
#include "kernels.hpp"

using namespace imm;

namespace {

thread_local std::string g_err;

imm_status fail(imm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? IMM_ENOMEM : IMM_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)

#define IMM_TRY(expr)                  \
    do {                               \
        imm_status s_ = (expr);        \
        if (s_ != IMM_OK) return s_;   \
    } while (0)

constexpr int64_t kMaxSets = (int64_t)INT32_MAX;   // RR index and counters fit int32

template <typename T>
imm_status dalloc(T** p, int64_t count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)count);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(IMM_ENOMEM, "hipMalloc of %lld bytes failed: %s",
                    (long long)(sizeof(T) * count), hipGetErrorString(e));
    }
    return IMM_OK;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Grow a device array to at least `need` elements, keeping the first `keep` elements.
template <typename T>
imm_status dgrow(T** p, int64_t* cap, int64_t need, int64_t keep, hipStream_t s) {
    if (need <= *cap) return IMM_OK;
    int64_t nc = *cap > 0 ? *cap : 1024;
    while (nc < need) nc *= 2;
    T* q = nullptr;
    IMM_TRY(dalloc(&q, nc));
    if (keep > *cap) keep = *cap;
    if (*p && keep > 0) {
        hipError_t e = hipMemcpyAsync(q, *p, sizeof(T) * (size_t)keep, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipFree(q);
            return fail(IMM_EDEVICE, "grow copy failed: %s", hipGetErrorString(e));
        }
    }
    if (*p) (void)hipFree(*p);
    *p = q;
    *cap = nc;
    return IMM_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ------------------------------------------------------------------------------------
// objects
// ------------------------------------------------------------------------------------
struct imm_graph {
    int device = 0;
    int32_t n = 0;
    int64_t m = 0;
    VRec* vrec = nullptr;
    int32_t* src = nullptr;
    uint32_t* thr = nullptr;     // IC thresholds (padded to a multiple of 4 edges)
    uint32_t* cum = nullptr;     // LT cumulative thresholds
    bool has_ic = false, has_lt = false;
    bool ic_uniform = false;     // every vertex has one common IC threshold
    int cus = 0;
};

struct imm_pool {
    const imm_graph* g = nullptr;
    imm_model model = IMM_IC;
    uint64_t seed = 0;
    int64_t count = 0;

    int64_t cap_sets = 0;
    int64_t* rr_start = nullptr;
    int32_t* rr_len = nullptr;
    int64_t cap_ids = 0;
    int32_t* ids = nullptr;
    uint32_t* hist = nullptr;
    PoolCounters* ctr = nullptr;
    PoolCounters* host_ctr = nullptr;   // pinned mirror

    int64_t cap_lists = 0;
    uint32_t* heavy_list = nullptr;     // light -> heavy queue
    uint32_t* cap_list = nullptr;       // id-buffer capacity misses
    uint32_t* retry_list = nullptr;

    int grid = 0;                       // light launch: blocks of 256 threads
    int64_t vis_words = 0;
    uint32_t* visited = nullptr;        // grid * 4 bitmaps
    int64_t hslots = 0;                 // heavy slots (IC: workgroups, LT: waves)
    uint32_t* hvisited = nullptr;
    int32_t* hlist = nullptr;
    int64_t budget = 4096;              // light-wave group budget per set
    int heavy_block = 256;              // threads per heavy set (256 or 1024)

    // selection workspace
    int32_t* h = nullptr;
    uint32_t* hist_tmp = nullptr;
    int64_t* inv_off = nullptr;
    int64_t* scan_tmp = nullptr;
    uint32_t* cursor = nullptr;
    int64_t cap_inv = 0;
    uint32_t* inv = nullptr;
    int64_t cap_cov = 0;
    uint8_t* covered = nullptr;
    int64_t cap_k = 0;
    unsigned long long* keys = nullptr;
    int32_t* seeds = nullptr;
    unsigned long long* n_covered = nullptr;
    int32_t* host_seeds = nullptr;      // pinned, cap_k
    unsigned long long* host_cov = nullptr;

    // HIP events bracketing each RR-generation kernel launch
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double kernel_s = 0.0;               // light kernel (IC) / walk kernel (LT)
    int64_t kernel_launches = 0;
    double heavy_s = 0.0;                // heavy kernel (IC) / HBM-list walk kernel (LT)
    int64_t heavy_launches = 0;
};

static unsigned long long sum64(const unsigned long long* v) {
    unsigned long long t = 0;
    for (int i = 0; i < 64; ++i) t += v[i];
    return t;
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

double log_binom(int64_t n, int64_t k) {
    double acc = 0.0;
    for (int64_t i = 0; i < k; ++i) acc += rt_log((double)(n - i)) - rt_log((double)(i + 1));
    return acc;
}
double ell_prime(int64_t n, double ell) { return ell * (1.0 + rt_log(2.0) / rt_log((double)n)); }
double lambda_prime(int64_t n, int64_t k, double eps, double lp) {
    const double ep = std::sqrt(2.0) * eps;
    const double lnc = log_binom(n, k);
    volatile double lg2n = std::log2((double)n);
    return (2.0 + 2.0 / 3.0 * ep) * (lnc + lp * rt_log((double)n) + rt_log(lg2n)) * (double)n /
           (ep * ep);
}
double lambda_star(int64_t n, int64_t k, double eps, double lp) {
    const double lnc = log_binom(n, k);
    const double alpha = std::sqrt(lp * rt_log((double)n) + rt_log(2.0));
    const double beta = std::sqrt((1.0 - 1.0 / kE) * (lnc + lp * rt_log((double)n) + rt_log(2.0)));
    return 2.0 * (double)n * ((1.0 - 1.0 / kE) * alpha + beta) * ((1.0 - 1.0 / kE) * alpha + beta) /
           (eps * eps);
}
// gIM Alg. 2 runs i = 1 .. log2(n) - 1; we read the bound as floor(log2 n) - 1.
int32_t estimation_rounds(int64_t n) {
    int32_t b = 0;
    while (b < 63 && ((int64_t)1 << b) <= n) ++b;
    return b - 2;
}
}  // namespace

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
    return IMM_OK;
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
    if (p->host_ctr) (void)hipHostFree(p->host_ctr);
    dfree(p->heavy_list);
    dfree(p->cap_list);
    dfree(p->retry_list);
    dfree(p->visited);
    dfree(p->hvisited);
    dfree(p->hlist);
    dfree(p->h);
    dfree(p->hist_tmp);
    dfree(p->inv_off);
    dfree(p->scan_tmp);
    dfree(p->cursor);
    dfree(p->inv);
    dfree(p->covered);
    dfree(p->keys);
    dfree(p->seeds);
    dfree(p->n_covered);
    if (p->host_seeds) (void)hipHostFree(p->host_seeds);
    if (p->host_cov) (void)hipHostFree(p->host_cov);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    delete p;
    return IMM_OK;
}

static imm_status pool_init(imm_pool* p) {
    const imm_graph* g = p->g;
    const bool lt = p->model == IMM_LT;
    p->grid = g->cus * gen_blocks_per_cu(lt ? 2 : 0);
    p->vis_words = ((int64_t)g->n + 31) / 32;
    // light visited bitmaps: at most ~4 GiB (fewer resident blocks on huge graphs)
    const int64_t vis_bytes_per_block = 4 * p->vis_words * 4;
    const int64_t max_blocks = std::max<int64_t>(g->cus, ((int64_t)4 << 30) / vis_bytes_per_block);
    if (p->grid > max_blocks) p->grid = (int)max_blocks;
    IMM_TRY(dalloc(&p->hist, g->n));
    IMM_TRY(dalloc(&p->ctr, 1));
    IMM_TRY(dalloc(&p->visited, (int64_t)p->grid * 4 * p->vis_words));
    HIP_TRY(hipMemset(p->hist, 0, sizeof(uint32_t) * (size_t)g->n));
    HIP_TRY(hipMemset(p->ctr, 0, sizeof(PoolCounters)));
    HIP_TRY(hipMemset(p->visited, 0, sizeof(uint32_t) * (size_t)(p->grid * 4 * p->vis_words)));
    HIP_TRY(hipHostMalloc((void**)&p->host_ctr, sizeof(PoolCounters), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void**)&p->host_cov, sizeof(unsigned long long), hipHostMallocDefault));
    memset(p->host_ctr, 0, sizeof(PoolCounters));
    HIP_TRY(hipEventCreate(&p->ev0));
    HIP_TRY(hipEventCreate(&p->ev1));
    if (const char* b = getenv("IMM_LIGHT_BUDGET")) p->budget = std::max(1ll, atoll(b));
    if (const char* b = getenv("IMM_HEAVY_BLOCK")) p->heavy_block = atoi(b) == 1024 ? 1024 : 256;
    return IMM_OK;
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

static imm_status read_counters(imm_pool* p, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(p->host_ctr, p->ctr, sizeof(PoolCounters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return IMM_OK;
}

extern "C" imm_status imm_pool_size(const imm_pool* p, int64_t* num_sets, int64_t* num_ids,
                                    int64_t* edges_examined) {
    if (!p) return fail(IMM_EINVAL, "pool is NULL");
    PoolCounters c;
    HIP_TRY(hipMemcpy(&c, p->ctr, sizeof c, hipMemcpyDeviceToHost));
    if (num_sets) *num_sets = p->count;
    if (num_ids) *num_ids = (int64_t)sum64(c.placed);
    if (edges_examined) *edges_examined = (int64_t)(sum64(c.edges) + sum64(c.hedges));
    return IMM_OK;
}

static GenArgs gen_args(imm_pool* p) {
    const imm_graph* g = p->g;
    GenArgs a{};
    a.vrec = g->vrec;
    a.src = g->src;
    a.thr = g->thr;
    a.cum = g->cum;
    a.n = g->n;
    a.k0 = (uint32_t)p->seed;
    a.k1 = (uint32_t)(p->seed >> 32);
    a.budget = p->budget;
    a.heavy_list = p->heavy_list;
    a.ids = p->ids;
    a.cap_ids = p->cap_ids;
    a.rr_start = p->rr_start;
    a.rr_len = p->rr_len;
    a.hist = p->hist;
    a.ctr = p->ctr;
    a.cap_list = p->cap_list;
    a.visited = p->visited;
    a.hvisited = p->hvisited;
    a.vis_words = p->vis_words;
    a.hlist = p->hlist;
    return a;
}

static double elapsed_s(imm_pool* p) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p->ev0, p->ev1) != hipSuccess) return 0.0;
    return ms * 1e-3;
}

// Light launch over RR indices first + i (or list[i]), i < count.
static imm_status run_light(imm_pool* p, int64_t first, int64_t count, const uint32_t* list,
                            hipStream_t s) {
    HIP_TRY(hipMemsetAsync(&p->ctr->work, 0, sizeof(unsigned long long), s));
    HIP_TRY(hipMemsetAsync(&p->ctr->n_heavy, 0, 2 * sizeof(unsigned int), s));
    GenArgs a = gen_args(p);
    a.first = first;
    a.count = count;
    a.list = list;
    int64_t grid = std::min<int64_t>(p->grid, (count + 3) / 4);
    if (grid < 1) grid = 1;
    HIP_TRY(hipEventRecord(p->ev0, s));
    if (p->model == IMM_IC) HIP_TRY(launch_ic_light(a, (int)grid, s));
    else HIP_TRY(launch_lt(a, false, (int)grid, s));
    HIP_TRY(hipEventRecord(p->ev1, s));
    IMM_TRY(read_counters(p, s));
    p->kernel_s += elapsed_s(p);
    p->kernel_launches += 1;
    return IMM_OK;
}

static imm_status ensure_heavy(imm_pool* p) {
    if (p->hlist) return IMM_OK;
    const int64_t n = p->g->n;
    const bool lt = p->model == IMM_LT;
    // slots: IC one per 1024-thread workgroup, LT one per wave; lists of n entries each,
    // bounded to ~4 GiB of lists
    int64_t want = lt ? (int64_t)p->g->cus * gen_blocks_per_cu(3) * 4
                      : (int64_t)p->g->cus * gen_blocks_per_cu(p->heavy_block == 1024 ? 1 : 4);
    int64_t cap = std::max<int64_t>(4, ((int64_t)4 << 30) / (4 * n + 4 * p->vis_words));
    int64_t slots = std::min(want, cap);
    if (lt) slots = std::max<int64_t>(4, (slots / 4) * 4);
    IMM_TRY(dalloc(&p->hlist, slots * n));
    IMM_TRY(dalloc(&p->hvisited, slots * p->vis_words));
    HIP_TRY(hipMemset(p->hvisited, 0, sizeof(uint32_t) * (size_t)(slots * p->vis_words)));
    p->hslots = slots;
    return IMM_OK;
}

// Heavy launch over the queue the last light launch filled.
static imm_status run_heavy(imm_pool* p, uint32_t n_queue, hipStream_t s) {
    IMM_TRY(ensure_heavy(p));
    HIP_TRY(hipMemsetAsync(&p->ctr->hwork, 0, sizeof(unsigned int), s));
    GenArgs a = gen_args(p);
    a.queue = p->heavy_list;
    a.n_queue = n_queue;
    a.first = 0;
    a.count = n_queue;
    a.list = p->heavy_list;
    HIP_TRY(hipEventRecord(p->ev0, s));
    if (p->model == IMM_IC) {
        int64_t grid = std::min<int64_t>(p->hslots, n_queue);
        HIP_TRY(launch_ic_heavy(a, p->heavy_block, (int)std::max<int64_t>(grid, 1), s));
    } else {
        // LT: sets too long for the on-chip list walk with their lists in HBM
        HIP_TRY(hipMemsetAsync(&p->ctr->work, 0, sizeof(unsigned long long), s));
        int64_t grid = std::min<int64_t>(p->hslots / 4, ((int64_t)n_queue + 3) / 4);
        HIP_TRY(launch_lt(a, true, (int)std::max<int64_t>(grid, 1), s));
    }
    HIP_TRY(hipEventRecord(p->ev1, s));
    IMM_TRY(read_counters(p, s));
    p->heavy_s += elapsed_s(p);
    p->heavy_launches += 1;
    return IMM_OK;
}

static imm_status pool_generate(imm_pool* p, int64_t upto, hipStream_t s) {
    if (upto <= p->count) return IMM_OK;
    if (upto > kMaxSets) return fail(IMM_ECAPACITY, "RR index %lld exceeds 2^31-1", (long long)upto);
    const int64_t first = p->count, cnt = upto - first;
    int64_t cap_sets = p->cap_sets;
    IMM_TRY(dgrow(&p->rr_start, &cap_sets, upto, p->count, s));
    cap_sets = p->cap_sets;
    IMM_TRY(dgrow(&p->rr_len, &cap_sets, upto, p->count, s));
    p->cap_sets = cap_sets;
    if (cnt > p->cap_lists) {
        dfree(p->heavy_list);
        dfree(p->cap_list);
        dfree(p->retry_list);
        IMM_TRY(dalloc(&p->heavy_list, cnt));
        IMM_TRY(dalloc(&p->cap_list, cnt));
        IMM_TRY(dalloc(&p->retry_list, cnt));
        p->cap_lists = cnt;
    }
    // id-buffer size from the mean set size seen so far, with room for the per-wave
    // reservation chunks left partly unused at the end of each launch
    const unsigned long long placed = sum64(p->host_ctr->placed);
    const double mean = p->count > 0 ? (double)placed / (double)p->count : 16.0;
    const int64_t slack = ((int64_t)p->grid * 4 + p->g->cus * 8) * (int64_t)2048;
    const int64_t need = (int64_t)p->host_ctr->tail + (int64_t)(mean * 1.3 * (double)cnt) + slack;
    IMM_TRY(dgrow(&p->ids, &p->cap_ids, need, (int64_t)p->host_ctr->tail, s));

    IMM_TRY(run_light(p, first, cnt, nullptr, s));
    for (int guard = 0; guard < 64; ++guard) {
        if (p->host_ctr->n_heavy > 0) IMM_TRY(run_heavy(p, p->host_ctr->n_heavy, s));
        const unsigned int n_cap = p->host_ctr->n_capacity;
        if (n_cap == 0) {
            p->count = upto;
            return IMM_OK;
        }
        // grow the id buffer and rerun the sets that did not fit
        const int64_t tail = (int64_t)p->host_ctr->tail;
        const int64_t want = tail + (int64_t)(std::max(mean, 64.0) * 2.0 * (double)n_cap) + slack;
        IMM_TRY(dgrow(&p->ids, &p->cap_ids, std::max(want, 2 * p->cap_ids), tail, s));
        HIP_TRY(hipMemcpyAsync(p->retry_list, p->cap_list, sizeof(uint32_t) * n_cap,
                               hipMemcpyDeviceToDevice, s));
        IMM_TRY(run_light(p, 0, n_cap, p->retry_list, s));
    }
    return fail(IMM_EDEVICE, "RR placement did not converge");
}

extern "C" imm_status imm_generate_rr(imm_pool* p, int64_t upto, void* stream) {
    if (!p) return fail(IMM_EINVAL, "pool is NULL");
    if (upto < 0) return fail(IMM_EINVAL, "upto < 0");
    return pool_generate(p, upto, (hipStream_t)stream);
}

static imm_status check_range(const imm_pool* p, int64_t first, int64_t count) {
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

static imm_status range_hist(imm_pool* p, int64_t first, int64_t count, const uint32_t** out,
                             hipStream_t s) {
    if (first == 0 && count == p->count) {
        *out = p->hist;
        return IMM_OK;
    }
    if (!p->hist_tmp) IMM_TRY(dalloc(&p->hist_tmp, p->g->n));
    HIP_TRY(launch_fill_u32(p->hist_tmp, p->g->n, 0u, s));
    HIP_TRY(launch_hist_range(p->rr_start, p->rr_len, p->ids, first, count, p->hist_tmp, s));
    *out = p->hist_tmp;
    return IMM_OK;
}

extern "C" imm_status imm_rr_histogram(const imm_pool* pc, int64_t first, int64_t count,
                                       uint32_t* hist_out) {
    if (!pc || !hist_out) return fail(IMM_EINVAL, "NULL argument");
    imm_pool* p = const_cast<imm_pool*>(pc);
    IMM_TRY(check_range(p, first, count));
    const uint32_t* h = nullptr;
    IMM_TRY(range_hist(p, first, count, &h, nullptr));
    HIP_TRY(hipMemcpy(hist_out, h, sizeof(uint32_t) * (size_t)p->g->n, hipMemcpyDeviceToHost));
    return IMM_OK;
}

// ------------------------------------------------------------------------------------
// selection
// ------------------------------------------------------------------------------------
static imm_status ensure_select(imm_pool* p, int64_t count, int32_t k) {
    const int64_t n = p->g->n;
    if (!p->h) {
        IMM_TRY(dalloc(&p->h, n));
        IMM_TRY(dalloc(&p->inv_off, n + 1));
        IMM_TRY(dalloc(&p->scan_tmp, scan_tmp_elems(n)));
        IMM_TRY(dalloc(&p->cursor, n));
        IMM_TRY(dalloc(&p->n_covered, 1));
    }
    const int64_t members = (int64_t)sum64(p->host_ctr->placed);
    if (members > p->cap_inv) {
        dfree(p->inv);
        int64_t c = members + members / 4 + 1024;
        IMM_TRY(dalloc(&p->inv, c));
        p->cap_inv = c;
    }
    if (count > p->cap_cov) {
        dfree(p->covered);
        int64_t c = count + count / 4 + 1024;
        IMM_TRY(dalloc(&p->covered, c));
        p->cap_cov = c;
    }
    if (k > p->cap_k) {
        dfree(p->keys);
        dfree(p->seeds);
        if (p->host_seeds) (void)hipHostFree(p->host_seeds);
        p->host_seeds = nullptr;
        IMM_TRY(dalloc(&p->keys, k));
        IMM_TRY(dalloc(&p->seeds, k));
        HIP_TRY(hipHostMalloc((void**)&p->host_seeds, sizeof(int32_t) * (size_t)k, hipHostMallocDefault));
        p->cap_k = k;
    }
    return IMM_OK;
}

static imm_status pool_select(imm_pool* p, int64_t first, int64_t count, int32_t k,
                              int32_t* seeds_out, int64_t* covered_out, hipStream_t s) {
    const int32_t n = p->g->n;
    IMM_TRY(ensure_select(p, count, k));
    const uint32_t* hsrc = nullptr;
    IMM_TRY(range_hist(p, first, count, &hsrc, s));
    HIP_TRY(launch_copy_hist(hsrc, p->h, n, s));
    HIP_TRY(launch_scan_u32(hsrc, n, p->inv_off, p->scan_tmp, s));
    HIP_TRY(launch_fill_u32(p->cursor, n, 0u, s));
    HIP_TRY(launch_inv_scatter(p->rr_start, p->rr_len, p->ids, first, count, p->inv_off, p->cursor,
                               p->inv, s));
    HIP_TRY(launch_fill_u8(p->covered, count, (uint8_t)0, s));
    HIP_TRY(launch_fill_u64(p->keys, k, 0ull, s));
    HIP_TRY(launch_fill_u64(p->n_covered, 1, 0ull, s));
    for (int32_t round = 0; round < k; ++round) {
        HIP_TRY(launch_argmax(p->h, n, round, p->seeds, p->keys, s));
        HIP_TRY(launch_cover(p->keys, round, p->inv_off, p->inv, p->rr_start, p->rr_len, p->ids,
                             first, p->covered, p->h, p->seeds, p->n_covered, s));
    }
    HIP_TRY(hipMemcpyAsync(p->host_seeds, p->seeds, sizeof(int32_t) * (size_t)k, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(p->host_cov, p->n_covered, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (seeds_out) memcpy(seeds_out, p->host_seeds, sizeof(int32_t) * (size_t)k);
    if (covered_out) *covered_out = (int64_t)*p->host_cov;
    return IMM_OK;
}

extern "C" imm_status imm_select_seeds(imm_pool* p, int64_t first, int64_t count, int32_t k,
                                       int32_t* seeds_out, int64_t* covered_out, void* stream) {
    if (!p) return fail(IMM_EINVAL, "pool is NULL");
    IMM_TRY(check_range(p, first, count));
    if (k < 1 || k > p->g->n) return fail(IMM_EINVAL, "k = %d outside [1, n]", k);
    return pool_select(p, first, count, k, seeds_out, covered_out, (hipStream_t)stream);
}

// ------------------------------------------------------------------------------------
// IMM driver
// ------------------------------------------------------------------------------------
static imm_status run_imm(imm_pool* p, int32_t k, double eps, double ell, int32_t fresh,
                          hipStream_t s, int32_t* seeds_out, imm_info* info) {
    const int64_t n = p->g->n;
    if (k < 1 || k > n) return fail(IMM_EINVAL, "k = %d outside [1, n]", k);
    if (!(eps > 0.0 && eps < 1.0)) return fail(IMM_EINVAL, "eps = %g outside (0, 1)", eps);
    if (!(ell > 0.0)) return fail(IMM_EINVAL, "ell = %g must be > 0", ell);
    if (!seeds_out) return fail(IMM_EINVAL, "seeds_out is NULL");
    const double t0 = now_s();
    double t_gen = 0.0, t_sel = 0.0;
    const double kernel_s0 = p->kernel_s, heavy_s0 = p->heavy_s;
    const int64_t launches0 = p->kernel_launches, heavy0 = p->heavy_launches;
    const double lp = ell_prime(n, ell);
    const double ep = std::sqrt(2.0) * eps;
    const double lam1 = lambda_prime(n, k, eps, lp);
    const double lam2 = lambda_star(n, k, eps, lp);
    const int32_t rounds = estimation_rounds(n);
    double lb = 1.0;
    int64_t used = 0, cov = 0;
    int32_t phases = 0;
    for (int32_t i = 1; i <= rounds; ++i) {
        const double x = (double)n / (double)((int64_t)1 << i);
        const double want = std::ceil(lam1 / x);
        if (want > (double)kMaxSets) return fail(IMM_ECAPACITY, "theta_%d = %g too large", i, want);
        const int64_t th = (int64_t)want;
        if (th > used) used = th;
        double ta = now_s();
        IMM_TRY(pool_generate(p, used, s));
        double tb = now_s();
        IMM_TRY(pool_select(p, 0, used, k, seeds_out, &cov, s));
        t_gen += tb - ta;
        t_sel += now_s() - tb;
        ++phases;
        if ((double)n * (double)cov / (double)used >= (1.0 + ep) * x) {
            lb = (double)n * (double)cov / (double)used / (1.0 + ep);
            break;
        }
    }
    const double want = std::ceil(lam2 / lb);
    if (want > (double)kMaxSets) return fail(IMM_ECAPACITY, "theta = %g too large", want);
    const int64_t theta = (int64_t)want;
    const int64_t first = fresh ? used : 0;
    const int64_t upto = fresh ? used + theta : (theta > used ? theta : used);
    if (upto > kMaxSets) return fail(IMM_ECAPACITY, "sample end %lld too large", (long long)upto);
    double ta = now_s();
    IMM_TRY(pool_generate(p, upto, s));
    double tb = now_s();
    IMM_TRY(pool_select(p, first, upto - first, k, seeds_out, &cov, s));
    t_gen += tb - ta;
    t_sel += now_s() - tb;
    ++phases;
    if (info) {
        memset(info, 0, sizeof *info);
        info->theta = theta;
        info->num_rr = upto;
        info->covered = cov;
        info->edges_examined = (int64_t)(sum64(p->host_ctr->edges) + sum64(p->host_ctr->hedges));
        info->edges_heavy = (int64_t)sum64(p->host_ctr->hedges);
        info->pool_ids = (int64_t)sum64(p->host_ctr->placed);
        info->phases = phases;
        info->lb = lb;
        info->spread_est = (double)n * (double)cov / (double)(upto - first);
        info->lambda_prime = lam1;
        info->lambda_star = lam2;
        info->t_generate_s = t_gen;
        info->t_select_s = t_sel;
        info->t_total_s = now_s() - t0;
        info->t_rr_kernel_s = p->kernel_s - kernel_s0;
        info->rr_kernel_launches = p->kernel_launches - launches0;
        info->t_rr_heavy_s = p->heavy_s - heavy_s0;
        info->rr_heavy_launches = p->heavy_launches - heavy0;
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
