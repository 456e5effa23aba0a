// Internal host-side declarations of libimm (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/imm.h"
#include "kernels.hpp"

namespace imm {

// ---- errors and device memory ---------------------------------------------------------
imm_status fail(imm_status st, const char* fmt, ...);

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::imm::fail(e_ == hipErrorOutOfMemory ? IMM_ENOMEM : IMM_EDEVICE,      \
                               "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,  \
                               __LINE__);                                                 \
    } while (0)

#define IMM_TRY(expr)                  \
    do {                               \
        imm_status s_ = (expr);        \
        if (s_ != IMM_OK) return s_;   \
    } while (0)

constexpr int64_t kMaxSets = (int64_t)INT32_MAX;   // RR index and counters fit int32

// Device memory goes through a caching allocator (devmem.cpp): blocks freed after their
// work completed are reused by later requests of similar size.
hipError_t dev_alloc(void** out, size_t bytes);
void dev_free(void* p);
size_t dev_cached_bytes();

// No-allocation calls (imm_select_seeds_noalloc) set a thread-local flag for their
// duration; every allocation attempted meanwhile fails with an error instead.
void set_no_alloc(bool on);
bool no_alloc_active();
imm_status noalloc_setup(int device);

template <typename T>
imm_status dalloc(T** p, int64_t count) {
    *p = nullptr;
    if (no_alloc_active()) return fail(IMM_ENOMEM, "device allocation inside a no-allocation call");
    if (count <= 0) count = 1;
    void* q = nullptr;
    hipError_t e = dev_alloc(&q, sizeof(T) * (size_t)count);
    if (e != hipSuccess)
        return fail(IMM_ENOMEM, "device allocation of %lld bytes failed: %s",
                    (long long)(sizeof(T) * count), hipGetErrorString(e));
    *p = static_cast<T*>(q);
    return IMM_OK;
}

template <typename T>
void dfree(T*& p) {
    dev_free((void*)p);
    p = nullptr;
}

// Small pinned host buffers (read-back of counters, coverage and seeds, launch tables) go
// through a cache of their own: hipHostMalloc / hipHostFree cost tens of microseconds each.
hipError_t host_alloc(void** out, size_t bytes);
void host_free(void* p);

template <typename T>
imm_status halloc(T** p, int64_t count) {
    *p = nullptr;
    if (no_alloc_active()) return fail(IMM_ENOMEM, "pinned host allocation inside a no-allocation call");
    if (count <= 0) count = 1;
    void* q = nullptr;
    hipError_t e = host_alloc(&q, sizeof(T) * (size_t)count);
    if (e != hipSuccess)
        return fail(IMM_ENOMEM, "pinned host allocation of %lld bytes failed: %s",
                    (long long)(sizeof(T) * count), hipGetErrorString(e));
    *p = static_cast<T*>(q);
    return IMM_OK;
}

template <typename T>
void hfree(T*& p) {
    host_free((void*)p);
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
            dfree(q);
            return fail(IMM_EDEVICE, "grow copy failed: %s", hipGetErrorString(e));
        }
    }
    dfree(*p);
    *p = q;
    *cap = nc;
    return IMM_OK;
}

double now_s();

inline unsigned long long sum64(const unsigned long long* v) {
    unsigned long long t = 0;
    for (int i = 0; i < 64; ++i) t += v[i];
    return t;
}

// ---- IMM sample sizes and the LB / theta state machine --------------------------------
double log_binom(int64_t n, int64_t k);
double ell_prime(int64_t n, double ell);
// `rounds` > 1: the multi-round problem (gIM Sec. IV-H), whose union bound runs over
// C(n,k)^rounds seed collections and whose greedy (a partition matroid) guarantees 1/2.
double lambda_prime(int64_t n, int64_t k, double eps, double lp, int32_t rounds = 1);
double lambda_star(int64_t n, int64_t k, double eps, double lp, int32_t rounds = 1);
int32_t estimation_rounds(int64_t n);

// One IMM solve as a sequence of selections (gIM Alg. 2, then Alg. 1).  next() names the
// RR range of the next selection and how far the pool must extend; complete() takes the
// covered count of that selection.  Every solve path (plain, served, batched) drives
// this one object, so they all compute the same doubles in the same order.
struct ImmPlan {
    int64_t n = 0;
    int32_t k = 0;                 // seeds per round
    int32_t mr = 1;                // rounds of a multi-round solve (selections take mr * k)
    double eps = 0, ell = 0;
    int32_t fresh = 0;
    double lp = 0, ep = 0, lam1 = 0, lam2 = 0;
    int32_t rounds = 0;
    // progress
    int32_t i = 1;
    int64_t used = 0;
    double x = 0.0;
    double lb = 1.0;
    bool final_phase = false, done = false;
    int64_t theta = 0, first = 0, upto = 0;
    int32_t phases = 0;
    int64_t covered = 0;
    // The final selection would run on exactly the sets of the estimation phase that passed
    // (no fresh sample and theta within the sets already drawn): greedy is deterministic,
    // so that phase's seeds and coverage are the final ones and no selection is run.
    bool reuse = false;

    imm_status init(int64_t n_, int32_t k_, double eps_, double ell_, int32_t fresh_,
                    int32_t mr_ = 1);
    imm_status next(int64_t* gen_upto, int64_t* sel_first, int64_t* sel_count);
    imm_status complete(int64_t cov);
    // Smallest coverage of the current estimation phase's selection that passes its test
    // (used + 1 when none does); 0 in the final phase.
    int64_t need_cov() const;
    bool reuses_last() const { return final_phase && reuse; }
    double spread_est() const { return (double)n * (double)covered / (double)(upto - first); }

  private:
    imm_status enter_final();
};

}  // namespace imm

// ---- library objects -------------------------------------------------------------------
namespace imm {
// Generation launch configuration chosen by imm_autotune for one model of a graph (zero:
// not tuned, library defaults).
struct GenTuning {
    int64_t budget = 0;
    int heavy_block = 0;
    int light_cap = 0;      // IC: on-chip members of a light set (frontier capacity)
    int lt_cap = 0;         // LT: on-chip members of a first-pass walk
    int fetch = 0;          // RR indices per work-counter fetch (queue depth)
};
}  // namespace imm

struct imm_graph {
    imm::GenTuning tuned[2];     // per model
    int device = 0;
    int32_t n = 0;
    int64_t m = 0;
    imm::VRec* vrec = nullptr;
    int32_t* src = nullptr;
    uint32_t* thr = nullptr;     // IC thresholds (padded to a multiple of 4 edges)
    uint32_t* cum = nullptr;     // LT cumulative thresholds
    imm::LtRec* lrec = nullptr;  // LT walk tables: edge records (m), guide records (2m
    imm::LtRec* grec = nullptr;  // pairs: the guide edge's record, then its successor's)
    uint32_t* gidx = nullptr;    // ... and guide positions (2m)
    bool has_ic = false, has_lt = false;
    bool ic_uniform = false;     // every vertex has one common IC threshold
    int cus = 0;
    // out-edge lists, built on first use by the forward spread simulations
    int64_t* out_off = nullptr;  // n + 1
    int32_t* out_dst = nullptr;  // m
    uint32_t* out_eid = nullptr; // m: in-edge index
};

namespace imm {

// Selection workspace: one per concurrent selection (a pool has one; a server has one per
// active query).
struct SelectWs {
    // One segment of the inverted index: the sets of one range, vertex-major.
    struct IndexSeg {
        int64_t* off = nullptr;               // n + 1
        uint32_t* inv = nullptr;              // relative set indices
        int64_t cap = 0;
    };
    int64_t n = 0;
    int32_t* h = nullptr;
    uint32_t* hist_tmp = nullptr;
    int64_t* scan_tmp = nullptr;
    uint32_t* cursor = nullptr;
    // The index covers sets [ix_first, ix_end) of pool ix_pool in nseg segments.  When the
    // next selection reads a longer prefix of the same pool, only the new sets are indexed
    // (their counts are the pool histogram minus snap, the histogram at ix_end).
    IndexSeg seg[kMaxSegs];
    int32_t nseg = 0;
    const imm_pool* ix_pool = nullptr;
    int64_t ix_first = 0, ix_end = 0;
    int64_t ix_members = 0;                   // pool members in [0, ix_end) (prefix index)
    uint32_t* snap = nullptr;
    bool snap_valid = false;
    int64_t cap_cov = 0;
    uint32_t* covered = nullptr;
    int32_t* taken = nullptr;                 // kMaxRounds partition counts
    int64_t cap_k = 0;
    unsigned long long* keys = nullptr;
    int32_t* seeds = nullptr;
    unsigned long long* n_covered = nullptr;
    int32_t* host_seeds = nullptr;            // pinned, cap_k
    unsigned long long* host_keys = nullptr;  // pinned, cap_k: each round's argmax key
                                              // (gain + 1 in the high word; 0: not run)
    unsigned long long* host_cov = nullptr;   // pinned
    int32_t k = 0;                            // of the prepared selection
    // hot set of single-instance selections (select.hip)
    unsigned long long* bcur = nullptr;       // kInvBuckets: bucketed index build cursors
    uint2* pairs = nullptr;                   // pair_cap: (entry, vertex) of the bucketed build
    int64_t pair_cap = 0;
    unsigned long long* hot_words = nullptr;  // (n + 31) / 32: hot bitmap | hot position << 32
    uint32_t* hot_blk = nullptr;              // hot_list_blocks(n) counts
    uint32_t* cnt_hist = nullptr;             // kSelectHotBuckets
    uint32_t* hot_n = nullptr;
    int32_t* hot_ids = nullptr;               // hot_cap
    int64_t hot_cap = 0;
    int32_t* hot_part = nullptr;              // part_cap: per-block decrement rows of dense rounds
    int64_t part_cap = 0;

    int64_t bytes() const;
    void release();
};

// Device descriptors + barrier of one cooperative selection launch (any number of
// instances up to the kernel's limit).
struct SelectLaunch {
    int64_t cap = 0;
    SelInst* d_inst = nullptr;
    GridBarrier* bar = nullptr;
    GridBarrier* host_bar = nullptr;          // pinned
    SelInst* host_inst = nullptr;             // pinned staging of the descriptors, or null
    void release();
};

// Launch state and scratch of RR-generation launches of one model over one or more pools
// (a plain pool owns one; a batch shares one across its instances).
struct GenCtx {
    int device = 0;
    imm_model model = IMM_IC;
    int cus = 0;
    int grid = 0;                       // light launch: blocks of 256 threads
    int64_t vis_n = 0;                  // vertices the bitmaps cover (largest graph seen)
    int64_t vis_words = 0;
    uint32_t* visited = nullptr;        // grid * 4 light bitmaps
    int64_t hslots = 0;                 // heavy slots (IC: workgroups, LT: waves)
    uint32_t* hvisited = nullptr;       // hslots bitmaps
    int32_t* hlist = nullptr;           // member lists: LT hslots x vis_n entries; IC
    int64_t hlist_words = 0;            // hlist_words entries shared by a launch's slots
    unsigned long long* over = nullptr; // IC heavy sets that outgrew their list (cap_queue)
    int64_t budget = 4096;              // light-wave group budget per set
    int heavy_block = 256;              // threads per heavy set (64, 128, 256 or 1024)
    int64_t heavy_scratch = (int64_t)16 << 30;   // bytes of heavy bitmaps + lists at most
    int64_t heavy_list = 0;             // IC heavy list entries per slot (0: chosen per launch)
    int32_t* lt_ext = nullptr;          // LT first pass: extension lists of the grid's walk slots
    int64_t lt_ext_words = 0;
    int lt_lds_cap = kLtLdsCap;         // members a first-pass walk keeps in LDS / extension
    int lt_ext_cap = kLtExtCap;
    int light_cap = 1024;               // IC light set's on-chip list (frontier capacity)
    int fetch = kGenFetch;              // RR indices per work fetch (queue depth)

    LaunchCounters* lc = nullptr;
    LaunchCounters* host_lc = nullptr;  // pinned
    int64_t cap_queue = 0;
    unsigned long long* queue = nullptr;  // light -> heavy queue
    uint32_t* handoff = nullptr;          // per queue entry (IC)
    int32_t* arena = nullptr;             // handed-off traversals (IC), kArenaWords
    int64_t cap_inst = 0;
    GenInst* d_inst = nullptr;
    GenInst* host_inst = nullptr;       // pinned
    int64_t* d_work_off = nullptr;
    int64_t* host_work_off = nullptr;   // pinned
    PoolSummary* d_sum = nullptr;
    PoolSummary* host_sum = nullptr;    // pinned

    // HIP events bracketing the light and heavy launches
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
    double kernel_s = 0.0;              // light kernel (IC) / walk kernel (LT)
    int64_t kernel_launches = 0;
    double heavy_s = 0.0;               // heavy kernel (IC) / HBM-list walk kernel (LT)
    int64_t heavy_launches = 0;
    int64_t heavy_overflow = 0;         // IC heavy sets drawn again in full lists

    // Defaults, then `tuning` (if given and set), then the IMM_LIGHT_BUDGET /
    // IMM_HEAVY_BLOCK / IMM_LIGHT_CAP / IMM_FETCH / IMM_HEAVY_SCRATCH_GIB / IMM_HEAVY_LIST /
    // IMM_LT_LDS_CAP / IMM_LT_EXT_CAP environment overrides.
    imm_status init(int device_, imm_model model_, int cus_, const GenTuning* tuning = nullptr);
    imm_status ready();
    int64_t bytes() const;
    // Device bytes of the heavy scratch that the first IC heavy launch on graphs of up to n
    // vertices allocates (0 once allocated, and for LT).
    int64_t heavy_bytes(int64_t n) const;
    void release();
};

}  // namespace imm

struct imm_pool {
    const imm_graph* g = nullptr;
    imm_model model = IMM_IC;
    uint64_t seed = 0;
    int64_t count = 0;
    uint32_t round = 0;                 // third counter word of this pool's edge draws

    // Multi-round pool (rounds > 1, gIM Sec. IV-H): set r is the union over t of round
    // pool sub[t]'s set r as elements t * n_base + u.  Generation extends the round pools
    // and lays their sets side by side in this pool's own arrays (contiguous, index
    // order); g is then `view`, a graph record with n = rounds * n_base and no arrays, so
    // histogram, index and selection run over the element space unchanged.
    int32_t rounds = 1;
    int32_t n_base = 0;
    imm_pool* sub[imm::kMaxRounds] = {};
    imm_graph* view = nullptr;

    int64_t cap_sets = 0;
    int64_t* rr_start = nullptr;
    int32_t* rr_len = nullptr;
    int64_t cap_ids = 0;
    int32_t* ids = nullptr;
    uint32_t* hist = nullptr;
    imm::PoolCounters* ctr = nullptr;
    imm::PoolSummary sum{};              // host copy, current after every generation call

    int64_t cap_lists = 0;
    uint32_t* cap_list = nullptr;       // id-buffer capacity misses
    uint32_t* retry_list = nullptr;

    imm::GenCtx gen;                    // generation scratch of this pool's own calls
    imm::SelectWs sel;                  // selection workspace of imm_select_seeds / solve
    imm::SelectLaunch launch;

    int64_t bytes() const;               // device memory held
};

namespace imm {

// Extends each pools[i] to upto[i] sets (no-op where it already holds that many) with
// shared light / heavy launches.  All pools must have the context's model.
imm_status gen_run(GenCtx* c, imm_pool* const* pools, const int64_t* upto, int32_t count,
                   hipStream_t s);
imm_status pool_generate(imm_pool* p, int64_t upto, hipStream_t s);
// Device arrays and generation context of a new pool (p->g, model, seed set).
imm_status pool_init(imm_pool* p);
// One IMM solve on pool p (CR-NAIMM on a multi-round pool): gIM Alg. 2 then Alg. 1.
// seeds_out holds p->rounds * k entries.
imm_status run_imm(imm_pool* p, int32_t k, double eps, double ell, int32_t fresh, hipStream_t s,
                   int32_t* seeds_out, imm_info* info);
// Multi-round pools: lays out sets [p->count, upto) from the round pools (mrim.cpp).
imm_status mr_merge(imm_pool* p, int64_t upto, hipStream_t s);
// Vertices of the graph a pool draws from (the part size of a multi-round pool).
inline int64_t pool_vertices(const imm_pool* p) { return p->rounds > 1 ? p->n_base : p->g->n; }
imm_status check_range(const imm_pool* p, int64_t first, int64_t count);

// Launches the per-selection setup kernels (counts, inverted index, clears) on `s` and
// fills `out` with the instance descriptor.
// segments: the index may be kept as segments across calls (single-instance launches only)
// hot: the selection runs alone in its launch and may keep a hot set (select.hip)
imm_status select_prepare(imm_pool* p, SelectWs* w, int64_t first, int64_t count, int32_t k,
                          hipStream_t s, SelInst* out, bool segments = false, bool hot = false);
// Hot-set size of a single-instance selection over n counters (0: off).  16384 by default
// (IMM_SELECT_HOT overrides; 0 turns it off), used only when n exceeds twice that (or the
// override), and at most kSelectHotPerBlock per block of the launch.
int32_t select_hot_max(int64_t n);
int32_t select_dense_gain();
// Runs all rounds of every prepared instance in one cooperative launch, then copies each
// instance's seeds and covered count to its workspace's pinned buffers (synchronises s).
imm_status select_run(SelectLaunch* L, SelectWs* const* ws, const SelInst* inst, int32_t ninst,
                      hipStream_t s);
// select_run in two halves: enqueue (descriptors, barrier reset, launch, read-backs; no
// synchronisation, so it may be captured into a graph: captured launches use an ordinary
// launch of the same grid) and wait (synchronises s, reports a barrier timeout).
imm_status select_enqueue(SelectLaunch* L, SelectWs* const* ws, const SelInst* inst, int32_t ninst,
                          hipStream_t s, bool captured = false);
imm_status select_wait(SelectLaunch* L, hipStream_t s);

}  // namespace imm
