// Greedy max coverage without allocation: imm_select_seeds_noalloc.
//
// The same selection as imm_select_seeds (gIM Alg. 1 greedy, Alg. 7 on the device), for
// callers that may not allocate (code under stream capture, tight serving loops, harnesses
// that forbid hipMalloc).  Its workspace -- counters, inverted index, covered flags,
// argmax keys, seeds, launch descriptor and grid barrier -- is carved out of one
// file-scope device array of kNoAllocScratchBytes per device, whose address is taken once
// per device with hipGetSymbolAddress (the array's name in host code is only a host-side
// stand-in).  While the call runs, any allocation the selection path would make is
// refused (thread-local guard in dalloc / halloc) and reported as an error, so the
// promise is checked rather than assumed.
//
// Every call on a device shares that device's array and leaves its contents behind; every
// region the selection reads is cleared or written by the call before use.  Calls that
// overlap on one device (other threads, other streams) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.hpp"

using namespace imm;

static __device__ __align__(256) unsigned char scratch[IMM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int64_t kNoAllocScratchBytes = IMM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device, with the
// device current).
imm_status scratch_ptr(int device, unsigned char** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return fail(IMM_EDEVICE, "device %d", device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(IMM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_ptr[device] = static_cast<unsigned char*>(p);
    }
    *out = g_ptr[device];
    return IMM_OK;
}

// Lays regions out at 256-byte boundaries; `base` null only measures.
struct Carver {
    unsigned char* base;
    int64_t used = 0;
    template <typename T>
    T* take(int64_t count) {
        if (count < 1) count = 1;
        used = (used + 255) / 256 * 256;
        T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
        used += (int64_t)sizeof(T) * count;
        return p;
    }
};

struct NoAllocGuard {
    NoAllocGuard() { set_no_alloc(true); }
    ~NoAllocGuard() { set_no_alloc(false); }
};

// The workspace of one selection of k per part over sets [first, first + count) of p.
int64_t carve(unsigned char* base, const imm_pool* p, int64_t count, int32_t k_total, bool prefix,
              SelectWs* w, SelectLaunch* L) {
    const int64_t n = p->g->n;
    const int64_t members = (int64_t)p->sum.placed;       // bounds the range's entries
    Carver c{base};
    w->n = n;
    w->h = c.take<int32_t>(n);
    w->hist_tmp = prefix ? nullptr : c.take<uint32_t>(n);
    w->scan_tmp = c.take<int64_t>(scan_tmp_elems(n));
    w->cursor = c.take<uint32_t>(n);
    w->n_covered = c.take<unsigned long long>(1);
    w->taken = c.take<int32_t>(kMaxRounds);
    w->covered = c.take<uint32_t>(count);
    w->cap_cov = count;
    w->keys = c.take<unsigned long long>(k_total);
    w->seeds = c.take<int32_t>(k_total);
    w->cap_k = k_total;
    w->seg[0].off = c.take<int64_t>(n + 1);
    w->seg[0].inv = c.take<uint32_t>(members);
    w->seg[0].cap = members;
    const int32_t hot_max = select_hot_max(n);
    w->hot_words = c.take<unsigned long long>((n + 31) / 32);
    w->hot_blk = c.take<uint32_t>(hot_list_blocks(n));
    w->cnt_hist = c.take<uint32_t>(kSelectHotBuckets);
    w->hot_n = c.take<uint32_t>(2);
    w->hot_ids = c.take<int32_t>(hot_max);
    w->hot_cap = hot_max;
    L->d_inst = c.take<SelInst>(1);
    L->bar = c.take<GridBarrier>(1);
    L->cap = 1;
    return c.used;
}

}  // namespace

namespace imm {
// Called by imm_init for the device it selects.
imm_status noalloc_setup(int device) {
    unsigned char* p = nullptr;
    return scratch_ptr(device, &p);
}
}  // namespace imm

extern "C" int64_t imm_select_noalloc_bytes(const imm_pool* p, int64_t first, int64_t count,
                                            int32_t k) {
    if (!p || count < 0) return -1;
    SelectWs w;
    SelectLaunch L;
    const bool prefix = first == 0 && count == p->count;
    return carve(nullptr, p, count, k * p->rounds, prefix, &w, &L);
}

extern "C" imm_status imm_select_seeds_noalloc(const imm_pool* pc, int64_t first, int64_t count,
                                               int32_t k, int32_t* seeds_out, int64_t* covered_out,
                                               void* stream) {
    if (!pc) return fail(IMM_EINVAL, "pool is NULL");
    if (!seeds_out) return fail(IMM_EINVAL, "seeds_out is NULL");
    imm_pool* p = const_cast<imm_pool*>(pc);
    IMM_TRY(check_range(p, first, count));
    if (k < 1 || k > pool_vertices(p)) return fail(IMM_EINVAL, "k = %d outside [1, n]", k);
    const int32_t k_total = k * p->rounds;
    const bool prefix = first == 0 && count == p->count;
    SelectWs w;
    SelectLaunch L;
    const int64_t need = carve(nullptr, p, count, k_total, prefix, &w, &L);
    if (need > kNoAllocScratchBytes)
        return fail(IMM_ECAPACITY,
                    "selection needs %lld bytes of workspace; the no-allocation scratch holds %lld",
                    (long long)need, (long long)kNoAllocScratchBytes);
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    unsigned char* base = nullptr;
    IMM_TRY(scratch_ptr(device, &base));
    w = SelectWs();
    L = SelectLaunch();
    carve(base, p, count, k_total, prefix, &w, &L);
    // read-back targets: the caller's seeds and stack variables (pageable host memory)
    unsigned long long cov = 0;
    GridBarrier bar_host{};
    w.host_seeds = seeds_out;
    w.host_cov = &cov;
    L.host_bar = &bar_host;

    const hipStream_t s = (hipStream_t)stream;
    imm_status st;
    {
        NoAllocGuard guard;
        SelInst si;
        st = select_prepare(p, &w, first, count, k, s, &si, false, true);
        if (st == IMM_OK) {
            SelectWs* wp = &w;
            st = select_run(&L, &wp, &si, 1, s);
        }
    }
    if (st != IMM_OK) {
        (void)hipStreamSynchronize(s);     // nothing of this call may still run on the array
        return st;
    }
    if (covered_out) *covered_out = (int64_t)cov;
    return IMM_OK;
}
