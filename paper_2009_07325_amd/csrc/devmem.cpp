// Device memory of libimm: a caching allocator over hipMalloc.
//
// An IMM solve allocates its RR pool, generation scratch (visited bitmaps and member lists
// of the concurrent sets, up to ~16 GiB on large graphs) and selection workspace, and
// frees them at the end; repeated solves, batches and served queries would otherwise pay
// hipMalloc/hipFree (page mapping, implicit device synchronisation) every time.  Freed
// blocks are kept per device and handed out again to requests of between half and all of
// their size.  The cache holds at most kCacheBytes per device (least recently freed blocks
// go first) and is emptied when hipMalloc fails or on imm_release_cached_memory().
//
// Blocks are only returned to the cache after the work that used them has completed
// (every library call synchronises its stream before it frees), so a cached block is
// never in use on the device.  Contents are not preserved: users clear what they need.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <list>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "host.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kCacheBytes = (size_t)64 << 30;

struct Block {
    int device;
    size_t bytes;
    void* ptr;
};

struct Cache {
    std::mutex mu;
    std::unordered_map<void*, Block> live;   // handed out
    std::list<Block> free;                   // most recently freed first
    size_t free_bytes[64] = {};              // per device
};

Cache& cache() {
    static Cache* c = new Cache();   // never destroyed: frees at exit are skipped
    return *c;
}

void drop_free(Cache& c, int device) {
    for (auto it = c.free.begin(); it != c.free.end();) {
        if (device < 0 || it->device == device) {
            (void)hipFree(it->ptr);
            c.free_bytes[it->device & 63] -= it->bytes;
            it = c.free.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace

namespace imm {

namespace {
thread_local bool t_no_alloc = false;
}  // namespace

void set_no_alloc(bool on) { t_no_alloc = on; }
bool no_alloc_active() { return t_no_alloc; }

hipError_t dev_alloc(void** out, size_t bytes) {
    *out = nullptr;
    if (t_no_alloc) return hipErrorOutOfMemory;
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return e;
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    if (bytes == 0) bytes = kAlign;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    // best fit among the cached blocks of this device that are at most twice the request
    auto best = c.free.end();
    for (auto it = c.free.begin(); it != c.free.end(); ++it) {
        if (it->device != device || it->bytes < bytes || it->bytes > 2 * bytes) continue;
        if (best == c.free.end() || it->bytes < best->bytes) best = it;
    }
    if (best != c.free.end()) {
        Block b = *best;
        c.free.erase(best);
        c.free_bytes[device & 63] -= b.bytes;
        c.live[b.ptr] = b;
        *out = b.ptr;
        return hipSuccess;
    }
    void* p = nullptr;
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        drop_free(c, device);      // give the cached memory back and retry once
        e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
    }
    c.live[p] = Block{device, bytes, p};
    *out = p;
    return hipSuccess;
}

// IMM_DEVICE_CACHE=0 turns the cache off (every free goes straight to hipFree).
bool cache_enabled() {
    static const bool on = [] {
        const char* e = getenv("IMM_DEVICE_CACHE");
        return !(e && e[0] == '0');
    }();
    return on;
}

void dev_free(void* p) {
    if (!p) return;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end() || !cache_enabled()) {
        if (it != c.live.end()) c.live.erase(it);
        (void)hipFree(p);
        return;
    }
    const Block b = it->second;
    c.live.erase(it);
    const int d = b.device & 63;
    c.free.push_front(b);
    c.free_bytes[d] += b.bytes;
    // keep the cache bounded: drop the least recently freed blocks of this device
    for (auto r = c.free.end(); c.free_bytes[d] > kCacheBytes && r != c.free.begin();) {
        --r;
        if ((r->device & 63) != d) continue;
        (void)hipFree(r->ptr);
        c.free_bytes[d] -= r->bytes;
        r = c.free.erase(r);
    }
}

// Pinned host buffers of up to 1 MiB are kept in power-of-two classes (256 B and up) once
// freed, and handed out again; larger ones are allocated and freed directly.  Like device
// blocks, a buffer is freed only after the copies into it have completed.
namespace {

constexpr int kHostMinClass = 8, kHostMaxClass = 20;

struct HostCache {
    std::mutex mu;
    std::unordered_map<void*, int> live;     // handed out: class, or -1 (not cached)
    std::vector<void*> free[kHostMaxClass + 1];
};

HostCache& host_cache() {
    static HostCache* c = new HostCache();   // never destroyed, like the device cache
    return *c;
}

void drop_host_free(HostCache& c) {
    for (std::vector<void*>& v : c.free) {
        for (void* p : v) (void)hipHostFree(p);
        v.clear();
    }
}

}  // namespace

hipError_t host_alloc(void** out, size_t bytes) {
    *out = nullptr;
    if (t_no_alloc) return hipErrorOutOfMemory;
    int cls = kHostMinClass;
    while (cls <= kHostMaxClass && ((size_t)1 << cls) < bytes) ++cls;
    HostCache& c = host_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (cls <= kHostMaxClass && !c.free[cls].empty()) {
        *out = c.free[cls].back();
        c.free[cls].pop_back();
        c.live[*out] = cls;
        return hipSuccess;
    }
    const size_t size = cls <= kHostMaxClass ? (size_t)1 << cls : bytes;
    void* p = nullptr;
    hipError_t e = hipHostMalloc(&p, size, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        drop_host_free(c);
        e = hipHostMalloc(&p, size, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
    }
    c.live[p] = cls <= kHostMaxClass ? cls : -1;
    *out = p;
    return hipSuccess;
}

void host_free(void* p) {
    if (!p) return;
    HostCache& c = host_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    const int cls = it == c.live.end() ? -1 : it->second;
    if (it != c.live.end()) c.live.erase(it);
    if (cls < 0 || !cache_enabled()) {
        (void)hipHostFree(p);
        return;
    }
    c.free[cls].push_back(p);
}

size_t dev_cached_bytes() {
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    size_t t = 0;
    for (const Block& b : c.free) t += b.bytes;
    return t;
}

}  // namespace imm

extern "C" imm_status imm_release_cached_memory(void) {
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    drop_free(c, -1);
    imm::HostCache& h = imm::host_cache();
    std::lock_guard<std::mutex> hk(h.mu);
    imm::drop_host_free(h);
    return IMM_OK;
}
