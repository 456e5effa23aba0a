// Greedy maximum coverage on the device (gIM Alg. 1 lines 6-10, Sec. III-H, Alg. 7).
//
// Per selection call over RR sets [first, first+count):
//   1. h[v]   = number of those sets containing v (Occur, gIM Sec. III-B), as int32;
//   2. an inverted index vertex -> RR indices (counting sort: scan of h, then the entries
//      grouped by buckets of vertices and placed bucket by bucket);
//   3. k rounds of
//        argmax  : u = the vertex outside S with the largest h, smallest id among equals
//                  (gIM Sec. III-H: a max reduction over Occur);
//        cover   : every set containing u that is not yet covered is flagged and each of
//                  its members' counters is decremented (gIM Alg. 7), using the inverted
//                  index so that a round touches only the sets that contain u.
// Integer decrements commute, so counters, seeds and the covered count are the same for
// any schedule.
#include <cstdlib>
#include <cstring>

#include "kernels.hpp"

namespace imm {

// ---- fills --------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
static hipError_t fill(T* p, int64_t n, T v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_fill<T><<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s) { return fill(p, n, v, s); }
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) { return fill(p, n, v, s); }
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
    return fill(p, n, v, s);
}

// ---- occurrence counts over a range of sets (one wave per set) ----------------------
__global__ void k_hist_range(const int64_t* __restrict__ rr_start, const int32_t* __restrict__ rr_len,
                             const int32_t* __restrict__ ids, int64_t first, int64_t count,
                             uint32_t* __restrict__ hist) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t i = wave; i < count; i += nwaves) {
        const int64_t s = rr_start[first + i];
        const int32_t len = rr_len[first + i];
        for (int32_t j = lane; j < len; j += kWave)
            __hip_atomic_fetch_add(hist + ids[s + j], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t launch_hist_range(const int64_t* rr_start, const int32_t* rr_len, const int32_t* ids,
                             int64_t first, int64_t count, uint32_t* hist, hipStream_t s) {
    if (count == 0) return hipSuccess;
    int64_t blocks = (count * kWave + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_hist_range<<<(unsigned)blocks, 256, 0, s>>>(rr_start, rr_len, ids, first, count, hist);
    return hipGetLastError();
}

// ---- exclusive scan into int64 (three passes: tile sums, scan of sums, tile scans) --
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanTile = kScanBlock * kScanItems;

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t& total) {
    // sh: kScanBlock / kWave + 1 entries
    const int lane = lane_id();
    const int wid = threadIdx.x / kWave;
    int64_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) sh[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int w = 0; w < kScanBlock / kWave; ++w) {
            int64_t t = sh[w];
            sh[w] = acc;
            acc += t;
        }
        sh[kScanBlock / kWave] = acc;
    }
    __syncthreads();
    total = sh[kScanBlock / kWave];
    int64_t res = incl - v + sh[wid];
    __syncthreads();
    return res;
}

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const T* __restrict__ in, int64_t n,
                                                           int64_t* __restrict__ tile_sum) {
    __shared__ int64_t sh[kScanBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) acc += (int64_t)in[base + i];
    int64_t total;
    block_excl_scan(acc, sh, total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int64_t* __restrict__ tile_sum, int64_t tiles) {
    __shared__ int64_t sh[kScanBlock / kWave + 1];
    int64_t carry = 0;
    for (int64_t b = 0; b < tiles; b += kScanBlock) {
        const int64_t i = b + threadIdx.x;
        const int64_t v = i < tiles ? tile_sum[i] : 0;
        int64_t total;
        const int64_t ex = block_excl_scan(v, sh, total);
        if (i < tiles) tile_sum[i] = ex + carry;
        carry += total;
    }
    if (threadIdx.x == 0) tile_sum[tiles] = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const T* __restrict__ in, int64_t n,
                                                           const int64_t* __restrict__ tile_sum,
                                                           int64_t* __restrict__ out) {
    __shared__ int64_t sh[kScanBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t vals[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        vals[i] = base + i < n ? (int64_t)in[base + i] : 0;
        acc += vals[i];
    }
    int64_t total;
    int64_t run = block_excl_scan(acc, sh, total) + tile_sum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += vals[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tile_sum[gridDim.x];
}

template <typename T>
static hipError_t scan(const T* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
    if (n == 0) {
        return fill(reinterpret_cast<unsigned long long*>(out), 1, 0ull, s);
    }
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    k_scan_tiles<T><<<(unsigned)tiles, kScanBlock, 0, s>>>(in, n, tmp);
    k_scan_sums<<<1, kScanBlock, 0, s>>>(tmp, tiles);
    k_scan_apply<T><<<(unsigned)tiles, kScanBlock, 0, s>>>(in, n, tmp, out);
    return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
    return scan(in, n, out, tmp, s);
}
hipError_t launch_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
    return scan(in, n, out, tmp, s);
}

// ---- inverted index: vertex -> relative RR indices (one wave per set) ---------------
// Entries hold rel0 + the set's index within [first, first + count).
__global__ void k_inv_scatter(const int64_t* __restrict__ rr_start, const int32_t* __restrict__ rr_len,
                              const int32_t* __restrict__ ids, int64_t first, int64_t count,
                              uint32_t rel0, const int64_t* __restrict__ inv_off,
                              uint32_t* __restrict__ cursor, uint32_t* __restrict__ inv) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t i = wave; i < count; i += nwaves) {
        const int64_t s = rr_start[first + i];
        const int32_t len = rr_len[first + i];
        for (int32_t j = lane; j < len; j += kWave) {
            const int32_t v = ids[s + j];
            const uint32_t at = atomic_add_agent(cursor + v, 1u);
            inv[inv_off[v] + at] = rel0 + (uint32_t)i;
        }
    }
}

hipError_t launch_inv_scatter(const int64_t* rr_start, const int32_t* rr_len, const int32_t* ids,
                              int64_t first, int64_t count, uint32_t rel0, const int64_t* inv_off,
                              uint32_t* cursor, uint32_t* inv, hipStream_t s) {
    if (count == 0) return hipSuccess;
    int64_t blocks = (count * kWave + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_inv_scatter<<<(unsigned)blocks, 256, 0, s>>>(rr_start, rr_len, ids, first, count, rel0,
                                                   inv_off, cursor, inv);
    return hipGetLastError();
}

// ---- inverted index by vertex buckets (no per-entry device atomics) -----------------
// Vertices are grouped in buckets of 2^shift consecutive ids (16 to 8192), at most
// kInvBuckets of them.
// Pass 1 (one block of 256 threads per 128 sets): each block counts its members per bucket in LDS, takes
// one range per bucket from the bucket's cursor (a device atomic per block and bucket), and
// writes (entry, vertex) pairs there; a bucket's pairs then fill exactly the index range of
// its vertices.  Pass 2 (one block per bucket): the bucket's vertices' next places are kept
// in LDS, so each pair goes to its vertex's list with an LDS atomic.
constexpr int kInvSetBlock = 256;
constexpr int kInvSets = 128;                // sets per block of pass 1
constexpr int kInvPlaceBlock = 512;
constexpr int kInvMaxShift = 13;

__global__ void k_inv_bucket_init(const int64_t* __restrict__ off, int64_t n, int32_t shift, int32_t nb,
                                  unsigned long long* __restrict__ bcur) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) bcur[b] = (unsigned long long)off[min((int64_t)b << shift, n)];
}

__global__ __launch_bounds__(kInvSetBlock) void k_inv_bucket(const int64_t* __restrict__ rr_start,
                                                             const int32_t* __restrict__ rr_len,
                                                             const int32_t* __restrict__ ids,
                                                             int64_t first, int64_t count, uint32_t rel0,
                                                             int32_t shift, int32_t nb,
                                                             unsigned long long* __restrict__ bcur,
                                                             uint2* __restrict__ pairs, int64_t pair_cap) {
    extern __shared__ unsigned char inv_lds[];
    uint32_t* cnt = reinterpret_cast<uint32_t*>(inv_lds);                        // nb
    unsigned long long* base = reinterpret_cast<unsigned long long*>(cnt + ((nb + 1) & ~1));  // nb
    __shared__ int64_t pre[kInvSetBlock + 1];
    __shared__ int64_t sst[kInvSetBlock];
    __shared__ int64_t sh[kScanBlock / kWave + 1];
    static_assert(kInvSetBlock == kScanBlock, "block_excl_scan spans the block");
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * kInvSets;
    const int64_t si = s0 + tid;
    int64_t len = 0;
    if (tid < kInvSets && si < count) {
        sst[tid] = rr_start[first + si];
        len = rr_len[first + si];
    }
    for (int32_t b = tid; b < nb; b += kInvSetBlock) cnt[b] = 0;
    int64_t total;
    pre[tid] = block_excl_scan(len, sh, total);
    if (tid == 0) pre[kInvSetBlock] = total;
    __syncthreads();
    // members q of the block's sets, flattened: set j with pre[j] <= q < pre[j + 1]
    auto member = [&](int64_t q, int& j) {
        int lo = 0, hi = kInvSetBlock;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= q) lo = mid; else hi = mid;
        }
        j = lo;
        return ids[sst[lo] + (q - pre[lo])];
    };
    for (int64_t q0 = 0; q0 < total; q0 += 4 * kInvSetBlock) {
        int32_t v[4];
        int j;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t q = q0 + u * kInvSetBlock + tid;
            v[u] = q < total ? member(q, j) : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (v[u] >= 0) atomicAdd(&cnt[v[u] >> shift], 1u);
    }
    __syncthreads();
    for (int32_t b = tid; b < nb; b += kInvSetBlock) {
        const uint32_t c = cnt[b];
        if (c) base[b] = atomic_add_agent(bcur + b, (unsigned long long)c);
        cnt[b] = 0;
    }
    __syncthreads();
    for (int64_t q0 = 0; q0 < total; q0 += 4 * kInvSetBlock) {
        int32_t v[4], js[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t q = q0 + u * kInvSetBlock + tid;
            js[u] = 0;
            v[u] = q < total ? member(q, js[u]) : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (v[u] >= 0) {
                const int32_t b = v[u] >> shift;
                const unsigned long long at = base[b] + atomicAdd(&cnt[b], 1u);
                if (at < (unsigned long long)pair_cap)
                    pairs[at] = make_uint2(rel0 + (uint32_t)(s0 + js[u]), (uint32_t)v[u]);
            }
    }
}

__global__ __launch_bounds__(kInvPlaceBlock) void k_inv_place(const int64_t* __restrict__ off, int64_t n,
                                                              int32_t shift, const uint2* __restrict__ pairs,
                                                              uint32_t* __restrict__ inv) {
    __shared__ uint32_t cur[1 << kInvMaxShift];
    const int tid = threadIdx.x;
    const int64_t v0 = (int64_t)blockIdx.x << shift;
    const int64_t v1 = min(v0 + ((int64_t)1 << shift), n);
    const int64_t r0 = off[v0], r1 = off[v1];
    for (int64_t v = v0 + tid; v < v1; v += kInvPlaceBlock) cur[v - v0] = (uint32_t)(off[v] - r0);
    __syncthreads();
    for (int64_t e0 = r0; e0 < r1; e0 += 4 * kInvPlaceBlock) {
        uint2 p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = e0 + u * kInvPlaceBlock + tid;
            p[u] = e < r1 ? pairs[e] : make_uint2(0u, 0xFFFFFFFFu);
        }
        // (the bounds tests only matter if the counts disagreed with the sets)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t vl = p[u].y - (uint32_t)v0;
            if (vl < (uint32_t)(v1 - v0)) {
                const int64_t at = r0 + atomicAdd(&cur[vl], 1u);
                if (at < r1) inv[at] = p[u].x;
            }
        }
    }
}

// Bucket shift for n vertices (0: the bucketed build does not apply): the narrowest buckets
// (at least 16 vertices) that make at most 1024 of them, so that small graphs still spread
// the placement over many blocks, else at most kInvBuckets.
int32_t inv_bucket_shift(int64_t n) {
    for (const int64_t most : {(int64_t)1024, (int64_t)kInvBuckets})
        for (int32_t shift = 4; shift <= kInvMaxShift; ++shift)
            if (((n + ((int64_t)1 << shift) - 1) >> shift) <= most) return shift;
    return 0;
}

hipError_t launch_inv_bucketed(const int64_t* rr_start, const int32_t* rr_len, const int32_t* ids,
                               int64_t first, int64_t count, uint32_t rel0, const int64_t* inv_off,
                               int64_t n, unsigned long long* bcur, uint2* pairs, int64_t pair_cap,
                               uint32_t* inv, hipStream_t s) {
    const int32_t shift = inv_bucket_shift(n);
    if (shift == 0 || n < 1) return hipErrorInvalidValue;
    if (count == 0) return hipSuccess;
    const int32_t nb = (int32_t)((n + ((int64_t)1 << shift) - 1) >> shift);
    k_inv_bucket_init<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(inv_off, n, shift, nb, bcur);
    const size_t lds = sizeof(uint32_t) * (size_t)((nb + 1) & ~1) + sizeof(unsigned long long) * (size_t)nb;
    const int64_t blocks = (count + kInvSets - 1) / kInvSets;
    k_inv_bucket<<<(unsigned)blocks, kInvSetBlock, lds, s>>>(rr_start, rr_len, ids, first, count, rel0, shift,
                                                            nb, bcur, pairs, pair_cap);
    k_inv_place<<<(unsigned)nb, kInvPlaceBlock, 0, s>>>(inv_off, n, shift, pairs, inv);
    return hipGetLastError();
}

__global__ void k_sub_u32(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                          uint32_t* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] - b[i];
}

hipError_t launch_sub_u32(const uint32_t* a, const uint32_t* b, uint32_t* out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_sub_u32<<<(unsigned)blocks, 256, 0, s>>>(a, b, out, n);
    return hipGetLastError();
}

__global__ void k_copy_hist(const uint32_t* __restrict__ hist, int32_t* __restrict__ h, int32_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        h[i] = (int32_t)hist[i];
}

hipError_t launch_copy_hist(const uint32_t* hist, int32_t* h, int32_t n, hipStream_t s) {
    int64_t blocks = ((int64_t)n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_copy_hist<<<(unsigned)blocks, 256, 0, s>>>(hist, h, n);
    return hipGetLastError();
}

// ---- greedy rounds ------------------------------------------------------------------
// key(v) = (h[v] + 1) << 32 | (2^32 - 1 - v): the largest key has the largest count and,
// among equal counts, the smallest id.  Chosen vertices hold h = -1 (key high part 0), so
// any vertex not chosen beats them; the vertex chosen in a round is set to -1 in that
// round's cover step, which never decrements it.
// ---- all rounds in one cooperative launch ---------------------------------------------
constexpr int kCoopBlock = 1024;
constexpr int kCoopWaves = kCoopBlock / kWave;
constexpr int kArgTile = kCoopBlock * 4;       // counters per argmax tile
constexpr int kArgGroup = 4;                     // tiles of a block loaded together
constexpr int kMaxInst = kCoopBlock;             // instances per launch (LDS tables)

template <typename T>
__device__ __forceinline__ T ld_co(const T* p) {        // coherent load (all XCDs)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_co(T* p, T v) {      // coherent store
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_co(const IMM_GLOBAL T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_co(IMM_GLOBAL T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier over all (co-resident) blocks.  Every block first waits for its own memory
// operations to complete, so once the last block has arrived, everything written before
// the barrier is visible to coherent (agent-scope) loads issued after it.  Data shared
// between blocks inside the kernel is only read and written with such loads, stores and
// atomics, so no cache write-back or invalidate is needed.  Counters are monotonic
// (epoch-based) and spread over 16 lines; a wait longer than kBarrierTimeout sets
// bar->err and every block leaves, so no wave spins forever.  The bound is a time, not a
// poll count: a cover step of many instances over RR sets of 10^5 members (trivalency IC
// on R-MAT scale 24) legitimately keeps some blocks busy for seconds, past the few
// seconds that 2^24 polls had allowed.
constexpr uint64_t kBarrierTimeout = 100000000ull * 120;   // s_memrealtime ticks (100 MHz): 120 s

__device__ __forceinline__ bool grid_sync(GridBarrier* bar, unsigned int& epoch) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        const unsigned int ngroups = gridDim.x < 16 ? gridDim.x : 16u;
        const unsigned int grp = blockIdx.x % ngroups;
        const unsigned int gsize = (gridDim.x - grp + ngroups - 1) / ngroups;
        const unsigned int old = __hip_atomic_fetch_add(&bar->sub[grp][0], 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == (epoch + 1) * gsize) {
            __builtin_amdgcn_s_waitcnt(0);
            __hip_atomic_fetch_add(&bar->top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const unsigned int target = (epoch + 1) * ngroups;
        int ok = 1;
        unsigned int polls = 0;
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (ld_co(&bar->top) < target) {
            if ((++polls & 63u) == 0u &&
                (ld_co(&bar->err) || __builtin_amdgcn_s_memrealtime() - t0 > kBarrierTimeout)) {
                st_co(&bar->err, 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        s_ok = ok;
    }
    ++epoch;
    __syncthreads();
    return s_ok != 0;
}

// Per-block combining of counter decrements.  In the first rounds the newly covered sets
// overlap heavily, so the same counters are decremented from many blocks; device-scope
// atomics on one address serialise across the XCDs.  Each block therefore adds its
// decrements into an LDS table keyed by (instance, vertex) (open addressing, two probes;
// a decrement that finds no slot goes straight to the device counter) and applies each
// slot's total with one device atomic at the end of the cover step.
constexpr int kDecSlots = 4096;
constexpr unsigned long long kDecEmpty = ~0ull;
struct DecCache {
    unsigned long long key[kDecSlots];
    int32_t cnt[kDecSlots];
};

__device__ __forceinline__ void dec_counter(DecCache& dc, const SelInst* inst, int32_t li,
                                            int32_t v) {
    const unsigned long long key = ((unsigned long long)(uint32_t)li << 32) | (uint32_t)v;
    uint32_t slot = (((uint32_t)v * 2654435761u) ^ ((uint32_t)li * 0x9E3779B9u)) >> 20;
#pragma unroll
    for (int probe = 0; probe < 2; ++probe) {
        unsigned long long cur = dc.key[slot];
        if (cur == kDecEmpty) cur = atomicCAS(&dc.key[slot], kDecEmpty, key);
        if (cur == kDecEmpty || cur == key) {
            atomicAdd(&dc.cnt[slot], 1);
            return;
        }
        slot = (slot + 1u) & (kDecSlots - 1u);
    }
    __hip_atomic_fetch_add(global(inst[li].h) + v, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Applies and clears the block's table (all threads of the block).
__device__ __forceinline__ void dec_flush(DecCache& dc, const SelInst* inst) {
    __syncthreads();
    for (int i = threadIdx.x; i < kDecSlots; i += blockDim.x) {
        const unsigned long long key = dc.key[i];
        if (key != kDecEmpty) {
            __hip_atomic_fetch_add(global(inst[(int32_t)(key >> 32)].h) + (int32_t)(uint32_t)key,
                                   -dc.cnt[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            dc.key[i] = kDecEmpty;
            dc.cnt[i] = 0;
        }
    }
}

// Exclusive prefix of one int64 per thread of the block into out[0..blockDim], with
// out[blockDim] the total.
__device__ __forceinline__ void block_excl_scan_i64(int64_t v, int64_t* out, int64_t* wsum) {
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int64_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        const int64_t t = lane < kCoopWaves ? wsum[lane] : 0;
        const int64_t ti = wave_incl_scan(t);
        if (lane < kCoopWaves) wsum[lane] = ti - t;
        if (lane == kCoopWaves - 1) out[kCoopBlock] = ti;
    }
    __syncthreads();
    out[tid] = incl - v + wsum[wid];
    __syncthreads();
}

// Block-wide maximum of every thread's key, merged into *key with one atomic (no-op when
// the maximum is 0).  Called by all threads of the block.
__device__ __forceinline__ void block_key_max(unsigned long long best,
                                              IMM_GLOBAL unsigned long long* key,
                                              unsigned long long* red, int lane, int wid, int tid) {
    best = wave_max_u64(best);
    if (lane == 0) red[wid] = best;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kCoopWaves; ++w) best = red[w] > best ? red[w] : best;
        if (best) __hip_atomic_fetch_max(key, best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// Block-wide maximum of every thread's key, stored (0 when the block saw no candidate) at
// *slot.  Called by all threads of the block.
__device__ __forceinline__ void block_key_store(unsigned long long best, unsigned long long* slot,
                                                unsigned long long* red, int lane, int wid, int tid) {
    best = wave_max_u64(best);
    if (lane == 0) red[wid] = best;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kCoopWaves; ++w) best = red[w] > best ? red[w] : best;
        st_co(slot, best);
    }
    __syncthreads();
}

// ---- hot set of a single-instance selection --------------------------------------------
// Counters only decrease, so a vertex whose count is at most C can be the argmax only once
// every other count is at most C.  With C the smallest threshold that leaves at most
// hot_max vertices above it ("hot"), a round whose best hot count exceeds C has found the
// exact argmax without reading any other counter, and the counters of cold vertices are
// not needed at all until then: they are not decremented.  On the R-MAT workloads the
// 16384 most frequent vertices leave every one of their greedy rounds in hot mode and
// carry 40-60% of the decrements.  The first round whose best hot count is at most C
// recounts every counter exactly (initial counts minus the covered sets, chosen vertices
// -1 again) and the selection continues over all vertices.
constexpr int kHotBuckets = kSelectHotBuckets;   // counts 0 .. 4094 exact, 4095: 4095 or more
constexpr int kHotPerThread = kSelectHotPerBlock / kCoopBlock;   // hot vertices per thread
static_assert(kHotBuckets == 4 * kCoopBlock, "the threshold search gives each thread 4 buckets");
static_assert(kHotPerThread * kCoopBlock == kSelectHotPerBlock, "hot vertices per block");
constexpr int32_t kHotOff = 0x7FFFFFFF;
constexpr int kHotListPer = 16;          // vertices per thread when the hot list is built

// h[v] = hist[v] for the selection's counters, and the histogram of those counts into
// cnt_hist (zeroed): counts 0..3 by wave ballots, the rest by LDS atomics, each block's
// non-zero buckets added to cnt_hist.
__global__ __launch_bounds__(kCoopBlock) void k_hot_counts(const uint32_t* __restrict__ hist,
                                                           int32_t* __restrict__ h, int64_t n,
                                                           uint32_t* __restrict__ cnt_hist) {
    __shared__ uint32_t chist[kHotBuckets];
    const int tid = threadIdx.x, lane = lane_id();
    for (int i = tid; i < kHotBuckets; i += kCoopBlock) chist[i] = 0;
    __syncthreads();
    uint32_t small[4] = {0u, 0u, 0u, 0u};
    for (int64_t b0 = (int64_t)blockIdx.x * kCoopBlock; b0 < n; b0 += (int64_t)gridDim.x * kCoopBlock) {
        const int64_t v = b0 + tid;
        int32_t c = -1;
        if (v < n) {
            c = (int32_t)hist[v];
            h[v] = c;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) small[q] += (uint32_t)__popcll(ballot(c == q));
        if (c >= 4) atomicAdd(&chist[c < kHotBuckets - 1 ? c : kHotBuckets - 1], 1u);
    }
    if (lane == 0)
        for (int q = 0; q < 4; ++q)
            if (small[q]) atomicAdd(&chist[q], small[q]);
    __syncthreads();
    for (int i = tid; i < kHotBuckets; i += kCoopBlock)
        if (chist[i]) atomicAdd(cnt_hist + i, chist[i]);
}

// The hot threshold C: the smallest count below the last bucket with at most hot_max counts
// above it (kHotOff: none).  All threads of the block.
__device__ int32_t hot_threshold(const uint32_t* __restrict__ cnt_hist, int32_t hot_max,
                                 int64_t* pre, int64_t* wsum) {
    __shared__ int32_t s_thr;
    const int tid = threadIdx.x;
    // thread t holds buckets kHotBuckets - 1 - (4t + j), j = 0..3 (descending)
    uint32_t cj[4];
    int64_t local = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        cj[j] = cnt_hist[kHotBuckets - 1 - (4 * tid + j)];
        local += cj[j];
    }
    block_excl_scan_i64(local, pre, wsum);
    int64_t above = pre[tid];                    // counts in the buckets above this thread's
    int32_t cand = kHotOff;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int32_t b = kHotBuckets - 1 - (4 * tid + j);
        if (b < kHotBuckets - 1 && above <= (int64_t)hot_max) cand = min(cand, b);
        above += cj[j];
    }
    if (tid == 0) s_thr = kHotOff;
    __syncthreads();
    if (cand != kHotOff) atomicMin(&s_thr, cand);
    __syncthreads();
    return s_thr;
}

// Hot vertices among the kHotListPer consecutive vertices v0, v0 + 1, ... (bit j: v0 + j).
__device__ __forceinline__ uint32_t hot_mask(const int32_t* __restrict__ h, int64_t n, int64_t v0,
                                             int32_t thr) {
    static_assert(kHotListPer == 16, "four 16-byte loads per thread");
    uint32_t m = 0;
    if (v0 + kHotListPer <= n) {
        const int4* p = reinterpret_cast<const int4*>(h + v0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int4 x = p[q];
            m |= ((uint32_t)(x.x > thr) | (uint32_t)(x.y > thr) << 1 | (uint32_t)(x.z > thr) << 2 |
                  (uint32_t)(x.w > thr) << 3) << (4 * q);
        }
    } else {
        for (int j = 0; j < kHotListPer; ++j)
            if (v0 + j < n && h[v0 + j] > thr) m |= 1u << j;
    }
    return m;
}

// The threshold C (hot_n[1], by block 0), each block's number of hot vertices {v : h[v] > C}
// in its range of kCoopBlock x kHotListPer vertices (blk_cnt), and their total (hot_n[0],
// zeroed before).
__global__ __launch_bounds__(kCoopBlock) void k_hot_threshold(const int32_t* __restrict__ h, int64_t n,
                                                              const uint32_t* __restrict__ cnt_hist,
                                                              int32_t hot_max,
                                                              uint32_t* __restrict__ blk_cnt,
                                                              uint32_t* __restrict__ hot_n) {
    __shared__ int64_t pre[kCoopBlock + 1];
    __shared__ int64_t wsum[kCoopWaves];
    const int tid = threadIdx.x;
    const int32_t thr = hot_threshold(cnt_hist, hot_max, pre, wsum);
    if (blockIdx.x == 0 && tid == 0) hot_n[1] = (uint32_t)thr;
    if (thr == kHotOff) return;
    const int64_t v0 = (int64_t)blockIdx.x * kCoopBlock * kHotListPer + (int64_t)tid * kHotListPer;
    block_excl_scan_i64(__popc(hot_mask(h, n, v0, thr)), pre, wsum);
    if (tid == 0) {
        blk_cnt[blockIdx.x] = (uint32_t)pre[kCoopBlock];
        if (pre[kCoopBlock]) atomicAdd(hot_n, (uint32_t)pre[kCoopBlock]);
    }
}

// The hot list in increasing vertex order (hot_ids) and, per 32 vertices, one word whose low
// half is their hot bitmap and whose high half the number of hot vertices before them
// (hot_words): the hot position of v is then high + popcount(low & (2^(v mod 32) - 1)).
__global__ __launch_bounds__(kCoopBlock) void k_hot_list(const int32_t* __restrict__ h, int64_t n,
                                                         const uint32_t* __restrict__ hot_n,
                                                         const uint32_t* __restrict__ blk_cnt,
                                                         int32_t* __restrict__ hot_ids,
                                                         unsigned long long* __restrict__ hot_words) {
    __shared__ int64_t pre[kCoopBlock + 1];
    __shared__ int64_t wsum[kCoopWaves];
    const int tid = threadIdx.x;
    const int32_t thr = (int32_t)hot_n[1];
    if (thr == kHotOff) return;
    // hot vertices of the blocks before this one
    int64_t before = 0;
    for (uint32_t b = tid; b < blockIdx.x; b += kCoopBlock) before += blk_cnt[b];
    block_excl_scan_i64(before, pre, wsum);
    const int64_t base = pre[kCoopBlock];
    const int64_t v0 = (int64_t)blockIdx.x * kCoopBlock * kHotListPer + (int64_t)tid * kHotListPer;
    const uint32_t m = hot_mask(h, n, v0, thr);
    block_excl_scan_i64(__popc(m), pre, wsum);
    const int64_t first = base + pre[tid];       // hot position of this thread's first one
    uint32_t at = (uint32_t)first;
    for (uint32_t r = m; r != 0; r &= r - 1) hot_ids[at++] = (int32_t)(v0 + __ffs(r) - 1);
    // two threads per word: the even one writes it
    const uint32_t hi = (uint32_t)__shfl_xor((int)m, 1);
    const int64_t w = v0 / 32;
    if ((tid & 1) == 0 && w < (n + 31) / 32)
        hot_words[w] = ((unsigned long long)(uint32_t)first << 32) | (unsigned long long)(m | (hi << 16));
}

hipError_t launch_hot_prepare(const uint32_t* hist, int32_t* h, int64_t n, int32_t hot_max,
                              uint32_t* cnt_hist, uint32_t* blk_cnt, unsigned long long* hot_words,
                              int32_t* hot_ids, uint32_t* hot_n, hipStream_t s) {
    int64_t blocks = (n + kCoopBlock - 1) / kCoopBlock;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    k_hot_counts<<<(unsigned)blocks, kCoopBlock, 0, s>>>(hist, h, n, cnt_hist);
    const int64_t lblocks = hot_list_blocks(n);
    k_hot_threshold<<<(unsigned)lblocks, kCoopBlock, 0, s>>>(h, n, cnt_hist, hot_max, blk_cnt, hot_n);
    k_hot_list<<<(unsigned)lblocks, kCoopBlock, 0, s>>>(h, n, hot_n, blk_cnt, hot_ids, hot_words);
    return hipGetLastError();
}

int64_t hot_list_blocks(int64_t n) {
    const int64_t per = (int64_t)kCoopBlock * kHotListPer;
    return n > 0 ? (n + per - 1) / per : 1;
}

struct CoopLds {
    int64_t tile_pre[kMaxInst + 1];     // argmax tiles per instance, prefix
    int64_t ent_pre[kMaxInst + 1];      // cover entries per instance, prefix
    int64_t ent_beg[kMaxInst];
    int32_t chosen[kMaxInst];           // each instance's vertex of this round
    unsigned long long red[kCoopWaves];
    int64_t wsum[kCoopWaves];
    int64_t set_pre[kCoopBlock + 1];    // decrement batch: prefix of its sets' sizes
    const int32_t* set_mem[kCoopBlock];
    int32_t set_inst[kCoopBlock];
    union {
        DecCache dc;                    // decrement combining of ordinary rounds
        int32_t dense[kSelectDenseHot]; // a dense round's decrements per hot position
    } u;
    unsigned char stopped[kMaxInst];    // estimation phase decided (failed)
    int64_t seg_pre[kMaxSegs + 1];      // single instance: its entries per segment
    int64_t seg_beg[kMaxSegs];
    unsigned long long key;             // single instance: this round's argmax key
    int32_t thr;
    int32_t hot_cnt;                    // this block's share of the hot list ...
    int32_t hot[kSelectHotPerBlock];    // ... kept for all rounds
    int32_t csum[2 * kCoopBlock];       // column sums of a dense round, per wave
};

// Decrements the counters of the members of every thread's set (len members at mem, of
// instance li; len 0: none): the block scans the sizes and its waves share the flattened
// members (consecutive lanes on consecutive members of a set, four per lane in flight),
// each member found by a binary search over the prefix.  Skips each instance's chosen
// vertex when skip_chosen, and, in batches of more than 4 x kCoopBlock members, vertices
// outside the hot set when hot_words is set.  In a dense round (a single instance) only hot
// vertices are decremented, each in the LDS count of its hot position.  All threads of the
// block.
__device__ __noinline__ void dec_batch(CoopLds& S, const SelInst* inst, int64_t len, const int32_t* mem, int li,
                          bool skip_chosen, const unsigned long long* hot_words,
                          bool dense = false) {
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    block_excl_scan_i64(len, S.set_pre, S.wsum);
    S.set_mem[tid] = mem;
    S.set_inst[tid] = li;
    __syncthreads();
    const int64_t total = S.set_pre[kCoopBlock];
    for (int64_t q0 = (int64_t)wid * (4 * kWave); q0 < total; q0 += 4 * kCoopBlock) {
        int32_t v[4], vi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t q = q0 + u * kWave + lane;
            v[u] = 0;
            vi[u] = -1;
            if (q < total) {
                int lo = 0, hi = kCoopBlock;       // set_pre[lo] <= q < set_pre[lo + 1]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (S.set_pre[mid] <= q) lo = mid; else hi = mid;
                }
                v[u] = global(S.set_mem[lo])[q - S.set_pre[lo]];
                vi[u] = S.set_inst[lo];
            }
        }
        if (dense) {
            unsigned long long hw[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) hw[u] = vi[u] >= 0 ? global(hot_words)[v[u] >> 5] : 0ull;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t b = (uint32_t)v[u] & 31u, lo = (uint32_t)hw[u];
                if (((lo >> b) & 1u) && v[u] != S.chosen[0])
                    atomicAdd(&S.u.dense[(uint32_t)(hw[u] >> 32) + __popc(lo & ((1u << b) - 1u))], 1);
            }
            continue;
        }
        if (hot_words && total > 4 * kCoopBlock) {
            // cold counters are never read in hot mode (and the recount resets them), so a
            // small batch skips the bitmap test and its dependent load
            uint32_t w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) w[u] = vi[u] >= 0 ? (uint32_t)global(hot_words)[v[u] >> 5] : 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (!((w[u] >> (v[u] & 31)) & 1u)) vi[u] = -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (vi[u] >= 0 && !(skip_chosen && v[u] == S.chosen[vi[u]]))
                dec_counter(S.u.dc, inst, vi[u], v[u]);
    }
    __syncthreads();                           // the batch tables are rewritten next
}

// One round's argmax over tiles of kArgTile counters, any instance still selecting.  A
// block's successive tiles of one instance share one block reduction (tiles are grouped by
// instance, so an instance's tiles are consecutive).  A single-instance launch leaves each
// block's maximum in bar->bkeys (reduced after the barrier); several instances merge theirs
// into the instance's key with an atomic.
__device__ void argmax_tiles(CoopLds& S, const SelInst* inst, int32_t ninst, int32_t round,
                             int64_t ntiles, GridBarrier* bar) {
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    unsigned long long best = 0;
    int cur = -1;                                    // instance of `best`, block-uniform
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int lo = 0, hi = ninst;                      // tile_pre[lo] <= t < tile_pre[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (S.tile_pre[mid] <= t) lo = mid; else hi = mid;
        }
        const SelInst& I = inst[lo];
        if (round >= I.k || S.stopped[lo]) continue;   // uniform across the block
        if (lo != cur) {
            if (cur >= 0) block_key_max(best, global(inst[cur].keys) + round, S.red, lane, wid, tid);
            cur = lo;
            best = 0;
        }
        // partition matroid: the parts that already hold part_k chosen elements
        uint64_t full = 0;
        if (I.part_n > 0) {
            const int32_t parts = I.n / I.part_n;
            const int32_t tk = lane < parts ? ld_co(global(I.taken) + lane) : 0;
            full = ballot(lane < parts && tk >= I.part_k);
        }
        const IMM_GLOBAL int32_t* h = global(I.h);
        // up to kArgGroup of the block's successive tiles of this instance are loaded
        // together
        const int64_t left = (S.tile_pre[lo + 1] - t + gridDim.x - 1) / gridDim.x;
        const int m = left < kArgGroup ? (int)left : kArgGroup;
        const int64_t base = (t - S.tile_pre[lo]) * kArgTile;
        const int64_t step = (int64_t)gridDim.x * kArgTile;
        int32_t c[4 * kArgGroup];
#pragma unroll
        for (int j = 0; j < 4 * kArgGroup; ++j) {
            const int64_t v = base + (j >> 2) * step + (j & 3) * kCoopBlock + tid;
            c[j] = (j >> 2) < m && v < I.n ? ld_co(h + v) : -1;
        }
#pragma unroll
        for (int j = 0; j < 4 * kArgGroup; ++j) {
            const int64_t v = base + (j >> 2) * step + (j & 3) * kCoopBlock + tid;
            if (full != 0 && c[j] >= 0 && ((full >> ((uint32_t)v / (uint32_t)I.part_n)) & 1ull))
                c[j] = -1;
            if (c[j] >= 0) {
                const unsigned long long key = ((unsigned long long)(uint32_t)(c[j] + 1) << 32) |
                                               (unsigned long long)(0xFFFFFFFFu - (uint32_t)v);
                best = key > best ? key : best;
            }
        }
        t += (int64_t)(m - 1) * gridDim.x;
    }
    if (ninst == 1) {
        block_key_store(best, bar->bkeys + blockIdx.x, S.red, lane, wid, tid);
    } else if (cur >= 0) {
        block_key_max(best, global(inst[cur].keys) + round, S.red, lane, wid, tid);
    }
}

// Single instance: the maximum of the blocks' keys, into S.key.  All threads of the block.
__device__ __forceinline__ void reduce_block_keys(CoopLds& S, GridBarrier* bar) {
    const int tid = threadIdx.x, lane = lane_id();
    if (tid < kWave) {
        unsigned long long k = 0;
        for (int b = lane; b < (int)gridDim.x; b += kWave) {
            const unsigned long long x = ld_co(bar->bkeys + b);
            k = x > k ? x : k;
        }
        k = wave_max_u64(k);
        if (lane == 0) S.key = k;
    }
    __syncthreads();
}

// Rows of hot_part: 16-bit counts (a block's count for one hot vertex in one round is at most
// its entries of the round, which a dense round keeps below 2^16), two per 32-bit word, rows
// of dense_words(total) words.
__device__ __forceinline__ int32_t dense_words(int32_t total) { return (total + 1) >> 1; }

// The new seed's entries in every index segment of a single instance: lane j of wave 0 loads
// segment j's range (all segments at once), into seg_beg / seg_pre and the entry count
// ent_pre[1].  All threads of the block.
__device__ __noinline__ void seg_ranges(CoopLds& S, const SelInst& I) {
    const int lane = lane_id();
    if (threadIdx.x < kWave) {
        const int32_t u = S.chosen[0];
        int64_t b = 0, c = 0;
        if (lane < I.nseg) {
            b = global(I.seg_off[lane])[u];
            c = global(I.seg_off[lane])[u + 1] - b;
        }
        const int64_t incl = wave_incl_scan(c);
        if (lane < I.nseg) {
            S.seg_beg[lane] = b;
            S.seg_pre[lane] = incl - c;
        }
        if (lane == I.nseg - 1) {
            S.seg_pre[I.nseg] = incl;
            S.ent_pre[1] = incl;
        }
    }
    __syncthreads();
}

// This block's row of hot_part from its LDS counts (every position, so no row needs
// clearing).  All threads of the block.
__device__ __noinline__ void dense_store_row(CoopLds& S, const SelInst& I, int32_t total) {
    const int32_t nw = dense_words(total);
    IMM_GLOBAL uint32_t* row =
        reinterpret_cast<IMM_GLOBAL uint32_t*>(global(I.hot_part)) + (int64_t)blockIdx.x * nw;
    for (int i = threadIdx.x; i < nw; i += kCoopBlock) {
        const uint32_t hi = 2 * i + 1 < total ? (uint32_t)S.u.dense[2 * i + 1] : 0u;
        st_co(row + i, (uint32_t)S.u.dense[2 * i] | hi << 16);
    }
}

// Column sums of hot_part over this block's hot positions [lo, lo + S.hot_cnt): acc[i] =
// sum over the grid's rows of the count at position lo + i.  A wave takes 64 consecutive
// words (128 positions) of every 16th row (8 loads per lane in flight); the 16 waves' sums
// are added in LDS.  All threads of the block.
__device__ __noinline__ void dense_column_sums(CoopLds& S, const SelInst& I, int32_t* acc,
                                               int32_t total, int32_t lo) {
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int32_t cnt = S.hot_cnt, rows = (int32_t)gridDim.x, stride = dense_words(total);
    const int32_t wlo = lo >> 1, whi = (lo + cnt + 1) >> 1;
    const IMM_GLOBAL uint32_t* part = reinterpret_cast<const IMM_GLOBAL uint32_t*>(global(I.hot_part));
    for (int32_t w0 = wlo; w0 < whi; w0 += kWave) {
        const int32_t w = w0 + lane;
        int32_t sum_lo = 0, sum_hi = 0;
        if (w < whi) {
            const IMM_GLOBAL uint32_t* p = part + w;
            const int64_t step = (int64_t)kCoopWaves * stride;
            for (int32_t r0 = wid; r0 < rows; r0 += kCoopWaves * 8) {
                uint32_t x[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int32_t r = r0 + j * kCoopWaves;
                    x[j] = r < rows ? ld_co(p + (int64_t)r0 * stride + j * step) : 0u;
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    sum_lo += (int32_t)(x[j] & 0xFFFFu);
                    sum_hi += (int32_t)(x[j] >> 16);
                }
            }
        }
        S.csum[wid * kWave + lane] = sum_lo;
        S.csum[kCoopBlock + wid * kWave + lane] = sum_hi;
        __syncthreads();
        if (tid < kWave && w0 + tid < whi) {
            int32_t a = 0, b = 0;
            for (int v = 0; v < kCoopWaves; ++v) {
                a += S.csum[v * kWave + tid];
                b += S.csum[kCoopBlock + v * kWave + tid];
            }
            const int32_t c = 2 * (w0 + tid) - lo;       // column of the low half
            if (c >= 0 && c < cnt) acc[c] = a;
            if (c + 1 >= 0 && c + 1 < cnt) acc[c + 1] = b;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kCoopBlock) void k_select_coop(const SelInst* __restrict__ inst,
                                                            int32_t ninst, int32_t maxk,
                                                            GridBarrier* bar) {
    __shared__ CoopLds S;
    if (threadIdx.x < kMaxInst) S.stopped[threadIdx.x] = 0;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const bool solo = ninst == 1;
    unsigned int epoch = 0;
    // instance prefixes are computed one instance per thread (kMaxInst == kCoopBlock); the
    // tables past ninst repeat the total
    block_excl_scan_i64(tid < ninst ? (inst[tid].n + kArgTile - 1) / kArgTile : 0, S.tile_pre, S.wsum);
    const int64_t ntiles = S.tile_pre[ninst];

    // ---- hot set (single instance with hot_max > 0), prepared by k_hot_counts and
    // k_hot_list: this block's share of the list is kept in LDS for all rounds ----
    int32_t thr = kHotOff;
    int32_t hot_total = 0, hot_lo = 0;          // hot list length; this block's first position
    bool dense_ok = false;                       // dense rounds possible (uniform)
    if (solo && inst[0].hot_max > 0) {
        const SelInst& I = inst[0];
        thr = (int32_t)I.hot_n[1];
        if (thr != kHotOff) {
            const int64_t H = I.hot_n[0];
            const int64_t per = (H + gridDim.x - 1) / gridDim.x;
            const int64_t lo = min(per * blockIdx.x, H);
            const int64_t cnt = min(per, H - lo);
            for (int64_t i = tid; i < cnt; i += kCoopBlock) S.hot[i] = I.hot_ids[lo + i];
            if (tid == 0) S.hot_cnt = (int32_t)cnt;
            hot_total = (int32_t)H;
            hot_lo = (int32_t)lo;
            dense_ok = I.hot_part && I.dense_gain > 0 && H <= kSelectDenseHot && per <= kSelectDenseShare;
        }
    }
    bool prev_dense = false;                     // the previous round was dense (uniform)
    static_assert(sizeof(S.set_pre) >= sizeof(int32_t) * kSelectDenseShare,
                  "the column sums of a block's hot positions fit the batch prefix table");
    for (int i = threadIdx.x; i < kDecSlots; i += blockDim.x) {
        S.u.dc.key[i] = kDecEmpty;
        S.u.dc.cnt[i] = 0;
    }
    __syncthreads();

    for (int32_t round = 0; round < maxk; ++round) {
        // coverage after the previous rounds (nothing adds to it before the next barrier);
        // thread i keeps instance i's
        const int64_t cov_before = tid < ninst ? (int64_t)ld_co(global(inst[tid].n_covered)) : 0;
        // ---- argmax (a second time, over every vertex, after leaving hot mode) ----
        for (;;) {
            if (thr != kHotOff) {
                const SelInst& I = inst[0];
                unsigned long long best = 0;
                if (round < I.k && !S.stopped[0]) {
                    uint64_t full = 0;
                    if (I.part_n > 0) {
                        const int32_t parts = I.n / I.part_n;
                        const int32_t tk = lane < parts ? ld_co(global(I.taken) + lane) : 0;
                        full = ballot(lane < parts && tk >= I.part_k);
                    }
                    // after a dense round: its decrements of this block's hot positions are
                    // the column sums of hot_part, accumulated in LDS (the batch prefix table
                    // is free until the cover step)
                    int32_t* acc = reinterpret_cast<int32_t*>(S.set_pre);
                    if (prev_dense) dense_column_sums(S, I, acc, hot_total, hot_lo);
                    int32_t c[kHotPerThread], hv[kHotPerThread];
#pragma unroll
                    for (int j = 0; j < kHotPerThread; ++j) {
                        const int i = tid + j * kCoopBlock;
                        hv[j] = i < S.hot_cnt ? S.hot[i] : -1;
                        c[j] = hv[j] >= 0 ? ld_co(global(I.h) + hv[j]) : -1;
                    }
                    if (prev_dense) {
                        // the counters of this block's hot vertices take the dense round's
                        // decrements (only this block writes them until the next barrier)
#pragma unroll
                        for (int j = 0; j < kHotPerThread; ++j) {
                            const int i = tid + j * kCoopBlock;
                            const int32_t d = hv[j] >= 0 ? acc[i] : 0;
                            if (d != 0) {
                                c[j] -= d;
                                st_co(global(I.h) + hv[j], c[j]);
                            }
                        }
                    }
#pragma unroll
                    for (int j = 0; j < kHotPerThread; ++j) {
                        const uint32_t v = (uint32_t)hv[j];
                        if (full != 0 && c[j] >= 0 && ((full >> (v / (uint32_t)I.part_n)) & 1ull)) c[j] = -1;
                        if (c[j] >= 0) {
                            const unsigned long long key = ((unsigned long long)(uint32_t)(c[j] + 1) << 32) |
                                                           (unsigned long long)(0xFFFFFFFFu - v);
                            best = key > best ? key : best;
                        }
                    }
                }
                block_key_store(best, bar->bkeys + blockIdx.x, S.red, lane, wid, tid);
            } else {
                argmax_tiles(S, inst, ninst, round, ntiles, bar);
            }
            if (!grid_sync(bar, epoch)) return;
            if (solo) reduce_block_keys(S, bar);
            if (thr == kHotOff || round >= inst[0].k || S.stopped[0] ||
                (S.key != 0 && (int64_t)(S.key >> 32) - 1 > (int64_t)thr))
                break;
            // the best hot count is no longer above every cold count: recount all counters
            // exactly and leave hot mode
            const SelInst& I = inst[0];
            IMM_GLOBAL int32_t* h = global(I.h);
            for (int64_t v = (int64_t)blockIdx.x * kCoopBlock + tid; v < I.n; v += (int64_t)gridDim.x * kCoopBlock)
                st_co(h + v, (int32_t)global(I.h0)[v]);
            if (!grid_sync(bar, epoch)) return;
            const int64_t s_lo = I.count * (int64_t)blockIdx.x / gridDim.x;
            const int64_t s_hi = I.count * ((int64_t)blockIdx.x + 1) / gridDim.x;
            for (int64_t sb = s_lo; sb < s_hi; sb += kCoopBlock) {
                const int64_t rel = sb + tid;
                int64_t len = 0;
                const int32_t* mem = nullptr;
                if (rel < s_hi && ld_co(global(I.covered) + rel) != 0u) {
                    mem = I.ids + global(I.rr_start)[I.first + rel];
                    len = global(I.rr_len)[I.first + rel];
                }
                dec_batch(S, inst, len, mem, 0, false, nullptr);
            }
            dec_flush(S.u.dc, inst);
            if (!grid_sync(bar, epoch)) return;
            if (blockIdx.x == 0)
                for (int j = tid; j < round; j += kCoopBlock) st_co(h + ld_co(global(I.seeds) + j), -1);
            thr = kHotOff;
            if (!grid_sync(bar, epoch)) return;
        }
        // ---- cover: sets containing each instance's new seed ----
        // Every block reads the same final keys and coverage, so every block takes the same
        // stop decisions.
        int64_t cnt = 0;
        bool live = false;
        if (tid < ninst && round < inst[tid].k && !S.stopped[tid]) {
            const SelInst& I = inst[tid];
            const unsigned long long key = solo ? S.key : ld_co(global(I.keys) + round);
            if (solo && blockIdx.x == 0) st_co(global(I.keys) + round, key);   // round's gain, for the caller
            const int64_t gain = key ? (int64_t)(key >> 32) - 1 : 0;
            const int64_t bound = cov_before + (int64_t)(I.k - round) * gain;
            if (I.need > 0 && bound < I.need) {
                S.stopped[tid] = 1;
                // the coverage all k rounds could reach at most (still below need): what
                // the caller reads as this failed phase's coverage
                if (blockIdx.x == 0) st_co(global(I.n_covered), (unsigned long long)bound);
            } else {
                live = true;
                const int32_t u = (int32_t)(0xFFFFFFFFu - (uint32_t)key);
                S.chosen[tid] = u;
                if (I.nseg > 1) {              // only in single-instance launches
                    S.ent_beg[tid] = 0;        // the segment table follows (wave 0)
                } else {
                    const int64_t beg = global(I.inv_off)[u];
                    S.ent_beg[tid] = beg;
                    cnt = global(I.inv_off)[u + 1] - beg;
                }
                if (blockIdx.x == 0) {
                    // u leaves the candidates now: its own counter is never decremented
                    // (every set holding it is covered in this round, and the cover step
                    // skips it), so the next argmax sees -1
                    st_co(global(I.seeds) + round, u);
                    st_co(global(I.h) + u, -1);
                    if (I.part_n > 0) atomic_add_agent(global(I.taken) + u / I.part_n, 1);
                }
            }
        }
        if (solo && tid == 0) {                         // one instance: no scan needed
            S.ent_pre[0] = 0;
            S.ent_pre[1] = cnt;
        }
        if (!__syncthreads_or(live)) return;            // every instance finished or stopped
        if (solo && inst[0].nseg > 1) seg_ranges(S, inst[0]);
        if (!solo) block_excl_scan_i64(cnt, S.ent_pre, S.wsum);
        const int64_t nent = S.ent_pre[ninst];
        // a dense round: a single instance in hot mode with a large gain (uniform: every block
        // holds the same key)
        const bool dense = dense_ok && thr != kHotOff && S.key != 0 && nent <= 65535ll * gridDim.x &&
                           (int64_t)(S.key >> 32) - 1 >= (int64_t)inst[0].dense_gain;
        if (dense) {
            for (int i = tid; i < hot_total; i += kCoopBlock) S.u.dense[i] = 0;
            __syncthreads();
        }
        // Block b takes entries [nent b / G, nent (b+1) / G) in batches of one per thread:
        // each thread tests and marks its entry's set, and the batch's newly covered sets
        // are decremented together.
        const int64_t e_lo = nent * (int64_t)blockIdx.x / gridDim.x;
        const int64_t e_hi = nent * ((int64_t)blockIdx.x + 1) / gridDim.x;
        const unsigned long long* hot_words = thr != kHotOff ? inst[0].hot_words : nullptr;
        unsigned long long mine = 0;
        int mine_inst = -1;
        for (int64_t eb = e_lo; eb < e_hi; eb += kCoopBlock) {
            const int64_t e = eb + tid;
            int li = -1;
            bool fresh = false;
            int64_t len = 0;
            const int32_t* mem = nullptr;
            if (e < e_hi) {
                int lo = 0, hi = ninst;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (S.ent_pre[mid] <= e) lo = mid; else hi = mid;
                }
                li = lo;
                const SelInst& I = inst[lo];
                uint32_t rel;
                if (I.nseg > 1) {
                    const int64_t q = e - S.ent_pre[lo];
                    int j = 0;
                    while (j + 1 < I.nseg && S.seg_pre[j + 1] <= q) ++j;
                    rel = global(I.seg_inv[j])[S.seg_beg[j] + (q - S.seg_pre[j])];
                } else {
                    rel = global(I.inv)[S.ent_beg[lo] + (e - S.ent_pre[lo])];
                }
                // the set's place is loaded together with its flag (most entries of late
                // rounds are covered already; the extra loads save a dependent latency)
                const int64_t st = global(I.rr_start)[I.first + rel];
                const int32_t ln = global(I.rr_len)[I.first + rel];
                fresh = ld_co(global(I.covered) + rel) == 0u;
                if (fresh) {
                    st_co(global(I.covered) + rel, 1u);
                    mem = I.ids + st;
                    len = ln;
                }
            }
            // covered counts per instance (an instance's entries are contiguous)
            uint64_t pending = ballot(fresh);
            while (pending) {
                const int x = __builtin_amdgcn_readlane(li, __ffsll((unsigned long long)pending) - 1);
                const uint64_t mx = ballot(fresh && li == x);
                if (x != mine_inst) {
                    if (mine && lane == 0) atomic_add_agent(global(inst[mine_inst].n_covered), mine);
                    mine = 0;
                    mine_inst = x;
                }
                mine += (unsigned long long)__popcll(mx);
                pending &= ~mx;
            }
            dec_batch(S, inst, len, mem, li, true, hot_words, dense);
        }
        if (mine && lane == 0) atomic_add_agent(global(inst[mine_inst].n_covered), mine);
        if (dense) {
            // the block's counts become its row of hot_part (every position, so no row needs
            // clearing), and the LDS table returns to its empty state
            __syncthreads();
            dense_store_row(S, inst[0], hot_total);
            __syncthreads();
            for (int i = tid; i < kDecSlots; i += kCoopBlock) {
                S.u.dc.key[i] = kDecEmpty;
                S.u.dc.cnt[i] = 0;
            }
        } else {
            dec_flush(S.u.dc, inst);
        }
        prev_dense = dense;
        if (!grid_sync(bar, epoch)) return;
    }
}

// One 1024-thread block per CU.  With this kernel's resources (about 141 KB of LDS and
// 128 VGPRs per lane, i.e. 4 waves per SIMD) one block per CU is also the most a CU can
// hold, so the grid is exactly the device's capacity and every block is resident while
// no other kernel occupies the CUs.
int select_coop_grid() {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus > 0 ? cus : 1;
}

int select_max_inst() { return kMaxInst; }

// Blocks of k_select_coop that the device can hold at once: its occupancy per CU times
// the CU count (0 if the runtime cannot tell).
static int select_coop_capacity() {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_select_coop, kCoopBlock, 0) != hipSuccess)
        return 0;
    return per_cu * cus;
}

// IMM_SELECT_LAUNCH=plain launches the same grid with an ordinary launch, for tools that
// do not handle cooperative launches (some profilers).  Either way a grid larger than the
// device can hold at once is refused before anything is launched: its blocks could not
// all reach the grid barrier.
static bool plain_launch() {
    static const bool plain = [] {
        const char* e = getenv("IMM_SELECT_LAUNCH");
        return e && strcmp(e, "plain") == 0;
    }();
    return plain;
}

hipError_t launch_select_coop(const SelInst* inst, int32_t ninst, int32_t maxk, GridBarrier* bar,
                              hipStream_t s, bool plain) {
    if (ninst < 1 || ninst > kMaxInst) return hipErrorInvalidValue;
    const int grid = select_coop_grid();
    const int capacity = select_coop_capacity();
    if (capacity < 1 || grid > capacity) return hipErrorCooperativeLaunchTooLarge;
    if (grid > kMaxCoopGrid) return hipErrorInvalidValue;
    if (plain || plain_launch()) {
        k_select_coop<<<grid, kCoopBlock, 0, s>>>(inst, ninst, maxk, bar);
        return hipGetLastError();
    }
    void* args[] = {(void*)&inst, (void*)&ninst, (void*)&maxk, (void*)&bar};
    return hipLaunchCooperativeKernel((const void*)k_select_coop, dim3(grid), dim3(kCoopBlock), args,
                                      0, s);
}

}  // namespace imm
