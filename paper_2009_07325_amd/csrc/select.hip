// Greedy maximum coverage on the device (gIM Alg. 1 lines 6-10, Sec. III-H, Alg. 7).
//
// Per selection call over RR sets [first, first+count):
//   1. h[v]   = number of those sets containing v (Occur, gIM Sec. III-B), as int32;
//   2. an inverted index vertex -> RR indices (counting sort: scan of h, then scatter);
//   3. k rounds of
//        argmax  : u = the vertex outside S with the largest h, smallest id among equals
//                  (gIM Sec. III-H: a max reduction over Occur);
//        cover   : every set containing u that is not yet covered is flagged and each of
//                  its members' counters is decremented (gIM Alg. 7), using the inverted
//                  index so that a round touches only the sets that contain u.
// Integer decrements commute, so counters, seeds and the covered count are the same for
// any schedule.
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
        return hipMemsetAsync(out, 0, sizeof(int64_t), s);
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
__global__ void k_inv_scatter(const int64_t* __restrict__ rr_start, const int32_t* __restrict__ rr_len,
                              const int32_t* __restrict__ ids, int64_t first, int64_t count,
                              const int64_t* __restrict__ inv_off, uint32_t* __restrict__ cursor,
                              uint32_t* __restrict__ inv) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t i = wave; i < count; i += nwaves) {
        const int64_t s = rr_start[first + i];
        const int32_t len = rr_len[first + i];
        for (int32_t j = lane; j < len; j += kWave) {
            const int32_t v = ids[s + j];
            const uint32_t at = atomic_add_agent(cursor + v, 1u);
            inv[inv_off[v] + at] = (uint32_t)i;
        }
    }
}

hipError_t launch_inv_scatter(const int64_t* rr_start, const int32_t* rr_len, const int32_t* ids,
                              int64_t first, int64_t count, const int64_t* inv_off,
                              uint32_t* cursor, uint32_t* inv, hipStream_t s) {
    if (count == 0) return hipSuccess;
    int64_t blocks = (count * kWave + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_inv_scatter<<<(unsigned)blocks, 256, 0, s>>>(rr_start, rr_len, ids, first, count, inv_off,
                                                   cursor, inv);
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

// ---- argmax over the counters ---------------------------------------------------------
// key(v) = (h[v] + 1) << 32 | (2^32 - 1 - v): the largest key has the largest count and,
// among equal counts, the smallest id.  Selected vertices hold h = -1 (key high part 0),
// so any unselected vertex beats them.  The vertex chosen in the previous round is set to
// -1 here, after its cover kernel has finished.
constexpr int kArgBlock = 256;

__global__ __launch_bounds__(kArgBlock) void k_argmax(int32_t* __restrict__ h, int32_t n, int32_t round,
                                                      const int32_t* __restrict__ seeds,
                                                      unsigned long long* __restrict__ keys) {
    __shared__ unsigned long long sh[kArgBlock / kWave];
    const int32_t prev = round > 0 ? seeds[round - 1] : -1;
    unsigned long long best = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t c = h[i];
        if ((int32_t)i == prev) {
            h[i] = -1;
            c = -1;
        }
        if (c >= 0) {
            const unsigned long long key = ((unsigned long long)(uint32_t)(c + 1) << 32) |
                                           (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
            best = key > best ? key : best;
        }
    }
    best = wave_max_u64(best);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kArgBlock / kWave; ++w) best = sh[w] > best ? sh[w] : best;
        if (best) __hip_atomic_fetch_max(keys + round, best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t launch_argmax(int32_t* h, int32_t n, int32_t round, const int32_t* seeds,
                         unsigned long long* keys, hipStream_t s) {
    int64_t blocks = ((int64_t)n + kArgBlock * 4 - 1) / (kArgBlock * 4);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    k_argmax<<<(unsigned)blocks, kArgBlock, 0, s>>>(h, n, round, seeds, keys);
    return hipGetLastError();
}

// ---- cover: flag the sets containing u, decrement their members' counters -----------
__global__ __launch_bounds__(256) void k_cover(const unsigned long long* __restrict__ keys, int32_t round,
                                               const int64_t* __restrict__ inv_off,
                                               const uint32_t* __restrict__ inv,
                                               const int64_t* __restrict__ rr_start,
                                               const int32_t* __restrict__ rr_len,
                                               const int32_t* __restrict__ ids, int64_t first,
                                               uint8_t* __restrict__ covered, int32_t* __restrict__ h,
                                               int32_t* __restrict__ seeds,
                                               unsigned long long* __restrict__ n_covered) {
    const int lane = lane_id();
    const unsigned long long key = keys[round];
    const int32_t u = (int32_t)(0xFFFFFFFFu - (uint32_t)key);
    if (blockIdx.x == 0 && threadIdx.x == 0) seeds[round] = u;
    const int64_t b = inv_off[u], e = inv_off[u + 1];
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    unsigned long long mine = 0;
    for (int64_t j = b + wave; j < e; j += nwaves) {
        const uint32_t rel = inv[j];
        if (covered[rel]) continue;          // uniform across the wave
        wave_sync();
        if (lane == 0) covered[rel] = 1;
        ++mine;
        const int64_t s = rr_start[first + rel];
        const int32_t len = rr_len[first + rel];
        for (int32_t t = lane; t < len; t += kWave)
            __hip_atomic_fetch_add(h + ids[s + t], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0 && mine) atomic_add_agent(n_covered, mine);
}

hipError_t launch_cover(const unsigned long long* keys, int32_t round, const int64_t* inv_off,
                        const uint32_t* inv, const int64_t* rr_start, const int32_t* rr_len,
                        const int32_t* ids, int64_t first, uint8_t* covered, int32_t* h,
                        int32_t* seeds, unsigned long long* n_covered, hipStream_t s) {
    k_cover<<<1024, 256, 0, s>>>(keys, round, inv_off, inv, rr_start, rr_len, ids, first, covered,
                                 h, seeds, n_covered);
    return hipGetLastError();
}

}  // namespace imm
