// Random RR-set generation on gfx950.
//
// IC (gIM Sec. II-E, Alg. 3-6): RR set r is every vertex that reaches root(r) in the
// live-edge instance drawn for r.  We enumerate it by a breadth-first search over in-edges
// in which every in-edge of an expanded vertex is tested once against its own Philox draw,
// and a visited test-and-set admits each vertex once (the duplicate-frontier hazard of gIM
// Sec. III-A).  Because each edge's draw is keyed by (r, e), the set does not depend on the
// order of expansion, so a whole wave can expand many frontier vertices at once.
//
// LT (gIM Sec. III-G): RR set r is the reverse walk from root(r) in which each vertex picks
// at most one in-edge (the first cumulative threshold above its draw) and the walk stops
// at a vertex with no in-edge, no pick, or a pick already on the walk.
//
// Launch shape (persistent, gIM Alg. 6 / Eq. 5 analogue): a grid sized to fill every CU;
// each wave pulls RR indices from an atomic work counter until the range is exhausted.
// Members of the current set live in an on-chip (LDS) list of kListCap entries; a set that
// outgrows it is abandoned and deferred to the big-set launch, which keeps member lists in
// HBM (the role of gIM's reservoir queue Q_res, Sec. III-C).  Finished sets are placed in
// the pool's id buffer at an atomically reserved offset (gIM Alg. 6's tail_RR), and the
// pool's occurrence counts are incremented for each member (gIM Sec. III-B, Occur).
#include "kernels.hpp"

namespace imm {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kListCap = 2048;

int rr_small_capacity() { return kListCap; }

struct FrontierLds {
    int32_t pre[kWave + 1];   // exclusive prefix of 4-edge group counts of the batch
    int64_t start[kWave];     // first in-edge of each batch vertex
    uint32_t deg[kWave];      // in-degree | uniform bit
    uint32_t thr[kWave];      // common threshold when uniform
};

template <bool kBig>
struct WaveLds {
    FrontierLds f;
    int32_t list[kBig ? 1 : kListCap];
};

__device__ __forceinline__ void vis_clear(uint32_t* vis, int32_t v) { vis[v >> 5] = 0u; }

__device__ __forceinline__ bool vis_test_and_set(uint32_t* vis, int32_t v) {
    const uint32_t bit = 1u << (v & 31);
    uint32_t old = __hip_atomic_fetch_or(vis + (v >> 5), bit, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return (old & bit) == 0u;
}

// Pull the next RR index of this launch (uniform across the wave); false when done.
__device__ __forceinline__ bool next_index(const GenArgs& a, uint32_t& r) {
    unsigned long long i = 0;
    if (lane_id() == 0) i = atomic_add_agent(&a.ctr->work, 1ull);
    i = uniform64(i);
    if ((int64_t)i >= a.count) return false;
    r = a.list ? a.list[i] : (uint32_t)(a.first + (int64_t)i);
    r = uniform(r);
    return true;
}

// Place a finished set: reserve space, copy members, count occurrences.  Returns false
// when the id buffer is full (the index is queued for a retry after the host grows it).
__device__ bool place_set(const GenArgs& a, uint32_t r, const int32_t* list, int32_t size,
                          uint64_t examined) {
    const int lane = lane_id();
    unsigned long long base = 0;
    if (lane == 0) base = atomic_add_agent(&a.ctr->tail, (unsigned long long)size);
    base = uniform64(base);
    if ((int64_t)(base + (unsigned long long)size) > a.cap_ids) {
        if (lane == 0) {
            unsigned int at = atomic_add_agent(&a.ctr->n_capacity, 1u);
            a.cap_list[at] = r;
        }
        return false;
    }
    for (int32_t i = lane; i < size; i += kWave) {
        int32_t v = list[i];
        a.ids[base + i] = v;
        __hip_atomic_fetch_add(a.hist + v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
        a.rr_start[r] = (int64_t)base;
        a.rr_len[r] = size;
        atomic_add_agent(&a.ctr->placed, (unsigned long long)size);
        atomic_add_agent(&a.ctr->edges, (unsigned long long)examined);
    }
    return true;
}

__device__ __forceinline__ void defer_overflow(const GenArgs& a, uint32_t r) {
    if (lane_id() == 0) {
        unsigned int at = atomic_add_agent(&a.ctr->n_overflow, 1u);
        a.ovf_list[at] = r;
    }
}

// ------------------------------------------------------------------------------------
// IC
// ------------------------------------------------------------------------------------
template <bool kBig>
__global__ __launch_bounds__(kBlock) void k_rr_ic(GenArgs a) {
    __shared__ WaveLds<kBig> lds_all[kWavesPerBlock];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    WaveLds<kBig>& L = lds_all[wib];
    const int64_t slot = (int64_t)blockIdx.x * kWavesPerBlock + wib;
    uint32_t* vis = a.visited + slot * a.vis_words;
    int32_t* list = kBig ? a.big_list + slot * (int64_t)a.n : L.list;
    const int32_t cap = kBig ? a.n : kListCap;
    const uint32_t k0 = a.k0, k1 = a.k1;

    uint32_t r;
    while (next_index(a, r)) {
        const int32_t root = (int32_t)root_of(r, (uint32_t)a.n, k0, k1);
        if (lane == 0) {
            list[0] = root;
            vis_test_and_set(vis, root);
        }
        int32_t size = 1, head = 0;
        uint64_t examined = 0;
        bool overflow = false;
        if (kBig) __threadfence(); else wave_sync();

        while (head < size && !overflow) {
            const int32_t nb = min(size - head, kWave);
            // -- batch of up to 64 frontier vertices: their in-edge groups, flattened --
            int32_t ng = 0;
            uint32_t dg = 0;
            if (lane < nb) {
                const int32_t v = list[head + lane];
                const VRec rec = a.vrec[v];
                dg = rec.deg & kDegMask;
                if (dg) ng = (int32_t)(((rec.start + dg - 1) >> 2) - (rec.start >> 2) + 1);
                L.f.start[lane] = rec.start;
                L.f.deg[lane] = rec.deg;
                L.f.thr[lane] = rec.thr;
            }
            const int32_t incl = wave_incl_scan(ng);
            if (lane < nb) L.f.pre[lane] = incl - ng;
            if (lane == nb - 1) L.f.pre[nb] = incl;
            const int32_t total = __shfl(incl, nb - 1, kWave);
            examined += (uint64_t)wave_sum((uint64_t)dg);
            wave_sync();

            for (int32_t base = 0; base < total && !overflow; base += kWave) {
                const int32_t q = base + lane;
                int32_t w[4] = {0, 0, 0, 0};
                bool fresh[4] = {false, false, false, false};
                if (q < total) {
                    int32_t lo = 0, hi = nb;   // pre[lo] <= q < pre[hi]
                    while (hi - lo > 1) {
                        const int32_t mid = (lo + hi) >> 1;
                        if (L.f.pre[mid] <= q) lo = mid; else hi = mid;
                    }
                    const int64_t s = L.f.start[lo];
                    const uint32_t dd = L.f.deg[lo];
                    const int64_t e_end = s + (dd & kDegMask);
                    const uint32_t g = (uint32_t)((s >> 2) + (q - L.f.pre[lo]));
                    const int64_t e0 = (int64_t)g << 2;
                    const Ctr4 x = philox10(Ctr4{r, g, 0u, kDomainIC}, k0, k1);
                    uint32_t t[4];
                    if (dd & kUniformBit) {
                        t[0] = t[1] = t[2] = t[3] = L.f.thr[lo];
                    } else {
                        const uint4 tv = *reinterpret_cast<const uint4*>(a.thr + e0);
                        t[0] = tv.x; t[1] = tv.y; t[2] = tv.z; t[3] = tv.w;
                    }
                    const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int64_t e = e0 + j;
                        const bool live = e >= s && e < e_end && (t[j] == kAlways || xs[j] < t[j]);
                        if (live) {
                            w[j] = a.src[e];
                            fresh[j] = vis_test_and_set(vis, w[j]);
                        }
                    }
                }
                // -- append the newly reached vertices (ballot + prefix count) --
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint64_t mask = ballot(fresh[j]);
                    const int32_t cnt = (int32_t)__popcll(mask);
                    if (cnt == 0) continue;
                    if (overflow || size + cnt > cap) {
                        overflow = true;
                        if (fresh[j]) vis_clear(vis, w[j]);
                        continue;
                    }
                    if (fresh[j]) list[size + (int32_t)lanes_below(mask)] = w[j];
                    size += cnt;
                }
                if (kBig) __threadfence(); else wave_sync();
            }
            head += nb;
        }

        bool placed = false;
        if (!overflow) placed = place_set(a, r, list, size, examined);
        else defer_overflow(a, r);
        (void)placed;
        for (int32_t i = lane; i < size; i += kWave) vis_clear(vis, list[i]);
        __threadfence();
    }
}

// ------------------------------------------------------------------------------------
// LT: reverse walk.  The wave finds the chosen in-edge of the current vertex: for short
// in-lists one coalesced load and a ballot; for long ones a 64-ary search over the
// non-decreasing cumulative thresholds.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ bool lt_hit(const GenArgs& a, int64_t j, uint32_t x) {
    const uint32_t c = a.cum[j];
    return c > x || c == kAlways;
}

// First j in [s, e) whose cumulative threshold is above the draw (a saturated entry always
// qualifies), or -1.  The predicate is monotone in j because cum is non-decreasing within
// an in-list, so a 64-ary search narrows [lo, hi) by a factor of 65 per step.
__device__ __forceinline__ int64_t lt_pick(const GenArgs& a, int64_t s, int64_t e, uint32_t x) {
    const int lane = lane_id();
    int64_t lo = s, hi = e;      // the answer lies in [lo, hi]; hi is a hit iff hi_hit
    bool hi_hit = false;
    while (hi - lo > kWave) {
        const int64_t span = hi - lo;
        const int64_t pos = lo + (span * (lane + 1)) / (kWave + 1);
        const uint64_t m = ballot(lt_hit(a, pos, x));
        if (m == 0) {
            lo = (int64_t)uniform64((uint64_t)__shfl(pos, kWave - 1, kWave)) + 1;
        } else {
            const int f = __ffsll((unsigned long long)m) - 1;
            const int64_t p_hit = (int64_t)uniform64((uint64_t)__shfl(pos, f, kWave));
            const int64_t p_miss = (int64_t)uniform64((uint64_t)__shfl(pos, f > 0 ? f - 1 : 0, kWave));
            hi = p_hit;
            hi_hit = true;
            if (f > 0) lo = p_miss + 1;
        }
    }
    const int64_t j = lo + lane;
    const uint64_t m = ballot(j < hi && lt_hit(a, j, x));
    if (m != 0) return lo + (__ffsll((unsigned long long)m) - 1);
    return hi_hit ? hi : -1;
}

template <bool kBig>
__global__ __launch_bounds__(kBlock) void k_rr_lt(GenArgs a) {
    __shared__ WaveLds<kBig> lds_all[kWavesPerBlock];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    WaveLds<kBig>& L = lds_all[wib];
    const int64_t slot = (int64_t)blockIdx.x * kWavesPerBlock + wib;
    uint32_t* vis = a.visited + slot * a.vis_words;
    int32_t* list = kBig ? a.big_list + slot * (int64_t)a.n : L.list;
    const int32_t cap = kBig ? a.n : kListCap;
    const uint32_t k0 = a.k0, k1 = a.k1;

    uint32_t r;
    while (next_index(a, r)) {
        int32_t v = (int32_t)root_of(r, (uint32_t)a.n, k0, k1);
        if (lane == 0) {
            list[0] = v;
            vis_test_and_set(vis, v);
        }
        int32_t size = 1;
        uint64_t examined = 0;
        bool overflow = false;
        if (kBig) __threadfence(); else wave_sync();
        for (;;) {
            const VRec rec = a.vrec[v];
            const uint32_t d = rec.deg & kDegMask;
            if (d == 0) break;
            examined += d;
            const uint32_t x = philox10(Ctr4{r, (uint32_t)v, 0u, kDomainLT}, k0, k1).x;
            const int64_t j = lt_pick(a, rec.start, rec.start + d, x);
            if (j < 0) break;
            const int32_t u = a.src[j];
            bool fresh = false;
            if (lane == 0) fresh = vis_test_and_set(vis, u);
            fresh = __shfl(fresh, 0, kWave);
            if (!fresh) break;
            if (size + 1 > cap) {
                overflow = true;
                if (lane == 0) vis_clear(vis, u);
                break;
            }
            if (lane == 0) list[size] = u;
            ++size;
            v = u;
            if (kBig) __threadfence(); else wave_sync();
        }
        if (kBig) __threadfence(); else wave_sync();
        if (!overflow) place_set(a, r, list, size, examined);
        else defer_overflow(a, r);
        for (int32_t i = lane; i < size; i += kWave) vis_clear(vis, list[i]);
        __threadfence();
    }
}

hipError_t launch_rr_ic(const GenArgs& a, bool big, int grid, hipStream_t s) {
    if (big) k_rr_ic<true><<<grid, kBlock, 0, s>>>(a);
    else k_rr_ic<false><<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_rr_lt(const GenArgs& a, bool big, int grid, hipStream_t s) {
    if (big) k_rr_lt<true><<<grid, kBlock, 0, s>>>(a);
    else k_rr_lt<false><<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

int rr_blocks_per_cu(bool lt, bool big) {
    int nb = 0;
    hipError_t e;
    if (lt) e = big ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rr_lt<true>, kBlock, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rr_lt<false>, kBlock, 0);
    else e = big ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rr_ic<true>, kBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rr_ic<false>, kBlock, 0);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

// ------------------------------------------------------------------------------------
// Export helpers: per-set sizes, and a canonical (sorted) copy of each set.
// ------------------------------------------------------------------------------------
__global__ void k_set_sizes(const int32_t* __restrict__ rr_len, int64_t first, int64_t count,
                            int64_t* __restrict__ sizes) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        sizes[i] = rr_len[first + i];
}

hipError_t launch_set_sizes(const int32_t* rr_len, int64_t first, int64_t count, int64_t* sizes,
                            hipStream_t s) {
    if (count == 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_set_sizes<<<(unsigned)blocks, 256, 0, s>>>(rr_len, first, count, sizes);
    return hipGetLastError();
}

// One wave per set: copy members, then sort them in place by rank counting (each member's
// position is the number of members smaller than it; members are distinct).
__global__ void k_gather_sets(const int64_t* __restrict__ rr_start, const int32_t* __restrict__ rr_len,
                              int64_t first, int64_t count, const int64_t* __restrict__ out_off,
                              const int32_t* __restrict__ ids, int32_t* __restrict__ out) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t i = wave; i < count; i += nwaves) {
        const int64_t src = rr_start[first + i];
        const int32_t len = rr_len[first + i];
        const int64_t dst = out_off[i];
        for (int32_t a = lane; a < len; a += kWave) {
            const int32_t v = ids[src + a];
            int32_t rank = 0;
            for (int32_t b = 0; b < len; ++b) rank += ids[src + b] < v;
            out[dst + rank] = v;
        }
    }
}

hipError_t launch_gather_sets(const int64_t* rr_start, const int32_t* rr_len, int64_t first,
                              int64_t count, const int64_t* out_off, const int32_t* ids,
                              int32_t* out_ids, hipStream_t s) {
    if (count == 0) return hipSuccess;
    int64_t blocks = (count * kWave + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_gather_sets<<<(unsigned)blocks, 256, 0, s>>>(rr_start, rr_len, first, count, out_off, ids,
                                                   out_ids);
    return hipGetLastError();
}

}  // namespace imm
