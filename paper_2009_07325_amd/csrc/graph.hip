// Graph upload checks and threshold encodings (run once per graph, on the device).
//
// IC (gIM Sec. II-B; Alg. 3 tests "p < p_uv"): edge e is live for RR set r when its 32-bit
// draw x satisfies x < floor(p_e * 2^32); p = 1 saturates to kAlways ("always live").
// For a float32 p, p * 2^32 is exact in double, so the floor is exact.
// LT (gIM Sec. II-B Eq. 1, Sec. III-G): a vertex activates through at most one in-edge,
// edge j with probability w_j / sum(w).  We store the scaled prefix sums
// floor(S_j * 2^32 / T) and saturate the last one, so the first entry above a uniform
// draw names the chosen in-edge.
#include "kernels.hpp"

namespace imm {

__global__ void k_validate_off(int32_t n, int64_t m, const int64_t* __restrict__ off,
                               uint32_t* err) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    bool bad = false;
    if (v == 0 && off[0] != 0) bad = true;
    if (v == n && off[n] != m) bad = true;
    if (v < n && off[v + 1] < off[v]) bad = true;
    if (bad) atomicOr(err, 1u);
}

__global__ void k_validate_edges(int32_t n, int64_t m, const int32_t* __restrict__ src,
                                 const float* __restrict__ p, const uint32_t* __restrict__ w,
                                 uint32_t* err) {
    uint32_t bits = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = src[e];
        if (s < 0 || s >= n) bits |= 2u;
        if (p) {
            float q = p[e];
            if (!(q >= 0.0f && q <= 1.0f)) bits |= 4u;
        }
        if (w && w[e] == 0u) bits |= 8u;
    }
    if (bits) atomicOr(err, bits);
}

hipError_t launch_validate(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                           const float* ic_p, const uint32_t* lt_w, uint32_t* err,
                           hipStream_t s) {
    k_validate_off<<<(unsigned)((n + 1 + 255) / 256), 256, 0, s>>>(n, m, in_off, err);
    if (m > 0) {
        int64_t blocks = (m + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        k_validate_edges<<<(unsigned)blocks, 256, 0, s>>>(n, m, in_src, ic_p, lt_w, err);
    }
    return hipGetLastError();
}

__global__ void k_encode_ic(int64_t m, const float* __restrict__ p, uint32_t* __restrict__ thr) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        double t = floor((double)p[e] * 4294967296.0);
        thr[e] = t >= 4294967296.0 ? kAlways : (uint32_t)t;
    }
}

hipError_t launch_encode_ic(int64_t m, const float* p, uint32_t* thr, hipStream_t s) {
    if (m == 0) return hipSuccess;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_encode_ic<<<(unsigned)blocks, 256, 0, s>>>(m, p, thr);
    return hipGetLastError();
}

// One wave per vertex: record (start, degree) and detect a common IC threshold.
__global__ void k_build_vrec(int32_t n, const int64_t* __restrict__ off,
                             const uint32_t* __restrict__ thr, VRec* __restrict__ vrec,
                             unsigned int* n_mixed) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t v = wave; v < n; v += nwaves) {
        int64_t s = off[v], e = off[v + 1];
        uint32_t deg = (uint32_t)(e - s);
        bool uniform = thr != nullptr;
        uint32_t t0 = 0;
        if (thr && e > s) {
            t0 = thr[s];
            bool same = true;
            for (int64_t j = s + lane; j < e; j += kWave) same &= thr[j] == t0;
            uniform = ballot(!same) == 0;
        }
        if (lane == 0) {
            VRec rec;
            rec.start = s;
            rec.deg = deg | (uniform ? kUniformBit : 0u);
            rec.thr = t0;
            vrec[v] = rec;
            if (!uniform && thr) atomicAdd(n_mixed, 1u);
        }
    }
}

hipError_t launch_build_vrec(int32_t n, const int64_t* in_off, const uint32_t* thr, VRec* vrec,
                             unsigned int* n_mixed, hipStream_t s) {
    int64_t blocks = ((int64_t)n * kWave + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_build_vrec<<<(unsigned)blocks, 256, 0, s>>>(n, in_off, thr, vrec, n_mixed);
    return hipGetLastError();
}

// floor(num * 2^32 / den) for num < den < 2^63, by 32 steps of restoring binary division.
__device__ __forceinline__ uint32_t scaled_ratio(uint64_t num, uint64_t den) {
    uint64_t rem = num;
    uint32_t q = 0;
    for (int i = 0; i < 32; ++i) {
        rem <<= 1;
        q <<= 1;
        if (rem >= den) {
            rem -= den;
            q |= 1u;
        }
    }
    return q;
}

// One wave per vertex: total weight by a wave reduction, then the scaled prefix sums
// chunk by chunk (64 edges per step, a wave scan per chunk).
__global__ void k_encode_lt(int32_t n, const int64_t* __restrict__ off,
                            const uint32_t* __restrict__ w, uint32_t* __restrict__ cum) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t v = wave; v < n; v += nwaves) {
        const int64_t s = off[v], e = off[v + 1];
        if (e == s) continue;
        uint64_t part = 0;
        for (int64_t j = s + lane; j < e; j += kWave) part += w ? (uint64_t)w[j] : 1ull;
        const uint64_t total = wave_sum(part);
        uint64_t carry = 0;
        for (int64_t base = s; base < e; base += kWave) {
            const int64_t j = base + lane;
            uint64_t wj = (j < e) ? (w ? (uint64_t)w[j] : 1ull) : 0ull;
            uint64_t incl = wave_incl_scan(wj) + carry;
            if (j < e) cum[j] = (j == e - 1) ? kAlways : scaled_ratio(incl, total);
            carry = __shfl(incl, kWave - 1, kWave);
        }
    }
}

hipError_t launch_encode_lt(int32_t n, const int64_t* in_off, const uint32_t* w, uint32_t* cum,
                            hipStream_t s) {
    int64_t blocks = ((int64_t)n * kWave + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_encode_lt<<<(unsigned)blocks, 256, 0, s>>>(n, in_off, w, cum);
    return hipGetLastError();
}

// ---- LT walk tables ---------------------------------------------------------------------
// The pick of a walk step is the first in-edge of v whose cumulative threshold exceeds the
// draw x (gIM Sec. III-G).  Instead of searching v's list, the walk looks its answer up in
// a guide table (the inverse-CDF guide of Chen and Asau, 1974): v's 2d buckets split the
// draws [0, 2^32) evenly, bucket b starting at L_b = ceil(b 2^32 / 2d), and the guide of b
// is the first edge whose threshold exceeds L_b.  Every x of bucket b has its pick at or
// after that edge (thresholds are non-decreasing), and it is that edge unless a threshold
// falls inside the bucket, so the walk reads one guide entry and, rarely, the edges after
// it: the same pick as the search, in about one dependent load.  The guide entries of v
// sit at [2 start_v, 2 start_v + 2d), each holding the edge record of its edge and, in a
// parallel array, the edge's position in v's list.

// lrec[e] = (cum[e], src[e], range of src)
__global__ void k_build_lrec(int64_t m, const uint32_t* __restrict__ cum, const int32_t* __restrict__ src,
                             const VRec* __restrict__ vrec, LtRec* __restrict__ lrec) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = src[e];
        const VRec r = vrec[u];
        lrec[e] = LtRec{cum[e], u, (uint32_t)r.start, r.deg & kDegMask};
    }
}

// One wave per vertex, lanes over its in-edges.  The guide of bucket b is the first edge j
// with cum_j > L_b (a saturated threshold counts as 2^32); bucket b's 32-byte slot holds
// edge j's record and then edge j+1's (j's again for the last edge), since a draw that
// passes cum_j inside the bucket most often picks j+1, which then costs a load from the
// same cache line rather than a second dependent one.  Edge j is the edge with
// cum_{j-1} <= L_b < cum_j, so edge j is the guide of exactly the buckets whose lower end
// lies in [cum_{j-1}, cum_j): b in [first(cum_{j-1}), first(cum_j)), where first(c), the
// smallest b with L_b >= c, is 0 for c = 0 and floor((c - 1) 2d / 2^32) + 1 otherwise
// (ceil(y) >= c iff y > c - 1).  Each edge writes its own buckets: O(d) per vertex.
__device__ __forceinline__ uint64_t first_bucket(uint64_t c, uint64_t nb) {
    return c == 0 ? 0 : (((c - 1) * nb) >> 32) + 1;
}

__global__ void k_build_guide(int32_t n, const VRec* __restrict__ vrec, const uint32_t* __restrict__ cum,
                              const LtRec* __restrict__ lrec, LtRec* __restrict__ grec,
                              uint32_t* __restrict__ gidx) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t v = wave; v < n; v += nwaves) {
        const int64_t s = vrec[v].start;
        const uint32_t d = vrec[v].deg & kDegMask;
        const uint64_t nb = 2ull * d;
        for (uint32_t j = lane; j < d; j += kWave) {
            const uint32_t cj = cum[s + j];
            const uint64_t hi_c = cj == kAlways ? (1ull << 32) : (uint64_t)cj;
            uint64_t lo_c = 0;
            if (j > 0) {
                const uint32_t cp = cum[s + j - 1];
                lo_c = cp == kAlways ? (1ull << 32) : (uint64_t)cp;
            }
            const uint64_t b_lo = first_bucket(lo_c, nb);
            const uint64_t b_hi = min(first_bucket(hi_c, nb), nb);
            if (b_lo >= b_hi) continue;
            const LtRec rec = lrec[s + j];
            const LtRec nxt = j + 1 < d ? lrec[s + j + 1] : rec;
            for (uint64_t b = b_lo; b < b_hi; ++b) {
                grec[2 * (2 * s + (int64_t)b)] = rec;
                grec[2 * (2 * s + (int64_t)b) + 1] = nxt;
                gidx[2 * s + (int64_t)b] = j;
            }
        }
    }
}

hipError_t launch_build_lt_tables(int32_t n, int64_t m, const uint32_t* cum, const int32_t* src,
                                  const VRec* vrec, LtRec* lrec, LtRec* grec, uint32_t* gidx,
                                  hipStream_t s) {
    if (m > 0) {
        int64_t blocks = (m + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        k_build_lrec<<<(unsigned)blocks, 256, 0, s>>>(m, cum, src, vrec, lrec);
    }
    int64_t blocks = ((int64_t)n * kWave + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_build_guide<<<(unsigned)blocks, 256, 0, s>>>(n, vrec, cum, lrec, grec, gidx);
    return hipGetLastError();
}

}  // namespace imm
