// Forward Monte-Carlo influence spread on the device (gIM Sec. II-C: E[I(S)] is the
// expected number of vertices reachable from S in an instance graph, estimated by
// simulating instances).  Used to score returned seed sets; not on the RR-set path.
//
// Draws (their own contract, independent of the RR sets'): in simulation j and round t,
//   IC : edge e (in-edge numbering) is kept iff word 0 of Philox(j, e, t, 4) < thr[e], or
//        thr[e] is saturated;
//   LT : vertex v keeps the first in-edge e with cum[e] above word 0 of Philox(j, v, t, 5)
//        (or saturated).  Because cum is non-decreasing within an in-list, e is that edge
//        iff e qualifies and its predecessor in v's list does not: one O(1) test per
//        examined out-edge, no search.
// A simulation's count is the number of vertices reached in at least one round.
//
// One 256-thread workgroup per simulation at a time (persistent, simulations pulled from a
// counter).  A round is a level-synchronous search over out-edges: the waves take frontier
// vertices one at a time from an LDS cursor and test their out-edges 64 at a time; reached
// vertices are admitted by a workgroup-scope test-and-set on the slot's bitmap and
// appended to its list in HBM.  Bitmaps are left clear by walking the lists.
#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace imm {

constexpr int kFwdBlock = 256;
constexpr uint32_t kDomainFwdIC = 4u, kDomainFwdLT = 5u;

// ---- out-edge lists (built once per graph) --------------------------------------------
__global__ void k_out_degree(int64_t m, const int32_t* __restrict__ src, uint32_t* __restrict__ deg) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(deg + src[e], 1u);
}

// One wave per vertex v: each in-edge (u -> v, e) goes to u's out-list.
__global__ void k_out_scatter(int32_t n, const VRec* __restrict__ vrec, const int32_t* __restrict__ src,
                              const int64_t* __restrict__ out_off, uint32_t* __restrict__ cursor,
                              int32_t* __restrict__ out_dst, uint32_t* __restrict__ out_eid) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t v = wave; v < n; v += nwaves) {
        const int64_t s = vrec[v].start;
        const uint32_t d = vrec[v].deg & kDegMask;
        for (uint32_t i = lane; i < d; i += kWave) {
            const int64_t e = s + i;
            const int32_t u = src[e];
            const uint32_t at = atomicAdd(cursor + u, 1u);
            out_dst[out_off[u] + at] = (int32_t)v;
            out_eid[out_off[u] + at] = (uint32_t)e;
        }
    }
}

hipError_t launch_out_degree(int64_t m, const int32_t* src, uint32_t* deg, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_out_degree<<<(unsigned)blocks, 256, 0, s>>>(m, src, deg);
    return hipGetLastError();
}

hipError_t launch_out_scatter(int32_t n, const VRec* vrec, const int32_t* src, const int64_t* out_off,
                              uint32_t* cursor, int32_t* out_dst, uint32_t* out_eid, hipStream_t s) {
    int64_t blocks = ((int64_t)n * kWave + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_out_scatter<<<(unsigned)blocks, 256, 0, s>>>(n, vrec, src, out_off, cursor, out_dst, out_eid);
    return hipGetLastError();
}

// ---- simulations ------------------------------------------------------------------------
__device__ __forceinline__ bool fwd_tas(uint32_t* vis, int32_t v) {
    const uint32_t bit = 1u << (v & 31);
    const uint32_t old = __hip_atomic_fetch_or(vis + (v >> 5), bit, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
    return (old & bit) == 0u;
}

__device__ __forceinline__ bool lt_qualifies(uint32_t c, uint32_t x) { return c == kAlways || x < c; }

__global__ __launch_bounds__(kFwdBlock) void k_spread_fwd(FwdLaunch L) {
    __shared__ int32_t s_size, s_next, s_count;
    __shared__ unsigned int s_j;
    const int tid = threadIdx.x, lane = lane_id();
    const int64_t slot = blockIdx.x;
    uint32_t* vis = L.vis + slot * L.vis_words;
    int32_t* list = L.list + slot * L.list_stride;
    uint32_t* uvis = L.rounds > 1 ? L.uvis + slot * L.vis_words : nullptr;
    int32_t* ulist = L.rounds > 1 ? L.ulist + slot * L.list_stride : nullptr;
    const IMM_GLOBAL uint32_t* w = global(L.w);
    const IMM_GLOBAL int64_t* out_off = global(L.out_off);
    const IMM_GLOBAL int32_t* out_dst = global(L.out_dst);
    const IMM_GLOBAL uint32_t* out_eid = global(L.out_eid);

    for (;;) {
        if (tid == 0) s_j = atomicAdd(L.work, 1u);
        __syncthreads();
        const unsigned int j = uniform(s_j);
        if ((int64_t)j >= L.sims) break;
        if (tid == 0) s_count = 0;
        for (int32_t t = 0; t < L.rounds; ++t) {
            if (tid == 0) s_size = 0;
            __syncthreads();
            for (int32_t i = tid; i < L.nelem; i += kFwdBlock) {
                const int32_t el = L.elems[i];
                if (el / L.n != t) continue;
                const int32_t u = el - t * L.n;
                if (fwd_tas(vis, u)) list[atomicAdd(&s_size, 1)] = u;
            }
            __syncthreads();
            int32_t head = 0;
            for (;;) {
                const int32_t end = uniform(s_size);
                if (head >= end) break;
                if (tid == 0) s_next = head;
                __syncthreads();
                for (;;) {
                    int32_t idx = 0;
                    if (lane == 0) idx = atomicAdd(&s_next, 1);
                    idx = __shfl(idx, 0, kWave);
                    if (idx >= end) break;
                    const int32_t u = list[idx];
                    const int64_t oo = out_off[u], oe = out_off[u + 1];
                    for (int64_t a0 = oo; a0 < oe; a0 += kWave) {
                        const int64_t a = a0 + lane;
                        bool fresh = false;
                        int32_t v = 0;
                        if (a < oe) {
                            v = out_dst[a];
                            const uint32_t e = out_eid[a];
                            bool live;
                            if (L.model == 0) {
                                const uint32_t x = philox10(Ctr4{j, e, (uint32_t)t, kDomainFwdIC}, L.k0, L.k1).x;
                                const uint32_t th = w[e];
                                live = th == kAlways || x < th;
                            } else {
                                const uint32_t x = philox10(Ctr4{j, (uint32_t)v, (uint32_t)t, kDomainFwdLT}, L.k0, L.k1).x;
                                live = lt_qualifies(w[e], x) &&
                                       ((int64_t)e == L.vrec[v].start || !lt_qualifies(w[e - 1], x));
                            }
                            if (live) fresh = fwd_tas(vis, v);
                        }
                        const uint64_t m = ballot(fresh);
                        if (m) {
                            int32_t at = 0;
                            if (lane == 0) at = atomicAdd(&s_size, (int32_t)__popcll(m));
                            at = __shfl(at, 0, kWave);
                            if (fresh) list[at + (int32_t)lanes_below(m)] = v;
                        }
                    }
                }
                __syncthreads();
                head = end;
            }
            const int32_t size = uniform(s_size);
            // this round's reach: counted (once over the rounds) and the bitmap cleared
            for (int32_t i = tid; i < size; i += kFwdBlock) {
                const int32_t v = list[i];
                if (uvis) {
                    if (fwd_tas(uvis, v)) ulist[atomicAdd(&s_count, 1)] = v;
                }
                vis[v >> 5] = 0u;
            }
            if (!uvis && tid == 0) s_count = size;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __syncthreads();
        }
        const int32_t count = uniform(s_count);
        if (uvis)
            for (int32_t i = tid; i < count; i += kFwdBlock) uvis[ulist[i] >> 5] = 0u;
        if (tid == 0) {
            L.counts[j] = (uint32_t)count;
            if (L.sums) {
                atomic_add_agent(L.sums, (unsigned long long)count);
                atomic_add_agent(L.sums + 1, (unsigned long long)count * (unsigned long long)count);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __syncthreads();
    }
}

hipError_t launch_spread_fwd(const FwdLaunch& a, int grid, hipStream_t s) {
    k_spread_fwd<<<grid, kFwdBlock, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace imm
