// Random RR-set generation on gfx950.
//
// IC (gIM Sec. II-E, Alg. 3-6): RR set r is every vertex that reaches root(r) in the
// live-edge instance drawn for r.  We enumerate it breadth-first over in-edges, testing
// every in-edge of an expanded vertex once against its own Philox draw; a visited
// test-and-set admits each vertex once (the duplicate-frontier hazard of gIM Sec. III-A).
// Draws are keyed by (r, e), so the set does not depend on the order of expansion: a wave
// expands up to 64 frontier vertices at once, their in-edges flattened into aligned 4-edge
// groups, one Philox4x32-10 call per lane per group.
//
// LT (gIM Sec. III-G): RR set r is the reverse walk from root(r) in which each vertex picks
// at most one in-edge (the first cumulative threshold above its draw); the walk stops at a
// vertex with no in-edge, no pick, or a pick already on the walk.  Walks run kLtWalks to a
// wave (k_lt_groups), each step one lookup in the vertex's guide table.
//
// Work split (the role of gIM's N_b persistent blocks, Alg. 6 / Eq. 5).  On skewed graphs
// the in-edges examined per set span five orders of magnitude and ~1% of the sets carry
// half of the work, so one set per block (the paper's choice) leaves the GPU waiting on a
// few sets.  Two kernels:
//   light : one wave per set, pulled 8 indices at a time from a work counter.  A set whose
//           examined 4-edge groups would exceed a budget, or whose members outgrow the
//           on-chip list, is abandoned and queued for the heavy kernel (its partial work is
//           redone there; the budget bounds the waste).
//   heavy : one workgroup (4 or 16 waves) per queued set, member list in HBM.
// Finished sets are written into the pool's id buffer at offsets reserved per wave in
// chunks (gIM Alg. 6's tail_RR, without a per-set atomic) and counted into the occurrence
// histogram (gIM Sec. III-B, Occur).  Counters that every wave updates are spread over 64
// addresses: device-scope atomics on one address serialise across the 8 XCDs.
#include "kernels.hpp"

namespace imm {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kLightCap = 1024;    // members a light set may hold on chip
constexpr int kIdChunk = kGenIdChunk;

int rr_light_capacity() { return kLightCap; }

// ------------------------------------------------------------------------------------
// shared helpers
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void vis_clear(uint32_t* vis, int32_t v) { vis[v >> 5] = 0u; }

__device__ __forceinline__ bool vis_test_and_set(uint32_t* vis, int32_t v) {
    const uint32_t bit = 1u << (v & 31);
    const uint32_t old = __hip_atomic_fetch_or(vis + (v >> 5), bit, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
    return (old & bit) == 0u;
}

// Orders the visited-bitmap clears of one set before the next set's test-and-sets.
__device__ __forceinline__ void vis_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// Wave-private state kept in (uniform) registers.
struct WaveState {
    int64_t cur = 0;                         // next fetched work item
    int32_t left = 0;                        // fetched work items not yet taken
    int32_t inst = -1;                       // instance of the current set
    int64_t inst_lo = 0, inst_hi = 0;        // its work items [inst_lo, inst_hi)
    int32_t place_inst = -1;                 // instance of the reserved chunk and counters
    int32_t chunk_left = 0;
    unsigned long long chunk_base = 0;
    unsigned long long placed = 0, edges = 0;
    unsigned long long heavy_buf = 0;        // lane i holds the i-th queued (instance, r)
    uint32_t heavy_ho = kNoHandoff;          // ... and its handoff offset
    int32_t heavy_n = 0;
    unsigned long long ar_base = 0;          // reserved handoff arena words
    int32_t ar_left = 0;
};

// Find the instance of work item w: largest i with work_off[i] <= w.
__device__ __forceinline__ int32_t find_inst(const GenLaunch& L, int64_t w) {
    int32_t lo = 0, hi = L.ninst;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (L.work_off[mid] <= w) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void flush_counters(const GenLaunch& L, WaveState& ws, int64_t slot) {
    if (ws.place_inst >= 0 && lane_id() == 0) {
        IMM_GLOBAL PoolCounters* c = global(L.inst[ws.place_inst].ctr);
        if (ws.placed) atomic_add_agent(&c->placed[slot & 63], ws.placed);
        if (ws.edges)
            atomic_add_agent(L.heavy_in ? &c->hedges[slot & 63] : &c->edges[slot & 63], ws.edges);
    }
    ws.placed = 0;
    ws.edges = 0;
}

// Next set of the launch: its instance (uniform) and RR index.  False when the launch's
// work is exhausted.
__device__ __forceinline__ bool next_set(const GenLaunch& L, WaveState& ws, int32_t& inst,
                                         uint32_t& r) {
    if (ws.left == 0) {
        unsigned long long i = 0;
        if (lane_id() == 0) i = atomic_add_agent(&L.lc->work, (unsigned long long)L.fetch);
        i = uniform64(i);
        if ((int64_t)i >= L.total) return false;
        ws.cur = (int64_t)i;
        ws.left = (int32_t)min((int64_t)L.fetch, L.total - (int64_t)i);
    }
    const int64_t w = ws.cur++;
    --ws.left;
    if (L.heavy_in) {
        const unsigned long long e = uniform64(L.heavy_in[w]);
        inst = (int32_t)(e >> 32);
        r = (uint32_t)e;
        return true;
    }
    if (ws.inst < 0 || w < ws.inst_lo || w >= ws.inst_hi) {
        ws.inst = uniform(find_inst(L, w));
        ws.inst_lo = (int64_t)uniform64((uint64_t)L.work_off[ws.inst]);
        ws.inst_hi = (int64_t)uniform64((uint64_t)L.work_off[ws.inst + 1]);
    }
    inst = ws.inst;
    const GenInst& I = L.inst[inst];
    const int64_t j = w - ws.inst_lo;
    r = uniform(I.list ? global(I.list)[j] : (uint32_t)(I.first + j));
    return true;
}

__device__ __forceinline__ void flush_heavy(const GenLaunch& L, WaveState& ws) {
    if (ws.heavy_n == 0) return;
    unsigned int at = 0;
    if (lane_id() == 0) at = atomic_add_agent(&L.lc->n_heavy, (unsigned int)ws.heavy_n);
    at = uniform(at);
    if (lane_id() < ws.heavy_n) {
        L.heavy_list[at + lane_id()] = ws.heavy_buf;
        if (L.handoff) L.handoff[at + lane_id()] = ws.heavy_ho;
    }
    ws.heavy_n = 0;
}

__device__ __forceinline__ void push_heavy(const GenLaunch& L, WaveState& ws, int32_t inst, uint32_t r,
                                           uint32_t ho = kNoHandoff) {
    if (lane_id() == ws.heavy_n) {
        ws.heavy_buf = ((unsigned long long)(uint32_t)inst << 32) | r;
        ws.heavy_ho = ho;
    }
    if (++ws.heavy_n == kWave) flush_heavy(L, ws);
}

// Copies a light set's partial traversal (members list[0, size), of which [0, head) are
// expanded, and the in-edges examined for them) to the handoff arena; wave-cooperative.  Arena space is
// reserved per wave in chunks of kArenaChunk words.  kNoHandoff when the arena is full.
constexpr int32_t kArenaChunk = 4096;
__device__ uint32_t hand_off(const GenLaunch& L, WaveState& ws, const int32_t* list, int32_t size,
                             int32_t head, unsigned long long examined) {
    if (!L.arena) return kNoHandoff;
    const int32_t need = size + 4;
    if (ws.ar_left < need) {
        const int32_t want = max(kArenaChunk, need);
        unsigned long long b = 0;
        if (lane_id() == 0) b = atomic_add_agent(&L.lc->arena, (unsigned long long)want);
        b = uniform64(b);
        if ((int64_t)(b + (unsigned long long)want) > L.arena_cap) {
            ws.ar_left = 0;
            return kNoHandoff;
        }
        ws.ar_base = b;
        ws.ar_left = want;
    }
    const unsigned long long o = ws.ar_base;
    ws.ar_base += (unsigned long long)need;
    ws.ar_left -= need;
    int32_t* p = L.arena + o;
    if (lane_id() == 0) {
        p[0] = size;
        p[1] = head;
        p[2] = (int32_t)(uint32_t)examined;
        p[3] = (int32_t)(uint32_t)(examined >> 32);
    }
    for (int32_t i = lane_id(); i < size; i += kWave) p[4 + i] = list[i];
    return (uint32_t)o;
}

__device__ __forceinline__ void push_capacity_miss(const GenInst& I, uint32_t r) {
    const unsigned int at = atomic_add_agent(&global(I.ctr)->n_capacity, 1u);
    global(I.cap_list)[at] = r;
}

// Write a finished set (members list[0..size)) into its pool; wave-cooperative.
// Members past `split` come from `ext` (an LT walk's extension list in HBM).
__device__ void place_wave(const GenLaunch& L, WaveState& ws, int64_t slot, int32_t inst,
                           uint32_t r, const int32_t* list, int32_t size, uint64_t examined,
                           const IMM_GLOBAL int32_t* ext = nullptr, int32_t split = 0x7FFFFFFF) {
    const int lane = lane_id();
    const GenInst& I = L.inst[inst];
    if (ws.place_inst != inst) {
        flush_counters(L, ws, slot);
        ws.place_inst = inst;
        ws.chunk_left = 0;
    }
    if (ws.chunk_left < size) {
        const int32_t want = max(kIdChunk, size);
        unsigned long long base = 0;
        if (lane == 0) base = atomic_add_agent(&global(I.ctr)->tail, (unsigned long long)want);
        base = uniform64(base);
        if ((int64_t)base + want > I.cap_ids) {
            if (lane == 0) push_capacity_miss(I, r);
            ws.chunk_left = 0;
            return;
        }
        ws.chunk_base = base;
        ws.chunk_left = want;
    }
    IMM_GLOBAL int32_t* ids = global(I.ids);
    IMM_GLOBAL uint32_t* hist = global(I.hist);
    for (int32_t i = lane; i < size; i += kWave) {
        const int32_t v = i < split ? list[i] : ext[i - split];
        ids[ws.chunk_base + i] = v;
        __hip_atomic_fetch_add(hist + v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
        global(I.rr_start)[r] = (int64_t)ws.chunk_base;
        global(I.rr_len)[r] = size;
    }
    ws.chunk_base += (unsigned long long)size;
    ws.chunk_left -= size;
    ws.placed += (unsigned long long)size;
    ws.edges += examined;
}

__device__ __forceinline__ void wave_exit(const GenLaunch& L, WaveState& ws, int64_t slot) {
    flush_heavy(L, ws);
    flush_counters(L, ws, slot);
}

// ------------------------------------------------------------------------------------
// IC: testing one 4-edge group and appending newly reached vertices
// ------------------------------------------------------------------------------------
// Vertices with at least this many 4-edge groups are expanded one at a time (all lanes on
// consecutive groups of that vertex, no lane -> vertex search); smaller ones are packed
// together and each lane finds its vertex by a search over the batch's group prefix.
constexpr int32_t kBigGroups = 48;

// The graph fields a set's traversal reads, loaded once per set into registers.
struct GraphView {
    const IMM_GLOBAL VRec* vrec;
    const IMM_GLOBAL int32_t* src;
    const IMM_GLOBAL uint32_t* w;       // IC thresholds or LT cumulative thresholds
    uint32_t k0, k1;
    int32_t n;
    uint32_t t;                         // round word of the edge draws
};

__device__ __forceinline__ GraphView ic_view(const GenInst& I) {
    return GraphView{global(I.vrec), global(I.src), global(I.thr), I.k0, I.k1, I.n, I.round};
}

// Draws the in-edges of group g (edges 4g .. 4g+3) for set r; bit j of the result is set
// when edge 4g + j lies in [s, e_end) and is live.  Pure ALU apart from the per-edge
// thresholds of a non-uniform vertex.
__device__ __forceinline__ uint32_t live_bits(const GraphView& a, uint32_t r, uint32_t g,
                                              uint32_t s, uint32_t e_end, bool uniform_thr,
                                              uint32_t uthr) {
    const Ctr4 x = philox10(Ctr4{r, g, a.t, kDomainIC}, a.k0, a.k1);
    const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
    // edge 4g + j is in the vertex's list iff its offset 4g + j - s (mod 2^32) is below d
    const uint32_t d = e_end - s, o = (g << 2) - s;
    uint32_t bits = 0;
    if (uniform_thr) {
        const bool always = uthr == kAlways;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bits |= (uint32_t)(o + j < d && (always || xs[j] < uthr)) << j;
    } else {
        const u32x4 tv = *reinterpret_cast<const IMM_GLOBAL u32x4*>(a.w + ((int64_t)g << 2));
        const uint32_t t[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bits |= (uint32_t)(o + j < d && (t[j] == kAlways || xs[j] < t[j])) << j;
    }
    return bits;
}

// Ballots of the draws of group g below the threshold t, one mask per word (the edges of a
// vertex with one threshold for its whole in-list): no per-edge range or threshold work.
__device__ __forceinline__ void live_masks_interior(const GraphView& a, uint32_t r, uint32_t g,
                                                    uint32_t t, uint64_t m[4]) {
    const Ctr4 x = philox10(Ctr4{r, g, a.t, kDomainIC}, a.k0, a.k1);
    m[0] = ballot(x.x < t);
    m[1] = ballot(x.y < t);
    m[2] = ballot(x.z < t);
    m[3] = ballot(x.w < t);
}

// Lanes [lo, hi) of a wave as a mask (0 <= lo <= hi <= 64).
__device__ __forceinline__ uint64_t lane_range(uint32_t lo, uint32_t hi) {
    const uint64_t below_hi = hi >= 64u ? ~0ull : (1ull << hi) - 1ull;
    return below_hi & ~((1ull << lo) - 1ull);
}

// Lanes L of a wave whose edge e0 + 4L + j lies in [s, e) (wave-uniform arguments):
// in[j] for word j.
__device__ __forceinline__ void edge_range_masks(uint32_t e0, uint32_t s, uint32_t e,
                                                 uint64_t in[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t ej = e0 + (uint32_t)j;
        const uint32_t lo = s > ej ? (s - ej + 3u) >> 2 : 0u;
        const uint32_t hi = e > ej ? min((e - ej + 3u) >> 2, 64u) : 0u;
        in[j] = lo < hi ? lane_range(lo, hi) : 0ull;
    }
}

__device__ __forceinline__ void masks_of_bits(uint32_t bits, uint64_t m[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) m[j] = ballot((bits >> j) & 1u);
}

// Live edges are staged in LDS (edge indices, per wave) and resolved in batches: the
// source loads and visited test-and-sets of a whole batch are issued together, so the
// group tests themselves never wait on memory.
constexpr int kStage = 256;

// Appends the live edges of one pass (ballot m[j] of word j of group g per lane) to the
// wave's stage, calling flush() first whenever they would not fit.
template <class Flush>
__device__ __forceinline__ void stage_masks(uint32_t* stage, int32_t& n, const uint64_t m[4],
                                            uint32_t g, Flush&& flush) {
    if ((m[0] | m[1] | m[2] | m[3]) == 0) return;
    const int lane = lane_id();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (m[j] == 0) continue;
        const int32_t c = (int32_t)__popcll(m[j]);
        if (n + c > kStage) flush();
        if ((m[j] >> lane) & 1u) stage[n + (int32_t)lanes_below(m[j])] = (g << 2) + j;
        n += c;
    }
}

template <class Flush>
__device__ __forceinline__ void stage_edges(uint32_t* stage, int32_t& n, uint32_t bits,
                                            uint32_t g, Flush&& flush) {
    uint64_t m[4];
    masks_of_bits(bits, m);
    stage_masks(stage, n, m, g, flush);
}

// Resolves up to 64 staged edges: source of edge stage[i] for i = i0 + lane < n, and
// whether this test-and-set visited it first.
__device__ __forceinline__ bool resolve_staged(const GraphView& a, const uint32_t* stage,
                                               int32_t i0, int32_t n, uint32_t* vis,
                                               int32_t& u) {
    const int32_t i = i0 + lane_id();
    if (i >= n) return false;
    u = a.src[stage[i]];
    return vis_test_and_set(vis, u);
}

// Light kernel: appends the new sources of the staged edges to the on-chip list; on
// overflow the set is abandoned (and the bits of the vertices not appended are cleared).
__device__ __forceinline__ void flush_light(const GraphView& a, uint32_t* stage, int32_t& n,
                                            int32_t* list, int32_t& size, bool& abandon,
                                            uint32_t* vis, int32_t cap) {
    wave_sync();
    for (int32_t i0 = 0; i0 < n; i0 += kWave) {
        int32_t u = 0;
        const bool fresh = resolve_staged(a, stage, i0, n, vis, u);
        const uint64_t m = ballot(fresh);
        const int32_t c = (int32_t)__popcll(m);
        if (c == 0) continue;
        if (abandon || size + c > cap) {
            abandon = true;
            if (fresh) vis_clear(vis, u);
            continue;
        }
        if (fresh) list[size + (int32_t)lanes_below(m)] = u;
        size += c;
    }
    n = 0;
    wave_sync();
}

// Vertex records of the most recently queued members of a heavy set, by list position
// modulo kRing: filled when a member is found, read when its batch starts, so a batch does
// not wait for its vertices' list entries and records.  Valid for positions [head, size)
// while size - head <= kRing (no later member has reused the slot yet).
constexpr int kRing = 256;
struct RecRing {
    uint32_t start[kRing];
    uint32_t deg[kRing];
    uint32_t thr[kRing];
};

__device__ __forceinline__ void ring_put(RecRing& ring, int32_t p, const VRec& rec) {
    const int32_t s = p & (kRing - 1);
    ring.start[s] = (uint32_t)rec.start;
    ring.deg[s] = rec.deg;
    ring.thr[s] = rec.thr;
}

// Heavy kernel: appends to the workgroup's HBM list (positions from an LDS counter) and
// puts each new member's vertex record in the ring.  The record is loaded for every
// resolved edge, in parallel with its test-and-set, so the two waits overlap.
// kBounded: members past `cap` are not stored (their bits are cleared again): the set has
// outgrown its list and is dropped at the end of the batch.
template <bool kBounded>
__device__ __forceinline__ void flush_block(const GraphView& a, uint32_t* stage, int32_t& n,
                                            int32_t* list, int32_t* s_size, uint32_t* vis,
                                            RecRing& ring, int32_t cap) {
    wave_sync();
    for (int32_t i0 = 0; i0 < n; i0 += kWave) {
        const int32_t i = i0 + lane_id();
        int32_t u = 0;
        VRec rec{};
        bool fresh = false;
        if (i < n) {
            u = a.src[stage[i]];
            rec = load_vrec(a.vrec + u);
            fresh = vis_test_and_set(vis, u);
        }
        const uint64_t m = ballot(fresh);
        const int32_t c = (int32_t)__popcll(m);
        if (c == 0) continue;
        int32_t at = 0;
        if (lane_id() == 0) at = atomicAdd(s_size, c);
        at = __shfl(at, 0, kWave);
        if (fresh) {
            const int32_t p = at + (int32_t)lanes_below(m);
            if (!kBounded || p < cap) {
                list[p] = u;
                ring_put(ring, p, rec);
            } else {
                vis_clear(vis, u);
            }
        }
    }
    n = 0;
    wave_sync();
}

__device__ __forceinline__ uint32_t groups_of(uint32_t start, uint32_t deg) {
    return deg ? ((start + deg - 1) >> 2) - (start >> 2) + 1 : 0u;
}

// ------------------------------------------------------------------------------------
// IC light kernel: one wave per set.
// ------------------------------------------------------------------------------------
struct FrontierLds {
    int32_t pre[kWave + 1];   // exclusive prefix of the small vertices' group counts
    uint32_t start[kWave];    // first in-edge of each batch vertex
    uint32_t deg[kWave];      // in-degree | uniform bit
    uint32_t thr[kWave];      // common threshold when uniform
};

struct LightLds {
    FrontierLds f;
    uint32_t stage[kStage];
    int32_t list[kLightCap];
};

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_ic_light(GenLaunch G) {
    __shared__ LightLds lds_all[kWavesPerBlock];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    LightLds& L = lds_all[wib];
    const int64_t slot = (int64_t)blockIdx.x * kWavesPerBlock + wib;
    uint32_t* vis = G.visited + slot * G.vis_words;
    int32_t* list = L.list;
    WaveState ws;

    int32_t inst;
    uint32_t r;
    while (next_set(G, ws, inst, r)) {
        const GraphView a = ic_view(G.inst[inst]);
        const int32_t root = (int32_t)root_of(r, (uint32_t)a.n, a.k0, a.k1);
        if (lane == 0) {
            list[0] = root;
            vis_test_and_set(vis, root);
        }
        int32_t size = 1, head = 0;
        uint64_t examined = 0;
        int64_t used = 0;
        bool abandon = false, resumable = false;
        wave_sync();

        while (head < size && !abandon) {
            const int32_t nb = min(size - head, kWave);
            uint32_t ng = 0, dg = 0, st = 0, dgf = 0, th = 0;
            if (lane < nb) {
                const VRec rec = load_vrec(a.vrec + list[head + lane]);
                dgf = rec.deg;
                th = rec.thr;
                dg = dgf & kDegMask;
                st = (uint32_t)rec.start;
                ng = groups_of(st, dg);
            }
            const bool big = ng >= (uint32_t)kBigGroups;
            const int32_t ngs = big ? 0 : (int32_t)ng;
            const int32_t incl = wave_incl_scan(ngs);
            if (lane < nb) {
                L.f.pre[lane] = incl - ngs;
                L.f.start[lane] = st;
                L.f.deg[lane] = dgf;
                L.f.thr[lane] = th;
            }
            if (lane == nb - 1) L.f.pre[nb] = incl;
            const int32_t total_small = __shfl(incl, nb - 1, kWave);
            const int64_t total = (int64_t)wave_sum((uint64_t)ng);
            const uint64_t level_edges = wave_sum((uint64_t)dg);
            wave_sync();
            if (used + total > G.budget) {
                abandon = true;                   // members [0, head) are expanded
                resumable = true;
                break;
            }
            used += total;
            examined += level_edges;

            int32_t nst = 0;
            auto flush = [&]() { flush_light(a, L.stage, nst, list, size, abandon, vis, G.light_cap); };
            // big vertices: one at a time, wave-uniform vertex data
            uint64_t bigmask = ballot(big);
            while (bigmask && !abandon) {
                const int b = __ffsll((unsigned long long)bigmask) - 1;
                bigmask &= bigmask - 1;
                const uint32_t s0 = __builtin_amdgcn_readlane(st, b);
                const uint32_t df = __builtin_amdgcn_readlane(dgf, b);
                const uint32_t t0 = __builtin_amdgcn_readlane(th, b);
                const uint32_t gb = __builtin_amdgcn_readlane(ng, b);
                const uint32_t e_end = s0 + (df & kDegMask);
                const uint32_t g0 = s0 >> 2;
                const bool uni = (df & kUniformBit) != 0;
                const bool plain = uni && t0 != kAlways;
                for (uint32_t base = 0; base < gb && !abandon; base += kWave) {
                    const uint32_t g = g0 + base + lane;
                    uint64_t m[4];
                    const int fast = uniform((int)(plain && (base > 0 || (s0 & 3u) == 0) &&
                                                   base + kWave < gb));
                    if (fast) {
                        live_masks_interior(a, r, g, t0, m);   // every lane a full group
                    } else {
                        masks_of_bits(base + lane < gb ? live_bits(a, r, g, s0, e_end, uni, t0) : 0u, m);
                    }
                    stage_masks(L.stage, nst, m, g, flush);
                }
            }

            // small vertices: packed, each lane searches for its vertex
            for (int32_t base = 0; base < total_small && !abandon; base += kWave) {
                const int32_t q = base + lane;
                uint32_t bits = 0, g = 0;
                if (q < total_small) {
                    int32_t lo = 0, hi = nb;   // pre[lo] <= q < pre[hi]
                    while (hi - lo > 1) {
                        const int32_t mid = (lo + hi) >> 1;
                        if (L.f.pre[mid] <= q) lo = mid; else hi = mid;
                    }
                    const uint32_t s0 = L.f.start[lo];
                    const uint32_t dd = L.f.deg[lo];
                    g = (s0 >> 2) + (uint32_t)(q - L.f.pre[lo]);
                    bits = live_bits(a, r, g, s0, s0 + (dd & kDegMask), (dd & kUniformBit) != 0,
                                     L.f.thr[lo]);
                }
                stage_edges(L.stage, nst, bits, g, flush);
            }
            if (nst > 0) flush();
            wave_sync();
            head += nb;
        }
        if (abandon) {
            // a set abandoned at the budget is handed over as it stands, with the in-edges
            // examined so far; the heavy kernel counts them for this launch when it places
            // the set (a set that misses the id buffer is drawn again and counts nothing)
            push_heavy(G, ws, inst, r, resumable ? hand_off(G, ws, list, size, head, examined)
                                                 : kNoHandoff);
        }
        else place_wave(G, ws, slot, inst, r, list, size, examined);
        for (int32_t i = lane; i < size; i += kWave) vis_clear(vis, list[i]);
        vis_fence();
        wave_sync();
    }
    wave_exit(G, ws, slot);
}

// ------------------------------------------------------------------------------------
// IC heavy kernel: one workgroup per set, member list in HBM.
// ------------------------------------------------------------------------------------
// Inclusive block scan of one uint64 per thread (up to 1024 threads).
template <int kHeavyBlock>
__device__ __forceinline__ uint64_t block_incl_scan(uint64_t v, uint64_t* wsum) {
    constexpr int kHeavyWaves = kHeavyBlock / kWave;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    uint64_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        const uint64_t t = lane < kHeavyWaves ? wsum[lane] : 0;
        const uint64_t ti = wave_incl_scan(t);
        if (lane < kHeavyWaves) wsum[lane] = ti - t;
    }
    __syncthreads();
    incl += wsum[wid];
    __syncthreads();
    return incl;
}

// Each batch of up to kHeavyBlock frontier vertices is split into work for independent
// waves: vertices with at least kWave groups ("big") are cut into chunks of kWave groups,
// chunk c going to wave c mod (waves per block); the other vertices are packed into
// windows of kWave groups, handed out the same way.  One block scan per batch yields, per
// vertex, its small-group prefix, its index among the big vertices and its first chunk,
// packed in one 64-bit value (fields of 16, 16 and 32 bits: a batch has at most 1024
// vertices, each with fewer than kWave groups in the first field).
// kBounded: member lists of list_stride entries that a set may outgrow (G.over_list);
// otherwise lists hold any set.
template <int kHeavyBlock, bool kBounded>
__global__ __launch_bounds__(kHeavyBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_ic_heavy(GenLaunch G) {
    constexpr int kHeavyWaves = kHeavyBlock / kWave;
    __shared__ int32_t pre[kHeavyBlock + 1];
    __shared__ uint32_t st[kHeavyBlock], dgs[kHeavyBlock], ths[kHeavyBlock];
    __shared__ uint32_t bst[kHeavyBlock], bdg[kHeavyBlock], bth[kHeavyBlock], bng[kHeavyBlock];
    __shared__ uint32_t bcp[kHeavyBlock + 1];
    __shared__ uint32_t stage_all[kHeavyWaves][kStage];
    __shared__ RecRing ring;
    __shared__ uint64_t wsum[kHeavyWaves];
    __shared__ unsigned long long wred[kHeavyWaves];
    __shared__ int32_t s_size;
    __shared__ uint32_t s_nchunks;
    __shared__ unsigned int s_idx;
    __shared__ int32_t s_head;
    __shared__ unsigned long long s_light;      // in-edges the light kernel examined
    __shared__ unsigned long long s_base;
    const int tid = threadIdx.x, lane = lane_id();
    const int wid = uniform(tid / kWave);
    const int64_t slot = blockIdx.x;
    uint32_t* vis = G.hvisited + slot * G.vis_words;
    int32_t* list = G.hlist + slot * G.list_stride;
    uint32_t* stage = stage_all[wid];

    for (;;) {
        if (tid == 0) s_idx = atomic_add_agent(&G.lc->hwork, 1u);
        __syncthreads();
        const unsigned int idx = uniform(s_idx);
        if (idx >= G.n_queue) break;
        const unsigned long long qe = uniform64(G.heavy_list[idx]);
        const GenInst& I = G.inst[(int32_t)(qe >> 32)];
        const GraphView a = ic_view(I);
        const uint32_t r = (uint32_t)qe;
        const uint32_t ho = G.handoff ? uniform(G.handoff[idx]) : kNoHandoff;
        if (ho != kNoHandoff) {
            // resume the light kernel's traversal: its members, of which [0, head) are
            // expanded, enter the list and the bitmap.  The ring receives the records of
            // the last kRing unexpanded members, positions [max(head, size - kRing),
            // size): whenever a later batch reads the ring (size' - head' <= kRing with
            // size' >= size), every position it reads at or past size - kRing holds its
            // own record, and positions past size are filled as members are found.
            const int32_t* hp = G.arena + ho;
            const int32_t hsize = uniform(hp[0]), hhead = uniform(hp[1]);
            const int32_t ring_from = max(hhead, hsize - kRing);
            for (int32_t i = tid; i < hsize; i += kHeavyBlock) {
                const int32_t v = hp[4 + i];
                list[i] = v;
                vis_test_and_set(vis, v);
                if (i >= ring_from) ring_put(ring, i, load_vrec(a.vrec + v));
            }
            if (tid == 0) {
                s_size = hsize;
                s_head = hhead;
                s_light = ((unsigned long long)(uint32_t)hp[3] << 32) | (uint32_t)hp[2];
            }
        } else if (tid == 0) {
            const int32_t root = (int32_t)root_of(r, (uint32_t)a.n, a.k0, a.k1);
            list[0] = root;
            ring_put(ring, 0, load_vrec(a.vrec + root));
            vis_test_and_set(vis, root);
            s_size = 1;
            s_head = 0;
            s_light = 0;
        }
        __syncthreads();
        int32_t head = s_head, size = s_size;
        unsigned long long examined = 0;
        while (head < size) {
            const int32_t nb = min(size - head, kHeavyBlock);
            uint32_t ng = 0, dg = 0, s0 = 0, dgf = 0, t0 = 0;
            if (tid < nb) {
                if (size - head <= kRing) {
                    const int32_t p = (head + tid) & (kRing - 1);
                    s0 = ring.start[p];
                    dgf = ring.deg[p];
                    t0 = ring.thr[p];
                } else {
                    const VRec rec = load_vrec(a.vrec + list[head + tid]);
                    dgf = rec.deg;
                    t0 = rec.thr;
                    s0 = (uint32_t)rec.start;
                }
                dg = dgf & kDegMask;
                ng = groups_of(s0, dg);
            }
            const bool big = ng >= (uint32_t)kWave;
            const uint64_t mine =
                big ? ((uint64_t)((ng + kWave - 1) / kWave) << 32) | (1ull << 16) : (uint64_t)ng;
            const unsigned long long dsum = wave_sum((unsigned long long)dg);
            if (lane == 0) wred[wid] = dsum;
            const uint64_t incl = block_incl_scan<kHeavyBlock>(mine, wsum);   // has barriers
            const uint64_t excl = incl - mine;
            if (tid < nb) {
                pre[tid] = (int32_t)(excl & 0xFFFFu);
                st[tid] = s0;
                dgs[tid] = dgf;
                ths[tid] = t0;
                if (big) {
                    const uint32_t k = (uint32_t)(excl >> 16) & 0xFFFFu;
                    bst[k] = s0;
                    bdg[k] = dgf;
                    bth[k] = t0;
                    bng[k] = ng;
                    bcp[k] = (uint32_t)(excl >> 32);
                }
            }
            if (tid == kHeavyBlock - 1) {          // block totals
                const uint32_t nbig = (uint32_t)(incl >> 16) & 0xFFFFu;
                pre[nb] = (int32_t)(incl & 0xFFFFu);
                bcp[nbig] = (uint32_t)(incl >> 32);
                s_nchunks = (uint32_t)(incl >> 32);
            }
            __syncthreads();
            if (tid == 0)
                for (int w = 0; w < kHeavyWaves; ++w) examined += wred[w];
            const uint32_t nchunks = uniform(s_nchunks);
            const int32_t total_small = uniform(pre[nb]);
            int32_t nst = 0;
            auto flush = [&]() {
                flush_block<kBounded>(a, stage, nst, list, &s_size, vis, ring, (int32_t)G.list_stride);
            };
            // big vertices: chunk c -> the vertex k with bcp[k] <= c < bcp[k + 1]; a wave's
            // chunks increase, so its vertex index only moves forward
            uint32_t k = ~0u, c_lo = 0, c_hi = 0;   // chunks [c_lo, c_hi) are vertex k's
            uint32_t bs = 0, be = 0, bt = 0, gb = 0;
            bool bu = false;
            for (uint32_t c = (uint32_t)wid; c < nchunks; c += kHeavyWaves) {
                if (c >= c_hi) {
                    do {
                        ++k;
                        c_hi = uniform(bcp[k + 1]);
                    } while (c_hi <= c);
                    c_lo = uniform(bcp[k]);
                    bs = uniform(bst[k]);
                    const uint32_t bd = uniform(bdg[k]);
                    be = bs + (bd & kDegMask);
                    bu = (bd & kUniformBit) != 0;
                    bt = uniform(bth[k]);
                    gb = uniform(bng[k]);
                }
                const uint32_t q0 = (c - c_lo) * kWave;        // chunk's first group, relative
                const uint32_t g = (bs >> 2) + q0 + (uint32_t)lane;
                uint64_t m[4];
                if (bu && bt != kAlways && c > c_lo && c + 1 < c_hi) {
                    // The wave's interior chunks of this vertex (every edge of every lane in
                    // the list, one threshold): a tight loop of draws and ballots, with the
                    // scalar work per chunk cut to the loop control and the live-edge test.
                    uint32_t gi = g;
                    for (; c + 1 < c_hi; c += kHeavyWaves, gi += (uint32_t)(kHeavyWaves * kWave)) {
                        const Ctr4 x = philox10(Ctr4{r, gi, a.t, kDomainIC}, a.k0, a.k1);
                        // one compare for "any live edge in the wave"; the per-word
                        // ballots only when there is one (rare on hub vertices)
                        const uint32_t lo = min(min(x.x, x.y), min(x.z, x.w));
                        if (ballot(lo < bt) != 0) {
                            m[0] = ballot(x.x < bt);
                            m[1] = ballot(x.y < bt);
                            m[2] = ballot(x.z < bt);
                            m[3] = ballot(x.w < bt);
                            stage_masks(stage, nst, m, gi, flush);
                        }
                    }
                    c -= kHeavyWaves;                  // the loop increment steps past it
                    continue;
                }
                if (bu) {
                    // One threshold for the whole list: the draws go straight into wave
                    // masks; only the vertex's first and last chunks need the lanes whose
                    // edges lie outside the list masked off.
                    uint64_t in[4] = {~0ull, ~0ull, ~0ull, ~0ull};
                    if (c == c_lo || c + 1 == c_hi) edge_range_masks(((bs >> 2) + q0) << 2, bs, be, in);
                    if (bt == kAlways) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) m[j] = in[j];
                    } else {
                        live_masks_interior(a, r, g, bt, m);
#pragma unroll
                        for (int j = 0; j < 4; ++j) m[j] &= in[j];
                    }
                } else {
                    masks_of_bits(q0 + (uint32_t)lane < gb ? live_bits(a, r, g, bs, be, false, 0u) : 0u, m);
                }
                stage_masks(stage, nst, m, g, flush);
            }
            // small vertices: windows of kWave groups, each lane searches for its vertex
            for (int32_t base = wid * kWave; base < total_small; base += kHeavyBlock) {
                const int32_t q = base + lane;
                uint32_t bits = 0, g = 0;
                if (q < total_small) {
                    int32_t lo = 0, hi = nb;   // pre[lo] <= q < pre[hi]
                    while (hi - lo > 1) {
                        const int32_t mid = (lo + hi) >> 1;
                        if (pre[mid] <= q) lo = mid; else hi = mid;
                    }
                    const uint32_t ss = st[lo];
                    const uint32_t dd = dgs[lo];
                    g = (ss >> 2) + (uint32_t)(q - pre[lo]);
                    bits = live_bits(a, r, g, ss, ss + (dd & kDegMask), (dd & kUniformBit) != 0,
                                     ths[lo]);
                }
                stage_edges(stage, nst, bits, g, flush);
            }
            if (nst > 0) flush();
            __syncthreads();
            head += nb;
            size = s_size;
            __syncthreads();
            if (kBounded && size > G.list_stride) size = head;   // outgrown: the traversal ends
        }
        if (kBounded && s_size > G.list_stride) {
            // outgrew the list (flush_block stored list_stride members and cleared the bits
            // of the rest): the queue entry goes to the full-list pass, which draws the set
            // again from its root, and the stored members' bits are cleared.  (A full list
            // holds any set; without an overflow list this would be a capacity miss.)
            if (tid == 0) {
                if (G.over_list) {
                    const unsigned int o = atomic_add_agent(&G.lc->n_over, 1u);
                    G.over_list[o] = G.heavy_list[s_idx];   // this set's queue entry
                } else {
                    push_capacity_miss(I, r);
                }
            }
            for (int32_t i = tid; i < (int32_t)G.list_stride; i += kHeavyBlock) vis_clear(vis, list[i]);
            vis_fence();
            __syncthreads();
            continue;
        }
        // place the set
        if (tid == 0) {
            IMM_GLOBAL PoolCounters* c = global(I.ctr);
            unsigned long long b = atomic_add_agent(&c->tail, (unsigned long long)size);
            if ((int64_t)b + size > I.cap_ids) {
                push_capacity_miss(I, r);
                b = ~0ull;
            } else {
                global(I.rr_start)[r] = (int64_t)b;
                global(I.rr_len)[r] = size;
                atomic_add_agent(&c->placed[slot & 63], (unsigned long long)size);
                atomic_add_agent(&c->hedges[slot & 63], (unsigned long long)examined);
                __hip_atomic_fetch_max(&c->max_len, (unsigned int)size, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                if (s_light) atomic_add_agent(&c->edges[slot & 63], s_light);
            }
            s_base = b;
        }
        __syncthreads();
        const unsigned long long b = s_base;
        IMM_GLOBAL int32_t* ids = global(I.ids);
        IMM_GLOBAL uint32_t* hist = global(I.hist);
        for (int32_t i = tid; i < size; i += kHeavyBlock) {
            const int32_t v = list[i];
            if (b != ~0ull) {
                ids[b + i] = v;
                __hip_atomic_fetch_add(hist + v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            vis_clear(vis, v);
        }
        vis_fence();
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// LT: reverse walks.
//
// A step reads its pick from the current vertex's guide table (graph.hip): one 16-byte
// record gives the picked edge's threshold (to confirm the pick), its source, and the
// source's in-edge range, so consecutive steps are one dependent load apart.  When a
// threshold falls inside the draw's bucket the pick is one of the following edges of the
// list (the last edge of a list is saturated, so the scan ends within it).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ bool lt_ok(uint32_t c, uint32_t x) { return c == kAlways || x < c; }

struct LtTables {
    const IMM_GLOBAL LtRec* grec;
    const IMM_GLOBAL uint32_t* gidx;
    const IMM_GLOBAL LtRec* lrec;
};

__device__ __forceinline__ LtTables lt_tables(const GenInst& I) {
    return LtTables{global(I.grec), global(I.gidx), global(I.lrec)};
}

// The in-edge of a vertex with in-edges [start, start + deg), deg > 0, that draw x picks.
__device__ __forceinline__ LtRec lt_step(const LtTables& T, uint32_t start, uint32_t deg, uint32_t x) {
    const int64_t gi = 2 * (int64_t)start + (int64_t)(((uint64_t)x * (2ull * deg)) >> 32);
    LtRec rec = load_ltrec(T.grec + 2 * gi);
    if (!lt_ok(rec.cum, x)) {
        rec = load_ltrec(T.grec + 2 * gi + 1);     // the successor (same cache line)
        if (!lt_ok(rec.cum, x)) {
            uint32_t pos = T.gidx[gi] + 1;
            do {
                ++pos;
                rec = load_ltrec(T.lrec + start + pos);
            } while (!lt_ok(rec.cum, x) && pos + 1 < deg);
        }
    }
    return rec;
}

// Walks longer than the first pass can hold (on-chip list plus extension): one walk per
// wave, its members in an HBM list and a visited bitmap (restarted from the root).
__global__ __launch_bounds__(kBlock) void k_rr_lt_hbm(GenLaunch G) {
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    const int64_t slot = (int64_t)blockIdx.x * kWavesPerBlock + wib;
    uint32_t* vis = G.hvisited + slot * G.vis_words;
    int32_t* list = G.hlist + slot * G.list_stride;
    WaveState ws;

    int32_t inst;
    uint32_t r;
    while (next_set(G, ws, inst, r)) {
        const GenInst& I = G.inst[inst];
        const LtTables T = lt_tables(I);
        const int32_t cap = I.n;
        const uint32_t k0 = I.k0, k1 = I.k1, t = I.round;
        int32_t v = (int32_t)root_of(r, (uint32_t)I.n, k0, k1);
        const VRec rv = load_vrec(global(I.vrec) + v);
        uint32_t start = (uint32_t)rv.start, deg = rv.deg & kDegMask;
        if (lane == 0) {
            list[0] = v;
            vis_test_and_set(vis, v);
        }
        int32_t size = 1;
        uint64_t examined = 0;
        bool abandon = false;
        while (deg > 0) {
            examined += deg;
            const uint32_t x = philox10(Ctr4{r, (uint32_t)v, t, kDomainLT}, k0, k1).x;
            const LtRec rec = lt_step(T, start, deg, x);
            const int32_t u = rec.src;
            bool fresh = false;
            if (lane == 0) fresh = vis_test_and_set(vis, u);
            fresh = __shfl(fresh, 0, kWave);
            if (!fresh) break;
            if (size + 1 > cap) {
                abandon = true;
                if (lane == 0) vis_clear(vis, u);
                break;
            }
            if (lane == 0) list[size] = u;
            ++size;
            v = u;
            start = rec.start;
            deg = rec.deg;
        }
        __threadfence();
        if (abandon) push_heavy(G, ws, inst, r);
        else place_wave(G, ws, slot, inst, r, list, size, examined);
        for (int32_t i = lane; i < size; i += kWave) vis_clear(vis, list[i]);
        vis_fence();
        wave_sync();
    }
    wave_exit(G, ws, slot);
}

// ------------------------------------------------------------------------------------
// LT: the first pass of every launch.  A group of kLtGroup lanes runs one walk (kLtWalks
// walks per wave), its first G.lt_lds_cap members in an LDS list and the next
// G.lt_ext_cap in the group's extension list in HBM; together they are the walk's revisit
// test (the group's lanes compare the picked vertex with the lists, kLtGroup entries per
// step of the scan).  Walks on RR sets are short (on R-MAT scale 22 the median is one
// member and the 99.99th percentile ~500), so the extension is rarely touched; it lets the
// few long walks finish here instead of being redrawn.  The group's lanes compute the same
// values (its draw, its loads, broadcast to the group); the wave places finished walks one
// at a time.  Walks longer than both lists are redrawn by k_rr_lt_hbm.
//
// Each step is one dependent load, so the kernel is organised to keep that load in flight
// while the wave does everything else: when a walk's pick u arrives, the draw and guide
// load of u's own step are issued at once, before u is tested against the walk (a revisit
// ends the walk once, so the speculation is almost always right; a wrong one costs one
// unused load), and the revisit scans, placements of finished walks and starts of new
// walks of the wave all run while those loads travel.  A new walk's root record is
// likewise loaded one iteration before its first draw.
//
// The scan runs only when the picked vertex may be on the walk: each walk keeps a
// 4096-bit filter in LDS (one bit per member, at a multiplicative hash of its id), and a
// clear bit proves the vertex new.  A walk of L members scans with probability at most
// L / 4096 per step, so long walks no longer pay a scan of their whole list (the
// extension part in HBM) at every step.
// ------------------------------------------------------------------------------------
constexpr int kLtGroup = 16;
constexpr int kLtWalks = kWave / kLtGroup;
constexpr int kLtFiltWords = 128;
constexpr int kLtFiltLog2 = 12;              // filter bits: 2^12 = kLtFiltWords x 32
static_assert((1 << kLtFiltLog2) == kLtFiltWords * 32, "filter hash width must match its words");

__device__ __forceinline__ uint32_t lt_filt_bit(int32_t u) {
    return ((uint32_t)u * 0x9E3779B1u) >> (32 - kLtFiltLog2);
}

__global__ __launch_bounds__(kBlock) void k_lt_groups(GenLaunch G) {
    __shared__ int32_t lists[kWavesPerBlock][kLtWalks][kLtLdsCap];
    __shared__ uint32_t filts[kWavesPerBlock][kLtWalks][kLtFiltWords];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    const int grp = lane / kLtGroup, gl = lane % kLtGroup;
    const uint64_t gmask = ((1ull << kLtGroup) - 1) << (grp * kLtGroup);
    int32_t* list = lists[wib][grp];
    uint32_t* filt = filts[wib][grp];
    const int64_t slot = (int64_t)blockIdx.x * kWavesPerBlock + wib;
    const int32_t lcap = G.lt_lds_cap, ecap = G.lt_ext_cap;
    IMM_GLOBAL int32_t* ext_wave = global(G.lt_ext) + slot * kLtWalks * (int64_t)ecap;
    IMM_GLOBAL int32_t* ext = ext_wave + grp * (int64_t)ecap;
    WaveState ws;

    // the group's walk (the same values in each of its lanes).  phase 0: the root's vertex
    // record `vr` is in flight; phase 1: the pick `rec` of the current vertex v (in-edges
    // [start, start + deg), draw x, guide entry gi) is in flight.
    bool active = false;
    int phase = 0;
    int32_t inst = 0, v = 0, size = 0;
    uint32_t r = 0, start = 0, deg = 0, x = 0, k0 = 0, k1 = 0, t = 0;
    int64_t gi = 0;
    uint64_t examined = 0;
    VRec vr{};
    LtRec rec{};
    LtTables T{nullptr, nullptr, nullptr};
    bool more = true;                      // the launch still has RR indices (uniform)

    for (;;) {
        // ---- one step of every walk whose load was issued in an earlier iteration ----
        bool done = false, abandon = false;
        if (active) {
            if (phase == 0) {
                start = (uint32_t)vr.start;
                deg = vr.deg & kDegMask;
                if (deg == 0) {
                    done = true;                        // the root has no in-edge
                } else {
                    examined += deg;
                    x = philox10(Ctr4{r, (uint32_t)v, t, kDomainLT}, k0, k1).x;
                    gi = 2 * (int64_t)start + (int64_t)(((uint64_t)x * (2ull * deg)) >> 32);
                    rec = load_ltrec(T.grec + 2 * gi);
                    phase = 1;
                }
            } else {
                if (!lt_ok(rec.cum, x)) {
                    // a threshold inside the draw's bucket: the pick is one of the next
                    // edges, most often the successor, whose record shares the guide's
                    // cache line (the list's last edge is saturated, so the scan ends)
                    rec = load_ltrec(T.grec + 2 * gi + 1);
                    if (!lt_ok(rec.cum, x)) {
                        uint32_t pos = T.gidx[gi] + 1;
                        do {
                            ++pos;
                            rec = load_ltrec(T.lrec + start + pos);
                        } while (!lt_ok(rec.cum, x) && pos + 1 < deg);
                    }
                }
                const int32_t u = rec.src;
                const uint32_t ustart = rec.start, udeg = rec.deg;
                // u's own step, issued before u is known to be new
                uint32_t ux = 0;
                int64_t ugi = 0;
                LtRec urec{};
                if (udeg > 0) {
                    ux = philox10(Ctr4{r, (uint32_t)u, t, kDomainLT}, k0, k1).x;
                    ugi = 2 * (int64_t)ustart + (int64_t)(((uint64_t)ux * (2ull * udeg)) >> 32);
                    urec = load_ltrec(T.grec + 2 * ugi);
                }
                const uint32_t hb = lt_filt_bit(u);
                bool hit = false;
                if ((filt[hb >> 5] >> (hb & 31)) & 1u) {    // u may be on the walk
                    const int32_t in_lds = min(size, lcap);
                    for (int32_t i = gl; i < in_lds; i += kLtGroup) hit |= list[i] == u;
                    for (int32_t i = gl; i < size - lcap; i += kLtGroup) hit |= ext[i] == u;
                }
                if ((ballot(hit) & gmask) != 0) {
                    done = true;                        // u is already on the walk
                } else if (size >= lcap + ecap) {
                    done = true;
                    abandon = true;
                } else {
                    if (gl == 0) {
                        if (size < lcap) list[size] = u;
                        else ext[size - lcap] = u;
                        filt[hb >> 5] |= 1u << (hb & 31);
                    }
                    ++size;
                    // the group's later scans read the extension entry written above
                    if (size > lcap) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    if (udeg == 0) {
                        done = true;                    // u has no in-edge
                    } else {
                        examined += udeg;
                        v = u;
                        start = ustart;
                        deg = udeg;
                        x = ux;
                        gi = ugi;
                        rec = urec;
                    }
                }
            }
        }
        wave_sync();
        // ---- finished walks, one group at a time ----
        uint64_t fin = ballot(done && gl == 0);
        while (fin) {
            const int b = __ffsll((unsigned long long)fin) - 1;
            fin &= fin - 1;
            const int32_t fi = __builtin_amdgcn_readlane(inst, b);
            const uint32_t fr = __builtin_amdgcn_readlane(r, b);
            const int32_t fs = __builtin_amdgcn_readlane(size, b);
            const uint64_t fe = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(examined >> 32), b) << 32) |
                                __builtin_amdgcn_readlane((uint32_t)examined, b);
            if (__builtin_amdgcn_readlane((int)abandon, b)) push_heavy(G, ws, fi, fr);
            else place_wave(G, ws, slot, fi, fr, lists[wib][b / kLtGroup], fs, fe,
                            ext_wave + (b / kLtGroup) * (int64_t)ecap, lcap);
        }
        if (done) active = false;
        wave_sync();
        // ---- idle groups start the launch's next walks: the root's record is loaded now
        // and read in the next iteration ----
        uint64_t idle = ballot(!active && gl == 0);
        while (idle && more) {
            int32_t wi;
            uint32_t wr;
            if (!next_set(G, ws, wi, wr)) {
                more = false;
                break;
            }
            const int g_new = (__ffsll((unsigned long long)idle) - 1) / kLtGroup;
            idle &= idle - 1;
            if (grp == g_new) {
                const GenInst& I = G.inst[wi];
                inst = wi;
                r = wr;
                T = lt_tables(I);
                k0 = I.k0;
                k1 = I.k1;
                t = I.round;
                v = (int32_t)root_of(r, (uint32_t)I.n, k0, k1);
                vr = load_vrec(global(I.vrec) + v);
                for (int i = gl; i < kLtFiltWords; i += kLtGroup) filt[i] = 0u;
                if (gl == 0) {
                    list[0] = v;
                    const uint32_t hb = lt_filt_bit(v);
                    filt[hb >> 5] |= 1u << (hb & 31);
                }
                size = 1;
                examined = 0;
                phase = 0;
                active = true;
            }
        }
        if (ballot(active) == 0) break;     // no walk left and no index left
        wave_sync();
    }
    wave_exit(G, ws, slot);
}

hipError_t launch_ic_light(const GenLaunch& a, int grid, hipStream_t s) {
    k_ic_light<<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

template <bool kBounded>
hipError_t launch_ic_heavy_t(const GenLaunch& a, int block, int grid, hipStream_t s) {
    switch (block) {
        case 64: k_ic_heavy<64, kBounded><<<grid, 64, 0, s>>>(a); break;
        case 128: k_ic_heavy<128, kBounded><<<grid, 128, 0, s>>>(a); break;
        case 256: k_ic_heavy<256, kBounded><<<grid, 256, 0, s>>>(a); break;
        case 1024: k_ic_heavy<1024, kBounded><<<grid, 1024, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ic_heavy(const GenLaunch& a, int block, int grid, hipStream_t s) {
    return a.over_list ? launch_ic_heavy_t<true>(a, block, grid, s) : launch_ic_heavy_t<false>(a, block, grid, s);
}

hipError_t launch_lt(const GenLaunch& a, bool big, int grid, hipStream_t s) {
    if (big) k_rr_lt_hbm<<<grid, kBlock, 0, s>>>(a);
    else k_lt_groups<<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

int lt_walks_per_block() { return kWavesPerBlock * kLtWalks; }

int gen_blocks_per_cu(int which) {
    int nb = 0;
    hipError_t e = hipSuccess;
    switch (which) {
        case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ic_light, kBlock, 0); break;
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ic_heavy<1024, true>, 1024, 0); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ic_heavy<256, true>, 256, 0); break;
        case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ic_heavy<128, true>, 128, 0); break;
        case 6: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ic_heavy<64, true>, 64, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_lt_groups, kBlock, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rr_lt_hbm, kBlock, 0); break;
    }
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

// One wave per instance.
__global__ void k_pool_summary(const GenInst* __restrict__ inst, int32_t ninst,
                               PoolSummary* __restrict__ out) {
    const int lane = lane_id();
    const int32_t i = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
    if (i >= ninst) return;
    PoolCounters* c = inst[i].ctr;
    const unsigned long long pl = wave_sum((uint64_t)c->placed[lane]);
    const unsigned long long ed = wave_sum((uint64_t)c->edges[lane]);
    const unsigned long long he = wave_sum((uint64_t)c->hedges[lane]);
    if (lane == 0) {
        PoolSummary o;
        o.tail = c->tail;
        o.placed = pl;
        o.edges = ed;
        o.hedges = he;
        o.n_capacity = c->n_capacity;
        o.max_len = c->max_len;
        out[i] = o;
        c->n_capacity = 0u;
    }
}

hipError_t launch_pool_summary(const GenInst* inst, int32_t ninst, PoolSummary* out,
                               hipStream_t s) {
    if (ninst <= 0) return hipSuccess;
    const int blocks = (ninst + kWavesPerBlock - 1) / kWavesPerBlock;
    k_pool_summary<<<blocks, kBlock, 0, s>>>(inst, ninst, out);
    return hipGetLastError();
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
