// Host-side launchers of libimm's HIP kernels (implemented in the .hip files).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace imm {

// Device-side counters of one pool (zeroed at pool creation).  Counters that every wave
// updates once per launch are spread over 64 slots (index = wave slot & 63).
struct alignas(64) PoolCounters {
    unsigned long long tail;       // next free entry of the id buffer (chunk reservations)
    unsigned int n_capacity;       // sets that found the id buffer full (this launch)
    unsigned int max_len;          // largest set the heavy kernel placed (all launches)
    unsigned int pad[12];
    unsigned long long placed[64]; // members written
    unsigned long long edges[64];  // in-edges examined by sets placed by the light kernel
    unsigned long long hedges[64]; // ... by the heavy kernel
};

// Counters of one generation launch (light + heavy), zeroed before the light launch.
struct alignas(64) LaunchCounters {
    unsigned long long work;       // light work-queue cursor
    unsigned int hwork;            // heavy work-queue cursor
    unsigned int n_heavy;          // sets the light launch queued for the heavy launch
    unsigned long long arena;      // handoff arena words in use
    unsigned int n_over;           // IC heavy sets that outgrew their slot's member list
    unsigned int pad[9];
};

// Host-bound summary of one pool's counters, written by launch_pool_summary.
struct PoolSummary {
    unsigned long long tail, placed, edges, hedges;
    unsigned int n_capacity;       // read and then cleared for the next launch
    unsigned int max_len;
};

constexpr int kGenFetch = 8;       // RR indices a wave takes per work-counter fetch (default)
constexpr int kGenFetchMax = 64;   // ... at most
constexpr int kGenIdChunk = 1024;  // id-buffer entries a light wave reserves at a time

// ---- graph.hip ----------------------------------------------------------------------
// Checks the CSR and weights; sets bits of *err: 1 offsets, 2 sources, 4 IC p, 8 LT w.
hipError_t launch_validate(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                           const float* ic_p, const uint32_t* lt_w, uint32_t* err,
                           hipStream_t s);
hipError_t launch_encode_ic(int64_t m, const float* p, uint32_t* thr, hipStream_t s);
// Per-vertex records; `thr` may be null (no IC encoding, no uniform detection).
hipError_t launch_build_vrec(int32_t n, const int64_t* in_off, const uint32_t* thr, VRec* vrec,
                             unsigned int* n_mixed, hipStream_t s);
hipError_t launch_encode_lt(int32_t n, const int64_t* in_off, const uint32_t* w, uint32_t* cum,
                            hipStream_t s);
// LT walk tables: edge records lrec[m], guide records grec[2m] and positions gidx[2m].
hipError_t launch_build_lt_tables(int32_t n, int64_t m, const uint32_t* cum, const int32_t* src,
                                  const VRec* vrec, LtRec* lrec, LtRec* grec, uint32_t* gidx,
                                  hipStream_t s);

// ---- rr_gen.hip ---------------------------------------------------------------------
// One (graph, pool) of a generation launch.  A launch covers any number of instances:
// its work items are the concatenation of every instance's RR indices.
struct GenInst {
    // graph
    const VRec* vrec;
    const int32_t* src;
    const uint32_t* thr;     // IC per-edge thresholds (padded to a multiple of 4 edges)
    const uint32_t* cum;     // LT cumulative thresholds
    const LtRec* lrec;       // LT walk tables (edge records, guide records and positions)
    const LtRec* grec;       // pairs: guide record, successor's record (4m)
    const uint32_t* gidx;
    int32_t n;
    uint32_t k0, k1;         // Philox key (pool seed)
    uint32_t round;          // third counter word of the edge draws (round of a
                             // multi-round set; 0 for plain sets)
    // RR indices of this launch: first + j, or list[j], for j in [0, count)
    int64_t first;
    const uint32_t* list;
    // pool outputs
    int32_t* ids;
    int64_t cap_ids;
    int64_t* rr_start;
    int32_t* rr_len;
    uint32_t* hist;
    PoolCounters* ctr;
    uint32_t* cap_list;      // RR indices that found the id buffer full
};

struct GenLaunch {
    const GenInst* inst;     // device array
    int32_t ninst;
    const int64_t* work_off; // device array [ninst + 1]: work items of instance i are
                             // [work_off[i], work_off[i+1])
    int64_t total;           // work_off[ninst]
    int64_t budget;          // 4-edge groups a light wave may examine for one set
    LaunchCounters* lc;
    unsigned long long* heavy_list;  // light -> heavy queue: instance << 32 | RR index
    // Per queue entry, the arena offset of the partial traversal the light kernel hands
    // over (IC sets abandoned at the budget: words size, head, in-edges examined (lo, hi),
    // then the members, of which [0, head) are expanded), or kNoHandoff: restart.  The
    // heavy kernel adds those in-edges to the light counters when it places the set.
    uint32_t* handoff;
    int32_t* arena;
    int64_t arena_cap;
    uint32_t n_queue;        // IC heavy launch: entries of heavy_list to process
    // IC heavy launch: sets whose members outgrow list_stride are dropped (their bitmap
    // bits cleared) and their queue entries appended here (count in lc->n_over), to be
    // drawn again from the root in slots of a full list; nullptr: list_stride holds any set
    unsigned long long* over_list;
    // LT walk over HBM lists: when set, the work items are heavy_in[0, total) (entries as
    // in heavy_list) instead of the instances' RR ranges
    const unsigned long long* heavy_in;
    // scratch, sized for the largest instance
    uint32_t* visited;       // light: one bitmap of vis_words words per wave slot
    uint32_t* hvisited;      // heavy: one bitmap per heavy slot
    int64_t vis_words;
    int32_t* hlist;          // heavy: one member list of list_stride entries per heavy slot
    int64_t list_stride;
    // LT first pass: members a walk keeps in LDS (at most kLtLdsCap), then in its group's
    // extension list in HBM (lt_ext_cap entries per walk slot of the grid)
    int32_t* lt_ext;
    int32_t lt_lds_cap;
    int32_t lt_ext_cap;
    int32_t light_cap;       // IC light kernel: members a set may hold on chip (<= 1024)
    int32_t fetch;           // RR indices a wave takes per work-counter fetch (queue depth)
};

constexpr int kLtLdsCap = 256;           // LDS entries per walk of the first LT pass
constexpr int kLtExtCap = 1024;          // extension entries per walk slot (default)

constexpr uint32_t kNoHandoff = 0xFFFFFFFFu;
constexpr int64_t kArenaWords = (int64_t)16 << 20;   // handoff arena: 64 MiB of int32
hipError_t launch_ic_light(const GenLaunch& a, int grid, hipStream_t s);   // 256-thread blocks
// block: threads per heavy set, 64, 128, 256 or 1024
hipError_t launch_ic_heavy(const GenLaunch& a, int block, int grid, hipStream_t s);
// big: walks too long for the on-chip list (HBM list and bitmap, one walk per wave);
// otherwise the first pass (several walks per wave, guide-table steps)
hipError_t launch_lt(const GenLaunch& a, bool big, int grid, hipStream_t s);
int lt_walks_per_block();          // walks one block of the first LT pass runs at once
                                   // (walk slots of a grid: grid x lt_walks_per_block())
int rr_light_capacity();
// Sums each instance's spread counters into out[i] and clears its n_capacity.
hipError_t launch_pool_summary(const GenInst* inst, int32_t ninst, PoolSummary* out,
                               hipStream_t s);
// occupancy in blocks per CU: 0 IC light, 1 IC heavy (1024), 2 LT, 3 LT with HBM lists,
// 4 IC heavy (256), 5 IC heavy (128), 6 IC heavy (64)
int gen_blocks_per_cu(int which);

// Sorts each set's members ascending into the host-bound export buffer.
hipError_t launch_gather_sets(const int64_t* rr_start, const int32_t* rr_len, int64_t first,
                              int64_t count, const int64_t* out_off, const int32_t* ids,
                              int32_t* out_ids, hipStream_t s);
hipError_t launch_set_sizes(const int32_t* rr_len, int64_t first, int64_t count, int64_t* sizes,
                            hipStream_t s);

// ---- select.hip ---------------------------------------------------------------------
hipError_t launch_hist_range(const int64_t* rr_start, const int32_t* rr_len, const int32_t* ids,
                             int64_t first, int64_t count, uint32_t* hist, hipStream_t s);
// Exclusive scan of int64 or uint32 values into int64 out[0..n] (out[n] = total).
hipError_t launch_scan_u32(const uint32_t* in, int64_t n, int64_t* out, int64_t* tmp,
                           hipStream_t s);
hipError_t launch_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* tmp,
                           hipStream_t s);
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_inv_scatter(const int64_t* rr_start, const int32_t* rr_len, const int32_t* ids,
                              int64_t first, int64_t count, uint32_t rel0, const int64_t* inv_off,
                              uint32_t* cursor, uint32_t* inv, hipStream_t s);
// The same index without per-entry device atomics: entries grouped by buckets of vertices,
// then placed per bucket (bcur: kInvBuckets cursors, pairs: one per entry).  Applies when
// inv_bucket_shift(n) != 0.
constexpr int kInvBuckets = 4096;  // vertex buckets of the bucketed index build at most
int32_t inv_bucket_shift(int64_t n);
hipError_t launch_inv_bucketed(const int64_t* rr_start, const int32_t* rr_len, const int32_t* ids,
                               int64_t first, int64_t count, uint32_t rel0, const int64_t* inv_off,
                               int64_t n, unsigned long long* bcur, uint2* pairs, int64_t pair_cap,
                               uint32_t* inv, hipStream_t s);
// out[v] = a[v] - b[v]
hipError_t launch_sub_u32(const uint32_t* a, const uint32_t* b, uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_copy_hist(const uint32_t* hist, int32_t* h, int32_t n, hipStream_t s);
// Hot set of a single-instance selection: h = hist (as launch_copy_hist), the histogram of
// the counts into cnt_hist (kSelectHotBuckets, zeroed), then the threshold and the hot list
// in increasing vertex order into hot_ids (hot_max) and hot_n (2 words, zeroed), and per 32
// vertices their hot bitmap and hot position into hot_words ((n + 31) / 32); blk_cnt holds
// hot_list_blocks(n) counts.
hipError_t launch_hot_prepare(const uint32_t* hist, int32_t* h, int64_t n, int32_t hot_max,
                              uint32_t* cnt_hist, uint32_t* blk_cnt, unsigned long long* hot_words,
                              int32_t* hot_ids, uint32_t* hot_n, hipStream_t s);
int64_t hot_list_blocks(int64_t n);
// All k rounds of greedy selection for one or more instances in one cooperative launch:
// per round a segmented argmax over every instance's counters, a grid barrier, the cover
// step of every instance, a grid barrier.
// Inverted-index segments one selection may read (sets of successive estimation phases).
constexpr int kMaxSegs = 16;
// Rounds of a multi-round RR set at most (parts of the selection's partition matroid).
constexpr int kMaxRounds = 32;

struct SelInst {
    int32_t n;
    int32_t k;
    int64_t first;                 // RR range [first, first + count) of the pool
    int64_t count;
    int32_t* h;                    // counters (n), -1 marks chosen vertices
    const int64_t* inv_off;        // inverted index (n + 1)
    const uint32_t* inv;           // relative RR indices
    const int64_t* rr_start;
    const int32_t* rr_len;
    const int32_t* ids;
    uint32_t* covered;             // count flags
    unsigned long long* keys;      // k argmax keys (zeroed)
    int32_t* seeds;                // k
    unsigned long long* n_covered; // zeroed
    // Estimation phases: the smallest coverage that passes the phase's test.  Greedy gains
    // never increase, so once (covered so far) + (rounds left) x (this round's gain) falls
    // below it the phase fails whatever the remaining seeds are, and the instance stops;
    // n_covered then receives that bound (below need: an upper bound of the coverage all
    // k rounds would have reached).  0: always run all k rounds.
    int64_t need;
    // A single-instance launch may read its index as segments: the entries of v are those
    // of every segment j, seg_inv[j][seg_off[j][v] .. seg_off[j][v + 1]).  nseg == 1 means
    // inv_off / inv alone (the only form multi-instance launches accept).
    int32_t nseg;
    // Partition matroid (multi-round sets, single-instance launches only): element v
    // belongs to part v / part_n, and a part whose taken[] count has reached part_k
    // offers no more elements.  part_n == 0: no constraint.
    int32_t part_n;
    int32_t part_k;
    int32_t pad0;
    int32_t* taken;                // per part (at most kMaxRounds), zeroed
    const int64_t* seg_off[kMaxSegs];
    const uint32_t* seg_inv[kMaxSegs];
    // Single-instance launches: hot set of at most hot_max vertices (0: off), prepared by
    // launch_hot_prepare (hot_n[0] vertices in hot_ids, in increasing order, hot_n[1] the
    // threshold; hot_words: per 32 vertices their hot bitmap (low half) and the hot position
    // of the first of them (high half)); h0 holds the initial counts (n).
    const uint32_t* h0;
    int32_t hot_max;
    int32_t pad1;
    const unsigned long long* hot_words;
    const uint32_t* hot_n;
    const int32_t* hot_ids;
    // Dense rounds (hot set of at most kSelectDenseHot vertices, hot_part non-null): a round
    // whose gain is at least dense_gain (0: never) counts each block's decrements of hot
    // vertices per hot position in LDS and stores them as the block's row of hot_part (grid
    // rows of hot_n[0] counts); the next argmax subtracts the column sums from the hot
    // counters.
    int32_t* hot_part;
    int32_t dense_gain;
    int32_t pad2;
};
constexpr int kSelectHotBuckets = 4096;   // entries of SelInst::cnt_hist
constexpr int kSelectHotPerBlock = 4096;  // hot vertices one block of the launch keeps at most
constexpr int kSelectDenseHot = 16384;    // hot set of dense rounds at most (LDS counts)
constexpr int kSelectDenseShare = 2048;   // ... and hot vertices per block at most
constexpr int kMaxCoopGrid = 1024;   // blocks of a cooperative selection launch at most
// Arrival counters of a hierarchical grid barrier (zeroed before each launch): block b
// arrives on sub[b % 16]; the last arrival of a group bumps top; all wait for top.
struct alignas(64) GridBarrier {
    unsigned int sub[16][16];      // one 64-byte line per group
    unsigned int top;
    unsigned int err;              // set when a barrier wait timed out
    unsigned int pad[14];
    unsigned long long bkeys[kMaxCoopGrid];  // single-instance selection: each block's argmax key
};
int select_coop_grid();            // blocks of the cooperative launch (co-resident)
int select_max_inst();             // instances one cooperative launch can take
// plain: an ordinary launch of the same grid (stream capture, some profilers)
hipError_t launch_select_coop(const SelInst* inst, int32_t ninst, int32_t maxk, GridBarrier* bar,
                              hipStream_t s, bool plain = false);
// ---- mr_sets.hip -----------------------------------------------------------------------
// The round pools of a multi-round pool (gIM Sec. IV-H): round t's sets, read by the merge.
struct MrSrc {
    const int64_t* start[kMaxRounds];
    const int32_t* len[kMaxRounds];
    const int32_t* ids[kMaxRounds];
    int32_t rounds;
    int32_t n_base;              // vertices of the graph: element of (u, t) is t * n_base + u
};
// sizes[i] = sum over t of the size of round t's set first + i.
hipError_t launch_mr_sizes(const MrSrc& src, int64_t first, int64_t count, int64_t* sizes,
                           hipStream_t s);
// Writes multi-round set first + i at ids[base + off[i] ...): the members of round 0, then
// round 1, ..., each member u of round t as t * n_base + u; sets rr_start / rr_len.
hipError_t launch_mr_copy(const MrSrc& src, int64_t first, int64_t count, const int64_t* off,
                          int64_t base, int64_t* rr_start, int32_t* rr_len, int32_t* ids,
                          hipStream_t s);

// ---- fwd_mc.hip ----------------------------------------------------------------------
// Out-edge lists of a graph, from its in-edge lists: out-degrees, then (after a scan into
// out_off) each in-edge (u -> v, e) placed in u's list as (v, e).
hipError_t launch_out_degree(int64_t m, const int32_t* src, uint32_t* deg, hipStream_t s);
hipError_t launch_out_scatter(int32_t n, const VRec* vrec, const int32_t* src, const int64_t* out_off,
                              uint32_t* cursor, int32_t* out_dst, uint32_t* out_eid, hipStream_t s);
// Forward Monte-Carlo simulations [0, sims) from a set of seed elements t * n + u.
struct FwdLaunch {
    const VRec* vrec;
    const uint32_t* w;            // IC thresholds or LT cumulative thresholds
    const int64_t* out_off;
    const int32_t* out_dst;
    const uint32_t* out_eid;      // in-edge index of each out-edge
    int32_t n;
    int32_t model;                // 0 IC, 1 LT
    int32_t rounds;
    uint32_t k0, k1;              // Philox key
    const int32_t* elems;
    int32_t nelem;
    int64_t sims;
    unsigned int* work;           // simulation cursor (zeroed)
    uint32_t* counts;             // per simulation: vertices reached in some round
    unsigned long long* sums;     // or null: [0] += count, [1] += count^2 per simulation
    uint32_t* vis;                // per slot: bitmap of the current round's search
    uint32_t* uvis;               // per slot: bitmap of the vertices reached so far (rounds > 1)
    int32_t* list;                // per slot: the round's reached vertices
    int32_t* ulist;               // per slot: vertices reached so far (rounds > 1)
    int64_t vis_words, list_stride;
};
hipError_t launch_spread_fwd(const FwdLaunch& a, int grid, hipStream_t s);

hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);

}  // namespace imm
