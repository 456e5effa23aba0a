// Host-side launchers of libimm's HIP kernels (implemented in the .hip files).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace imm {

// Device-side counters of one pool (one 64-byte block, zeroed at pool creation).
struct alignas(64) PoolCounters {
    unsigned long long tail;       // next free slot of the id buffer (reservations)
    unsigned long long placed;     // members written (sum of sizes of placed sets)
    unsigned long long edges;      // in-edges examined
    unsigned long long work;       // work-queue cursor of the current launch
    unsigned int n_overflow;       // sets deferred by the current launch
    unsigned int n_capacity;       // sets that found the id buffer full
    unsigned int pad[6];
};

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

// ---- rr_gen.hip ---------------------------------------------------------------------
struct GenArgs {
    // graph
    const VRec* vrec;
    const int32_t* src;
    const uint32_t* thr;     // IC per-edge thresholds (null when every vertex is uniform)
    const uint32_t* cum;     // LT cumulative thresholds
    int32_t n;
    uint32_t k0, k1;         // Philox key
    // work: RR indices first + i for i in [0, count), or list[i] when list is set
    int64_t first;
    int64_t count;
    const uint32_t* list;
    // outputs
    int32_t* ids;
    int64_t cap_ids;
    int64_t* rr_start;
    int32_t* rr_len;
    uint32_t* hist;
    PoolCounters* ctr;
    uint32_t* ovf_list;      // deferred RR indices (too big for the on-chip list)
    uint32_t* cap_list;      // RR indices that found the id buffer full
    // scratch
    uint32_t* visited;       // one n-bit bitmap per wave slot
    int64_t vis_words;       // words per bitmap
    int32_t* big_list;       // one n-entry member list per wave slot (big-set launch)
};

// Launches the on-chip-list generator (sets larger than its list are deferred) or the
// big-set generator (member lists in HBM).  `grid` blocks of 256 threads.
hipError_t launch_rr_ic(const GenArgs& a, bool big, int grid, hipStream_t s);
hipError_t launch_rr_lt(const GenArgs& a, bool big, int grid, hipStream_t s);
int rr_small_capacity();           // members held on chip per set
int rr_blocks_per_cu(bool lt, bool big);

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
                              int64_t first, int64_t count, const int64_t* inv_off,
                              uint32_t* cursor, uint32_t* inv, hipStream_t s);
hipError_t launch_copy_hist(const uint32_t* hist, int32_t* h, int32_t n, hipStream_t s);
hipError_t launch_argmax(int32_t* h, int32_t n, int32_t round, const int32_t* seeds,
                         unsigned long long* keys, hipStream_t s);
hipError_t launch_cover(const unsigned long long* keys, int32_t round, const int64_t* inv_off,
                        const uint32_t* inv, const int64_t* rr_start, const int32_t* rr_len,
                        const int32_t* ids, int64_t first, uint8_t* covered, int32_t* h,
                        int32_t* seeds, unsigned long long* n_covered, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);

}  // namespace imm
