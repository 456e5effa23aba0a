// Multi-round RR sets (gIM Sec. IV-H, Table 3: multi-round influence maximisation, the
// CR-NAIMM algorithm of Sun et al., KDD'18).
//
// Influence spreads in T rounds, each an independent diffusion from that round's seeds; a
// multi-round RR set draws one root and runs one reverse search per round from it, in that
// round's own live-edge instance, and its elements are (vertex, round) pairs.  The library
// generates round t's searches as an ordinary pool whose draws carry t in the third counter
// word, so every round's set is produced by the same light / heavy / walk kernels; the
// kernels here lay the T searches of each index side by side as one set of elements
// t * n + u, the form the greedy (a partition matroid over the rounds) reads.
#include "kernels.hpp"

namespace imm {

__global__ void k_mr_sizes(MrSrc src, int64_t first, int64_t count, int64_t* __restrict__ sizes) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t acc = 0;
        for (int32_t t = 0; t < src.rounds; ++t) acc += src.len[t][first + i];
        sizes[i] = acc;
    }
}

hipError_t launch_mr_sizes(const MrSrc& src, int64_t first, int64_t count, int64_t* sizes,
                           hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_mr_sizes<<<(unsigned)blocks, 256, 0, s>>>(src, first, count, sizes);
    return hipGetLastError();
}

// One wave per set: the rounds' members are copied in round order, coalesced per round.
__global__ void k_mr_copy(MrSrc src, int64_t first, int64_t count, const int64_t* __restrict__ off,
                          int64_t base, int64_t* __restrict__ rr_start, int32_t* __restrict__ rr_len,
                          int32_t* __restrict__ ids) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t i = wave; i < count; i += nwaves) {
        const int64_t r = first + i;
        const int64_t dst = base + off[i];
        int64_t at = dst;
        for (int32_t t = 0; t < src.rounds; ++t) {
            const int64_t s0 = src.start[t][r];
            const int32_t len = src.len[t][r];
            const int32_t add = t * src.n_base;
            for (int32_t j = lane; j < len; j += kWave) ids[at + j] = src.ids[t][s0 + j] + add;
            at += len;
        }
        if (lane == 0) {
            rr_start[r] = dst;
            rr_len[r] = (int32_t)(at - dst);
        }
    }
}

hipError_t launch_mr_copy(const MrSrc& src, int64_t first, int64_t count, const int64_t* off,
                          int64_t base, int64_t* rr_start, int32_t* rr_len, int32_t* ids,
                          hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count * kWave + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_mr_copy<<<(unsigned)blocks, 256, 0, s>>>(src, first, count, off, base, rr_start, rr_len, ids);
    return hipGetLastError();
}

}  // namespace imm
