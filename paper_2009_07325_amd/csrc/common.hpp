// Shared device/host helpers of libimm (HIP, gfx950 wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imm {

constexpr int kWave = 64;
constexpr uint32_t kAlways = 0xFFFFFFFFu;   // saturated threshold: the edge is always live
constexpr uint32_t kDomainRoot = 1u, kDomainIC = 2u, kDomainLT = 3u;

// Per-vertex record of the in-edge CSR: one aligned 16-byte load per expanded vertex.
//   start   first in-edge index
//   deg     in-degree (bit 31 set when every in-edge of the vertex has the same IC
//           threshold, stored in `thr`; weighted cascade gives this for every vertex)
//   thr     that common threshold (valid only with the uniform bit)
struct alignas(16) VRec {
    int64_t start;
    uint32_t deg;
    uint32_t thr;
};
// Pointers read from device memory (per-instance descriptors) are generic to the
// compiler, which then emits flat accesses; global() restates that they address HBM so
// that loads, stores and atomics through them are global_* instructions.
#define IMM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ IMM_GLOBAL T* global(T* p) {
    return (IMM_GLOBAL T*)p;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte load of a vertex record.
__device__ __forceinline__ VRec load_vrec(const IMM_GLOBAL VRec* p) {
    const u32x4 v = *reinterpret_cast<const IMM_GLOBAL u32x4*>(p);
    VRec r;
    r.start = (int64_t)(((uint64_t)v.y << 32) | v.x);
    r.deg = v.z;
    r.thr = v.w;
    return r;
}

constexpr uint32_t kUniformBit = 0x80000000u;
constexpr uint32_t kDegMask = 0x7FFFFFFFu;

// LT in-edge record: everything one reverse-walk step needs from the edge it picks, in
// one aligned 16-byte load -- the edge's cumulative threshold, its source, and the
// source's in-edge range (so the next step needs no vertex-record load).
struct alignas(16) LtRec {
    uint32_t cum;
    int32_t src;
    uint32_t start;     // first in-edge of src (edge indices fit 32 bits)
    uint32_t deg;       // in-degree of src
};

__device__ __forceinline__ LtRec load_ltrec(const IMM_GLOBAL LtRec* p) {
    const u32x4 v = *reinterpret_cast<const IMM_GLOBAL u32x4*>(p);
    return LtRec{v.x, (int32_t)v.y, v.z, v.w};
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) -------------------------------
// Ten rounds of the Philox S-box on a 128-bit counter with a 64-bit key, the key advanced
// by the Weyl constants between rounds.
struct Ctr4 {
    uint32_t x, y, z, w;
};

// Three-input XOR in one instruction (v_bitop3_b32 with truth table 0x96); the compiler
// emits two v_xor_b32 for a ^ b ^ c.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

__device__ __forceinline__ Ctr4 philox10(Ctr4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t a = (uint64_t)c.x * 0xD2511F53u;
        const uint64_t b = (uint64_t)c.z * 0xCD9E8D57u;
        Ctr4 o;
        o.x = xor3((uint32_t)(b >> 32), c.y, k0);
        o.y = (uint32_t)b;
        o.z = xor3((uint32_t)(a >> 32), c.w, k1);
        o.w = (uint32_t)a;
        c = o;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint32_t root_of(uint32_t r, uint32_t n, uint32_t k0,
                                                     uint32_t k1) {
    Ctr4 w = philox10(Ctr4{r, 0u, 0u, kDomainRoot}, k0, k1);
    return (uint32_t)(((uint64_t)w.x * n) >> 32);
}

// ---- wave-level helpers --------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Orders this wave's LDS/global accesses across lanes (the role of __syncwarp in the
// paper's Sec. III-F): a wavefront-scope fence plus a scheduling barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Inclusive prefix sum over the 64 lanes.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        uint64_t o = __shfl_xor(v, d, kWave);
        v = o > v ? o : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T uniform(T v) {
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T atomic_add_agent(T* p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T atomic_add_agent(IMM_GLOBAL T* p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace imm
