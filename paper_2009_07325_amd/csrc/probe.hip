// Measured peak of the IC generation roofline: the device's throughput of Philox4x32-10 as
// the generation kernels use it (a draw per 4 in-edges, its four words compared with a
// threshold and ballotted), with nothing else in the loop: no memory traffic, two
// independent draws per lane in flight.  bench.py prices the IC kernels against the
// arithmetic peak (40 VALU instructions per draw at one instruction per lane-cycle); this
// probe shows how much of that a real draw loop reaches.
#include <hip/hip_runtime.h>

#include "host.hpp"

namespace imm {

__global__ __launch_bounds__(256) void k_philox_rate(uint32_t k0, uint32_t k1, int64_t draws,
                                                     uint32_t thr, unsigned long long* out) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long acc = 0;
    for (int64_t i = 0; i < draws; i += 2) {
        const Ctr4 a = philox10(Ctr4{r, (uint32_t)i, 0u, kDomainIC}, k0, k1);
        const Ctr4 b = philox10(Ctr4{r, (uint32_t)i + 1u, 0u, kDomainIC}, k0, k1);
        acc += ballot(a.x < thr) ^ ballot(a.y < thr) ^ ballot(a.z < thr) ^ ballot(a.w < thr);
        acc += ballot(b.x < thr) ^ ballot(b.y < thr) ^ ballot(b.z < thr) ^ ballot(b.w < thr);
    }
    if (acc == 0x5A5A5A5A5A5A5A5Aull) out[0] = acc;   // keeps every draw live
}

}  // namespace imm

using namespace imm;

extern "C" imm_status imm_philox_rate(int64_t draws_per_lane, double* gphilox_s) {
    if (!gphilox_s) return fail(IMM_EINVAL, "gphilox_s is NULL");
    if (draws_per_lane < 2 || draws_per_lane > (1ll << 24))
        return fail(IMM_EINVAL, "draws_per_lane outside [2, 2^24]");
    draws_per_lane &= ~1ll;
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = cus * 8;                     // 8 waves per SIMD
    unsigned long long* out = nullptr;
    IMM_TRY(dalloc(&out, 1));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    imm_status st = IMM_OK;
    float ms = 0.0f;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = fail(IMM_EDEVICE, "hipEventCreate failed");
    } else {
        // one untimed launch, then the timed one
        k_philox_rate<<<grid, 256>>>(0x12345678u, 0x9ABCDEF0u, draws_per_lane, 0x01000000u, out);
        hipError_t e = hipEventRecord(e0, nullptr);
        k_philox_rate<<<grid, 256>>>(0x12345678u, 0x9ABCDEF0u, draws_per_lane, 0x01000000u, out);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess || ms <= 0.0f)
            st = fail(IMM_EDEVICE, "philox probe: %s", hipGetErrorString(e));
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dfree(out);
    if (st != IMM_OK) return st;
    *gphilox_s = (double)grid * 256.0 * (double)draws_per_lane / (ms * 1e-3) / 1e9;
    return IMM_OK;
}
