// Device probes beside the step kernels: the rate of random integer atomics.
// The update kernel's count additions are such atomics (one per destination
// that receives molecules, at random places of the next count buffer), and
// they execute at the memory side, so this rate bounds the update the way the
// copy kernel's bandwidth bounds a streaming kernel.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "rdos_internal.h"

namespace {

// A counter-based 32-bit hash (the "lowbias32" integer hash published by
// C. Wellons): spreads the probe's addresses uniformly without any state.
__device__ __forceinline__ uint32_t probe_hash(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

constexpr int kProbeBlocks = 1024, kProbeLanes = 256;

// Each lane adds 1 at per_lane random int32 slots of cnt[0, n); n < 2^32, so
// (h * n) >> 32 < n.  No result is returned to the lane, as in the update.
__global__ __launch_bounds__(kProbeLanes) void atomic_probe_kernel(int32_t *cnt, uint64_t n, int32_t per_lane,
                                                                   uint32_t seed)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int32_t k = 0; k < per_lane; ++k) {
        const uint32_t h = probe_hash((gid * (uint32_t)per_lane + (uint32_t)k) ^ seed);
        atomicAdd(cnt + (((uint64_t)h * n) >> 32), 1);
    }
}

}  // namespace

extern "C" rdos_status rdos_atomic_probe(int device, size_t bytes, int64_t n_atomics, int reps, double *per_s)
{
    const uint64_t n = bytes / sizeof(int32_t);
    if (!per_s || reps < 1 || n < 1 || n >= (uint64_t(1) << 32) || n_atomics < 1 || n_atomics > (int64_t(1) << 34))
        return RDOS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return RDOS_EDEVICE;
    const int64_t lanes = (int64_t)kProbeBlocks * kProbeLanes;
    const int32_t per_lane = (int32_t)((n_atomics + lanes - 1) / lanes);
    int32_t *cnt = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rdos_status rc = RDOS_OK;
    float ms = 0.f;
    bool allocated;
    {
        std::lock_guard<std::mutex> g(rdos::device_api_mutex());
        allocated = hipMalloc(&cnt, n * sizeof(int32_t)) == hipSuccess;
    }
    if (!allocated) {
        rc = RDOS_ENOMEM;
    } else if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
               hipEventCreate(&e1) != hipSuccess || hipMemsetAsync(cnt, 0, n * sizeof(int32_t), st) != hipSuccess) {
        rc = RDOS_EDEVICE;
    } else {
        // one untimed launch, then reps timed ones on fresh addresses
        atomic_probe_kernel<<<kProbeBlocks, kProbeLanes, 0, st>>>(cnt, n, per_lane, 0x9e3779b9u);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e0, st) != hipSuccess) rc = RDOS_EDEVICE;
        for (int i = 0; i < reps && rc == RDOS_OK; ++i) {
            atomic_probe_kernel<<<kProbeBlocks, kProbeLanes, 0, st>>>(cnt, n, per_lane, 0x85ebca6bu * (uint32_t)(i + 1));
            if (hipGetLastError() != hipSuccess) rc = RDOS_EDEVICE;
        }
        if (rc == RDOS_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f)))
            rc = RDOS_EDEVICE;
    }
    if (rc == RDOS_OK) *per_s = (double)lanes * per_lane * reps / ((double)ms * 1e-3);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    {
        std::lock_guard<std::mutex> g(rdos::device_api_mutex());
        if (cnt) (void)hipFree(cnt);
    }
    return rc;
}
