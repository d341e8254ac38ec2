// Stepping without device allocation: the occupied-tet queue that the scan
// and update kernels share (entries, counts, segment lengths, work header)
// lives in a file-scope device array instead of the simulation's own queue.
// For callers that cannot allocate device memory around the step.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "rdos_internal.h"
#include "rdos_sim.h"

namespace rdos {

// The queue of one call: header (256 B), segment lengths (2 x kMaxSegments x
// kLenStride int32), then the entries and their count rows.  Each device
// holds its own copy until the process ends.
constexpr size_t kStaticBytes = size_t(8) << 20;
constexpr size_t kStaticLenOffset = 256;
constexpr size_t kStaticEntryOffset = kStaticLenOffset + 2 * (size_t)kMaxSegments * kLenStride * sizeof(int32_t);

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, taken once per
// device: in host code the array's name is not a device address.
hipError_t scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// Zeroes both halves of the segment lengths and writes the work header (a
// kernel, not a memset or copy, so that the call can be captured).
__global__ __launch_bounds__(256) void static_queue_init(WorkHeader *hdr, int32_t *len, WorkHeader h)
{
    const int32_t n = 2 * kMaxSegments * kLenStride;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) len[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *hdr = h;
}

}  // namespace
}  // namespace rdos

using namespace rdos;

extern "C" rdos_status rdos_step_static(rdos_sim *s, int64_t n_steps)
{
    if (!s) return RDOS_EINVAL;
    if (s->engine_owned) return fail(s, RDOS_EBUSY, "simulation is owned by an engine");
    if (s->state != SimState::Ready) return fail(s, RDOS_ESTATE, "step before finalize");
    if (n_steps < 0) return fail(s, RDOS_EINVAL, "negative step count");
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_fail(s, e, "set device");
    // the queue geometry of the simulation's own work list
    int32_t nseg, seg_cap;
    queue_shape(s->n_tiles, &nseg, &seg_cap);
    const int64_t qcap = (int64_t)nseg * seg_cap;
    const int32_t rows = s->queue.species;
    const size_t need = kStaticEntryOffset + (size_t)qcap * (1 + (size_t)rows) * sizeof(int32_t);
    if (need > kStaticBytes)
        return fail(s, RDOS_EINVAL,
                    "work list too large for the static queue: %lld tiled tets x %d count rows need %zu bytes, "
                    "the static queue holds %zu (use rdos_step)",
                    (long long)qcap, rows, need, kStaticBytes);
    void *base = nullptr;
    e = scratch_address(s->device, &base);
    if (e != hipSuccess) return hip_fail(s, e, "static queue address");
    unsigned char *p = static_cast<unsigned char *>(base);
    QueueView q{};
    q.hdr = reinterpret_cast<WorkHeader *>(p);
    q.len = reinterpret_cast<int32_t *>(p + kStaticLenOffset);
    q.tet = reinterpret_cast<int32_t *>(p + kStaticEntryOffset);
    q.counts = q.tet + qcap;
    q.nseg = nseg;
    q.seg_cap = seg_cap;
    q.qcap = qcap;
    q.species = rows;
    q.scaled = s->queue.scaled;
    q.work = nullptr;
    q.owned = s->n_tiles <= kMaxSegments ? 1 : 0;
    WorkHeader h{};
    h.n_tiles = s->n_tiles;
    h.n_sims = 1;
    h.nseg = nseg;
    h.seg_cap = seg_cap;
    h.qcap = qcap;
    h.tile0 = 0;
    static_queue_init<<<64, 256, 0, s->stream>>>(q.hdr, q.len, h);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, "static queue set-up");
    for (int64_t i = 0; i < n_steps; ++i) {
        rdos_status st = ensure_mask(s);
        if (st != RDOS_OK) return st;
        e = launch_step(s->d_desc, s->d_tiles, s->step, -1, 0.0, q, (int32_t)(i & 1), scan_blocks_for(s->n_tiles),
                        s->update_bps, q.nseg, s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "launch period");
        s->step += 1;
    }
    return RDOS_OK;
}
