// Host side of the rdos C ABI: handles, call-order checks, mesh topology,
// device set-up and the stepping loop (Algorithm 1, Steps 1 and 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "rdos_internal.h"
#include "rdos_sim.h"

using namespace rdos;

namespace rdos {

rdos_status fail(rdos_sim *s, rdos_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->error = buf;
    return code;
}

rdos_status hip_fail(rdos_sim *s, hipError_t e, const char *what)
{
    return fail(s, e == hipErrorOutOfMemory ? RDOS_ENOMEM : RDOS_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(sim, expr, what)                         \
    do {                                                 \
        hipError_t e__ = (expr);                         \
        if (e__ != hipSuccess) return hip_fail(sim, e__, what); \
    } while (0)

int64_t padded_tets(int32_t T) { return ((int64_t)T + 3) & ~(int64_t)3; }

// Device memory of simulations, their queues and their set-up comes from a
// stream-ordered pool per device: allocation and release are ordered on the
// simulation's stream and never synchronise the whole device (hipFree can,
// which stalled admissions behind the engine's running chunks), and freed
// memory stays in the pool for the next simulation.
static hipMemPool_t pool_for(int device)
{
    static std::mutex mu;
    static hipMemPool_t pools[64] = {};
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> g(mu);
    if (!pools[device]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = device;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) != hipSuccess) return nullptr;
        uint64_t keep = ~0ull;  // never hand freed memory back to the driver
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        pools[device] = pool;
    }
    return pools[device];
}

hipError_t dev_alloc(void **p, size_t bytes, hipStream_t st)
{
    *p = nullptr;
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return e;
    hipMemPool_t pool = pool_for(device);
    if (!pool) return hipErrorOutOfMemory;
    return hipMallocFromPoolAsync(p, bytes ? bytes : 16, pool, st);
}

void dev_free(void *p, hipStream_t st)
{
    if (p) (void)hipFreeAsync(p, st);
}

size_t queue_bytes(int64_t n_tiles, int32_t n_species)
{
    int32_t nseg, seg_cap;
    queue_shape(n_tiles, &nseg, &seg_cap);
    return (size_t)nseg * seg_cap * (1 + (size_t)n_species) * sizeof(int32_t) +
           2 * (size_t)kMaxSegments * kLenStride * sizeof(int32_t) + sizeof(WorkHeader) +
           kPersistSyncWords * sizeof(uint32_t);
}

// Room for a work list of up to capacity_tiles tiles and n_species count rows.
hipError_t alloc_queue(QueueView *q, int64_t capacity_tiles, int32_t n_species, hipStream_t st)
{
    *q = QueueView{};
    queue_shape(capacity_tiles, &q->nseg, &q->seg_cap);
    q->qcap = (int64_t)q->nseg * q->seg_cap;
    q->species = std::max(n_species, 1);
    hipError_t e = dev_alloc((void **)&q->tet, (size_t)q->qcap * sizeof(int32_t), st);
    if (e == hipSuccess) e = dev_alloc((void **)&q->counts, (size_t)q->qcap * q->species * sizeof(int32_t), st);
    const size_t len_bytes = 2 * (size_t)kMaxSegments * kLenStride * sizeof(int32_t);
    if (e == hipSuccess) e = dev_alloc((void **)&q->len, len_bytes, st);
    if (e == hipSuccess) e = dev_alloc((void **)&q->hdr, sizeof(WorkHeader), st);
    if (e == hipSuccess) e = dev_alloc((void **)&q->sync, kPersistSyncWords * sizeof(uint32_t), st);
    if (e == hipSuccess) e = hipMemsetAsync(q->len, 0, len_bytes, st);
    return e;
}

// Points the queue at a work list of n_tiles tiles (<= its capacity) and
// n_sims descriptors; the kernels read these sizes from q->hdr.
hipError_t set_queue_work(QueueView *q, int64_t n_tiles, int32_t n_sims, hipStream_t st, int32_t tile0)
{
    int32_t nseg, seg_cap;
    queue_shape(n_tiles, &nseg, &seg_cap);
    if ((int64_t)nseg * seg_cap > q->qcap) return hipErrorInvalidValue;
    q->nseg = nseg;
    q->seg_cap = seg_cap;
    WorkHeader h{};
    h.n_tiles = (int32_t)n_tiles;
    h.n_sims = n_sims;
    h.nseg = nseg;
    h.seg_cap = seg_cap;
    h.qcap = q->qcap;
    h.tile0 = tile0;
    hipError_t e = hipMemcpyAsync(q->hdr, &h, sizeof h, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // h lives on this stack frame
    return e;
}

void free_queue(QueueView *q, hipStream_t st)
{
    dev_free(q->tet, st);
    dev_free(q->counts, st);
    dev_free(q->len, st);
    dev_free(q->hdr, st);
    dev_free(q->sync, st);
    *q = QueueView{};
}

static int64_t tiles_of(const rdos_sim *s) { return (int64_t)s->Rz * ((s->T + kTetsPerTile - 1) / kTetsPerTile); }

size_t state_bytes(const rdos_sim *s)
{
    const int64_t Tp = padded_tets(s->T);
    const size_t counts = (size_t)s->Rz * s->D.size() * (size_t)Tp * sizeof(int32_t);
    const size_t tiles = (size_t)tiles_of(s) * sizeof(Tile);
    const size_t masks = s->regions.empty() ? 0 : (size_t)s->T * sizeof(uint32_t);
    const size_t occupancy = 2 * (size_t)s->Rz * s->D.size() * mask_stride(Tp);
    return (size_t)s->T * sizeof(MeshRec) + 2 * counts + tiles + queue_bytes(tiles_of(s), (int32_t)s->D.size()) +
           masks + occupancy + sizeof(DevSim) + 64;
}

// Face-matching results are cached by mesh connectivity (the cell array):
// requests that share a lattice but move its vertices reuse them.  An entry
// shares the cell array of the simulation that made it and its neighbour
// table ([T][4] ints) with the simulations set up from it; nothing is copied.
struct TopologyCache {
    struct Entry {
        int32_t cell_verts = 4;
        std::shared_ptr<const std::vector<int32_t>> cells;
        std::shared_ptr<const int32_t> nbr;
        uint64_t last_use = 0;
    };
    std::mutex mu;
    std::multimap<uint64_t, Entry> entries;  // by hash of the cell array
    size_t bytes = 0;
    uint64_t clock = 0;
    static constexpr size_t kMaxBytes = size_t(1) << 30;
};

static TopologyCache &topology_cache()
{
    static TopologyCache c;
    return c;
}

static uint64_t hash_tets(const std::vector<int32_t> &tv)
{
    // Four independent multiply-rotate lanes over 64-bit words, folded at the
    // end: a hit is confirmed by comparing the arrays, so the hash only has to
    // spread keys, and independent lanes keep it near memory speed (a
    // byte-serial hash took about 15 ms for a million tetrahedra).
    const uint64_t m = 0x9e3779b97f4a7c15ull;
    const size_t nb = tv.size() * sizeof(int32_t);
    const unsigned char *p = reinterpret_cast<const unsigned char *>(tv.data());
    uint64_t h[4] = {0x243f6a8885a308d3ull, 0x13198a2e03707344ull, 0xa4093822299f31d0ull, 0x082efa98ec4e6c89ull};
    size_t i = 0;
    for (; i + 32 <= nb; i += 32)
        for (int j = 0; j < 4; ++j) {
            uint64_t w;
            std::memcpy(&w, p + i + 8 * j, 8);
            const uint64_t x = h[j] ^ w;
            h[j] = ((x << 29) | (x >> 35)) * m;
        }
    uint64_t r = nb;
    for (; i < nb; ++i) r = (r ^ p[i]) * 1099511628211ull;
    for (int j = 0; j < 4; ++j) {
        r = (r ^ h[j]) * m;
        r ^= r >> 31;
    }
    return r;
}

// A neighbour table of n ints, left uninitialized for its producer to fill.
static std::shared_ptr<int32_t> new_table(size_t n)
{
    return std::shared_ptr<int32_t>(new int32_t[n], std::default_delete<int32_t[]>());
}

// The cached neighbour table of this simulation's connectivity, or null;
// *hash receives the key for topology_insert.
static std::shared_ptr<const int32_t> topology_lookup(rdos_sim *s, uint64_t *hash)
{
    TopologyCache &c = topology_cache();
    const uint64_t h = hash_tets(*s->tet_verts) ^ (uint64_t)s->cell_verts;
    *hash = h;
    std::lock_guard<std::mutex> g(c.mu);
    auto range = c.entries.equal_range(h);
    for (auto it = range.first; it != range.second; ++it)
        if (it->second.cell_verts == s->cell_verts &&
            (it->second.cells == s->tet_verts || *it->second.cells == *s->tet_verts)) {
            it->second.last_use = ++c.clock;
            return it->second.nbr;
        }
    return nullptr;
}

// Adds a table made for this simulation's connectivity (least recently used
// entries make room).
static void topology_insert(rdos_sim *s, uint64_t h, std::shared_ptr<const int32_t> nbr)
{
    TopologyCache &c = topology_cache();
    std::lock_guard<std::mutex> g(c.mu);
    const size_t add = (s->tet_verts->size() + 4 * (size_t)s->T) * sizeof(int32_t);
    while (!c.entries.empty() && c.bytes + add > TopologyCache::kMaxBytes) {
        auto old = c.entries.begin();
        for (auto it = c.entries.begin(); it != c.entries.end(); ++it)
            if (it->second.last_use < old->second.last_use) old = it;
        c.bytes -= (old->second.cells->size() + 4 * (old->second.cells->size() / old->second.cell_verts)) *
                   sizeof(int32_t);
        c.entries.erase(old);
    }
    if (add > TopologyCache::kMaxBytes) return;
    TopologyCache::Entry en;
    en.cell_verts = s->cell_verts;
    en.cells = s->tet_verts;
    en.nbr = std::move(nbr);
    en.last_use = ++c.clock;
    c.entries.emplace(h, std::move(en));
    c.bytes += add;
}

// Face matching runs on the device (launch_face_match) for meshes of at least
// 16384 cells whose vertex ids pack into a 64-bit key (*bits: bits per vertex
// id).  The sort makes it O(T) where the host sort is O(T log T): about a
// second on the host for a million tetrahedra.
static bool device_match_applies(const rdos_sim *s, int32_t *bits)
{
    int32_t b = 1;
    while (b < 31 && ((int64_t)1 << b) < (int64_t)s->n_verts) ++b;
    *bits = b;
    return s->T >= 16384 && !(s->cell_verts == 4 && b > 21) && (int64_t)s->T * 4 <= 0x7fffffff;
}

rdos_status build_topology_uncached(rdos_sim *s, std::vector<int32_t> &nbr);

// Edge matching for a surface of triangles: each edge (opposite local vertex
// e) keyed by its sorted vertex pair; slot 3 of every triangle is a boundary.
static rdos_status build_edges(rdos_sim *s, std::vector<int32_t> &nbr)
{
    struct EdgeKey {
        int32_t a, b;
        int32_t slot;  // 4 * triangle + edge
    };
    const int32_t T = s->T;
    std::vector<EdgeKey> keys((size_t)T * 3);
    for (int32_t t = 0; t < T; ++t) {
        const int32_t *v = &(*s->tet_verts)[3 * (size_t)t];
        for (int e = 0; e < 3; ++e) {
            const int32_t p = v[e == 0 ? 1 : 0], q = v[e <= 1 ? 2 : 1];
            keys[3 * (size_t)t + e] = {std::min(p, q), std::max(p, q), 4 * t + e};
        }
    }
    std::sort(keys.begin(), keys.end(), [](const EdgeKey &x, const EdgeKey &y) {
        if (x.a != y.a) return x.a < y.a;
        if (x.b != y.b) return x.b < y.b;
        return x.slot < y.slot;
    });
    nbr.assign((size_t)T * 4, -1);
    for (size_t i = 0; i < keys.size();) {
        size_t j = i + 1;
        while (j < keys.size() && keys[j].a == keys[i].a && keys[j].b == keys[i].b) ++j;
        if (j - i > 2)
            return fail(s, RDOS_EINVAL, "edge (%d,%d) is shared by %zu triangles", keys[i].a, keys[i].b, j - i);
        if (j - i == 2) {
            const int32_t t0 = keys[i].slot / 4, t1 = keys[i + 1].slot / 4;
            if (t0 == t1) return fail(s, RDOS_EINVAL, "triangle %d repeats an edge", t0);
            nbr[keys[i].slot] = t1;
            nbr[keys[i + 1].slot] = t0;
        }
        i = j;
    }
    return RDOS_OK;
}

// Face matching: each face is keyed by its sorted vertex triple; two tets with
// the same key are neighbours across it.  A key seen three times is an error.
rdos_status build_topology_uncached(rdos_sim *s, std::vector<int32_t> &nbr)
{
    if (s->cell_verts == 3) return build_edges(s, nbr);
    struct FaceKey {
        int32_t a, b, c;
        int32_t slot;  // 4 * tet + face
    };
    const int32_t T = s->T;
    std::vector<FaceKey> keys((size_t)T * 4);
    for (int32_t t = 0; t < T; ++t) {
        const int32_t *v = &(*s->tet_verts)[4 * (size_t)t];
        for (int f = 0; f < 4; ++f) {
            std::array<int32_t, 3> tri;
            int q = 0;
            for (int i = 0; i < 4; ++i)
                if (i != f) tri[q++] = v[i];
            std::sort(tri.begin(), tri.end());
            keys[4 * (size_t)t + f] = {tri[0], tri[1], tri[2], 4 * t + f};
        }
    }
    std::sort(keys.begin(), keys.end(), [](const FaceKey &x, const FaceKey &y) {
        if (x.a != y.a) return x.a < y.a;
        if (x.b != y.b) return x.b < y.b;
        if (x.c != y.c) return x.c < y.c;
        return x.slot < y.slot;
    });
    nbr.assign((size_t)T * 4, -1);
    const size_t nF = keys.size();
    for (size_t i = 0; i < nF;) {
        size_t j = i + 1;
        while (j < nF && keys[j].a == keys[i].a && keys[j].b == keys[i].b && keys[j].c == keys[i].c) ++j;
        if (j - i > 2)
            return fail(s, RDOS_EINVAL, "face (%d,%d,%d) is shared by %zu tetrahedra", keys[i].a, keys[i].b,
                        keys[i].c, j - i);
        if (j - i == 2) {
            const int32_t t0 = keys[i].slot / 4, t1 = keys[i + 1].slot / 4;
            if (t0 == t1) return fail(s, RDOS_EINVAL, "tetrahedron %d repeats a face", t0);
            nbr[keys[i].slot] = t1;
            nbr[keys[i + 1].slot] = t0;
        }
        i = j;
    }
    return RDOS_OK;
}

rdos_status upload_desc(rdos_sim *s)
{
    HIP_TRY(s, hipMemcpyAsync(s->d_desc, &s->desc, sizeof(DevSim), hipMemcpyHostToDevice, s->stream),
            "upload simulation descriptor");
    HIP_TRY(s, hipStreamSynchronize(s->stream), "upload simulation descriptor");
    return RDOS_OK;
}

// The kernels read the state of period k from buf[k & 1]; the descriptor's
// buf[] follows the handle's buffers, which swap when set_state changes the
// parity of the period index (the other buffer is all zero between periods).
rdos_status match_parity(rdos_sim *s)
{
    if (s->desc.buf[0] == s->d_buf[0] && s->desc.buf[1] == s->d_buf[1] && s->desc.mask[0] == s->d_mask[0] &&
        s->desc.mask[1] == s->d_mask[1])
        return RDOS_OK;
    s->desc.buf[0] = s->d_buf[0];
    s->desc.buf[1] = s->d_buf[1];
    s->desc.mask[0] = s->d_mask[0];
    s->desc.mask[1] = s->d_mask[1];
    return upload_desc(s);
}

// The scan reads only count vectors whose occupancy byte is set; after the
// host wrote counts, the map of the current buffer is rebuilt from them
// (and the other one cleared) before the next period runs.
rdos_status ensure_mask(rdos_sim *s)
{
    if (!s->mask_dirty) return RDOS_OK;
    const int64_t Tp = padded_tets(s->T);
    const int p = (int)(s->step & 1);
    HIP_TRY(s, launch_mask_build(s->d_buf[p], s->d_mask[p], s->d_mask[p ^ 1], occupancy_tag(s->step), s->Rz,
                                 (int32_t)s->D.size(), Tp, s->stream),
            "rebuild occupancy");
    s->mask_dirty = false;
    return RDOS_OK;
}

rdos_status check_flags(rdos_sim *s)
{
    int32_t flags = 0;
    HIP_TRY(s, hipMemcpyAsync(&flags, s->d_flags, sizeof flags, hipMemcpyDeviceToHost, s->stream),
            "read flags");
    HIP_TRY(s, hipStreamSynchronize(s->stream), "synchronize");
    if (flags & 1) return fail(s, RDOS_EOVERFLOW, "a molecule count overflowed int32");
    if (flags & 4) return fail(s, RDOS_EDEVICE, "occupied-tet queue overflowed (internal error)");
    if (flags & 8) return fail(s, RDOS_EDEVICE, "a grid barrier of the one-launch path timed out (internal error)");
    if (flags & 2)
        return fail(s, RDOS_EOVERFLOW, "a tet fired more than %u reactions in one period; shorten tau",
                    kMaxEventsPerPeriod);
    return RDOS_OK;
}

rdos_status enqueue_period(rdos_sim *s, int64_t period, int64_t partial, double tau_last)
{
    rdos_status st = ensure_mask(s);
    if (st != RDOS_OK) return st;
    if (s->launch_mode == 3 && s->queue.species <= kFusedSpecies) {
        // one fused launch; the queue's length halves stay as they are, so
        // the two-launch path that may follow keeps its parity
        HIP_TRY(s, launch_fused(s->d_desc, s->d_tiles, period, partial, tau_last, s->queue,
                                scan_blocks_for(s->n_tiles), s->stream),
                "launch period");
        return RDOS_OK;
    }
    HIP_TRY(s, launch_step(s->d_desc, s->d_tiles, period, partial, tau_last, s->queue, (int32_t)(s->launches & 1),
                           scan_blocks_for(s->n_tiles), s->update_bps, s->queue.nseg, s->stream),
            "launch period");
    s->launches += 1;
    return RDOS_OK;
}

// Grid of the one-launch path for this simulation, or 0 when it does not
// apply (launch mode 0: work lists of at most kPersistTiles tiles; 1 and 3:
// never; 2: always).  Blocks beyond what a cooperative launch may hold stride over
// the tiles and queue segments.
int32_t persist_grid(rdos_sim *s)
{
    if (s->launch_mode == 1 || s->launch_mode == 3 || (s->launch_mode == 0 && s->n_tiles > kPersistTiles)) return 0;
    if (s->persist_limit < 0) s->persist_limit = persist_grid_limit(s->queue);
    // four blocks per queue segment, so that a segment's tets are shared by
    // 1024 lanes
    const int32_t need = std::max(4 * s->queue.nseg, scan_blocks_for(s->n_tiles));
    return s->persist_limit > 0 ? std::min(need, s->persist_limit) : 0;
}

// n periods from the current one; the last lasts tau_last when `partial`
// (Algorithm 1, Step 1), all others tau.
rdos_status enqueue_run(rdos_sim *s, int64_t n, bool partial, double tau_last)
{
    if (n <= 0) return RDOS_OK;
    const int32_t grid = persist_grid(s);
    if (grid <= 0) {
        for (int64_t i = 0; i < n; ++i) {
            const bool last = partial && i == n - 1;
            rdos_status st = enqueue_period(s, s->step, last ? s->step : -1, last ? tau_last : 0.0);
            if (st != RDOS_OK) return st;
            s->step += 1;
        }
        return RDOS_OK;
    }
    rdos_status st = ensure_mask(s);
    if (st != RDOS_OK) return st;
    const int64_t partial_index = partial ? s->step + n - 1 : -1;
    while (n > 0) {
        const int32_t len = (int32_t)std::min<int64_t>(n, kPersistPeriods);
        HIP_TRY(s, launch_persist(s->d_desc, s->d_tiles, s->step, len, (int32_t)(s->launches & 1), partial_index,
                                  tau_last, s->queue, grid, s->queue.sync, s->stream),
                "launch periods");
        s->launches += len;
        s->step += len;
        n -= len;
    }
    return RDOS_OK;
}

double time_of(const rdos_sim *s, int64_t k)
{
    return s->anchor_t + (double)(k - s->anchor_step) * s->tau;
}

void free_device(rdos_sim *s)
{
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    std::lock_guard<std::mutex> g(device_api_mutex());
    void *ptrs[] = {s->d_mesh, s->d_buf[0], s->d_buf[1], s->d_mask[0], s->d_mask[1], s->d_flags, s->d_desc,
                    s->d_tiles, s->d_allowed};
    for (void *p : ptrs) dev_free(p, s->stream);
    free_queue(&s->queue, s->stream);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    s->d_mask[0] = s->d_mask[1] = nullptr;
    s->d_mesh = nullptr;
    s->d_allowed = nullptr;
    s->d_buf[0] = s->d_buf[1] = s->d_flags = nullptr;
    s->d_desc = nullptr;
    s->d_tiles = nullptr;
    if (s->stream && s->own_stream) (void)hipStreamDestroy(s->stream);
    s->stream = nullptr;
}

}  // namespace rdos

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#define CHECK_HANDLE(s)                                   \
    do {                                                  \
        if (!(s)) return RDOS_EINVAL;                     \
        if ((s)->engine_owned) return fail(s, RDOS_EBUSY, "simulation is owned by an engine"); \
    } while (0)

extern "C" {

rdos_status rdos_create(rdos_sim **out, int device, uint64_t seed, int32_t n_realizations)
{
    if (!out) return RDOS_EINVAL;
    *out = nullptr;
    if (n_realizations < 1) return RDOS_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RDOS_EDEVICE;
    rdos_sim *s = new (std::nothrow) rdos_sim();
    if (!s) return RDOS_ENOMEM;
    s->device = device;
    s->seed = seed;
    s->Rz = n_realizations;
    *out = s;
    return RDOS_OK;
}

rdos_status rdos_set_mesh(rdos_sim *s, int32_t n_verts, const double *xyz, int32_t n_tets,
                          const int32_t *tet_verts)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Created) return fail(s, RDOS_ESTATE, "set_mesh after the mesh was set");
    if (n_verts < 4 || n_tets < 1 || !xyz || !tet_verts)
        return fail(s, RDOS_EINVAL, "mesh needs >= 4 vertices and >= 1 tetrahedron");
    for (int64_t i = 0; i < 3 * (int64_t)n_verts; ++i)
        if (!std::isfinite(xyz[i])) return fail(s, RDOS_EINVAL, "vertex coordinate %lld is not finite", (long long)i);
    for (int64_t i = 0; i < 4 * (int64_t)n_tets; ++i)
        if (tet_verts[i] < 0 || tet_verts[i] >= n_verts)
            return fail(s, RDOS_EINVAL, "vertex id %d out of range at %lld", tet_verts[i], (long long)i);
    s->xyz.assign(xyz, xyz + 3 * (size_t)n_verts);
    s->tet_verts = std::make_shared<const std::vector<int32_t>>(tet_verts, tet_verts + 4 * (size_t)n_tets);
    s->n_verts = n_verts;
    s->T = n_tets;
    s->state = SimState::Meshed;
    return RDOS_OK;
}

rdos_status rdos_set_surface_mesh(rdos_sim *s, int32_t n_verts, const double *xyz, int32_t n_tris,
                                  const int32_t *tri_verts)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Created) return fail(s, RDOS_ESTATE, "set_surface_mesh after the mesh was set");
    if (n_verts < 3 || n_tris < 1 || !xyz || !tri_verts)
        return fail(s, RDOS_EINVAL, "surface needs >= 3 vertices and >= 1 triangle");
    for (int64_t i = 0; i < 3 * (int64_t)n_verts; ++i)
        if (!std::isfinite(xyz[i])) return fail(s, RDOS_EINVAL, "vertex coordinate %lld is not finite", (long long)i);
    for (int64_t i = 0; i < 3 * (int64_t)n_tris; ++i)
        if (tri_verts[i] < 0 || tri_verts[i] >= n_verts)
            return fail(s, RDOS_EINVAL, "vertex id %d out of range at %lld", tri_verts[i], (long long)i);
    s->xyz.assign(xyz, xyz + 3 * (size_t)n_verts);
    s->tet_verts = std::make_shared<const std::vector<int32_t>>(tri_verts, tri_verts + 3 * (size_t)n_tris);
    s->cell_verts = 3;
    s->n_verts = n_verts;
    s->T = n_tris;
    s->state = SimState::Meshed;
    return RDOS_OK;
}

rdos_status rdos_add_species(rdos_sim *s, double D, int32_t *out_id)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Meshed) return fail(s, RDOS_ESTATE, "add_species needs a mesh and no finalize yet");
    if (!(D >= 0.0) || !std::isfinite(D)) return fail(s, RDOS_EINVAL, "D must be finite and >= 0");
    if ((int)s->D.size() >= kMaxSpecies) return fail(s, RDOS_EINVAL, "at most %d species", kMaxSpecies);
    s->D.push_back(D);
    if (out_id) *out_id = (int32_t)s->D.size() - 1;
    return RDOS_OK;
}

rdos_status rdos_add_reaction(rdos_sim *s, int32_t n_reac, const int32_t *reac, int32_t n_prod,
                              const int32_t *prod, double k, int32_t *out_id)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Meshed) return fail(s, RDOS_ESTATE, "add_reaction needs a mesh and no finalize yet");
    if (n_reac < 0 || n_reac > 2 || n_prod < 0 || n_prod > 3)
        return fail(s, RDOS_EINVAL, "0..2 reactants and 0..3 products");
    if ((n_reac && !reac) || (n_prod && !prod)) return fail(s, RDOS_EINVAL, "null species list");
    if (!(k >= 0.0) || !std::isfinite(k)) return fail(s, RDOS_EINVAL, "rate constant must be finite and >= 0");
    if ((int)s->rx.size() >= kMaxReactions) return fail(s, RDOS_EINVAL, "at most %d reactions", kMaxReactions);
    Reaction r;
    r.rn = n_reac;
    r.pn = n_prod;
    for (int i = 0; i < n_reac; ++i) {
        if (reac[i] < 0 || reac[i] >= (int32_t)s->D.size()) return fail(s, RDOS_EINVAL, "reactant id out of range");
        r.r[i] = reac[i];
    }
    for (int i = 0; i < n_prod; ++i) {
        if (prod[i] < 0 || prod[i] >= (int32_t)s->D.size()) return fail(s, RDOS_EINVAL, "product id out of range");
        r.p[i] = prod[i];
    }
    r.k = k;
    s->rx.push_back(r);
    if (out_id) *out_id = (int32_t)s->rx.size() - 1;
    return RDOS_OK;
}

rdos_status rdos_set_method(rdos_sim *s, int32_t occupancy_correction, int32_t split_threshold,
                            int32_t tau_outliers)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Meshed) return fail(s, RDOS_ESTATE, "set_method needs a mesh and no finalize yet");
    if (split_threshold < 1 || tau_outliers < 0)
        return fail(s, RDOS_EINVAL, "split_threshold must be >= 1 and tau_outliers >= 0");
    s->first_order = occupancy_correction ? 0 : 1;
    s->split_threshold = split_threshold;
    s->tau_outliers = tau_outliers;
    return RDOS_OK;
}

rdos_status rdos_set_transfer_form(rdos_sim *s, int32_t form)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Meshed)
        return fail(s, RDOS_ESTATE, "set_transfer_form needs a mesh and no finalize yet");
    if (form != 0 && form != 1) return fail(s, RDOS_EINVAL, "transfer form must be 0 or 1");
    s->transfer_form = form;
    return RDOS_OK;
}

rdos_status rdos_set_reaction_region(rdos_sim *s, int32_t reaction, int32_t n_tets, const int32_t *tets)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Meshed)
        return fail(s, RDOS_ESTATE, "set_reaction_region needs a mesh and no finalize yet");
    if (reaction < 0 || reaction >= (int32_t)s->rx.size()) return fail(s, RDOS_EINVAL, "reaction id out of range");
    if (n_tets < 0 || (n_tets > 0 && !tets)) return fail(s, RDOS_EINVAL, "bad tet list");
    std::vector<int32_t> v(tets, tets + n_tets);
    for (int32_t t : v)
        if (t < 0 || t >= s->T) return fail(s, RDOS_EINVAL, "tet id %d out of range", t);
    s->regions[reaction] = std::move(v);
    return RDOS_OK;
}

rdos_status rdos_finalize(rdos_sim *s, double tau_scale, double *out_tau)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Meshed) return fail(s, RDOS_ESTATE, "finalize needs a mesh and must run once");
    if (s->D.empty()) return fail(s, RDOS_EINVAL, "no species");
    if (!(tau_scale > 0.0 && tau_scale <= 1.0)) return fail(s, RDOS_EINVAL, "tau_scale must be in (0, 1]");
    for (const Reaction &r : s->rx)
        for (int i = 0; i < r.pn; ++i)
            if (r.p[i] >= (int32_t)s->D.size()) return fail(s, RDOS_EINVAL, "product id out of range");
    // one realization's counts are addressed with 32-bit byte offsets
    if ((int64_t)s->D.size() * padded_tets(s->T) * 4 > 0x7fffffff)
        return fail(s, RDOS_EINVAL, "tets x species of one realization exceed 2^29");
    // queue entries are int32 (tile * kTetsPerTile + offset): the tiled work
    // list, not only realizations x tets, must stay below 2^31
    if (tiles_of(s) * kTetsPerTile > 0x7fffffff)
        return fail(s, RDOS_EINVAL, "realizations x tiled tets exceed 2^31");
    HIP_TRY(s, hipSetDevice(s->device), "set device");
    if (!s->stream) {
        HIP_TRY(s, hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "create stream");
        s->own_stream = true;
    }
    // Face matching (step a0): the cached table of this connectivity, else
    // matching on the device in the set-up buffers below, else on the host.
    const int32_t T = s->T;
    const size_t nbr_n = 4 * (size_t)T;
    uint64_t topo_hash = 0;
    std::shared_ptr<const int32_t> nbr_table = topology_lookup(s, &topo_hash);
    const bool fresh = !nbr_table;
    int32_t bits = 0;
    bool on_device = fresh && device_match_applies(s, &bits);
    rdos_status st = RDOS_OK;
    if (fresh && !on_device) {
        std::vector<int32_t> host;
        st = build_topology_uncached(s, host);
        if (st != RDOS_OK) return st;
        std::shared_ptr<int32_t> t = new_table(nbr_n);
        std::memcpy(t.get(), host.data(), nbr_n * sizeof(int32_t));
        nbr_table = t;
    }
    const int S = (int)s->D.size();
    const int64_t Tp = padded_tets(T);
    const size_t count_bytes = (size_t)s->Rz * S * (size_t)Tp * sizeof(int32_t);
    const size_t mask_bytes = (size_t)s->Rz * S * mask_stride(Tp);

    // temporary set-up buffers
    double *d_xyz = nullptr, *d_vol = nullptr, *d_bc = nullptr, *d_area = nullptr, *d_D = nullptr;
    int32_t *d_tv = nullptr, *d_nbr = nullptr, *d_match_err = nullptr;
    void *d_match = nullptr;
    unsigned long long *d_tau = nullptr;
    std::unique_lock<std::mutex> alloc_lock(device_api_mutex(), std::defer_lock);
    auto cleanup = [&]() {
        if (s->stream) (void)hipStreamSynchronize(s->stream);
        std::unique_lock<std::mutex> g(device_api_mutex(), std::defer_lock);
        if (!alloc_lock.owns_lock()) g.lock();
        void *p[] = {d_xyz, d_vol, d_bc, d_area, d_D, d_tv, d_nbr, d_tau, d_match_err, d_match};
        for (void *q : p) dev_free(q, s->stream);
    };
#define SETUP_TRY(expr, what)                               \
    do {                                                    \
        hipError_t e__ = (expr);                            \
        if (e__ != hipSuccess) {                            \
            if (alloc_lock.owns_lock()) alloc_lock.unlock(); \
            cleanup();                                      \
            free_device(s);                                 \
            return hip_fail(s, e__, what);                  \
        }                                                   \
    } while (0)
    alloc_lock.lock();
    SETUP_TRY(dev_alloc((void **)&s->d_mesh, (size_t)T * sizeof(MeshRec), s->stream), "allocate mesh tables");
    SETUP_TRY(dev_alloc((void **)&s->d_buf[0], count_bytes, s->stream), "allocate counts");
    SETUP_TRY(dev_alloc((void **)&s->d_buf[1], count_bytes, s->stream), "allocate counts");
    SETUP_TRY(dev_alloc((void **)&s->d_mask[0], mask_bytes, s->stream), "allocate occupancy");
    SETUP_TRY(dev_alloc((void **)&s->d_mask[1], mask_bytes, s->stream), "allocate occupancy");
    SETUP_TRY(dev_alloc((void **)&s->d_flags, 64, s->stream), "allocate flags");
    SETUP_TRY(dev_alloc((void **)&s->d_desc, sizeof(DevSim), s->stream), "allocate descriptor");
    SETUP_TRY(alloc_queue(&s->queue, tiles_of(s), S, s->stream), "allocate queue");
    s->queue.owned = tiles_of(s) <= kMaxSegments ? 1 : 0;  // a segment and a scan wavefront per tile
    SETUP_TRY(dev_alloc((void **)&d_xyz, s->xyz.size() * sizeof(double), s->stream), "allocate set-up");
    SETUP_TRY(dev_alloc((void **)&d_tv, s->tet_verts->size() * sizeof(int32_t), s->stream), "allocate set-up");
    SETUP_TRY(dev_alloc((void **)&d_nbr, nbr_n * sizeof(int32_t), s->stream), "allocate set-up");
    if (on_device) {
        SETUP_TRY(dev_alloc((void **)&d_match_err, 64, s->stream), "allocate face matching");
        SETUP_TRY(dev_alloc(&d_match, face_match_scratch_bytes(T, s->cell_verts), s->stream), "allocate face matching");
    }
    SETUP_TRY(dev_alloc((void **)&d_vol, (size_t)T * sizeof(double), s->stream), "allocate set-up");
    SETUP_TRY(dev_alloc((void **)&d_bc, (size_t)T * 3 * sizeof(double), s->stream), "allocate set-up");
    SETUP_TRY(dev_alloc((void **)&d_area, (size_t)T * 4 * sizeof(double), s->stream), "allocate set-up");
    SETUP_TRY(dev_alloc((void **)&d_D, (size_t)S * sizeof(double), s->stream), "allocate set-up");
    SETUP_TRY(dev_alloc((void **)&d_tau, sizeof(unsigned long long) + 8, s->stream), "allocate set-up");
    alloc_lock.unlock();
    SETUP_TRY(hipMemsetAsync(s->d_buf[0], 0, count_bytes, s->stream), "clear counts");
    SETUP_TRY(hipMemsetAsync(s->d_buf[1], 0, count_bytes, s->stream), "clear counts");
    SETUP_TRY(hipMemsetAsync(s->d_mask[0], 0, mask_bytes, s->stream), "clear occupancy");
    SETUP_TRY(hipMemsetAsync(s->d_mask[1], 0, mask_bytes, s->stream), "clear occupancy");
    SETUP_TRY(hipMemsetAsync(s->d_flags, 0, 64, s->stream), "clear flags");
    SETUP_TRY(hipMemsetAsync(d_tau, 0xff, sizeof(unsigned long long), s->stream), "clear tau");
    SETUP_TRY(hipMemcpyAsync(d_xyz, s->xyz.data(), s->xyz.size() * sizeof(double), hipMemcpyHostToDevice, s->stream),
              "upload vertices");
    SETUP_TRY(hipMemcpyAsync(d_tv, s->tet_verts->data(), s->tet_verts->size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s->stream),
              "upload tetrahedra");
    if (on_device) {
        // keys of each face's sorted vertex ids, a radix sort, pairs of equal keys
        int32_t match_err = 1;
        SETUP_TRY(hipMemsetAsync(d_nbr, 0xff, nbr_n * sizeof(int32_t), s->stream), "face matching");
        SETUP_TRY(hipMemsetAsync(d_match_err, 0, sizeof(int32_t), s->stream), "face matching");
        SETUP_TRY(launch_face_match(d_tv, T, s->cell_verts, bits, d_nbr, d_match, d_match_err, s->stream),
                  "face matching");
        SETUP_TRY(hipMemcpyAsync(&match_err, d_match_err, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream),
                  "face matching");
        SETUP_TRY(hipStreamSynchronize(s->stream), "face matching");
        if (match_err == 0) {
            // the table stays on the device for the geometry pass; a host copy goes to the cache
            std::shared_ptr<int32_t> t = new_table(nbr_n);
            SETUP_TRY(hipMemcpyAsync(t.get(), d_nbr, nbr_n * sizeof(int32_t), hipMemcpyDeviceToHost, s->stream),
                      "read neighbours");
            nbr_table = t;
        } else {
            // a bad face: the host matching names the first one in key order
            std::vector<int32_t> host;
            st = build_topology_uncached(s, host);
            if (st != RDOS_OK) {
                cleanup();
                free_device(s);
                return st;
            }
            std::shared_ptr<int32_t> t = new_table(nbr_n);
            std::memcpy(t.get(), host.data(), nbr_n * sizeof(int32_t));
            nbr_table = t;
            on_device = false;
        }
    }
    if (!on_device)
        SETUP_TRY(hipMemcpyAsync(d_nbr, nbr_table.get(), nbr_n * sizeof(int32_t), hipMemcpyHostToDevice, s->stream),
                  "upload neighbours");
    SETUP_TRY(hipMemcpyAsync(d_D, s->D.data(), (size_t)S * sizeof(double), hipMemcpyHostToDevice, s->stream),
              "upload D");
    if (s->cell_verts == 3)
        SETUP_TRY(launch_geometry_tri(d_xyz, d_tv, d_nbr, T, d_vol, d_bc, d_area, s->d_mesh, s->d_flags + 1,
                                      s->stream),
                  "geometry");
    else
        SETUP_TRY(launch_geometry(d_xyz, d_tv, d_nbr, T, d_vol, d_bc, d_area, s->d_mesh, s->d_flags + 1, s->stream),
                  "geometry");
    if (s->tau_outliers > 0) {
        // Sec. II.A outlier relaxation: the (k+1)-th smallest 1/(D g) sets tau
        void *scratch = nullptr;
        hipError_t e_sel;
        {
            std::lock_guard<std::mutex> g(device_api_mutex());
            e_sel = dev_alloc(&scratch, tau_select_scratch_bytes(T, S), s->stream);
        }
        if (e_sel == hipSuccess) {
            e_sel = launch_tau_select(s->d_mesh, T, d_D, S, s->tau_outliers, scratch, d_tau, s->stream);
            (void)hipStreamSynchronize(s->stream);
            std::lock_guard<std::mutex> g(device_api_mutex());
            dev_free(scratch, s->stream);
        }
        SETUP_TRY(e_sel, "tau selection");
    } else {
        SETUP_TRY(launch_tau_min(s->d_mesh, T, d_D, S, d_tau, s->stream), "tau");
    }
    unsigned long long tau_bits = 0;
    int32_t bad[2] = {0, 0};
    SETUP_TRY(hipMemcpyAsync(&tau_bits, d_tau, sizeof tau_bits, hipMemcpyDeviceToHost, s->stream), "read tau");
    SETUP_TRY(hipMemcpyAsync(bad, s->d_flags, sizeof bad, hipMemcpyDeviceToHost, s->stream), "read flags");
    SETUP_TRY(hipStreamSynchronize(s->stream), "set-up");
    SETUP_TRY(hipMemsetAsync(s->d_flags, 0, 64, s->stream), "clear flags");
    cleanup();
#undef SETUP_TRY
    if (bad[1]) {
        free_device(s);
        return fail(s, RDOS_EINVAL, s->cell_verts == 3 ? "degenerate triangle (zero area)"
                                                       : "degenerate tetrahedron (zero volume)");
    }
    if (tau_bits == ~0ull) {
        free_device(s);
        return fail(s, RDOS_EINVAL, "no diffusing species on a connected cell: tau is undefined");
    }
    double tmin;
    std::memcpy(&tmin, &tau_bits, sizeof tmin);
    s->tau = tau_scale * tmin;

    // kernel-side description
    DevSim &d = s->desc;
    std::memset(&d, 0, sizeof d);
    d.mesh = s->d_mesh;
    d.buf[0] = s->d_buf[0];
    d.buf[1] = s->d_buf[1];
    d.mask[0] = s->d_mask[0];
    d.mask[1] = s->d_mask[1];
    d.flags = s->d_flags;
    d.T = T;
    d.mstride = mask_stride(Tp);
    d.S = S;
    d.R = (int32_t)s->rx.size();
    d.Rz = s->Rz;
    d.key0 = (uint32_t)s->seed;
    d.key1 = (uint32_t)(s->seed >> 32);
    d.tau = s->tau;
    d.step0 = 0;
    d.step_end = std::numeric_limits<int64_t>::max();
    for (int m = 0; m < S; ++m) {
        d.D[m] = s->D[m];
        if (s->D[m] > 0.0) d.diff_mask |= 1u << m;
    }
    d.first_order = s->first_order ? 1u : 0u;
    d.split_threshold = s->split_threshold;
    d.transfer_form = s->transfer_form;
    s->queue.scaled = s->transfer_form == 1 ? 1 : 0;
    if (!s->regions.empty()) {
        std::vector<uint32_t> allowed((size_t)T, 0xFFFFFFFFu);
        for (const auto &kv : s->regions) {
            const uint32_t bit = 1u << kv.first;
            for (uint32_t &a : allowed) a &= ~bit;
            for (int32_t t : kv.second) allowed[t] |= bit;
        }
        hipError_t e_al;
        {
            std::lock_guard<std::mutex> g(device_api_mutex());
            e_al = dev_alloc((void **)&s->d_allowed, allowed.size() * sizeof(uint32_t), s->stream);
        }
        if (e_al == hipSuccess)
            e_al = hipMemcpyAsync(s->d_allowed, allowed.data(), allowed.size() * sizeof(uint32_t),
                                  hipMemcpyHostToDevice, s->stream);
        if (e_al == hipSuccess) e_al = hipStreamSynchronize(s->stream);
        if (e_al != hipSuccess) {
            free_device(s);
            return hip_fail(s, e_al, "upload reaction regions");
        }
        d.allowed = s->d_allowed;
    }
    for (size_t q = 0; q < s->rx.size(); ++q) {
        const Reaction &r = s->rx[q];
        d.rn[q] = r.rn;
        d.pn[q] = r.pn;
        d.r0[q] = r.rn > 0 ? r.r[0] : -1;
        d.r1[q] = r.rn > 1 ? r.r[1] : -1;
        d.p0[q] = r.pn > 0 ? r.p[0] : -1;
        d.p1[q] = r.pn > 1 ? r.p[1] : -1;
        d.p2[q] = r.pn > 2 ? r.p[2] : -1;
        uint32_t inv = 0;
        for (int i = 0; i < r.rn; ++i) inv |= 1u << r.r[i];
        for (int i = 0; i < r.pn; ++i) inv |= 1u << r.p[i];
        d.involved[q] = inv;
        d.k[q] = r.k;
        if (r.rn == 0) d.zeroth = 1;
    }
    // work list: one tile per 1024 tets of each realization
    std::vector<Tile> tiles;
    for (int32_t r = 0; r < s->Rz; ++r)
        for (int32_t t0 = 0; t0 < T; t0 += kTetsPerTile)
            tiles.push_back({0, r, t0, std::min<int32_t>(kTetsPerTile, T - t0)});
    s->n_tiles = (int32_t)tiles.size();
    hipError_t e;
    {
        std::lock_guard<std::mutex> g(device_api_mutex());
        e = dev_alloc((void **)&s->d_tiles, tiles.size() * sizeof(Tile), s->stream);
    }
    if (e != hipSuccess) {
        free_device(s);
        return hip_fail(s, e, "allocate work list");
    }
    e = hipMemcpyAsync(s->d_tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) {
        free_device(s);
        return hip_fail(s, e, "upload work list");
    }
    e = set_queue_work(&s->queue, s->n_tiles, 1, s->stream);
    if (e != hipSuccess) {
        free_device(s);
        return hip_fail(s, e, "queue header");
    }
    st = upload_desc(s);
    if (st != RDOS_OK) {
        free_device(s);
        return st;
    }
    if (fresh) topology_insert(s, topo_hash, std::move(nbr_table));  // the read-back was waited for above
    s->state = SimState::Ready;
    s->step = 0;
    s->anchor_step = 0;
    s->anchor_t = 0.0;
    // counts staged before finalize
    for (auto &kv : s->staged) {
        const int32_t r = kv.first / kMaxSpecies, m = kv.first % kMaxSpecies;
        int32_t *dst = s->d_buf[0] + ((int64_t)r * S + m) * Tp;
        HIP_TRY(s, hipMemcpyAsync(dst, kv.second.data(), (size_t)T * sizeof(int32_t), hipMemcpyHostToDevice, s->stream),
                "upload counts");
    }
    HIP_TRY(s, hipStreamSynchronize(s->stream), "upload counts");
    s->mask_dirty = true;
    s->staged.clear();
    s->xyz.clear();
    s->xyz.shrink_to_fit();
    if (out_tau) *out_tau = s->tau;
    return RDOS_OK;
}

rdos_status rdos_set_counts(rdos_sim *s, int32_t realization, int32_t species, const int32_t *counts)
{
    CHECK_HANDLE(s);
    if (s->state == SimState::Created) return fail(s, RDOS_ESTATE, "set_counts needs a mesh");
    if (realization < 0 || realization >= s->Rz || species < 0 || species >= (int32_t)s->D.size() || !counts)
        return fail(s, RDOS_EINVAL, "realization or species out of range");
    int64_t total = 0;
    for (int32_t t = 0; t < s->T; ++t) {
        if (counts[t] < 0) return fail(s, RDOS_EINVAL, "negative count at tet %d", t);
        total += counts[t];
    }
    if (total > 0x3fffffff) return fail(s, RDOS_EOVERFLOW, "more than 2^30 molecules of one species");
    if ((int64_t)s->Rz * s->T > 0x7fffffff) return fail(s, RDOS_EINVAL, "realizations x tets exceeds 2^31");
    if (s->state == SimState::Meshed) {
        s->staged[realization * kMaxSpecies + species].assign(counts, counts + s->T);
        return RDOS_OK;
    }
    HIP_TRY(s, hipSetDevice(s->device), "set device");
    int32_t *dst = s->d_buf[s->step & 1] + ((int64_t)realization * (int64_t)s->D.size() + species) * padded_tets(s->T);
    HIP_TRY(s, hipMemcpyAsync(dst, counts, (size_t)s->T * sizeof(int32_t), hipMemcpyHostToDevice, s->stream),
            "upload counts");
    HIP_TRY(s, hipStreamSynchronize(s->stream), "upload counts");
    s->mask_dirty = true;
    return RDOS_OK;
}

rdos_status rdos_get_counts(rdos_sim *s, int32_t realization, int32_t species, int32_t *out)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Ready) return fail(s, RDOS_ESTATE, "get_counts before finalize");
    if (realization < 0 || realization >= s->Rz || species < 0 || species >= (int32_t)s->D.size() || !out)
        return fail(s, RDOS_EINVAL, "realization or species out of range");
    HIP_TRY(s, hipSetDevice(s->device), "set device");
    const int32_t *src =
        s->d_buf[s->step & 1] + ((int64_t)realization * (int64_t)s->D.size() + species) * padded_tets(s->T);
    HIP_TRY(s, hipMemcpyAsync(out, src, (size_t)s->T * sizeof(int32_t), hipMemcpyDeviceToHost, s->stream),
            "download counts");
    return check_flags(s);
}

rdos_status rdos_device_counts(rdos_sim *s, int32_t realization, int32_t species, int32_t **out)
{
    CHECK_HANDLE(s);
    if (!out) return fail(s, RDOS_EINVAL, "null output");
    *out = nullptr;
    if (s->state != SimState::Ready) return fail(s, RDOS_ESTATE, "device_counts before finalize");
    if (realization < 0 || realization >= s->Rz || species < 0 || species >= (int32_t)s->D.size())
        return fail(s, RDOS_EINVAL, "realization or species out of range");
    *out = s->d_buf[s->step & 1] + ((int64_t)realization * (int64_t)s->D.size() + species) * padded_tets(s->T);
    s->mask_dirty = true;  // the caller may write through the view
    return RDOS_OK;
}

rdos_status rdos_set_state(rdos_sim *s, int64_t step_index, double t)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Ready) return fail(s, RDOS_ESTATE, "set_state before finalize");
    if (step_index < 0 || !std::isfinite(t)) return fail(s, RDOS_EINVAL, "bad state");
    HIP_TRY(s, hipSetDevice(s->device), "set device");
    HIP_TRY(s, hipStreamSynchronize(s->stream), "set state");
    if ((step_index & 1) != (s->step & 1)) {  // the state moves with k & 1
        std::swap(s->d_buf[0], s->d_buf[1]);
        std::swap(s->d_mask[0], s->d_mask[1]);
    }
    s->step = step_index;
    s->anchor_step = step_index;
    s->anchor_t = t;
    s->mask_dirty = true;  // the occupancy bytes hold tags of the period index
    return match_parity(s);
}

rdos_status rdos_get_time(rdos_sim *s, double *t, int64_t *step_index)
{
    CHECK_HANDLE(s);  // an engine's worker moves the period index of the simulations it owns
    if (t) *t = time_of(s, s->step);
    if (step_index) *step_index = s->step;
    return RDOS_OK;
}

rdos_status rdos_step(rdos_sim *s, int64_t n_steps)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Ready) return fail(s, RDOS_ESTATE, "step before finalize");
    if (n_steps < 0) return fail(s, RDOS_EINVAL, "negative step count");
    HIP_TRY(s, hipSetDevice(s->device), "set device");
    return enqueue_run(s, n_steps, false, 0.0);
}

rdos_status rdos_run_until(rdos_sim *s, double t_end)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Ready) return fail(s, RDOS_ESTATE, "run_until before finalize");
    if (!std::isfinite(t_end)) return fail(s, RDOS_EINVAL, "t_end must be finite");
    HIP_TRY(s, hipSetDevice(s->device), "set device");
    // full periods while one more fits, then (Step 1) a last period shortened
    // to end at t_end
    int64_t k = s->step;
    while (time_of(s, k) < t_end && !(time_of(s, k) + s->tau > t_end)) ++k;
    const bool partial = time_of(s, k) < t_end;
    const double tau_last = partial ? t_end - time_of(s, k) : 0.0;
    rdos_status st = enqueue_run(s, k - s->step + (partial ? 1 : 0), partial, tau_last);
    if (st != RDOS_OK) return st;
    if (partial) {
        s->anchor_step = s->step;
        s->anchor_t = t_end;
    }
    return RDOS_OK;
}

rdos_status rdos_set_launch_mode(rdos_sim *s, int32_t mode)
{
    CHECK_HANDLE(s);
    if (mode < 0 || mode > 3) return fail(s, RDOS_EINVAL, "launch mode must be 0, 1, 2 or 3");
    s->launch_mode = mode;
    return RDOS_OK;
}

rdos_status rdos_synchronize(rdos_sim *s)
{
    CHECK_HANDLE(s);
    if (s->state != SimState::Ready) return RDOS_OK;
    HIP_TRY(s, hipSetDevice(s->device), "set device");
    return check_flags(s);
}

rdos_status rdos_set_stream(rdos_sim *s, void *hip_stream)
{
    CHECK_HANDLE(s);
    HIP_TRY(s, hipSetDevice(s->device), "set device");
    if (s->stream) HIP_TRY(s, hipStreamSynchronize(s->stream), "drain old stream");
    if (s->stream && s->own_stream) (void)hipStreamDestroy(s->stream);
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
        s->own_stream = false;
    } else if (s->state == SimState::Ready) {
        HIP_TRY(s, hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "create stream");
        s->own_stream = true;
    } else {
        s->stream = nullptr;
        s->own_stream = false;
    }
    return RDOS_OK;
}

rdos_status rdos_get_geometry(rdos_sim *s, int32_t *nbr, double *w, double *g, double *nav)
{
    if (!s) return RDOS_EINVAL;
    if (s->state != SimState::Ready) return fail(s, RDOS_ESTATE, "get_geometry before finalize");
    HIP_TRY(s, hipSetDevice(s->device), "set device");
    std::vector<MeshRec> m((size_t)s->T);
    HIP_TRY(s, hipMemcpyAsync(m.data(), s->d_mesh, m.size() * sizeof(MeshRec), hipMemcpyDeviceToHost, s->stream),
            "download mesh tables");
    HIP_TRY(s, hipStreamSynchronize(s->stream), "download mesh tables");
    for (int32_t t = 0; t < s->T; ++t) {
        for (int f = 0; f < 4; ++f) {
            if (nbr) nbr[4 * (size_t)t + f] = m[t].nbr[f];
            if (w) w[4 * (size_t)t + f] = m[t].w[f];
        }
        if (g) g[t] = m[t].g;
        if (nav) nav[t] = m[t].nav;
    }
    return RDOS_OK;
}

rdos_status rdos_get_info(rdos_sim *s, int32_t *n_tets, int32_t *n_species, int32_t *n_reactions,
                          int32_t *n_realizations, size_t *device_bytes)
{
    if (!s) return RDOS_EINVAL;
    if (n_tets) *n_tets = s->T;
    if (n_species) *n_species = (int32_t)s->D.size();
    if (n_reactions) *n_reactions = (int32_t)s->rx.size();
    if (n_realizations) *n_realizations = s->Rz;
    if (device_bytes) *device_bytes = state_bytes(s);
    return RDOS_OK;
}

const char *rdos_last_error(const rdos_sim *s) { return s ? s->error.c_str() : "null handle"; }

void rdos_destroy(rdos_sim *s)
{
    if (!s) return;
    free_device(s);
    delete s;
}

}  // extern "C"
