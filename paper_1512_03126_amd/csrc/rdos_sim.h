// Host-side state of one simulation handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "rdos_internal.h"

namespace rdos {

enum class SimState { Created, Meshed, Ready };

struct Reaction {
    int32_t rn = 0, pn = 0;
    int32_t r[2] = {-1, -1};
    int32_t p[3] = {-1, -1, -1};
    double k = 0.0;
};

}  // namespace rdos

struct rdos_sim {
    int device = 0;
    uint64_t seed = 0;
    int32_t Rz = 1;
    rdos::SimState state = rdos::SimState::Created;
    std::string error;
    bool engine_owned = false;

    // model (host copy)
    int32_t n_verts = 0, T = 0;
    std::vector<double> xyz;
    std::shared_ptr<const std::vector<int32_t>> tet_verts;  // cells: [T][4] tetrahedra, or [T][3] triangles of a
                                                            // surface (shared with the topology cache)
    int32_t cell_verts = 4;
    std::vector<double> D;
    std::vector<rdos::Reaction> rx;
    std::map<int32_t, std::vector<int32_t>> staged;  // (r * kMaxSpecies + s) -> counts before finalize
    // method options (set before finalize)
    int32_t first_order = 0;
    int32_t split_threshold = rdos::kSplitOneByOne;
    int32_t tau_outliers = 0;
    int32_t transfer_form = 0;
    std::map<int32_t, std::vector<int32_t>> regions;  // reaction -> tets where it may fire

    // time: time(k) = anchor_t + (k - anchor_step) * tau
    double tau = 0.0;
    int64_t step = 0;
    int64_t anchor_step = 0;
    double anchor_t = 0.0;

    // device
    hipStream_t stream = nullptr;
    bool own_stream = false;
    rdos::MeshRec *d_mesh = nullptr;
    uint32_t *d_allowed = nullptr;  // per-tet reaction masks (only with regions)
    int32_t *d_buf[2] = {nullptr, nullptr};  // counts; the state of period k is d_buf[k & 1]
    uint8_t *d_mask[2] = {nullptr, nullptr};   // occupancy maps of d_buf[0], d_buf[1]
    bool mask_dirty = false;                 // counts were written from the host: rebuild d_mask
    int32_t *d_flags = nullptr;
    rdos::DevSim *d_desc = nullptr;
    rdos::Tile *d_tiles = nullptr;
    int32_t n_tiles = 0;
    rdos::QueueView queue{};      // occupied tets of one period (tet ids + counts + segment lengths)
    int64_t launches = 0;         // periods launched on this handle (selects the queue length half)
    int32_t update_bps = 1;       // update blocks per queue segment
    int32_t launch_mode = 0;      // 0: one launch for small work lists, two per period otherwise; 1: always two
    int32_t persist_limit = -1;   // blocks a cooperative launch of the one-launch kernel may have (-1: not asked)
    rdos::DevSim desc{};
};

namespace rdos {
rdos_status fail(rdos_sim *s, rdos_status code, const char *fmt, ...);
rdos_status hip_fail(rdos_sim *s, hipError_t e, const char *what);
int64_t padded_tets(int32_t T);
size_t state_bytes(const rdos_sim *s);
size_t queue_bytes(int64_t n_tiles, int32_t n_species);
hipError_t alloc_queue(rdos::QueueView *q, int64_t capacity_tiles, int32_t n_species, hipStream_t st);
hipError_t set_queue_work(rdos::QueueView *q, int64_t n_tiles, int32_t n_sims, hipStream_t st, int32_t tile0 = 0);
void free_queue(rdos::QueueView *q, hipStream_t st);
// Device memory from the per-device stream-ordered pool (ordered on st).
hipError_t dev_alloc(void **p, size_t bytes, hipStream_t st);
void dev_free(void *p, hipStream_t st);
rdos_status match_parity(rdos_sim *s);
rdos_status ensure_mask(rdos_sim *s);
rdos_status check_flags(rdos_sim *s);
double time_of(const rdos_sim *s, int64_t k);
rdos_status rdos_finalize_internal(rdos_sim *s, double tau_scale);
// Work lists of at most this many tiles run all their periods in one
// cooperative launch (launch_persist), up to kPersistPeriods per launch.
// Beyond it the one-launch path loses: every grid barrier needs each block's
// agent-scope release, which writes back its L2, and two launches per period
// are cheaper (measured: 16.4 against 22 us per period on 1 tile, 18.5
// against 16.8 on 17 tiles, 50 against 21 on 129 tiles).
constexpr int64_t kPersistTiles = 8;
constexpr int64_t kPersistPeriods = 4096;
}  // namespace rdos
