// Shared host/device definitions of the rdos library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/rdos.h"

namespace rdos {

constexpr int kMaxSpecies = RDOS_MAX_SPECIES;
constexpr int kMaxReactions = RDOS_MAX_REACTIONS;
constexpr uint32_t kSsaStream = 0x80000000u;   // Philox stream id of the SSA draws
constexpr int kSplitOneByOne = 10;             // Sec. II.B: n below this moves one by one
constexpr double kAvogadro = 6.02214076e23;    // 1/mol (SI 2019)
constexpr uint32_t kMaxEventsPerPeriod = 1u << 24;  // SSA events of one tet in one period

// One tetrahedron's tables: one 64-byte line, read only when the tet holds
// molecules (or has a 0th-order reaction).
struct alignas(64) MeshRec {
    int32_t nbr[4];   // neighbour across face f (opposite local vertex f), -1 = boundary
    double w[4];      // direction weights, sum 1 over interior faces
    double g;         // sum_f A_f / (V delta_f), 1/m^2; local rate d = D g
    double nav;       // N_A * volume in litres
};
static_assert(sizeof(MeshRec) == 64, "MeshRec must be one cache line");

// The value an occupancy byte holds to mark period k (1..255, never 0).
// Bytes are not cleared after they are read: a byte marks its group only in
// the period whose tag it holds.  A byte left from 510 periods earlier (the
// tags repeat every 255 periods, and each of the two maps serves every other
// period) can match again; the scan then reads an all-zero count vector and
// queues nothing, so a stale byte costs a read, never a result.
__host__ __device__ inline uint8_t occupancy_tag(int64_t period) { return (uint8_t)(period % 255 + 1); }

// One simulation as the step kernel sees it (device memory).
struct alignas(16) DevSim {
    const MeshRec *mesh;       // [T]
    int32_t *buf[2];           // [Rz][S][Tp] counts; period k reads buf[k & 1] and fills buf[(k + 1) & 1]
    uint8_t *mask[2];          // [Rz][S][mstride] occupancy of buf[k & 1]: byte t >> 2 of row (r, s)
                               // equals occupancy_tag(k) when species s of tets 4 (t >> 2) .. + 3 may
                               // be non-zero in period k
    int32_t *flags;            // bit 0: count overflow; bit 1: SSA event cap; bit 2: queue overflow
    int32_t T, S, R, Rz;
    int32_t mstride;           // occupancy bytes per species row (Tp / 4 rounded up to 16)
    uint32_t key0, key1;       // Philox key words before the realization is mixed in
    double tau;                // full period
    int64_t step0;             // period index of launch iteration 0
    int64_t step_end;          // periods >= step_end are not run
    double D[kMaxSpecies];
    uint32_t diff_mask;        // species with D > 0
    uint32_t zeroth;           // 1 if some reaction has no reactant (every tet active)
    uint32_t first_order;      // 1: n from the count at the end of the period instead of Nbar
    int32_t split_threshold;   // below this n molecules are split one by one (Sec. II.B: 10)
    int32_t transfer_form;     // 0: n = binomial then split (eq. 3); 1: one split scaled by zeta
    const uint32_t *allowed;   // [T] bit r: reaction r may fire in the tet (null: everywhere)
    // reactions
    int32_t rn[kMaxReactions], r0[kMaxReactions], r1[kMaxReactions];
    int32_t pn[kMaxReactions], p0[kMaxReactions], p1[kMaxReactions], p2[kMaxReactions];
    uint32_t involved[kMaxReactions];   // bit m: species m is a reactant or a product
    double k[kMaxReactions];
};

// A block's unit of work: up to kTetsPerTile consecutive tets of one
// realization of one simulation.
struct Tile {
    int32_t sim;
    int32_t realization;
    int32_t tet0;
    int32_t ntet;
};

constexpr int kBlock = 256;        // threads per block (4 wavefronts)
constexpr int kTetsPerLane = 4;    // one 16-byte load per species and lane
constexpr int kTetsPerTile = kBlock * kTetsPerLane;

// One realization of one simulation in a work list, for building the tile
// list on the device: its tiles are tiles[first .. first + ceil(T / kTetsPerTile)).
struct WorkUnit {
    int32_t sim;
    int32_t realization;
    int32_t T;
    int32_t first;
};

// Held while a graph is captured and around device allocations and frees
// made by other threads, so neither can interfere with a capture.
inline std::mutex &device_api_mutex()
{
    static std::mutex m;
    return m;
}

// Kernel launchers (rdos_kernels.hip).
hipError_t launch_geometry(const double *xyz, const int32_t *tet_verts, const int32_t *nbr,
                           int32_t T, double *scratch_vol, double *scratch_bc,
                           double *scratch_area, MeshRec *mesh, int32_t *bad_volume,
                           hipStream_t st);
// The same for triangles (surface diffusion): area instead of volume, edge
// lengths instead of face areas, N_A A as the unit of amount.
hipError_t launch_geometry_tri(const double *xyz, const int32_t *tri_verts, const int32_t *nbr, int32_t T,
                               double *scratch_area, double *scratch_bc, double *scratch_len, MeshRec *mesh,
                               int32_t *bad_area, hipStream_t st);
// Face matching on the device for cells of cell_verts (4: tetrahedra, 3:
// triangles) vertices with ids below 2^bits (bits <= 21 for tetrahedra, <= 31
// for triangles): nbr[4 T] (filled with -1 by the caller) gets the cell
// across each face; *err (zero on entry) becomes non-zero when a face lies on
// more than two cells or twice on one.  scratch holds
// face_match_scratch_bytes(T, cell_verts) bytes.
size_t face_match_scratch_bytes(int32_t T, int32_t cell_verts);
hipError_t launch_face_match(const int32_t *cells, int32_t T, int32_t cell_verts, int32_t bits, int32_t *nbr,
                             void *scratch, int32_t *err, hipStream_t st);
hipError_t launch_tau_min(const MeshRec *mesh, int32_t T, const double *D, int32_t S,
                          unsigned long long *out_bits, hipStream_t st);
// Writes the k-th smallest (0-based, clamped to the last) of 1/(D_m g_t)
// over diffusing species and connected tets to *out_bits (as its bit
// pattern); scratch must hold tau_select_scratch_bytes(T, S) bytes.
size_t tau_select_scratch_bytes(int32_t T, int32_t S);
hipError_t launch_tau_select(const MeshRec *mesh, int32_t T, const double *D, int32_t S, int64_t k, void *scratch,
                             unsigned long long *out_bits, hipStream_t st);
// Work-list sizes and queue geometry, read by the kernels from device memory
// so that a captured graph stays valid when the work list changes.
struct alignas(16) WorkHeader {
    int32_t n_tiles;   // tiles in the work list
    int32_t n_sims;    // simulation descriptors
    int32_t nseg;      // queue segments in use, 1..kMaxSegments
    int32_t seg_cap;   // entries per segment
    int64_t qcap;      // stride between the count rows of the queue (allocated entries)
    int32_t tile0;     // this work list starts at tiles[tile0] (kernels get the array's base)
    int32_t pad;
};

// Occupied-tet queue of one launch pair (device memory, see the scan kernel).
struct QueueView {
    int32_t *tet;       // [qcap] tile * kTetsPerTile + offset
    int32_t *counts;    // [species][qcap] counts at the start of the period
    int32_t *len;       // [2][kMaxSegments] segment lengths, one per kLenStride ints (own cache
                        // line); both halves zero before the first launch
    WorkHeader *hdr;    // device copy of the sizes below
    int32_t nseg;       // host copies
    int32_t seg_cap;
    int64_t qcap;       // allocated entries per count row
    int32_t species;    // allocated count rows
    int32_t scaled;     // some simulation of the work list uses transfer form 1 (picks the update kernel)
    uint32_t *sync;     // [kPersistSyncWords] grid-barrier counters and failure word of the one-launch path
    unsigned long long *work;  // null, or [3] device totals the update kernel adds to: tets, count additions,
                               // additions that are transfers across a face
    int32_t owned;      // the work lists launched on it have a segment per tile and a scan wavefront per
                        // tile (at most kMaxSegments tiles): the scan instance that fills segments by its
                        // own count (checked again on the device)
};
constexpr int kMaxSegments = 1024;
constexpr int kPersistSyncWords = 64 * 32 + 32;  // 64 barrier counters on lines of their own, the failure word
constexpr int kLenStride = 32;  // 128 bytes between segment lengths: no two share a line

// Queue geometry for a work list of n_tiles tiles: tiles ti with
// ti % nseg == k fill segment k.
inline void queue_shape(int64_t n_tiles, int32_t *nseg, int32_t *seg_cap)
{
    const int64_t ns = n_tiles < kMaxSegments ? (n_tiles > 0 ? n_tiles : 1) : kMaxSegments;
    *nseg = (int32_t)ns;
    *seg_cap = (int32_t)(((n_tiles + ns - 1) / ns) * kTetsPerTile);
}

// One period for every tile: period index = sims[i].step0 + iter; the period
// whose index equals `partial` lasts tau_last instead of tau.  Consecutive
// launches on one queue alternate qsel = 0, 1, 0, ...
// scan_grid blocks stride over the tiles named in q.hdr (> 0 required).
hipError_t launch_scan(const DevSim *sims, const Tile *tiles, int64_t iter, const QueueView &q, int32_t qsel,
                       int32_t scan_grid, hipStream_t st);
// The update grid is grid_segments (1..kMaxSegments) x blocks_per_segment
// blocks, one block column per queue segment: grid_segments must be at least
// the segments of the work list (else the kernel updates nothing and raises
// bit 2 of the first simulation's flags).
hipError_t launch_update(const DevSim *sims, const Tile *tiles, int64_t iter, int64_t partial, double tau_last,
                         const QueueView &q, int32_t qsel, int32_t blocks_per_segment, int32_t grid_segments,
                         hipStream_t st);
hipError_t launch_step(const DevSim *sims, const Tile *tiles, int64_t iter, int64_t partial, double tau_last,
                       const QueueView &q, int32_t qsel, int32_t scan_grid, int32_t blocks_per_segment,
                       int32_t grid_segments, hipStream_t st);
// One launch per period (scan and update fused; no queue in device memory):
// grid blocks of four wavefronts stride over the tiles named in q.hdr; the
// queue supplies the header, the species bound and the work tallies only.
// Queues of up to kFusedSpecies species rows (hipErrorInvalidValue beyond).
constexpr int kFusedSpecies = 8;
hipError_t launch_fused(const DevSim *sims, const Tile *tiles, int64_t iter, int64_t partial, double tau_last,
                        const QueueView &q, int32_t grid, hipStream_t st);
// Scan blocks needed to give every tile of a work list its own wavefront.
inline int32_t scan_blocks_for(int64_t n_tiles)
{
    const int64_t b = (n_tiles + kBlock / 64 - 1) / (kBlock / 64);
    return (int32_t)(b < 1 ? 1 : (b > (1 << 20) ? (1 << 20) : b));
}
hipError_t launch_advance(DevSim *sims, const WorkHeader *hdr, int64_t by, hipStream_t st);
// Writes tiles[0 .. n_tiles) from n_units work units whose `first` fields
// ascend from 0 and leave no gaps (each unit has at least one tile).
hipError_t launch_expand_tiles(const WorkUnit *units, int32_t n_units, int32_t n_tiles, Tile *tiles, hipStream_t st);
// Small work lists: n_periods periods in one cooperative launch of `grid`
// blocks (at most persist_grid_limit(q), every block resident), grid-wide
// barriers between the scan and update phases.  Period i uses queue half
// (phase + i) & 1.  sync points at kPersistSyncWords words of device memory
// (barrier counters, failure word) that no other launch uses meanwhile; a
// barrier that times out raises bit 3 of every simulation's flags.
int32_t persist_grid_limit(const QueueView &q);
hipError_t launch_persist(const DevSim *sims, const Tile *tiles, int64_t iter0, int32_t n_periods, int32_t phase,
                          int64_t partial, double tau_last, const QueueView &q, int32_t grid, uint32_t *sync,
                          hipStream_t st);
// Rebuilds the occupancy bytes of buf[parity] from the counts of every
// realization and species and clears those of the other buffer (after
// counts were set from the host).
hipError_t launch_mask_build(const int32_t *counts, uint8_t *mask_cur, uint8_t *mask_other, uint8_t tag, int32_t Rz,
                             int32_t S,
                             int64_t Tp, hipStream_t st);
// Bytes of one species row of the occupancy map: one per four tets, padded
// to 16 bytes so that the scan reads four bytes at a time.
inline int32_t mask_stride(int64_t Tp) { return (int32_t)(((Tp / 4) + 15) & ~(int64_t)15); }
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st);
// blocks x 256 lanes each split n molecules reps times, one-by-one or by
// sequential binomials; sink holds blocks * 256 int64.
hipError_t launch_split_cost(bool one_by_one, int64_t n, int32_t reps, int64_t *sink, int32_t blocks, hipStream_t st);


}  // namespace rdos
