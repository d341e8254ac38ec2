// Batching and serving engine: every admitted simulation ("slot") advances
// one of its own periods per launch pair, all slots in the same launches.
// Chunks of periods are captured into a hipGraph and replayed.  The kernels
// read the work-list sizes from a small device header, so the graph survives
// changes of the slot set: admitting or retiring a simulation only rewrites
// descriptors, tiles and the header; a new capture is needed only when a
// buffer has to grow or the tuner picks another launch shape.  An admission
// thread admits queued simulations while their device memory fits the budget
// (finalizing them on their own streams), and the worker adds them to the
// work list at its next chunk (continuous batching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "rdos_internal.h"
#include "rdos_sim.h"

using namespace rdos;
using Clock = std::chrono::steady_clock;

namespace {

struct Ticket {
    rdos_sim *sim = nullptr;
    int64_t n_steps = 0;
    double tau_scale = 1.0;
    Clock::time_point submitted;
    Clock::time_point admit_start;  // the admission thread took it (set-up begins)
    Clock::time_point admit_end;    // set up and handed to the worker
    Clock::time_point started;      // its first periods were launched
    Clock::time_point finished;
    bool admitted = false;
    bool done = false;
    bool failed = false;
    size_t bytes = 0;
    int64_t end_step = 0;  // the simulation's period index when done
    std::string error;
};

// Launch-shape choices the tuner tries on live work (results do not depend on them).
struct Shape {
    int32_t chunk;       // periods per graph replay (even: the queue length halves alternate)
    int32_t scan_grid;   // blocks of the scan launch (grid-stride over the tiles)
    int32_t update_bps;  // update blocks per queue segment; 0: one fused launch per period (no update kernel)
    int32_t chains;      // 1, or 2 independent halves of the realizations on two streams
    bool operator==(const Shape &o) const
    {
        return chunk == o.chunk && scan_grid == o.scan_grid && update_bps == o.update_bps && chains == o.chains;
    }
};

// Work lists of up to this many tiles (size buckets below it) are not tuned:
// all candidates clamp to about the same grids there.
constexpr int32_t kSmallWorkTiles = 1024;
constexpr Shape kSmallWorkShape{32, 2048, 1, 1};

// Tuning results shared by every engine of the process, by work-list size
// bucket: an engine that meets a bucket another engine has tuned starts
// with its shape instead of tuning again.
struct TuneCache {
    std::mutex mu;
    std::map<std::pair<int, int>, Shape> shapes;
};
TuneCache &tune_cache()
{
    static TuneCache c;
    return c;
}

}  // namespace

struct rdos_engine {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    hipStream_t stream = nullptr;
    hipStream_t stream2 = nullptr;  // second chain of a two-chain chunk
    hipEvent_t fork = nullptr, join = nullptr;
    std::string error;

    std::mutex mu;
    std::condition_variable cv_work;   // wakes the worker
    std::condition_variable cv_admit;  // wakes the admission thread
    std::condition_variable cv_done;   // wakes drain()
    std::thread worker;
    // admission threads: they finalize admitted simulations while the worker keeps launching, two so
    // that a small request need not wait while a large one is set up
    static constexpr int kAdmitters = 2;
    std::thread admitters[kAdmitters];
    int admitting = 0;            // tickets being finalized right now
    int64_t admitting_tiled = 0;  // their tiled tets
    bool stop = false;
    bool worker_dead = false;  // the worker left its loop after a device error
    bool stalled = false;      // nothing runs and the next request does not fit the budget
    bool admit_blocked = false;  // the next waiting request does not fit the budget now
    bool held = false;         // rdos_engine_hold: start no chunk

    uint64_t next_ticket = 1;
    std::map<uint64_t, Ticket> tickets;
    std::deque<uint64_t> waiting;  // submitted, not admitted (FIFO)
    std::vector<uint64_t> ready;   // admitted and finalized, joining at the next chunk
    std::vector<uint64_t> slots;   // running

    // device work list of the current slot set (buffers only grow)
    DevSim *d_sims = nullptr;
    int64_t cap_sims = 0;
    Tile *d_tiles = nullptr;
    int64_t cap_tiles = 0;
    WorkUnit *d_units = nullptr;  // the work list's units, expanded into d_tiles on the device
    int64_t cap_units = 0;
    QueueView queue{};   // chain 0 (all tiles when there is one chain)
    QueueView queue2{};  // chain 1
    int32_t n_tiles = 0;
    int32_t n_sims = 0;
    int32_t n_tiles0 = 0;   // tiles of chain 0 when split: they come first in d_tiles
    int32_t hdr_chains = 0; // chain count the queue headers currently describe
    int32_t max_species = 1;
    // instantiated chunk graphs by (shape, grid_tiles): a graph sized for a
    // bucket serves every work list that fits it, so buckets that come back
    // (serving) reuse their graphs
    std::map<std::array<int32_t, 5>, hipGraphExec_t> graphs;
    int32_t grid_tiles = 1;        // launch grids serve work lists of up to this many tiles (size bucket)
    double last_chunk_ms = 0.0;    // device time of the last full chunk
    double last_period_ms = 0.0;   // device time per period of the last one-launch run
    int32_t persist_limit = -1;    // blocks of a cooperative one-launch kernel (-1: not asked)
    int32_t persist_key = -1;      // queue species bound and transfer form it was asked for
    int32_t qphase = 0;            // queue half (qsel) of the next period; graphs start at 0
    bool graph_stale = true;  // a buffer the graphs name was reallocated
    bool rebuild = true;      // the slot set changed

    // tuner, per work-list size bucket: a first pass runs each candidate for
    // two chunks (the first replays a freshly captured graph and is not
    // scored), a second pass scores each once more; the lowest mean time per
    // period wins
    std::vector<Shape> candidates;
    bool fixed_shape = false;  // set_shape: no tuning, always `best`
    std::map<std::pair<int, int>, Shape> tuned;
    std::pair<int, int> bucket{-1, -1};
    size_t trial = 0;  // chunks of tuning done in this bucket (tune_candidate maps them to candidates)
    std::vector<double> trial_ms[2];  // ms per period of each candidate's scored chunk, by pass
    Shape best{16, 2048, 2, 1};
    int32_t shape_source = RDOS_SHAPE_DEFAULT;  // where `best` comes from
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    // per-kernel timing: chunks launched directly with events between launches
    int profiling = 0;             // 0 off; 1 timed launches with work tallies; 2 timed launches only
    std::vector<hipEvent_t> kev;
    double scan_ms = 0.0, update_ms = 0.0;
    int64_t scan_n = 0, update_n = 0;
    unsigned long long *d_work = nullptr;  // [3] tets updated, count additions, face transfers (timing pass only)

    // stats
    int64_t launches = 0;
    double updates = 0.0;
    double busy_s = 0.0;
};

namespace {

rdos_status efail(rdos_engine *e, rdos_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    e->error = buf;
    return code;
}

#define ENGINE_HIP(e, expr, what)                                                                    \
    do {                                                                                             \
        hipError_t err__ = (expr);                                                                   \
        if (err__ != hipSuccess)                                                                     \
            return efail(e, err__ == hipErrorOutOfMemory ? RDOS_ENOMEM : RDOS_EDEVICE, "%s: %s", what, \
                         hipGetErrorString(err__));                                                  \
    } while (0)

// Grows a device array to hold `need` elements (x1.5 headroom); a move
// makes the captured graph stale.
template <typename T>
rdos_status ensure(rdos_engine *e, T **buf, int64_t *cap, int64_t need, const char *what)
{
    if (need <= *cap) return RDOS_OK;
    ENGINE_HIP(e, hipStreamSynchronize(e->stream), what);
    std::lock_guard<std::mutex> g(device_api_mutex());
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    const int64_t n = std::max<int64_t>(need, need + need / 2);
    ENGINE_HIP(e, hipMalloc(buf, (size_t)n * sizeof(T)), what);
    *cap = n;
    e->graph_stale = true;
    return RDOS_OK;
}

// Species rows of the queue, which also size the scan's register arrays.
int species_bound(int s)
{
    return s <= 2 ? 2 : (s == 3 ? 3 : (s <= 4 ? 4 : (s <= 6 ? 6 : (s <= 8 ? 8 : (s <= 10 ? 10 : kMaxSpecies)))));
}

// Chunks of tuning per size bucket: two per candidate, then one more each.
size_t tune_end(const rdos_engine *e) { return 3 * e->candidates.size(); }
// The candidate that tuning chunk `trial` runs.
size_t tune_candidate(const rdos_engine *e)
{
    const size_t m = e->candidates.size();
    return e->trial < 2 * m ? e->trial / 2 : e->trial - 2 * m;
}

// Rewrites the device work list for the current slots (lock held).
rdos_status build_work(rdos_engine *e)
{
    // Realizations never exchange molecules, so the (simulation, realization)
    // units split into two independent chains; units are dealt to the chain
    // with fewer tiles so far, chain 0's tiles first in the list.  The host
    // lists the units; a kernel expands them into tiles.
    std::vector<DevSim> sims;
    std::vector<WorkUnit> part[2];
    int64_t part_tiles[2] = {0, 0};
    int32_t max_species = 1;
    int32_t any_scaled = 0;  // some slot uses transfer form 1: the update kernel instance that handles it
    for (size_t i = 0; i < e->slots.size(); ++i) {
        Ticket &tk = e->tickets[e->slots[i]];
        rdos_sim *s = tk.sim;
        DevSim d = s->desc;
        d.step0 = s->step;
        d.step_end = tk.end_step;
        sims.push_back(d);
        const int64_t per = (s->T + kTetsPerTile - 1) / kTetsPerTile;
        for (int32_t r = 0; r < s->Rz; ++r) {
            const int c = part_tiles[0] <= part_tiles[1] ? 0 : 1;
            part[c].push_back({(int32_t)i, r, s->T, 0});
            part_tiles[c] += per;
        }
        max_species = std::max(max_species, (int32_t)s->D.size());
        if (s->desc.transfer_form == 1) any_scaled = 1;
    }
    std::vector<WorkUnit> units = part[0];
    units.insert(units.end(), part[1].begin(), part[1].end());
    int64_t n_tiles = 0;
    for (WorkUnit &u : units) {
        u.first = (int32_t)n_tiles;
        n_tiles += (u.T + kTetsPerTile - 1) / kTetsPerTile;
    }
    e->n_tiles0 = (int32_t)part_tiles[0];
    rdos_status st = ensure(e, &e->d_sims, &e->cap_sims, (int64_t)std::max<size_t>(sims.size(), 1), "engine slots");
    if (st != RDOS_OK) return st;
    st = ensure(e, &e->d_tiles, &e->cap_tiles, std::max<int64_t>(n_tiles, 1), "engine tiles");
    if (st != RDOS_OK) return st;
    st = ensure(e, &e->d_units, &e->cap_units, (int64_t)std::max<size_t>(units.size(), 1), "engine work units");
    if (st != RDOS_OK) return st;
    // chain 0's queue can hold every tile (one chain); chain 1's the second half
    const int64_t need[2] = {std::max<int64_t>(n_tiles, 1), std::max<int64_t>(part_tiles[1], 1)};
    QueueView *qs[2] = {&e->queue, &e->queue2};
    for (int c = 0; c < 2; ++c) {
        int32_t nseg, seg_cap;
        queue_shape(need[c], &nseg, &seg_cap);
        if ((int64_t)nseg * seg_cap > qs[c]->qcap || species_bound(max_species) > qs[c]->species) {
            ENGINE_HIP(e, hipStreamSynchronize(e->stream), "drain before reallocating the queue");
            std::lock_guard<std::mutex> g(device_api_mutex());
            free_queue(qs[c], e->stream);
            ENGINE_HIP(e, alloc_queue(qs[c], need[c] + need[c] / 2, species_bound(max_species), e->stream),
                       "engine queue");
            e->graph_stale = true;
        }
        if (qs[c]->scaled != any_scaled) {  // the captured graph names the other kernel instance
            qs[c]->scaled = any_scaled;
            e->graph_stale = true;
        }
    }
    if (!sims.empty())
        ENGINE_HIP(e, hipMemcpyAsync(e->d_sims, sims.data(), sims.size() * sizeof(DevSim), hipMemcpyHostToDevice,
                                     e->stream),
                   "upload slots");
    if (!units.empty()) {
        ENGINE_HIP(e, hipMemcpyAsync(e->d_units, units.data(), units.size() * sizeof(WorkUnit),
                                     hipMemcpyHostToDevice, e->stream),
                   "upload work units");
        ENGINE_HIP(e, launch_expand_tiles(e->d_units, (int32_t)units.size(), (int32_t)n_tiles, e->d_tiles, e->stream),
                   "expand tiles");
    }
    e->n_tiles = (int32_t)n_tiles;
    e->n_sims = (int32_t)sims.size();
    e->max_species = max_species;
    e->hdr_chains = 0;  // headers are written for the chain count of the next chunk
    return RDOS_OK;
}

// Points the queue headers at one chain over all tiles or two chains.
rdos_status set_chains(rdos_engine *e, int32_t chains)
{
    if (chains == e->hdr_chains) return RDOS_OK;
    if (chains == 1) {
        ENGINE_HIP(e, set_queue_work(&e->queue, e->n_tiles, e->n_sims, e->stream), "work header");
    } else {
        ENGINE_HIP(e, set_queue_work(&e->queue, e->n_tiles0, e->n_sims, e->stream), "work header");
        ENGINE_HIP(e, set_queue_work(&e->queue2, e->n_tiles - e->n_tiles0, e->n_sims, e->stream, e->n_tiles0),
                   "work header");
    }
    e->hdr_chains = chains;
    return RDOS_OK;
}

// Launch grids for the current size bucket: no more scan wavefronts than
// tiles, no more update block columns than queue segments.
int32_t scan_grid_of(const rdos_engine *e, const Shape &sh)
{
    return std::min(sh.scan_grid, scan_blocks_for(e->grid_tiles));
}
int32_t update_segments_of(const rdos_engine *e) { return std::min<int32_t>(e->grid_tiles, kMaxSegments); }

// The launches of `len` periods: a scan and an update launch per period (or
// one fused launch, which leaves the queue halves alone), the first on
// queue half `phase`, then one launch that moves every slot's period index
// on by `len`.  With `timed`, events separate every launch (direct launches
// only: event records are not captured into the graph).
hipError_t enqueue_periods(rdos_engine *e, const Shape &sh, int32_t len, int32_t phase, bool timed)
{
    hipError_t err = hipSuccess;
    const int32_t sg = scan_grid_of(e, sh), gseg = update_segments_of(e);
    if (sh.chains == 2) {
        // two independent chains: fork the second stream off the first, join before the advance
        err = hipEventRecord(e->fork, e->stream);
        if (err == hipSuccess) err = hipStreamWaitEvent(e->stream2, e->fork, 0);
        for (int32_t i = 0; i < len && err == hipSuccess; ++i) {
            const int32_t qs = (phase + i) & 1;
            if (sh.update_bps == 0) {
                err = launch_fused(e->d_sims, e->d_tiles, i, -1, 0.0, e->queue, sg, e->stream);
                if (err == hipSuccess) err = launch_fused(e->d_sims, e->d_tiles, i, -1, 0.0, e->queue2, sg, e->stream2);
                continue;
            }
            err = launch_step(e->d_sims, e->d_tiles, i, -1, 0.0, e->queue, qs, sg, sh.update_bps, gseg, e->stream);
            if (err == hipSuccess)
                err = launch_step(e->d_sims, e->d_tiles, i, -1, 0.0, e->queue2, qs, sg, sh.update_bps, gseg,
                                  e->stream2);
        }
        if (err == hipSuccess) err = hipEventRecord(e->join, e->stream2);
        if (err == hipSuccess) err = hipStreamWaitEvent(e->stream, e->join, 0);
        if (err == hipSuccess) err = launch_advance(e->d_sims, e->queue.hdr, len, e->stream);
        return err;
    }
    if (timed) err = hipEventRecord(e->kev[0], e->stream);
    for (int32_t i = 0; i < len && err == hipSuccess; ++i) {
        const int32_t qs = (phase + i) & 1;
        if (sh.update_bps == 0) {  // fused: timed as an update with an empty scan before it
            if (timed) err = hipEventRecord(e->kev[2 * i + 1], e->stream);
            if (err == hipSuccess) err = launch_fused(e->d_sims, e->d_tiles, i, -1, 0.0, e->queue, sg, e->stream);
            if (err == hipSuccess && timed) err = hipEventRecord(e->kev[2 * i + 2], e->stream);
            continue;
        }
        err = launch_scan(e->d_sims, e->d_tiles, i, e->queue, qs, sg, e->stream);
        if (err == hipSuccess && timed) err = hipEventRecord(e->kev[2 * i + 1], e->stream);
        if (err == hipSuccess)
            err = launch_update(e->d_sims, e->d_tiles, i, -1, 0.0, e->queue, qs, sh.update_bps, gseg, e->stream);
        if (err == hipSuccess && timed) err = hipEventRecord(e->kev[2 * i + 2], e->stream);
    }
    if (err == hipSuccess) err = launch_advance(e->d_sims, e->queue.hdr, len, e->stream);
    return err;
}

void drop_graphs(rdos_engine *e)
{
    for (auto &kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    e->graphs.clear();
}

// The graph of one chunk of shape `sh` at the current grid size, captured on
// first use.
rdos_status graph_for(rdos_engine *e, const Shape &sh, hipGraphExec_t *out)
{
    std::lock_guard<std::mutex> lock(device_api_mutex());
    if (e->graph_stale) {
        drop_graphs(e);
        e->graph_stale = false;
    }
    const std::array<int32_t, 5> key{sh.chunk, sh.scan_grid, sh.update_bps, sh.chains, e->grid_tiles};
    auto it = e->graphs.find(key);
    if (it != e->graphs.end()) {
        *out = it->second;
        return RDOS_OK;
    }
    if (e->graphs.size() >= 32) drop_graphs(e);
    hipGraph_t g = nullptr;
    ENGINE_HIP(e, hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t err = enqueue_periods(e, sh, sh.chunk, 0, false);
    hipError_t err2 = hipStreamEndCapture(e->stream, &g);
    if (err != hipSuccess || err2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return efail(e, RDOS_EDEVICE, "capture: %s", hipGetErrorString(err != hipSuccess ? err : err2));
    }
    hipGraphExec_t x = nullptr;
    err = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) return efail(e, RDOS_EDEVICE, "instantiate: %s", hipGetErrorString(err));
    e->graphs[key] = x;
    *out = x;
    return RDOS_OK;
}

double slot_updates(const rdos_sim *s) { return (double)s->Rz * (double)s->T * (double)s->D.size(); }

int64_t tiled_tets(const rdos_sim *q)
{
    return (int64_t)q->Rz * ((q->T + kTetsPerTile - 1) / kTetsPerTile) * kTetsPerTile;
}

// Admission threads: each takes the first waiting ticket while its device
// memory fits the budget, finalizes it if it is not finalized yet (with the
// lock released, on the simulation's own stream) and hands it to the
// worker, which adds it to the work list at its next chunk.
void admitter_main(rdos_engine *e)
{
    (void)hipSetDevice(e->device);
    std::unique_lock<std::mutex> lk(e->mu);
    while (!e->stop) {
        bool progressed = false;
        if (!e->waiting.empty()) {
            const uint64_t id = e->waiting.front();
            Ticket &tk = e->tickets[id];
            // queue entries are int32 (tile * kTetsPerTile + offset): keep the work list below 2^31 tets
            const int64_t own_tiled = tiled_tets(tk.sim);
            int64_t tiled = own_tiled + e->admitting_tiled;
            for (uint64_t sid : e->slots) tiled += tiled_tets(e->tickets[sid].sim);
            for (uint64_t sid : e->ready) tiled += tiled_tets(e->tickets[sid].sim);
            const bool fits = e->used + tk.bytes <= e->budget &&
                              (tiled <= 0x7fffffff || (e->slots.empty() && e->ready.empty() && e->admitting == 0));
            if (fits) {
                tk.admit_start = Clock::now();
                e->waiting.pop_front();
                e->used += tk.bytes;
                ++e->admitting;
                e->admitting_tiled += own_tiled;
                rdos_sim *s = tk.sim;
                const double tau_scale = tk.tau_scale;
                rdos_status st = RDOS_OK;
                std::string err;
                lk.unlock();
                if (s->state != SimState::Ready) {
                    s->engine_owned = false;
                    st = rdos_finalize(s, tau_scale, nullptr);
                    s->engine_owned = true;
                }
                if (st == RDOS_OK) st = ensure_mask(s);  // occupancy of counts set from the host
                if (st == RDOS_OK && hipStreamSynchronize(s->stream) != hipSuccess)
                    st = fail(s, RDOS_EDEVICE, "occupancy rebuild failed");
                if (st != RDOS_OK) err = s->error;
                lk.lock();
                --e->admitting;
                e->admitting_tiled -= own_tiled;
                Ticket &t2 = e->tickets[id];
                t2.admit_end = Clock::now();
                if (st == RDOS_OK) {
                    t2.end_step = s->step + t2.n_steps;
                    t2.admitted = true;
                    if (t2.n_steps == 0) {
                        t2.done = true;
                        t2.finished = Clock::now();
                        e->cv_done.notify_all();
                    } else {
                        e->ready.push_back(id);
                        e->cv_work.notify_all();
                    }
                } else {
                    t2.failed = t2.done = true;
                    t2.error = err;
                    t2.finished = Clock::now();
                    e->used -= t2.bytes;
                    e->cv_done.notify_all();
                }
                progressed = true;
            }
        }
        // nothing runs or waits to join and the next request does not fit: only a release can help
        e->stalled = !progressed && !e->waiting.empty() && e->slots.empty() && e->ready.empty() &&
                     e->admitting == 0;
        e->admit_blocked = !progressed && !e->waiting.empty();
        if (e->stalled || !progressed) e->cv_done.notify_all();
        if (!progressed) e->cv_admit.wait(lk);
    }
}

void fail_slots(rdos_engine *e)
{
    for (uint64_t id : e->slots) {
        Ticket &tk = e->tickets[id];
        tk.failed = tk.done = true;
        tk.error = e->error;
        tk.finished = Clock::now();
    }
    e->slots.clear();
    e->cv_done.notify_all();
}

void worker_main(rdos_engine *e)
{
    (void)hipSetDevice(e->device);
    std::unique_lock<std::mutex> lk(e->mu);
    while (!e->stop) {
        if (e->held) {  // rdos_engine_hold: admissions go on, no chunk starts
            e->cv_work.wait(lk);
            continue;
        }
        if (!e->ready.empty()) {  // continuous batching: newly admitted simulations join here
            const auto joined = Clock::now();
            for (uint64_t id : e->ready) {
                e->slots.push_back(id);
                e->tickets[id].started = joined;
            }
            e->ready.clear();
            e->rebuild = true;
        }
        if (e->slots.empty()) {
            e->cv_work.wait(lk);
            continue;
        }
        if (e->rebuild) {
            if (build_work(e) != RDOS_OK) {
                fail_slots(e);
                break;
            }
            e->rebuild = false;
            const int lg = (int)std::ilogb((double)std::max(e->n_tiles, 1));
            const std::pair<int, int> b{lg, species_bound(e->max_species)};
            // launch grids cover every work list of this size bucket
            e->grid_tiles = (int32_t)std::min<int64_t>(int64_t(1) << (lg + 1), int64_t(1) << 30);
            // every work list of a bucket this small has a segment per tile, and the scan grids
            // give each tile a wavefront (the graphs of the bucket keep this scan instance)
            e->queue.owned = e->queue2.owned = e->grid_tiles <= kMaxSegments ? 1 : 0;
            if (b != e->bucket && !e->fixed_shape && e->grid_tiles <= kSmallWorkTiles) {
                // small work lists: every candidate clamps to about the same
                // grids and launch latency dominates; no tuning, long chunks
                e->bucket = b;
                e->best = kSmallWorkShape;
                e->shape_source = RDOS_SHAPE_SMALL_WORK;
                e->trial = tune_end(e);
                for (auto &v : e->trial_ms) v.assign(e->candidates.size(), 0.0);  // nothing measured here
            } else if (b != e->bucket) {
                e->bucket = b;
                auto hit = e->tuned.find(b);
                bool found = hit != e->tuned.end();
                Shape cached{};
                if (found) {
                    cached = hit->second;
                } else {
                    TuneCache &tc = tune_cache();
                    std::lock_guard<std::mutex> g(tc.mu);
                    auto it = tc.shapes.find(b);
                    if (it != tc.shapes.end()) {
                        found = true;
                        cached = it->second;
                        e->tuned[b] = cached;
                    }
                }
                if (found) {
                    if (!e->fixed_shape) {
                        e->best = cached;
                        e->shape_source = RDOS_SHAPE_CACHED;
                    }
                    e->trial = tune_end(e);
                    for (auto &v : e->trial_ms) v.assign(e->candidates.size(), 0.0);  // measured elsewhere
                } else {
                    e->trial = 0;
                    for (auto &v : e->trial_ms) v.assign(e->candidates.size(), 0.0);
                    if (!e->fixed_shape) e->shape_source = RDOS_SHAPE_DEFAULT;
                }
            }
        }
        // the tuner tries each candidate per size bucket, then keeps the best
        const bool tuning = !e->fixed_shape && e->trial < tune_end(e);
        Shape sh = tuning ? e->candidates[tune_candidate(e)] : e->best;
        const bool timed = e->profiling != 0;
        if (timed || e->n_tiles0 == 0 || e->n_tiles0 == e->n_tiles) sh.chains = 1;  // nothing to split
        if (sh.update_bps == 0 && e->queue.species > kFusedSpecies) sh.update_bps = 1;  // too wide to fuse
        // fused periods leave the queue's length halves alone: any phase suits them
        const bool fused = sh.update_bps == 0;
        if (set_chains(e, sh.chains) != RDOS_OK) {
            fail_slots(e);
            break;
        }
        // A full chunk replays the captured graph, which starts on queue half
        // 0.  The last periods of the slots (fewer than a chunk) are launched
        // directly, as many as are left, so no launch runs idle; after an odd
        // number of them one direct period puts the queue halves back in step
        // with the graph.  The timing pass always launches directly.
        int64_t left_max = 1;
        for (uint64_t id : e->slots) {
            const Ticket &tk = e->tickets[id];
            left_max = std::max<int64_t>(left_max, tk.end_step - tk.sim->step);
        }
        bool replay = !timed && (fused || e->qphase == 0) && left_max >= sh.chunk;
        int32_t len = replay ? sh.chunk : (int32_t)std::min<int64_t>(left_max, sh.chunk);
        if (!replay && !timed && !fused && e->qphase == 1 && left_max >= sh.chunk) len = 1;
        // Small work lists run their periods in one cooperative launch: as
        // many as the slot nearest its end has left, or (when requests wait
        // to join) at most a chunk, or about 2 ms of device time.
        int32_t persist = 0;
        if (!timed && e->shape_source == RDOS_SHAPE_SMALL_WORK && sh.chains == 1 && e->n_tiles <= kPersistTiles) {
            const int32_t key = e->queue.species * 2 + e->queue.scaled;
            if (key != e->persist_key) {
                e->persist_limit = persist_grid_limit(e->queue);
                e->persist_key = key;
            }
            if (e->persist_limit > 0)
                persist = std::min(e->persist_limit, std::max(4 * e->queue.nseg, scan_blocks_for(e->n_tiles)));
        }
        if (persist > 0) {
            replay = false;
            const bool pending = !e->ready.empty() || !e->waiting.empty() || e->admitting > 0;
            int64_t left_min = left_max;
            for (uint64_t id : e->slots) {
                const Ticket &tk = e->tickets[id];
                left_min = std::min<int64_t>(left_min, tk.end_step - tk.sim->step);
            }
            int64_t cap = sh.chunk;
            if (!pending && e->last_period_ms > 0.0)
                cap = std::max<int64_t>(cap, (int64_t)(2.0 / e->last_period_ms));
            len = (int32_t)std::max<int64_t>(1, std::min<int64_t>({left_min, cap, kPersistPeriods}));
        }
        // the timing pass launches directly and tallies its work; captured graphs never do
        e->queue.work = e->queue2.work = e->profiling == 1 ? e->d_work : nullptr;
        if (timed) {
            bool ok = true;
            while (ok && (int32_t)e->kev.size() < 2 * len + 1) {
                hipEvent_t ev;
                ok = hipEventCreate(&ev) == hipSuccess;
                if (ok) e->kev.push_back(ev);
            }
            if (!ok) {
                e->error = "create profiling events";
                fail_slots(e);
                break;
            }
        }
        hipGraphExec_t gx = nullptr;
        if (replay && graph_for(e, sh, &gx) != RDOS_OK) {
            fail_slots(e);
            break;
        }
        // When no slot ends within them and no request waits to join, up to
        // 8 chunks (about 2 ms of device time) are replayed back to back, so
        // the host's turn between chunks does not leave the device idle.
        // When those replays take every slot to within a chunk of its end and
        // all slots end together, the remaining periods are launched directly
        // behind them, so the run ends without another turn of the host.
        int32_t reps = 1, tail = 0;
        if (replay && !tuning && e->ready.empty() && e->waiting.empty() && e->admitting == 0) {
            int64_t left_min = left_max;
            for (uint64_t id : e->slots) {
                const Ticket &tk = e->tickets[id];
                left_min = std::min<int64_t>(left_min, tk.end_step - tk.sim->step);
            }
            int64_t r = left_min / sh.chunk;
            if (e->last_chunk_ms > 0.0) r = std::min<int64_t>(r, (int64_t)(2.0 / e->last_chunk_ms));
            reps = (int32_t)std::max<int64_t>(1, std::min<int64_t>(r, 8));
            if (left_min == left_max && (int64_t)reps * sh.chunk + sh.chunk > left_max)
                tail = (int32_t)(left_max - (int64_t)reps * sh.chunk);
        }
        len = len * reps + tail;
        double work = 0.0;
        for (uint64_t id : e->slots) {
            Ticket &tk = e->tickets[id];
            const int64_t left = tk.end_step - tk.sim->step;
            work += slot_updates(tk.sim) * (double)std::min<int64_t>(left, len);
        }
        const int32_t phase = e->qphase;
        lk.unlock();
        hipError_t err = hipEventRecord(e->ev0, e->stream);
        if (err == hipSuccess) {
            if (persist > 0) {
                err = launch_persist(e->d_sims, e->d_tiles, 0, len, phase, -1, 0.0, e->queue, persist, e->queue.sync,
                                     e->stream);
                if (err == hipSuccess) err = launch_advance(e->d_sims, e->queue.hdr, len, e->stream);
            } else if (replay) {
                for (int32_t k = 0; k < reps && err == hipSuccess; ++k) err = hipGraphLaunch(gx, e->stream);
                if (err == hipSuccess && tail > 0)
                    err = enqueue_periods(e, sh, tail, (phase + reps * sh.chunk) & 1, false);
            } else {
                err = enqueue_periods(e, sh, len, phase, timed);
            }
        }
        if (err == hipSuccess) err = hipEventRecord(e->ev1, e->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e->ev1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e->ev0, e->ev1);
        lk.lock();
        if (err != hipSuccess) {
            e->error = std::string("chunk: ") + hipGetErrorString(err);
            fail_slots(e);
            break;
        }
        if (!fused || persist > 0) e->qphase = (phase + len) & 1;
        if (timed) {
            for (int32_t i = 0; i < len; ++i) {
                float a = 0.f, b = 0.f;
                if (hipEventElapsedTime(&a, e->kev[2 * i], e->kev[2 * i + 1]) == hipSuccess &&
                    hipEventElapsedTime(&b, e->kev[2 * i + 1], e->kev[2 * i + 2]) == hipSuccess) {
                    e->scan_ms += a;
                    e->update_ms += b;
                    ++e->scan_n;
                    ++e->update_n;
                }
            }
        }
        if (replay && tail == 0) e->last_chunk_ms = (double)ms / reps;
        if (persist > 0) e->last_period_ms = (double)ms / len;
        if (tuning && replay) {  // only full graph-replayed chunks are scored
            const size_t m = e->candidates.size();
            if (e->trial >= 2 * m || (e->trial & 1)) e->trial_ms[e->trial >= 2 * m][tune_candidate(e)] = ms / len;
            ++e->trial;
            if (e->trial == tune_end(e)) {
                double best_ms = 0.0;
                for (size_t c = 0; c < m; ++c) {
                    const double t = 0.5 * (e->trial_ms[0][c] + e->trial_ms[1][c]);
                    if (c == 0 || t < best_ms) {
                        best_ms = t;
                        e->best = e->candidates[c];
                    }
                }
                e->tuned[e->bucket] = e->best;
                e->shape_source = RDOS_SHAPE_TUNED;
                TuneCache &tc = tune_cache();
                std::lock_guard<std::mutex> g(tc.mu);
                tc.shapes[e->bucket] = e->best;
            }
        }
        e->launches += len;
        e->updates += work;
        e->busy_s += ms * 1e-3;
        // progress and retirement
        const auto now = Clock::now();
        std::vector<uint64_t> keep;
        for (uint64_t id : e->slots) {
            Ticket &tk = e->tickets[id];
            rdos_sim *s = tk.sim;
            s->step = std::min<int64_t>(s->step + len, tk.end_step);
            if (s->step >= tk.end_step) {
                tk.done = true;
                tk.finished = now;
                e->rebuild = true;
            } else {
                keep.push_back(id);
            }
        }
        if (keep.size() != e->slots.size()) {
            e->cv_done.notify_all();
            e->cv_admit.notify_all();  // lets the admission thread re-check whether it is stalled
        }
        e->slots.swap(keep);
    }
    e->worker_dead = !e->stop;
    e->cv_done.notify_all();
}

}  // namespace

extern "C" {

rdos_status rdos_engine_create(rdos_engine **out, int device, size_t hbm_budget_bytes)
{
    if (!out) return RDOS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RDOS_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return RDOS_EDEVICE;
    rdos_engine *e = new (std::nothrow) rdos_engine();
    if (!e) return RDOS_ENOMEM;
    e->device = device;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        delete e;
        return RDOS_EDEVICE;
    }
    e->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
    if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&e->stream2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&e->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e->join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&e->ev0) != hipSuccess || hipEventCreate(&e->ev1) != hipSuccess ||
        hipStreamSynchronize(e->stream) != hipSuccess) {
        delete e;
        return RDOS_EDEVICE;
    }
    // Two-launch shapes only: the fused shape (update_bps 0) lost to them on every tuned size measured,
    // and under a profiler, which taxes each launch, it scored first; it stays available by set_shape.
    // One 32-period shape: fewer graph launches per period, at the cost of a longer wait to join.
    e->candidates = {{16, 2048, 2, 1}, {16, 1024, 2, 2}, {16, 2048, 2, 2}, {16, 4096, 1, 2}, {32, 4096, 1, 2}};
    e->worker = std::thread(worker_main, e);
    for (std::thread &t : e->admitters) t = std::thread(admitter_main, e);
    *out = e;
    return RDOS_OK;
}

rdos_status rdos_engine_submit(rdos_engine *e, rdos_sim *sim, int64_t n_steps, double tau_scale, uint64_t *ticket)
{
    if (!e || !sim || n_steps < 0) return RDOS_EINVAL;
    if (sim->engine_owned) return efail(e, RDOS_EBUSY, "simulation already owned by an engine");
    if (sim->state == SimState::Created) return efail(e, RDOS_ESTATE, "simulation has no mesh");
    if (sim->D.empty()) return efail(e, RDOS_ESTATE, "simulation has no species");
    if (sim->state == SimState::Ready && sim->device != e->device)
        return efail(e, RDOS_EINVAL, "simulation lives on another device");
    if (!(tau_scale > 0.0 && tau_scale <= 1.0)) return efail(e, RDOS_EINVAL, "tau_scale must be in (0, 1]");
    const size_t bytes = state_bytes(sim);
    if ((int64_t)sim->Rz * ((sim->T + kTetsPerTile - 1) / kTetsPerTile) * kTetsPerTile > 0x7fffffff)
        return efail(e, RDOS_EINVAL, "realizations x tets exceeds 2^31");
    std::lock_guard<std::mutex> g(e->mu);
    if (bytes > e->budget) return efail(e, RDOS_ENOMEM, "simulation needs %zu bytes, budget is %zu", bytes, e->budget);
    sim->engine_owned = true;
    sim->device = e->device;
    const uint64_t id = e->next_ticket++;
    Ticket &tk = e->tickets[id];
    tk.sim = sim;
    tk.n_steps = n_steps;
    tk.tau_scale = tau_scale;
    tk.bytes = bytes;
    tk.submitted = Clock::now();
    e->waiting.push_back(id);
    e->admit_blocked = false;  // the admission thread looks again
    if (ticket) *ticket = id;
    e->cv_admit.notify_all();
    return RDOS_OK;
}

rdos_status rdos_engine_poll(rdos_engine *e, uint64_t ticket, int *done, double *latency_s)
{
    if (!e) return RDOS_EINVAL;
    std::lock_guard<std::mutex> g(e->mu);
    auto it = e->tickets.find(ticket);
    if (it == e->tickets.end()) return efail(e, RDOS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const Ticket &tk = it->second;
    if (done) *done = tk.done ? 1 : 0;
    if (latency_s)
        *latency_s = tk.done ? std::chrono::duration<double>(tk.finished - tk.submitted).count() : 0.0;
    if (tk.failed) return efail(e, RDOS_EDEVICE, "ticket failed: %s", tk.error.c_str());
    return RDOS_OK;
}

rdos_status rdos_engine_ticket_times(rdos_engine *e, uint64_t ticket, double *wait_s, double *setup_s,
                                     double *join_s, double *run_s)
{
    if (!e) return RDOS_EINVAL;
    std::lock_guard<std::mutex> g(e->mu);
    auto it = e->tickets.find(ticket);
    if (it == e->tickets.end()) return efail(e, RDOS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const Ticket &tk = it->second;
    if (!tk.done || tk.failed || tk.n_steps == 0)
        return efail(e, RDOS_ESTATE, "ticket %llu has not run to completion", (unsigned long long)ticket);
    auto sec = [](Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); };
    if (wait_s) *wait_s = sec(tk.submitted, tk.admit_start);
    if (setup_s) *setup_s = sec(tk.admit_start, tk.admit_end);
    if (join_s) *join_s = sec(tk.admit_end, tk.started);
    if (run_s) *run_s = sec(tk.started, tk.finished);
    return RDOS_OK;
}

rdos_status rdos_engine_hold(rdos_engine *e, int32_t on)
{
    if (!e) return RDOS_EINVAL;
    std::unique_lock<std::mutex> lk(e->mu);
    if (on) {
        e->held = true;
        return RDOS_OK;
    }
    // every queued request that fits is admitted before the worker goes on
    e->cv_done.wait(lk, [&] {
        return (e->admitting == 0 && (e->waiting.empty() || e->admit_blocked)) || e->worker_dead || e->stop;
    });
    e->held = false;
    e->cv_work.notify_all();
    return RDOS_OK;
}

rdos_status rdos_engine_drain(rdos_engine *e)
{
    if (!e) return RDOS_EINVAL;
    std::unique_lock<std::mutex> lk(e->mu);
    e->cv_done.wait(lk, [&] {
        return (e->waiting.empty() && e->ready.empty() && e->slots.empty() && e->admitting == 0) ||
               e->worker_dead || e->stalled;
    });
    for (auto &kv : e->tickets)
        if (kv.second.failed) return efail(e, RDOS_EDEVICE, "a ticket failed: %s", kv.second.error.c_str());
    if (e->worker_dead) return efail(e, RDOS_EDEVICE, "engine stopped: %s", e->error.c_str());
    if (e->stalled)
        return efail(e, RDOS_ENOMEM, "queued simulations do not fit the budget until finished ones are released");
    return RDOS_OK;
}

rdos_status rdos_engine_release(rdos_engine *e, uint64_t ticket, rdos_sim **sim)
{
    if (!e || !sim) return RDOS_EINVAL;
    std::lock_guard<std::mutex> g(e->mu);
    auto it = e->tickets.find(ticket);
    if (it == e->tickets.end()) return efail(e, RDOS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.done) return efail(e, RDOS_EBUSY, "ticket %llu is still running", (unsigned long long)ticket);
    rdos_sim *s = it->second.sim;
    s->engine_owned = false;
    e->used -= it->second.bytes;
    *sim = s;
    e->tickets.erase(it);
    e->stalled = false;  // budget was freed: the admission thread re-checks
    e->admit_blocked = false;
    e->cv_admit.notify_all();
    return RDOS_OK;
}

rdos_status rdos_engine_stats(rdos_engine *e, int64_t *launches, double *updates, double *busy_s)
{
    if (!e) return RDOS_EINVAL;
    std::lock_guard<std::mutex> g(e->mu);
    if (launches) *launches = e->launches;
    if (updates) *updates = e->updates;
    if (busy_s) *busy_s = e->busy_s;
    return RDOS_OK;
}

rdos_status rdos_engine_launch_shape(rdos_engine *e, int32_t *chunk, int32_t *scan_grid, int32_t *update_bps,
                                     int32_t *chains, int32_t *source)
{
    if (!e) return RDOS_EINVAL;
    std::lock_guard<std::mutex> g(e->mu);
    if (chunk) *chunk = e->best.chunk;
    if (scan_grid) *scan_grid = e->best.scan_grid;
    if (update_bps) *update_bps = e->best.update_bps;
    if (chains) *chains = e->best.chains;
    if (source) *source = e->shape_source;
    return RDOS_OK;
}

rdos_status rdos_engine_tuner_scores(rdos_engine *e, int32_t cap, int32_t *n, int32_t *shapes, double *ms_first,
                                     double *ms_second)
{
    if (!e || cap < 0) return RDOS_EINVAL;
    std::lock_guard<std::mutex> g(e->mu);
    const int32_t m = (int32_t)e->candidates.size();
    if (n) *n = m;
    for (int32_t c = 0; c < std::min(cap, m); ++c) {
        const Shape &sh = e->candidates[c];
        if (shapes) {
            shapes[4 * c] = sh.chunk;
            shapes[4 * c + 1] = sh.scan_grid;
            shapes[4 * c + 2] = sh.update_bps;
            shapes[4 * c + 3] = sh.chains;
        }
        const bool have = e->trial_ms[0].size() == (size_t)m;
        if (ms_first) ms_first[c] = have ? e->trial_ms[0][c] : 0.0;
        if (ms_second) ms_second[c] = have ? e->trial_ms[1][c] : 0.0;
    }
    return RDOS_OK;
}

rdos_status rdos_engine_set_shape(rdos_engine *e, int32_t chunk, int32_t scan_grid, int32_t update_bps,
                                  int32_t chains)
{
    if (!e) return RDOS_EINVAL;
    if (chunk < 0) return efail(e, RDOS_EINVAL, "negative chunk");
    std::lock_guard<std::mutex> g(e->mu);
    if (chunk == 0) {  // back to tuning
        e->fixed_shape = false;
        e->bucket = {-1, -1};
        e->rebuild = true;  // the worker re-enters the size bucket (cache or tuner)
        e->shape_source = RDOS_SHAPE_DEFAULT;
        return RDOS_OK;
    }
    if (chunk % 2 != 0 || chunk > 1024 || scan_grid < 1 || scan_grid > (1 << 20) || update_bps < 0 ||
        update_bps > 64 || (chains != 1 && chains != 2))
        return efail(e, RDOS_EINVAL, "launch shape out of range");
    e->best = Shape{chunk, scan_grid, update_bps, chains};
    e->fixed_shape = true;
    e->shape_source = RDOS_SHAPE_FIXED;
    return RDOS_OK;
}

rdos_status rdos_engine_set_profiling(rdos_engine *e, int on)
{
    if (!e) return RDOS_EINVAL;
    if (on < 0 || on > 2) return efail(e, RDOS_EINVAL, "profiling mode must be 0, 1 or 2");
    std::lock_guard<std::mutex> g(e->mu);
    if (on == 1 && !e->d_work) {
        hipError_t err;
        {
            std::lock_guard<std::mutex> dg(device_api_mutex());
            err = hipMalloc(&e->d_work, 3 * sizeof(unsigned long long));
        }
        if (err != hipSuccess) return efail(e, RDOS_ENOMEM, "work counters: %s", hipGetErrorString(err));
    }
    if (on == 1) {
        ENGINE_HIP(e, hipMemsetAsync(e->d_work, 0, 3 * sizeof(unsigned long long), e->stream), "clear work counters");
        ENGINE_HIP(e, hipStreamSynchronize(e->stream), "clear work counters");
    }
    e->profiling = on;
    e->scan_ms = e->update_ms = 0.0;
    e->scan_n = e->update_n = 0;
    return RDOS_OK;
}

rdos_status rdos_engine_work_counts(rdos_engine *e, int64_t *tets, int64_t *additions, int64_t *transfers)
{
    if (!e) return RDOS_EINVAL;
    std::lock_guard<std::mutex> g(e->mu);
    unsigned long long w[3] = {0, 0, 0};
    if (e->d_work) {
        ENGINE_HIP(e, hipMemcpyAsync(w, e->d_work, sizeof w, hipMemcpyDeviceToHost, e->stream), "read work counters");
        ENGINE_HIP(e, hipStreamSynchronize(e->stream), "read work counters");
    }
    if (tets) *tets = (int64_t)w[0];
    if (additions) *additions = (int64_t)w[1];
    if (transfers) *transfers = (int64_t)w[2];
    return RDOS_OK;
}

rdos_status rdos_engine_kernel_times(rdos_engine *e, double *scan_ms, int64_t *scan_launches, double *update_ms,
                                     int64_t *update_launches)
{
    if (!e) return RDOS_EINVAL;
    std::lock_guard<std::mutex> g(e->mu);
    if (scan_ms) *scan_ms = e->scan_ms;
    if (scan_launches) *scan_launches = e->scan_n;
    if (update_ms) *update_ms = e->update_ms;
    if (update_launches) *update_launches = e->update_n;
    return RDOS_OK;
}

rdos_status rdos_bandwidth_probe(int device, size_t bytes, int reps, double *gbps)
{
    if (!gbps || reps < 1 || bytes < 16) return RDOS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return RDOS_EDEVICE;
    void *a = nullptr, *b = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rdos_status rc = RDOS_OK;
    float ms = 0.f;
    bool allocated;
    {
        std::lock_guard<std::mutex> g(device_api_mutex());
        allocated = hipMalloc(&a, bytes) == hipSuccess && hipMalloc(&b, bytes) == hipSuccess;
    }
    if (!allocated) {
        rc = RDOS_ENOMEM;
    } else if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
               hipEventCreate(&e1) != hipSuccess || hipMemsetAsync(a, 1, bytes, st) != hipSuccess ||
               launch_copy(a, b, bytes, st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess) {
        rc = RDOS_EDEVICE;
    } else {
        for (int i = 0; i < reps && rc == RDOS_OK; ++i)
            if (launch_copy((i & 1) ? b : a, (i & 1) ? a : b, bytes, st) != hipSuccess) rc = RDOS_EDEVICE;
        if (rc == RDOS_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = RDOS_EDEVICE;
    }
    if (rc == RDOS_OK) *gbps = 2.0 * (double)(bytes / 16 * 16) * reps / ((double)ms * 1e-3) / 1e9;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    {
        std::lock_guard<std::mutex> g(device_api_mutex());
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
    }
    return rc;
}

rdos_status rdos_tune_split_threshold(int device, int32_t n_max, int32_t *threshold, double *ms_one_by_one,
                                      double *ms_sequential)
{
    if (!threshold || n_max < 2 || n_max > 256) return RDOS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return RDOS_EDEVICE;
    constexpr int32_t kBlocks = 1024, kReps = 4;
    int64_t *sink = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<double> one((size_t)n_max + 1, 0.0), seq((size_t)n_max + 1, 0.0);
    rdos_status rc = RDOS_OK;
    {
        std::lock_guard<std::mutex> g(device_api_mutex());
        if (hipMalloc(&sink, (size_t)kBlocks * 256 * sizeof(int64_t)) != hipSuccess) rc = RDOS_ENOMEM;
    }
    if (rc == RDOS_OK && (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                          hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = RDOS_EDEVICE;
    // warm-up, then each method at each n, timed on its own
    if (rc == RDOS_OK && (launch_split_cost(true, 8, kReps, sink, kBlocks, st) != hipSuccess ||
                          launch_split_cost(false, 8, kReps, sink, kBlocks, st) != hipSuccess))
        rc = RDOS_EDEVICE;
    for (int32_t n = 1; n <= n_max && rc == RDOS_OK; ++n)
        for (int m = 0; m < 2 && rc == RDOS_OK; ++m) {
            float ms = 0.f;
            if (hipEventRecord(e0, st) != hipSuccess || launch_split_cost(m == 0, n, kReps, sink, kBlocks, st) != hipSuccess ||
                hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = RDOS_EDEVICE;
            (m == 0 ? one : seq)[(size_t)n] = ms;
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (sink) {
        std::lock_guard<std::mutex> g(device_api_mutex());
        (void)hipFree(sink);
    }
    if (rc != RDOS_OK) return rc;
    // the switch point: from here on the binomial chain is never slower
    int32_t t = n_max + 1;
    for (int32_t n = n_max; n >= 1 && seq[(size_t)n] <= one[(size_t)n]; --n) t = n;
    *threshold = t;
    for (int32_t n = 1; n <= n_max; ++n) {
        if (ms_one_by_one) ms_one_by_one[n - 1] = one[(size_t)n];
        if (ms_sequential) ms_sequential[n - 1] = seq[(size_t)n];
    }
    return RDOS_OK;
}

const char *rdos_engine_last_error(const rdos_engine *e) { return e ? e->error.c_str() : "null engine"; }

void rdos_engine_destroy(rdos_engine *e)
{
    if (!e) return;
    {
        std::lock_guard<std::mutex> g(e->mu);
        e->stop = true;
    }
    e->cv_work.notify_all();
    e->cv_admit.notify_all();
    if (e->worker.joinable()) e->worker.join();
    for (std::thread &t : e->admitters)
        if (t.joinable()) t.join();
    (void)hipSetDevice(e->device);
    (void)hipStreamSynchronize(e->stream);
    for (auto &kv : e->tickets) {  // simulations never released are destroyed with the engine
        kv.second.sim->engine_owned = false;
        rdos_destroy(kv.second.sim);
    }
    drop_graphs(e);
    void *p[] = {e->d_sims, e->d_tiles, e->d_units, e->d_work};
    for (void *q : p)
        if (q) (void)hipFree(q);
    free_queue(&e->queue, e->stream);
    free_queue(&e->queue2, e->stream);
    (void)hipStreamSynchronize(e->stream);
    for (hipEvent_t ev : e->kev) (void)hipEventDestroy(ev);
    if (e->fork) (void)hipEventDestroy(e->fork);
    if (e->join) (void)hipEventDestroy(e->join);
    if (e->stream2) (void)hipStreamDestroy(e->stream2);
    if (e->ev0) (void)hipEventDestroy(e->ev0);
    if (e->ev1) (void)hipEventDestroy(e->ev1);
    if (e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

}  // extern "C"
