/*
 * rdos -- operator-split stochastic reaction-diffusion on tetrahedral meshes,
 * on one AMD Instinct MI355X (gfx950).
 *
 * The method is that of Hepburn, Chen & De Schutter, "Accurate
 * Reaction-Diffusion Operator Splitting on Tetrahedral Meshes for Parallel
 * Stochastic Molecular Simulations" (arXiv:1512.03126), Algorithm 1: every
 * period tau each tetrahedron runs an exact SSA of its own reactions while
 * recording the time-mean population ("occupancy", Sec. II.C, eq. 2); then,
 * per diffusing species, n = binomial(Nbar, zeta) molecules leave (eq. 3,
 * zeta = tau d, Sec. II.A) and are split multinomially over the face
 * neighbours (Sec. II.B).
 *
 * Conventions shared by every call
 *   - Plain C99 ABI: opaque handles, host pointers for inputs/outputs, status
 *     codes <= 0.  No exception crosses the ABI.  rdos_last_error() returns a
 *     message for the last failing call on a handle (valid until the next
 *     call on it).
 *   - The caller owns every host array it passes; the library copies in and
 *     out and keeps no caller pointer after a call returns.
 *   - The library owns all device memory of a simulation from
 *     rdos_finalize() to rdos_destroy().
 *   - A handle is not thread-safe: use one handle per host thread.
 *   - Call order is enforced (RDOS_ESTATE otherwise):
 *       create -> set_mesh -> add_species / add_reaction -> finalize
 *              -> set_counts -> step / run_until -> get_counts
 *     set_counts may also be called before finalize (the counts are staged
 *     on the host and uploaded by finalize).
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 *     (low 32 bits of seed, high 32 bits of seed XOR realization) and counter
 *     (draw block, stream, tet, low 32 bits of the period index).  Stream m
 *     is species m's diffusion draws; stream 0x80000000 the tet's SSA draws.
 *     Results therefore do not depend on launch shape, batching or order.
 *   - Units: SI.  Coordinates in metres, D in m^2/s, rate constants in
 *     M/s (0th order), 1/s (1st order), 1/(M s) (2nd order).
 */
#ifndef RDOS_H
#define RDOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rdos_sim rdos_sim;
typedef struct rdos_engine rdos_engine;

typedef enum {
    RDOS_OK = 0,
    RDOS_EINVAL = -1,     /* invalid argument or mesh                         */
    RDOS_ENOMEM = -2,     /* device or host allocation failed                 */
    RDOS_EDEVICE = -3,    /* a HIP call failed                                */
    RDOS_ESTATE = -4,     /* call out of order                                */
    RDOS_EOVERFLOW = -5,  /* a molecule count left the int32 range            */
    RDOS_EBUSY = -6       /* the simulation is owned by an engine             */
} rdos_status;

/* Limits of one simulation. */
#define RDOS_MAX_SPECIES 16
#define RDOS_MAX_REACTIONS 32

/* New simulation on HIP device `device` with n_realizations independent
 * realizations (realization r uses Philox key (seed, r)).  Each realization is
 * one run of Algorithm 1 from its own initial counts; the validations of
 * Sec. III average over many such runs of one model.
 *   out             receives the handle (NULL on failure); the caller frees it
 *                   with rdos_destroy
 *   n_realizations  >= 1
 * RDOS_EINVAL for a null out or n_realizations < 1, RDOS_EDEVICE for a
 * device index that does not exist.  No device memory is taken until
 * rdos_finalize. */
rdos_status rdos_create(rdos_sim **out, int device, uint64_t seed, int32_t n_realizations);

/* Tetrahedral mesh (Sec. II.A: subvolumes with up to 4 face neighbours).
 *   xyz        [n_verts][3] vertex coordinates, metres
 *   tet_verts  [n_tets][4]  vertex ids; face f of a tet is the triangle
 *                           opposite its local vertex f
 * Faces on no other tet are reflecting boundaries.  RDOS_EINVAL for ids out
 * of range, a face shared by more than two tets (detected at finalize), or
 * a tet of zero volume (detected at finalize). */
rdos_status rdos_set_mesh(rdos_sim *s, int32_t n_verts, const double *xyz, int32_t n_tets,
                          const int32_t *tet_verts);

/* A surface instead of a volume (the transfer between surface triangles of
 * Sec. III.A, Fig. 5(c)-(d)): xyz[n_verts][3] (m), tri_verts[n_tris][3].
 * Triangles are the subvolumes: neighbours across edges (edge e opposite
 * local vertex e), r_e = L_e / (A delta_e), g = sum r_e, w_e = r_e / g, and
 * the unit of amount is N_A A with A in m^2, so reaction rates are SI per
 * area: mol/(m^2 s) (0th order), 1/s (1st), m^2/(mol s) (2nd).  Everything
 * else (species, reactions, counts, stepping, engine) is the same as for a
 * volume mesh.  RDOS_EINVAL for bad ids; finalize rejects degenerate
 * triangles and edges on three triangles.  Call instead of rdos_set_mesh. */
rdos_status rdos_set_surface_mesh(rdos_sim *s, int32_t n_verts, const double *xyz, int32_t n_tris,
                                  const int32_t *tri_verts);

/* A species with diffusion coefficient D >= 0 in m^2/s (0 = immobile).
 * Sec. II.A: in subvolume t the species' local diffusion rate is
 * d = D g_t (g_t from the mesh, see rdos_finalize); the period tau and the
 * transfer probability zeta = tau d follow from it, and Step 3 of
 * Algorithm 1 runs for every species with D > 0.  Writes the species id
 * (0, 1, ... in call order) to *out_id when non-NULL.  Between set_mesh and
 * finalize; RDOS_ESTATE otherwise, RDOS_EINVAL for D < 0, a non-finite D or
 * more than RDOS_MAX_SPECIES species. */
rdos_status rdos_add_species(rdos_sim *s, double D, int32_t *out_id);

/* A mass-action reaction with 0..2 reactants and 0..3 products (species
 * ids), rate constant k >= 0.  A reactant listed twice is a homodimer
 * reaction with k[A]^2 kinetics (propensity k N (N-1) / (N_A V)).
 * These are the reactions each subvolume's SSA fires during a period
 * (Algorithm 1, Step 2; Sec. II.C): propensity c h with h the reactant
 * count product and c = k N_A V (no reactant), k (one), k / (N_A V) (two),
 * V in litres.  reac[n_reac] and prod[n_prod] are read during the call only.
 * Writes the reaction id to *out_id when non-NULL.  Between set_mesh and
 * finalize; RDOS_EINVAL for ids out of range, k < 0 or non-finite, or more
 * than RDOS_MAX_REACTIONS reactions. */
rdos_status rdos_add_reaction(rdos_sim *s, int32_t n_reac, const int32_t *reac, int32_t n_prod,
                              const int32_t *prod, double k, int32_t *out_id);

/* Method options, before finalize (defaults: 1, 10, 0).
 *   occupancy_correction  1: n = binomial(Nbar, zeta) with Nbar the mean
 *                         population over the period (Sec. II.C, eqs. 2-3);
 *                         0: "first-order" splitting, n drawn from the count
 *                         at the end of the period (the comparison method of
 *                         Sec. III.B, Fig. 7)
 *   split_threshold       n below which the split moves molecules one by one
 *                         (Sec. II.B: 10 in the paper); >= 1.  The law does
 *                         not depend on it, the draws do.
 *   tau_outliers          k >= 0: tau from the (k+1)-th smallest 1/(D g)
 *                         instead of the smallest, so zeta is held at 1 in the
 *                         k fastest tet-species (outlier relaxation, Sec. II.A).
 * RDOS_EINVAL for split_threshold < 1 or tau_outliers < 0. */
rdos_status rdos_set_method(rdos_sim *s, int32_t occupancy_correction, int32_t split_threshold,
                            int32_t tau_outliers);

/* Transfer form (the alternative named at the end of Sec. II.B: the whole
 * population of the subvolume is split at once, each direction's weight
 * scaled down by zeta, which has the same law).  0 (default):
 * n = binomial(SR(Nbar), zeta), then the multinomial split of Step 3.3.  1: SR(Nbar) split at once over the faces
 * with weights zeta w_f and "stay" with 1 - zeta; if more than the molecules
 * present would leave, those present are split as in form 0.  Same law,
 * different draws.  Before finalize; RDOS_EINVAL for other values. */
rdos_status rdos_set_transfer_form(rdos_sim *s, int32_t form);

/* Restricts reaction `reaction` to the tets tets[0..n_tets) (a localized
 * reaction, e.g. the influx at both ends of the tube of Sec. III.B);
 * before finalize.  Without a call a reaction may fire in every tet. */
rdos_status rdos_set_reaction_region(rdos_sim *s, int32_t reaction, int32_t n_tets, const int32_t *tets);

/* Builds the mesh tables on the device and fixes the period
 *   tau = tau_scale * min over tets t and diffusing species m of 1/(D_m g_t)
 * (Algorithm 1, "precompute tau"; the local rate is d = D g with
 * g = sum_f A_f / (V delta_f), delta_f the distance between barycentres).
 * tau_scale in (0, 1] shortens tau below the paper's upper limit (Sec. II.A).
 * Writes tau to *out_tau when non-NULL. */
rdos_status rdos_finalize(rdos_sim *s, double tau_scale, double *out_tau);

/* Counts of one species in one realization, counts[n_tets] >= 0: the
 * population N of the species in every subvolume (Sec. II.C), the state
 * that Step 2 (SSA) and Step 3 (diffusion) of Algorithm 1 act on.  Sets the
 * state at the current period boundary; before finalize the counts are
 * staged on the host.  counts is copied during the call.  RDOS_EINVAL for a
 * negative count or ids out of range, RDOS_EOVERFLOW for more than 2^30
 * molecules of one species in one realization. */
rdos_status rdos_set_counts(rdos_sim *s, int32_t realization, int32_t species,
                            const int32_t *counts);

/* Reads the population N of one species in every subvolume (Sec. II.C)
 * into out[n_tets] at the current period boundary, i.e. after Step 4 of
 * the last period run (synchronises).  RDOS_ESTATE before finalize,
 * RDOS_EINVAL for ids out of range, RDOS_EOVERFLOW if any count overflowed
 * since the last check. */
rdos_status rdos_get_counts(rdos_sim *s, int32_t realization, int32_t species, int32_t *out);

/* Zero-copy view: *out is the device address of counts[n_tets] (int32) of
 * one species in one realization at the current period boundary.  The
 * library owns the memory; the address is valid until the next step,
 * run_until, set_state or destroy (the count buffers alternate between
 * periods).  Work is asynchronous: synchronise the simulation's stream before
 * reading it.  Writing non-negative counts through it sets the state like
 * set_counts. */
rdos_status rdos_device_counts(rdos_sim *s, int32_t realization, int32_t species, int32_t **out);

/* Time bookkeeping of Algorithm 1, Step 4 (t += tau after each period) and
 * resume support.  rdos_get_time writes the simulated time t and the index
 * of the next period to run; rdos_set_state sets both.  The period index
 * keys the random streams, so get_counts + get_time on one handle and
 * set_counts + set_state on a new one continue bit-identically.  t is the
 * simulated time of period step_index; full periods after it end at
 * t + i tau.  RDOS_EBUSY while an engine owns the simulation; set_state
 * needs a finalized simulation (RDOS_ESTATE) and step_index >= 0, finite t
 * (RDOS_EINVAL). */
rdos_status rdos_set_state(rdos_sim *s, int64_t step_index, double t);
rdos_status rdos_get_time(rdos_sim *s, double *t, int64_t *step_index);

/* n full periods of Algorithm 1 (asynchronous on the simulation's stream). */
rdos_status rdos_step(rdos_sim *s, int64_t n_steps);

/* Runs to t_end; the last period is shortened to end exactly at t_end
 * (Algorithm 1, Step 1).  Asynchronous. */
rdos_status rdos_run_until(rdos_sim *s, double t_end);

/* For callers that cannot allocate device memory around the step (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same periods as rdos_step, with the occupied-tet queue that the step
 * kernels share (entries, counts, segment lengths, work header) in a static
 * device array of 8 MiB per device, held until the process ends, instead of
 * the simulation's own queue.  Allocates nothing; the queue is cleared and
 * its header written by a kernel at the start of every call (no memset or
 * host copy).  Results are bit-identical to rdos_step.  The array holds
 * (1 + rows) x 4 B per tiled tet (tets rounded up to 1024 per realization,
 * rows = the simulation's species rounded up to 2, 3, 4, 6 or 8): about
 * 406,000 tiled tets with up to 4 species, 225,000 with 8.  Larger work
 * lists get RDOS_EINVAL with the sizes in the message.  Every call on one GPU uses
 * that GPU's array: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  Asynchronous. */
rdos_status rdos_step_static(rdos_sim *s, int64_t n_steps);

/* How rdos_step and rdos_run_until launch the periods (results never depend
 * on it).  0 (default): a work list of at most 8 tiles (1024 tets per
 * realization and tile) runs all its periods in one cooperative launch, the
 * scan and update phases of each period separated by grid-wide barriers;
 * larger ones launch a scan and an update kernel per period.  1: always two
 * launches per period.  2: always one cooperative launch.  3: one fused
 * launch per period (each wavefront scans its tiles and updates the tets it
 * queued, no queue in device memory; simulations of more than 8 species
 * launch two kernels instead).  The one-launch path exists for small meshes,
 * where the gaps between launches dominate a period (the 1 um cube of
 * Sec. II.A's Fig. 2 example: 750 tets).  RDOS_EINVAL for other values. */
rdos_status rdos_set_launch_mode(rdos_sim *s, int32_t mode);

/* Waits for all queued work; reports RDOS_EOVERFLOW if raised. */
rdos_status rdos_synchronize(rdos_sim *s);

/* Use a caller-owned HIP stream (e.g. a PyTorch stream) for all work of
 * this simulation; NULL returns to the library's own stream. */
rdos_status rdos_set_stream(rdos_sim *s, void *hip_stream);

/* The mesh tables built by finalize, for inspection:
 * nbr[n_tets][4] (-1 = boundary), w[n_tets][4] direction weights,
 * g[n_tets] (1/m^2), nav[n_tets] (N_A times volume in litres).
 * Any pointer may be NULL. */
rdos_status rdos_get_geometry(rdos_sim *s, int32_t *nbr, double *w, double *g, double *nav);

/* Sizes: tets, species, reactions, realizations; bytes of device memory the
 * simulation holds (or will hold once finalized). */
rdos_status rdos_get_info(rdos_sim *s, int32_t *n_tets, int32_t *n_species, int32_t *n_reactions,
                          int32_t *n_realizations, size_t *device_bytes);

const char *rdos_last_error(const rdos_sim *s);
void rdos_destroy(rdos_sim *s);

/* ------------------------------------------------------------------------ */
/* Batching and serving: many simulations advance together, one launch per   */
/* period for all of them (hipGraph-captured in chunks of periods).          */
/* ------------------------------------------------------------------------ */

/* An engine on `device` that admits simulations while their device memory
 * fits in hbm_budget_bytes (0 = 90% of the free device memory). */
rdos_status rdos_engine_create(rdos_engine **out, int device, size_t hbm_budget_bytes);

/* Queues n_steps full periods of `sim`.  The simulation may be finalized
 * already or not (then the engine finalizes it with tau_scale on admission,
 * uploading the counts staged by set_counts).  The engine owns the handle
 * until rdos_engine_release(); calls on it meanwhile return RDOS_EBUSY. */
rdos_status rdos_engine_submit(rdos_engine *e, rdos_sim *sim, int64_t n_steps, double tau_scale,
                               uint64_t *ticket);

/* Non-blocking: *done = 1 once the ticket's periods have all run;
 * *latency_s = seconds from submit to completion (valid when done). */
rdos_status rdos_engine_poll(rdos_engine *e, uint64_t ticket, int *done, double *latency_s);

/* Where a completed ticket's latency went (seconds): waiting for admission
 * (the HBM budget, earlier requests in the FIFO), set-up on admission
 * (finalize and the occupancy map), waiting to join the running work list
 * (the next chunk boundary), and running its periods.  The four add up to
 * the latency rdos_engine_poll reports.  RDOS_ESTATE for a ticket that has
 * not completed (or failed, or asked for no periods).  Any pointer may be
 * NULL. */
rdos_status rdos_engine_ticket_times(rdos_engine *e, uint64_t ticket, double *wait_s, double *setup_s,
                                     double *join_s, double *run_s);

/* Starts a set of requests together.  on = 1: the engine starts no new chunk
 * of periods (the running one finishes; admissions go on).  on = 0: waits
 * until every queued request that fits the HBM budget has been admitted,
 * then lets the engine run them all from the same chunk on.  Without it the
 * first request admitted starts at once, and those admitted after it join
 * at later chunks (continuous batching). */
rdos_status rdos_engine_hold(rdos_engine *e, int32_t on);

/* Blocks until every submitted ticket is done. */
rdos_status rdos_engine_drain(rdos_engine *e);

/* Returns a completed simulation to the caller (its device state is kept;
 * read it with rdos_get_counts, then rdos_destroy it). */
rdos_status rdos_engine_release(rdos_engine *e, uint64_t ticket, rdos_sim **sim);

/* Engine counters: periods launched, tet-species updates done, seconds the
 * device was busy. */
rdos_status rdos_engine_stats(rdos_engine *e, int64_t *launches, double *updates, double *busy_s);

/* Per-kernel timing.  on = 1 or 2: chunks are launched directly (not
 * replayed from the graph) with HIP events between every scan and update
 * launch; rdos_engine_kernel_times returns the summed milliseconds and launch
 * counts since profiling was last switched.  With on = 1 the update kernel
 * also tallies its work (rdos_engine_work_counts, cleared here); the tally
 * adds about 8% to the update's time, so on = 2 times the kernel as graph
 * replays run it and leaves the last tallies readable.  0 switches it off.
 * Results do not change.  RDOS_EINVAL for other values. */
rdos_status rdos_engine_set_profiling(rdos_engine *e, int on);
rdos_status rdos_engine_kernel_times(rdos_engine *e, double *scan_ms, int64_t *scan_launches,
                                     double *update_ms, int64_t *update_launches);

/* Work the timed update launches did since profiling was switched on, counted
 * on the device: `tets` tet-realization entries taken from the queue (Step 2
 * of Algorithm 1 then Step 3 for every species), `additions` molecule-count
 * additions into the next buffer (the synchronous application of all
 * transfers of Step 3, one per non-empty destination, the molecules that stay
 * included), `transfers` the additions across a face (Step 3.3's non-zero
 * n_i).  All are zero when profiling never ran.  Any pointer may be NULL. */
rdos_status rdos_engine_work_counts(rdos_engine *e, int64_t *tets, int64_t *additions, int64_t *transfers);

/* Where an engine's launch shape comes from. */
enum {
    RDOS_SHAPE_DEFAULT = 0,  /* the tuner has not finished on this work-list size: built-in
                                default, or the best candidate so far                    */
    RDOS_SHAPE_TUNED = 1,    /* tuned by this engine on live work of this size           */
    RDOS_SHAPE_CACHED = 2,   /* tuned earlier in this process (any engine) for this size */
    RDOS_SHAPE_FIXED = 3,    /* fixed by rdos_engine_set_shape                           */
    RDOS_SHAPE_SMALL_WORK = 4 /* work list of at most 1024 tiles: not tuned, 32-period
                                 chunks (launch latency dominates there)                 */
};

/* The launch shape of the current work list: periods per graph replay, scan
 * blocks, update blocks per queue segment (0: fused, see
 * rdos_engine_set_shape), 1 or 2 independent chains
 * (halves of the realizations on two streams, so one half's update overlaps
 * the other's scan), and where it comes from (RDOS_SHAPE_*).  The tuner
 * scores each candidate on full graph-replayed chunks of live work, per
 * work-list size bucket (power of two of the tile count, species bound).
 * Grids are clamped to the size bucket: never more scan wavefronts than
 * tiles nor update block columns than queue segments.  A run's last
 * periods, fewer than a chunk, are launched directly, as many as are left.
 * Results never depend on the shape.  Any pointer may be NULL. */
rdos_status rdos_engine_launch_shape(rdos_engine *e, int32_t *chunk, int32_t *scan_grid,
                                     int32_t *update_bps, int32_t *chains, int32_t *source);

/* What the tuner measured for the work list's current size bucket.  Per
 * work-list size bucket it runs each candidate shape for two chunks of
 * graph replays and scores the second (the first replays a freshly captured
 * graph), then scores each once more in a second pass, and keeps the lowest
 * mean time per period.  Writes the number of candidates to *n and, for the
 * first min(cap, *n) of them in the order tried: shapes[4 c .. 4 c + 3] =
 * chunk, scan_grid, update_bps, chains, and the device time per period (ms)
 * of the scored chunk of each pass to ms_first[c] and ms_second[c] (0 where
 * not measured: a bucket not tuned, taken from the cache, or still being
 * tuned).  Any pointer may be NULL.  RDOS_EINVAL for a NULL engine or cap < 0. */
rdos_status rdos_engine_tuner_scores(rdos_engine *e, int32_t cap, int32_t *n, int32_t *shapes, double *ms_first,
                                     double *ms_second);

/* Fixes the launch shape instead of tuning it: chunk (even, 2..1024)
 * periods per graph, scan_grid (1..2^20) blocks, update_bps (1..64) update
 * blocks per queue segment or 0 for one fused launch per period (scan_grid
 * blocks scan their tiles and update what they queued; work lists of more
 * than 8 species rows launch two kernels with one update block per segment
 * instead), chains 1 or 2.  chunk 0 returns to the tuner.
 * Results never depend on it; it exists for tests and for callers that
 * tune offline.  RDOS_EINVAL for values out of range. */
rdos_status rdos_engine_set_shape(rdos_engine *e, int32_t chunk, int32_t scan_grid, int32_t update_bps,
                                  int32_t chains);

/* Sec. II.B: the split switches from one categorical draw per molecule to
 * sequential binomials at a threshold (10 in the paper, measured on its
 * hardware).  This measures both methods on the device for n = 1..n_max
 * (2..256) molecules over a tet with four interior faces and writes the
 * switch point to *threshold: the smallest n from which the binomial chain
 * is never slower (n_max + 1 if it never wins).  The per-launch times (ms)
 * go to ms_one_by_one[n_max] and ms_sequential[n_max] when non-NULL.  Pass
 * the result to rdos_set_method; any threshold gives the same law. */
rdos_status rdos_tune_split_threshold(int device, int32_t n_max, int32_t *threshold, double *ms_one_by_one,
                                      double *ms_sequential);

/* Measures the device's streaming copy bandwidth (read + write bytes per
 * second / 1e9) with a 16-byte-per-lane copy kernel over `bytes`, `reps`
 * times.  The same kernel calibrates hardware byte counters. */
rdos_status rdos_bandwidth_probe(int device, size_t bytes, int reps, double *gbps);

/* Measures the device's rate of random integer atomics (additions per
 * second): 262,144 lanes each add 1 at ceil(n_atomics / 262,144) slots of an
 * int32 buffer of `bytes` (fewer than 2^32 slots) chosen by a counter-based
 * hash, with no result returned to the lane, `reps` timed launches after one
 * untimed.  The update step's count additions are such atomics, so this rate
 * bounds them as the copy kernel's bandwidth bounds a streaming kernel.
 * RDOS_EINVAL for bad sizes, RDOS_ENOMEM if the buffer cannot be allocated. */
rdos_status rdos_atomic_probe(int device, size_t bytes, int64_t n_atomics, int reps, double *per_s);

const char *rdos_engine_last_error(const rdos_engine *e);
void rdos_engine_destroy(rdos_engine *e);

#ifdef __cplusplus
}
#endif
#endif
