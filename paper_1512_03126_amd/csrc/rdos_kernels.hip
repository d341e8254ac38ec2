// gfx950 kernels of the operator-split reaction-diffusion step.
//
// Layout in HBM (one simulation, Rz realizations, S species, T tets, rows
// padded to Tp = T rounded up to a multiple of 4 so that a lane can read four
// consecutive tets with one 16-byte load):
//   buf[2][r][s][Tp]  int32  molecule counts, double-buffered: the state at the
//                            start of period k is buf[k & 1]; buf[(k + 1) & 1]
//                            is all zero then and receives, by integer
//                            atomics, every molecule that stays or arrives.
//                            Species rows are separate so that the atomics of
//                            one tet's species fall on different cache lines.
//   mask[2][r][s][Tp/4]  uint8  occupancy of the four-tet groups of buf[k & 1], per species:
//                            a byte marks period k when it holds occupancy_tag(k)
//   mesh[T]           64 B   neighbours, weights, g, N_A V (one line)
#include <hip/hip_runtime.h>

#include <cstdint>

#include <hipcub/hipcub.hpp>

#include "rdos_internal.h"
#include "rdos_sampling.h"

#pragma clang fp contract(off)

namespace rdos {

typedef int32_t v4i __attribute__((ext_vector_type(4)));

// A pointer into device (global) memory.  Accesses through generic pointers
// become flat instructions, which also count against the scalar-load wait
// counter, so a wait for a scalar load would wait for them too.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> global(T *p)
{
    return (gptr<T>)p;
}

// ---------------------------------------------------------------------------
// Set-up (Sec. II.A): volumes, face areas, barycentres, then per face
// r_f = A_f / (V delta_f), g = sum_f r_f, w_f = r_f / g.
// ---------------------------------------------------------------------------
struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 vsub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 vcross(V3 a, V3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double vdot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ double vnorm(V3 a) { return sqrt((a.x * a.x + a.y * a.y) + a.z * a.z); }

__global__ __launch_bounds__(256) void geometry_pass1(const double *__restrict__ xyz,
                                                      const int32_t *__restrict__ tet_verts, int32_t T,
                                                      double *__restrict__ vol, double *__restrict__ bc,
                                                      double *__restrict__ area, MeshRec *__restrict__ mesh,
                                                      int32_t *__restrict__ bad)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    V3 P[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t id = tet_verts[4 * (int64_t)t + v];
        P[v] = {xyz[3 * id], xyz[3 * id + 1], xyz[3 * id + 2]};
    }
    const double V = fabs(vdot(vcross(vsub(P[1], P[0]), vsub(P[2], P[0])), vsub(P[3], P[0]))) / 6.0;
    if (!(V > 0.0)) atomicOr(bad, 1);
    vol[t] = V;
    mesh[t].nav = kAvogadro * (V * 1000.0);
    bc[3 * (int64_t)t + 0] = ((P[0].x + P[1].x) + (P[2].x + P[3].x)) * 0.25;
    bc[3 * (int64_t)t + 1] = ((P[0].y + P[1].y) + (P[2].y + P[3].y)) * 0.25;
    bc[3 * (int64_t)t + 2] = ((P[0].z + P[1].z) + (P[2].z + P[3].z)) * 0.25;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        // the face opposite vertex f, its vertices in increasing local order
        const V3 a = P[f == 0 ? 1 : 0];
        const V3 b = P[f <= 1 ? 2 : 1];
        const V3 c = P[f <= 2 ? 3 : 2];
        area[4 * (int64_t)t + f] = 0.5 * vnorm(vcross(vsub(b, a), vsub(c, a)));
    }
}

__global__ __launch_bounds__(256) void geometry_pass2(const int32_t *__restrict__ nbr, int32_t T,
                                                      const double *__restrict__ vol,
                                                      const double *__restrict__ bc,
                                                      const double *__restrict__ area,
                                                      MeshRec *__restrict__ mesh)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const V3 me = {bc[3 * (int64_t)t], bc[3 * (int64_t)t + 1], bc[3 * (int64_t)t + 2]};
    const double V = vol[t];
    double r[4];
    int32_t nb[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        nb[f] = nbr[4 * (int64_t)t + f];
        if (nb[f] < 0) {
            r[f] = 0.0;
        } else {
            const int64_t u = nb[f];
            const V3 other = {bc[3 * u], bc[3 * u + 1], bc[3 * u + 2]};
            const double delta = vnorm(vsub(other, me));
            r[f] = area[4 * (int64_t)t + f] / (V * delta);
        }
    }
    const double g = ((r[0] + r[1]) + r[2]) + r[3];
    MeshRec &m = mesh[t];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        m.nbr[f] = nb[f];
        m.w[f] = g > 0.0 ? r[f] / g : 0.0;
    }
    m.g = g;
}

// Triangles (surface diffusion): area, barycentre and edge lengths, edge e
// opposite local vertex e; slot 3 is a boundary (length 0).  The unit of
// amount is N_A A (A in m^2).  Pass 2 is shared: r_e = L_e / (A d_e).
__global__ __launch_bounds__(256) void geometry_tri_pass1(const double *__restrict__ xyz,
                                                          const int32_t *__restrict__ tri_verts, int32_t T,
                                                          double *__restrict__ area, double *__restrict__ bc,
                                                          double *__restrict__ len, MeshRec *__restrict__ mesh,
                                                          int32_t *__restrict__ bad)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    V3 P[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const int64_t id = tri_verts[3 * (int64_t)t + v];
        P[v] = {xyz[3 * id], xyz[3 * id + 1], xyz[3 * id + 2]};
    }
    const double A = 0.5 * vnorm(vcross(vsub(P[1], P[0]), vsub(P[2], P[0])));
    if (!(A > 0.0)) atomicOr(bad, 1);
    area[t] = A;
    mesh[t].nav = kAvogadro * A;
    bc[3 * (int64_t)t + 0] = ((P[0].x + P[1].x) + P[2].x) / 3.0;
    bc[3 * (int64_t)t + 1] = ((P[0].y + P[1].y) + P[2].y) / 3.0;
    bc[3 * (int64_t)t + 2] = ((P[0].z + P[1].z) + P[2].z) / 3.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        // the edge opposite vertex e, its end points in increasing local order
        const V3 a = P[e == 0 ? 1 : 0];
        const V3 b = P[e <= 1 ? 2 : 1];
        len[4 * (int64_t)t + e] = vnorm(vsub(b, a));
    }
    len[4 * (int64_t)t + 3] = 0.0;
}

hipError_t launch_geometry_tri(const double *xyz, const int32_t *tri_verts, const int32_t *nbr, int32_t T,
                               double *scratch_area, double *scratch_bc, double *scratch_len, MeshRec *mesh,
                               int32_t *bad_area, hipStream_t st)
{
    const int grid = (T + 255) / 256;
    geometry_tri_pass1<<<grid, 256, 0, st>>>(xyz, tri_verts, T, scratch_area, scratch_bc, scratch_len, mesh,
                                             bad_area);
    geometry_pass2<<<grid, 256, 0, st>>>(nbr, T, scratch_area, scratch_bc, scratch_len, mesh);
    return hipGetLastError();
}

hipError_t launch_geometry(const double *xyz, const int32_t *tet_verts, const int32_t *nbr, int32_t T,
                           double *scratch_vol, double *scratch_bc, double *scratch_area, MeshRec *mesh,
                           int32_t *bad_volume, hipStream_t st)
{
    const int grid = (T + 255) / 256;
    geometry_pass1<<<grid, 256, 0, st>>>(xyz, tet_verts, T, scratch_vol, scratch_bc, scratch_area, mesh,
                                         bad_volume);
    geometry_pass2<<<grid, 256, 0, st>>>(nbr, T, scratch_vol, scratch_bc, scratch_area, mesh);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Face matching (the neighbours of Sec. II.A's subvolumes): each face of a
// cell becomes a key, its vertex ids sorted and packed (bits per id), with
// its slot 4 cell + face; after a radix sort the two cells of an interior
// face sit side by side.  Triangles (surfaces) match edges the same way.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void face_keys_kernel(const int32_t *__restrict__ cells, int32_t T,
                                                        int32_t cell_verts, int32_t bits,
                                                        unsigned long long *__restrict__ keys,
                                                        int32_t *__restrict__ slots)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)T * cell_verts) return;
    const int32_t t = (int32_t)(i / cell_verts), f = (int32_t)(i % cell_verts);
    uint32_t v[3];
    int k = 0;
    for (int j = 0; j < cell_verts; ++j)
        if (j != f) v[k++] = (uint32_t)cells[(int64_t)t * cell_verts + j];
    unsigned long long key;
    if (cell_verts == 4) {  // sort three ids
        uint32_t a = v[0], b = v[1], c = v[2], x;
        if (a > b) { x = a; a = b; b = x; }
        if (b > c) { x = b; b = c; c = x; }
        if (a > b) { x = a; a = b; b = x; }
        key = ((unsigned long long)a << (2 * bits)) | ((unsigned long long)b << bits) | (unsigned long long)c;
    } else {
        const uint32_t a = v[0] < v[1] ? v[0] : v[1], b = v[0] < v[1] ? v[1] : v[0];
        key = ((unsigned long long)a << bits) | (unsigned long long)b;
    }
    keys[i] = key;
    slots[i] = 4 * t + f;
}

// Thread i looks at the run of equal keys that starts at i: two slots are
// neighbours across that face; more than two, or one cell twice, raises
// *err (the caller then reports the first offending face in key order).
__global__ __launch_bounds__(256) void face_pair_kernel(const unsigned long long *__restrict__ keys,
                                                        const int32_t *__restrict__ slots, int64_t n,
                                                        int32_t *__restrict__ nbr, int32_t *__restrict__ err)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || (i > 0 && keys[i - 1] == keys[i])) return;
    if (i + 1 >= n || keys[i + 1] != keys[i]) return;  // a face on no other cell: boundary
    if (i + 2 < n && keys[i + 2] == keys[i]) {
        atomicOr(err, 1);
        return;
    }
    const int32_t s0 = slots[i], s1 = slots[i + 1];
    if (s0 / 4 == s1 / 4) {
        atomicOr(err, 2);
        return;
    }
    nbr[s0] = s1 / 4;
    nbr[s1] = s0 / 4;
}

static size_t face_sort_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const unsigned long long *)nullptr,
                                             (unsigned long long *)nullptr, (const int32_t *)nullptr,
                                             (int32_t *)nullptr, (int)n, 0, 64);
    return bytes;
}

size_t face_match_scratch_bytes(int32_t T, int32_t cell_verts)
{
    const int64_t n = (int64_t)T * cell_verts;
    return 2 * (size_t)n * (sizeof(unsigned long long) + sizeof(int32_t)) + 512 + face_sort_temp_bytes(n);
}

hipError_t launch_face_match(const int32_t *cells, int32_t T, int32_t cell_verts, int32_t bits, int32_t *nbr,
                             void *scratch, int32_t *err, hipStream_t st)
{
    const int64_t n = (int64_t)T * cell_verts;
    char *p = static_cast<char *>(scratch);
    unsigned long long *k0 = reinterpret_cast<unsigned long long *>(p);
    unsigned long long *k1 = k0 + n;
    int32_t *s0 = reinterpret_cast<int32_t *>(k1 + n);
    int32_t *s1 = s0 + n;
    void *temp = reinterpret_cast<char *>(s1 + n) + 256;
    size_t temp_bytes = face_sort_temp_bytes(n);
    const unsigned grid = (unsigned)((n + 255) / 256);
    face_keys_kernel<<<grid, 256, 0, st>>>(cells, T, cell_verts, bits, k0, s0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int end_bit = (cell_verts == 4 ? 3 : 2) * bits;
    e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, k0, k1, s0, s1, (int)n, 0, end_bit, st);
    if (e != hipSuccess) return e;
    face_pair_kernel<<<grid, 256, 0, st>>>(k1, s1, n, nbr, err);
    return hipGetLastError();
}

// tau upper limit: min over tets and diffusing species of 1/(D g).  Positive
// doubles order like their bit patterns, so an integer atomic min is exact.
__global__ __launch_bounds__(256) void tau_min_kernel(const MeshRec *__restrict__ mesh, int32_t T,
                                                      const double *__restrict__ D, int32_t S,
                                                      unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long best[256];
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long mine = ~0ull;
    if (t < T) {
        const double g = mesh[t].g;
        if (g > 0.0) {
            for (int s = 0; s < S; ++s) {
                if (!(D[s] > 0.0)) continue;
                const unsigned long long bits = (unsigned long long)__double_as_longlong(1.0 / (D[s] * g));
                mine = bits < mine ? bits : mine;
            }
        }
    }
    best[threadIdx.x] = mine;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off && best[threadIdx.x + off] < best[threadIdx.x])
            best[threadIdx.x] = best[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && best[0] != ~0ull) atomicMin(out, best[0]);
}

hipError_t launch_tau_min(const MeshRec *mesh, int32_t T, const double *D, int32_t S,
                          unsigned long long *out_bits, hipStream_t st)
{
    tau_min_kernel<<<(T + 255) / 256, 256, 0, st>>>(mesh, T, D, S, out_bits);
    return hipGetLastError();
}

// 1/(D_m g_t) for every (species, tet) as sortable bit patterns; pairs that
// set no rate (D = 0 or an isolated tet) become all-ones and sort last.
__global__ __launch_bounds__(256) void tau_values_kernel(const MeshRec *__restrict__ mesh, int32_t T,
                                                         const double *__restrict__ D, int32_t S,
                                                         unsigned long long *__restrict__ out,
                                                         unsigned long long *__restrict__ n_valid)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)T * S) return;
    const int32_t m = (int32_t)(i / T), t = (int32_t)(i % T);
    const double g = mesh[t].g;
    unsigned long long v = ~0ull;
    if (D[m] > 0.0 && g > 0.0) {
        v = (unsigned long long)__double_as_longlong(1.0 / (D[m] * g));
        atomicAdd(n_valid, 1ull);
    }
    out[i] = v;
}

__global__ void tau_pick_kernel(const unsigned long long *sorted, const unsigned long long *n_valid, int64_t k,
                                unsigned long long *out_bits)
{
    const unsigned long long n = *n_valid;
    if (n == 0) {
        *out_bits = ~0ull;
        return;
    }
    const unsigned long long idx = (unsigned long long)k < n ? (unsigned long long)k : n - 1;
    *out_bits = sorted[idx];
}

static size_t tau_sort_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, (const unsigned long long *)nullptr,
                                            (unsigned long long *)nullptr, (int)n, 0, 64);
    return bytes;
}

size_t tau_select_scratch_bytes(int32_t T, int32_t S)
{
    const int64_t n = (int64_t)T * S;
    return 2 * (size_t)n * sizeof(unsigned long long) + 256 + tau_sort_temp_bytes(n);
}

hipError_t launch_tau_select(const MeshRec *mesh, int32_t T, const double *D, int32_t S, int64_t k, void *scratch,
                             unsigned long long *out_bits, hipStream_t st)
{
    const int64_t n = (int64_t)T * S;
    char *p = static_cast<char *>(scratch);
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(p);
    unsigned long long *sorted = keys + n;
    unsigned long long *n_valid = sorted + n;
    void *temp = p + 2 * (size_t)n * sizeof(unsigned long long) + 256;
    size_t temp_bytes = tau_sort_temp_bytes(n);
    hipError_t e = hipMemsetAsync(n_valid, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    tau_values_kernel<<<(int)((n + 255) / 256), 256, 0, st>>>(mesh, T, D, S, keys, n_valid);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipcub::DeviceRadixSort::SortKeys(temp, temp_bytes, keys, sorted, (int)n, 0, 64, st);
    if (e != hipSuccess) return e;
    tau_pick_kernel<<<1, 1, 0, st>>>(sorted, n_valid, k, out_bits);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The period update of one tet (Algorithm 1, Steps 2-3).
// ---------------------------------------------------------------------------
// Per-lane working state lives in LDS slots with a stride of kBlock between
// species, so species can be indexed at run time without private memory.
// per-block tallies of the update kernel in the timing pass (its queue's `work` set):
// tets taken from the queue, count additions, and the additions that are
// transfers across a face
__shared__ uint32_t block_tets, block_adds, block_moves;

// One count for tally `which` (0 tets, 1 additions, 2 face transfers) of the
// timing pass, whose totals are work[0..2].  Instances of up to 6 species
// count per block in LDS; from 8 species on, where the per-lane state sets
// how many blocks fit a CU (the 8-species one fills a quarter of the LDS to
// the byte), they add per wavefront straight to the totals (a ballot over the
// lanes that count, one atomic by the first of them).
template <int KS>
constexpr bool block_tallies()
{
    return KS <= 6;
}
template <int KS>
__device__ __forceinline__ void tally_count(unsigned long long *work, int which)
{
    if constexpr (block_tallies<KS>()) {
        atomicAdd(which == 0 ? &block_tets : (which == 1 ? &block_adds : &block_moves), 1u);
    } else {
        const uint64_t m = __ballot(1);
        if (__lane_id() == (unsigned)__builtin_ctzll(m)) atomicAdd(&work[which], (unsigned long long)__popcll(m));
    }
}

struct LaneState {
    int32_t *N;     // counts during the period
    double *occ;    // occupancy integral since the start of the period
    double *last;   // time of the last change
    __device__ __forceinline__ int32_t &n(int s) const { return N[s * kBlock]; }
};

// propensity a_r = c_r h_r of reaction q with the tet's counts (mass action);
// zero where the reaction is not allowed in tet t (bit q of its `allowed`
// word).  The counts are tested first, and the tet's N_A V and allowed word
// are read from memory only when they matter: most tets hold no reactant
// pair, and then their update does not wait for those loads.
__device__ __forceinline__ double propensity(const DevSim &sm, int q, const LaneState &ls, const MeshRec *mr,
                                             int32_t t)
{
    const int order = sm.rn[q];
    double h;
    if (order == 0) {
        h = 1.0;
    } else {
        const int32_t na = ls.n(sm.r0[q]);
        if (order == 1) {
            h = (double)na;
        } else if (sm.r0[q] == sm.r1[q]) {
            h = (double)na * (double)(na - 1);
        } else {
            h = (double)na * (double)ls.n(sm.r1[q]);
        }
    }
    if (h == 0.0) return 0.0;  // c_r * 0 == 0 for every finite c_r
    if (sm.allowed && !((sm.allowed[t] >> q) & 1u)) return 0.0;
    if (order == 1) return sm.k[q] * h;
    const double nav = mr->nav;
    const double c = order == 0 ? sm.k[q] * nav : sm.k[q] / nav;
    return c * h;
}

// nxt and mnxt point at one realization's counts and occupancy rows; the
// offsets into them are 32-bit (finalize keeps S Tp below 2^29), which keeps
// the kernel within its register budget.
template <bool ANY_SCALED, int KS>
__device__ __forceinline__ void update_tet(const DevSim &sm, int32_t t, int64_t period, double tau_k,
                                           uint32_t key1, int32_t *__restrict__ nxt, int32_t Tp,
                                           uint8_t *__restrict__ mnxt, uint8_t mark, const LaneState &ls,
                                           unsigned long long *work)
{
    const bool tally = work != nullptr;
    const int S = sm.S;
    const int R = sm.R;
    const uint32_t period32 = (uint32_t)period;
    // a pointer, not a reference: a reference would tell the compiler the
    // record may be read anywhere, and the SSA's conditional read of N_A V
    // would then be made for every tet
    const MeshRec *mr = sm.mesh + t;

    // Step 2: Gillespie direct method over [0, tau_k); the first event at or
    // past tau_k is discarded.  Step 2.1: on each event the occupancy
    // integral of every reactant and product is brought up to the event time.
    // occ/last of species s are meaningful once bit s of `touched` is set;
    // before that they stand for 0 (no stores for tets without events).
    uint32_t touched = 0;
    if (R > 0) {
        Stream ssa(sm.key0, key1, kSsaStream, (uint32_t)t, period32);
        double now = 0.0;
        for (uint32_t events = 0;; ++events) {
            if (events >= kMaxEventsPerPeriod) {  // runaway rates: stop and report, never hang
                atomicOr(sm.flags, 2);
                break;
            }
            double a0 = 0.0;
            for (int q = 0; q < R; ++q) a0 = a0 + propensity(sm, q, ls, mr, t);
            if (!(a0 > 0.0)) break;
            const double dt = -log_basic(1.0 - ssa.uniform()) / a0;
            if (now + dt >= tau_k) break;
            now = now + dt;
            const double x = ssa.uniform() * a0;
            int chosen = -1;
            double cum = 0.0;
            for (int q = 0; q < R; ++q) {
                cum = cum + propensity(sm, q, ls, mr, t);
                if (x < cum) {
                    chosen = q;
                    break;
                }
            }
            if (chosen < 0) {  // x rounded up to a0: the last reaction able to fire
                for (int q = R - 1; q >= 0; --q)
                    if (propensity(sm, q, ls, mr, t) > 0.0) {
                        chosen = q;
                        break;
                    }
            }
            // the chosen reaction's fields, read with a wavefront-uniform index
            // (scalar loads) and selected per lane
            uint32_t inv = 0;
            int a = -1, b = -1, c0 = -1, c1 = -1, c2 = -1;
            for (int q = 0; q < R; ++q) {
                const int rn = sm.rn[q], pn = sm.pn[q];
                const bool is = q == chosen;
                inv = is ? sm.involved[q] : inv;
                a = is && rn > 0 ? sm.r0[q] : a;
                b = is && rn > 1 ? sm.r1[q] : b;
                c0 = is && pn > 0 ? sm.p0[q] : c0;
                c1 = is && pn > 1 ? sm.p1[q] : c1;
                c2 = is && pn > 2 ? sm.p2[q] : c2;
            }
            for (int s = 0; s < S; ++s) {
                if (!((inv >> s) & 1u)) continue;
                const bool seen = (touched >> s) & 1u;
                const double o = seen ? ls.occ[s * kBlock] : 0.0;
                const double l = seen ? ls.last[s * kBlock] : 0.0;
                int32_t &ns = ls.n(s);
                ls.occ[s * kBlock] = o + (double)ns * (now - l);
                ls.last[s * kBlock] = now;
                ns += (int)(s == c0) + (int)(s == c1) + (int)(s == c2) - (int)(s == a) - (int)(s == b);
                if (ns > 0x3fffffff) atomicOr(sm.flags, 1);
            }
            touched |= inv;
        }
    }

    // Step 3, per diffusing species: mean occupancy (eq. 2), stochastic
    // rounding to an integer population, n = binomial(Nbar, zeta) (eq. 3)
    // limited to the molecules present, then the multinomial split.
    // Each lane walks only the species its tet holds (lowest first), so the
    // wavefront runs as many rounds as its busiest lane has species, not S;
    // every species draws from its own stream, so the order is immaterial.
    int32_t nb[4];
    double w[4];
    bool have_faces = false;
    double g = 0.0;
    uint32_t present = 0;
    for (int s = 0; s < S; ++s)
        if (ls.n(s) > 0) present |= 1u << s;
    while (present) {
        const int s = __builtin_ctz(present);
        present &= present - 1u;
        const int32_t Ns = ls.n(s);
        if ((sm.diff_mask >> s) & 1u) {  // Ns == 0 never gets here: n = min(binomial(.), 0) = 0
            const bool hit = ((touched >> s) & 1u) && !sm.first_order;
            const double nbar = hit ? (ls.occ[s * kBlock] + (double)Ns * (tau_k - ls.last[s * kBlock])) / tau_k
                                    : (double)Ns;
            Stream rng(sm.key0, key1, (uint32_t)s, (uint32_t)t, period32);
            int32_t ni = (int32_t)floor(nbar);
            const double frac = nbar - (double)ni;
            if (frac > 0.0 && rng.uniform() < frac) ni += 1;
            if (!have_faces) {
                const int4 n4 = *reinterpret_cast<const int4 *>(mr->nbr);
                nb[0] = n4.x;
                nb[1] = n4.y;
                nb[2] = n4.z;
                nb[3] = n4.w;
#pragma unroll
                for (int f = 0; f < 4; ++f) w[f] = mr->w[f];
                g = mr->g;
                have_faces = true;
            }
            // D of species s, read with uniform indices (scalar loads) and
            // selected per lane, instead of one vector load per species
            double Ds = 0.0;
#pragma unroll
            for (int k = 0; k < KS; ++k)
                if (k < S) Ds = k == s ? sm.D[k] : Ds;
            double zeta = (tau_k * Ds) * g;
            if (zeta > 1.0) zeta = 1.0;
            // Step 3.2-3.3: n = min(binomial(SR(Nbar), zeta), N) split over the
            // faces; or (transfer form 1) SR(Nbar) split at once with weights
            // zeta w_f, and if more would leave than are present, those
            // present split as in Step 3.3.  The second form is compiled only
            // into the kernel instance launched when some simulation uses it,
            // so the first keeps its registers.
            int32_t out[4];
            int32_t n;
            if constexpr (ANY_SCALED) {
                bool scaled = sm.transfer_form == 1;
                int32_t pop = ni;
                if (!scaled) {
                    pop = binomial(ni, zeta, rng);
                    if (pop > Ns) pop = Ns;
                }
                for (;;) {
                    n = split_faces(pop, nb, w, scaled ? zeta : 1.0, scaled, sm.split_threshold, rng, out);
                    if (!(scaled && n > Ns)) break;
                    pop = Ns;
                    scaled = false;
                }
            } else {
                n = binomial(ni, zeta, rng);
                if (n > Ns) n = Ns;
                if (n > 0) split_over_faces(n, nb, w, sm.split_threshold, rng, out);
            }
            if (n > 0) {
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    if (out[f] > 0) {
                        atomicAdd(&nxt[(uint32_t)(s * Tp + nb[f])], (int32_t)out[f]);
                        mnxt[(uint32_t)(s * sm.mstride + (nb[f] >> 2))] = mark;
                        if (tally) {
                            tally_count<KS>(work, 1);
                            tally_count<KS>(work, 2);
                        }
                    }
                ls.n(s) = Ns - (int32_t)n;
            }
        }
        if (ls.n(s) > 0) {  // the molecules that stay
            atomicAdd(&nxt[(uint32_t)(s * Tp + t)], ls.n(s));
            mnxt[(uint32_t)(s * sm.mstride + (t >> 2))] = mark;
            if (tally) tally_count<KS>(work, 1);
        }
    }
}

// Each period is two launches.
//  scan:   one wavefront per tile of 1024 tets.  Each lane sweeps the
//          occupancy bytes of 16 tets (four groups of four) and compares
//          them with the period's tag; the tile's flagged groups are ranked over the wavefront and
//          listed in LDS, and the lanes then take the listed groups in turn:
//          a lane reads its group's flagged count vectors (16 bytes per
//          species), the group's tets that hold any molecule (all of them if
//          a reaction has no reactant) are ranked with ballots, staged in LDS
//          and written to the queue in tet order with coalesced stores after
//          an atomic reservation on the tile's segment (one per chunk of 64
//          groups), and the vectors read
//          are cleared, so the buffer is all zero by the time it is refilled.
//          The map is not cleared: a byte marks its group in the period
//          whose tag it holds.  A tile per wavefront keeps the chain of dependent loads
//          (tile, map, counts, reservation) short relative to the work it
//          covers.
//  update: each lane takes queued tets of its segment in turn (reading the
//          next entry one tet ahead), runs Steps 2-3 on them, adds what
//          stays and what leaves into the other buffer and sets the
//          occupancy bytes of the tets it added to.
// The queue has nseg segments of seg_cap entries (tiles ti with
// ti % nseg == k fill segment k, so seg_cap = tets of those tiles suffices);
// entry i of segment k is qtet[k * seg_cap + i] with counts
// qcnt[s * qcap + k * seg_cap + i].  Segment lengths live in
// len[(qsel * kMaxSegments + k) * kLenStride]; the update launch clears the
// other half for the next scan, so consecutive launches alternate qsel.
struct Queue {
    int32_t *tet;     // [qcap]
    int32_t *counts;  // [rows][qcap]
    int32_t *len;     // [2][kMaxSegments] * kLenStride
    const WorkHeader *hdr;
    unsigned long long *work;  // null, or [3] totals of the timing pass: tets updated, count additions, face transfers
    int32_t rows;     // count rows allocated: at least the species of every simulation served
};

// Raw buffer resource word 3 for gfx950 (untyped 32-bit data) and the cache
// policy of the scan's count loads: device scope (sc1) without the
// non-temporal hint, so that a line stays in L2 for the clear that follows
// (with the hint, more lines were filled twice).
constexpr int32_t kBufferWord3 = 0x00020000;
constexpr int32_t kScanLoadPolicy = 16;

constexpr int kScanWaves = kBlock / 64;
constexpr int kTileGroups = kTetsPerTile / 4;    // 256 four-tet groups per tile

// The map sweep of one tile by one wavefront: the tile's flagged four-tet
// groups, listed in glist (group | species mask << 8) in tet order.  Returns
// how many, uniform over the wavefront.
template <int MAXS>
__device__ __forceinline__ int32_t list_groups(const DevSim &sm, const Tile &tile, int64_t period,
                                               int32_t *__restrict__ glist)
{
    constexpr int kLaneTets = kTetsPerTile / 64;   // 16 consecutive tets per lane in the map sweep
    constexpr int kGroups = kLaneTets / 4;           // its four-tet groups
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int32_t off = lane * kLaneTets;
    const int32_t valid = tile.ntet - off;  // tets of this lane inside the tile (may be <= 0)
    const int64_t t0 = tile.tet0 + off;
    const int S = sm.S;
    // Per species, the four occupancy bytes of this lane's groups in one load
    // (rows are padded to 16 bytes, t0 / 4 is a multiple of 4), all species
    // together.  A byte flags its group when it holds this period's tag;
    // nothing is cleared.
    const gptr<const uint8_t> mrow =
        global((const uint8_t *)sm.mask[period & 1]) + (int64_t)tile.realization * S * sm.mstride + (t0 >> 2);
    const uint32_t tag = occupancy_tag(period);
    // this lane's flagged groups and the species flagged in each (all of
    // them in every group if a reaction has no reactants: every tet runs)
    uint32_t sp[kGroups];
#pragma unroll
    for (int k = 0; k < kGroups; ++k) sp[k] = 0u;
    if constexpr (MAXS > 10) {
        // one species row at a time (all rows at once take some 200 registers)
        for (int s = 0; s < S; ++s) {
            const uint32_t mb = valid > 0 ? *(gptr<const uint32_t>)(mrow + (int64_t)s * sm.mstride) : 0u;
#pragma unroll
            for (int k = 0; k < kGroups; ++k)
                if (((mb >> (8 * k)) & 0xFFu) == tag) sp[k] |= 1u << s;
        }
    } else {
        uint32_t mb[MAXS];
#pragma unroll
        for (int s = 0; s < MAXS; ++s) {
            mb[s] = 0u;
            if (s < S && valid > 0) mb[s] = *(gptr<const uint32_t>)(mrow + (int64_t)s * sm.mstride);
        }
#pragma unroll
        for (int k = 0; k < kGroups; ++k)
#pragma unroll
            for (int s = 0; s < MAXS; ++s)
                if (s < S && ((mb[s] >> (8 * k)) & 0xFFu) == tag) sp[k] |= 1u << s;
    }
    uint32_t fl = 0;
#pragma unroll
    for (int k = 0; k < kGroups; ++k) {
        if (sm.zeroth) sp[k] = (1u << S) - 1u;
        if (4 * k >= valid) sp[k] = 0u;
        if (sp[k] != 0u) fl |= 1u << k;
    }
    // rank the flagged groups over the wavefront (lane order, then group
    // order: tet order) and list them in LDS
    const uint32_t fc = (uint32_t)__popc(fl);
    int32_t fbefore = 0, F = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint64_t plane = __ballot((fc >> k) & 1u);
        fbefore += __popcll(plane & below) << k;
        F += __popcll(plane) << k;
    }
    if (F == 0) return 0;  // uniform over the wavefront
    {
        int32_t r = fbefore;
#pragma unroll
        for (int k = 0; k < kGroups; ++k)
            if (sp[k] != 0u) {
                glist[r] = (lane * kGroups + k) | (int32_t)(sp[k] << 8);
                ++r;
            }
    }
    // LDS operations of one wavefront complete in order; the fences keep
    // the compiler from moving LDS reads and writes across each other
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return F;
}

// One lane's group of a chunk of 64 listed groups: its flagged count
// vectors (16 bytes per species, the others zero), which of its tets hold
// molecules (all of them if a reaction has no reactant) and their rank over
// the wavefront (before: tets of lower lanes; total: the chunk's).
// The 16-species instance keeps no count vectors across the chunk (16 of
// them are 64 registers): it notes which were non-zero and reads them again,
// from L2, when it stages them.  The instances up to 10 species keep theirs
// (the 10-species scan holds 108 VGPRs, four wavefronts per SIMD, and beat
// the re-reading form on a ten-species mix, 1.40 against 1.45 ms per period).
template <int MAXS>
struct ChunkGroup {
    static constexpr bool kWide = MAXS > 10;
    v4i c[kWide ? 1 : MAXS];
    int32_t gid;
    uint32_t gsp;   // flagged species (their vectors were read)
    uint32_t nz;    // species whose vector was non-zero
    uint32_t bits;
    int32_t before, total;
};

__device__ __forceinline__ v4i load_counts(const __amdgpu_buffer_rsrc_t &rs, int64_t Tp, int32_t tg, int s)
{
    return __builtin_bit_cast(v4i,
                              __builtin_amdgcn_raw_buffer_load_b128(rs, (int32_t)((s * Tp + tg) * 4), 0, kScanLoadPolicy));
}

template <int MAXS>
__device__ __forceinline__ void read_chunk(const DevSim &sm, const Tile &tile, const __amdgpu_buffer_rsrc_t &rs,
                                           int64_t Tp, const int32_t *__restrict__ glist, int32_t c0, int32_t F,
                                           ChunkGroup<MAXS> &g)
{
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const bool act = c0 + lane < F;
    const int32_t gl = act ? glist[c0 + lane] : 0;
    g.gid = gl & 0xFF;
    const uint32_t gsp = act ? ((uint32_t)gl >> 8) : 0u;
    g.gsp = gsp;
    g.nz = 0u;
    const int32_t tg = tile.tet0 + 4 * g.gid;  // the group's first tet
    uint32_t bits = 0;
    int32_t sign = 0;  // a negative count was wrapped by an overflowing atomic add
    if constexpr (ChunkGroup<MAXS>::kWide) {
        // the flagged species one at a time
        for (uint32_t left = gsp; left; left &= left - 1u) {
            const int s = __builtin_ctz(left);
            const v4i c = load_counts(rs, Tp, tg, s);
            const uint32_t b = (uint32_t)(c.x != 0) | ((uint32_t)(c.y != 0) << 1) | ((uint32_t)(c.z != 0) << 2) |
                               ((uint32_t)(c.w != 0) << 3);
            bits |= b;
            if (b) g.nz |= 1u << s;
            sign |= c.x | c.y | c.z | c.w;
        }
    } else {
#pragma unroll
        for (int s = 0; s < MAXS; ++s) {
            g.c[s] = v4i{0, 0, 0, 0};
            if ((gsp >> s) & 1u) g.c[s] = load_counts(rs, Tp, tg, s);
            bits |= (uint32_t)(g.c[s].x != 0) | ((uint32_t)(g.c[s].y != 0) << 1) |
                    ((uint32_t)(g.c[s].z != 0) << 2) | ((uint32_t)(g.c[s].w != 0) << 3);
        }
#pragma unroll
        for (int s = 0; s < MAXS; ++s) sign |= g.c[s].x | g.c[s].y | g.c[s].z | g.c[s].w;
    }
    if (sm.zeroth && act) bits = 0xFu;  // a reaction without reactants: every tet runs
    const int32_t in_group = tile.ntet - 4 * g.gid;
    if (in_group < 4) bits &= in_group > 0 ? (1u << in_group) - 1u : 0u;
    if (sign < 0) atomicOr(sm.flags, 1);
    g.bits = bits;
    const uint32_t cnt = (uint32_t)__popc(bits);
    int32_t before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint64_t plane = __ballot((cnt >> k) & 1u);
        before += __popcll(plane & below) << k;
        total += __popcll(plane) << k;
    }
    g.before = before;
    g.total = total;
}

// The queued molecules now live in the queue: clear the vectors read so the
// buffer is all zero when it is next filled.
template <int MAXS>
__device__ __forceinline__ void clear_chunk(int32_t *cur, const Tile &tile, int64_t Tp, const ChunkGroup<MAXS> &g)
{
    const int32_t tg = tile.tet0 + 4 * g.gid;
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
        bool nz;
        if constexpr (ChunkGroup<MAXS>::kWide)
            nz = (g.nz >> s) & 1u;
        else
            nz = (g.c[s].x | g.c[s].y | g.c[s].z | g.c[s].w) != 0;
        if (nz) *(gptr<v4i>)(global(cur) + s * Tp + tg) = v4i{0, 0, 0, 0};
    }
}

// Rows of a wavefront's staging area: the tet row and the species rows of
// one pass.  Instances for more than 4 species stage four species at a time,
// so that their LDS (24 KB per block), and with it their occupancy, stays
// that of the 4-species one.
template <int MAXS>
constexpr int stage_rows()
{
    return MAXS > 4 ? 1 + 4 : 1 + MAXS;
}

// Writes the chunk's occupied tets to the queue from `base` on, in rank
// order: each row is staged in LDS at the tets' ranks, then stored with one
// coalesced store per row (tet: tile index * kTetsPerTile + offset; then the
// counts of species 0 .. S - 1).
template <int MAXS>
__device__ __forceinline__ void write_chunk(const __amdgpu_buffer_rsrc_t &rs, int64_t Tp, const Tile &tile, int32_t ti,
                                            int S, const ChunkGroup<MAXS> &g, const Queue &q, const WorkHeader &h,
                                            int64_t base, int32_t (*__restrict__ stage)[kTileGroups])
{
    const int lane = threadIdx.x & 63;
    const gptr<int32_t> qtet = global(q.tet);
    const gptr<int32_t> qcnt = global(q.counts);
    const int32_t total = g.total;
    if constexpr (ChunkGroup<MAXS>::kWide) {
        const int32_t tg = tile.tet0 + 4 * g.gid;
        int32_t k = g.before;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((g.bits >> b) & 1u) stage[0][k++] = 4 * g.gid + b;
        for (int s0 = 0; s0 < S; s0 += 4) {
            // four species rows, each vector read again (from L2)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (s0 + j >= S) break;
                const int s = s0 + j;
                const v4i c = ((g.gsp >> s) & 1u) ? load_counts(rs, Tp, tg, s) : v4i{0, 0, 0, 0};
                k = g.before;
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if ((g.bits >> b) & 1u) stage[1 + j][k++] = b == 0 ? c.x : b == 1 ? c.y : b == 2 ? c.z : c.w;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int32_t e = lane; e < total; e += 64) {
                if (s0 == 0) qtet[base + e] = ti * kTetsPerTile + stage[0][e];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (s0 + j < S) qcnt[(s0 + j) * h.qcap + base + e] = stage[1 + j][e];
            }
            // the rows are read before the next pass writes them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    } else if constexpr (MAXS > 4) {
        // species rows four at a time, from the vectors held in registers
#pragma unroll
        for (int s0 = 0; s0 < MAXS; s0 += 4) {
            if (s0 >= S) break;
            int32_t k = g.before;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (!((g.bits >> b) & 1u)) continue;
                if (s0 == 0) stage[0][k] = 4 * g.gid + b;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (s0 + j >= MAXS || s0 + j >= S) break;
                    const v4i &c = g.c[s0 + j];
                    stage[1 + j][k] = b == 0 ? c.x : b == 1 ? c.y : b == 2 ? c.z : c.w;
                }
                ++k;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int32_t e = lane; e < total; e += 64) {
                if (s0 == 0) qtet[base + e] = ti * kTetsPerTile + stage[0][e];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (s0 + j < MAXS && s0 + j < S) qcnt[(s0 + j) * h.qcap + base + e] = stage[1 + j][e];
            }
            // the rows are read before the next pass writes them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    } else {
        int32_t k = g.before;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (!((g.bits >> b) & 1u)) continue;
            stage[0][k] = 4 * g.gid + b;
#pragma unroll
            for (int s = 0; s < MAXS; ++s) {
                if (s >= S) break;
                stage[1 + s][k] = b == 0 ? g.c[s].x : b == 1 ? g.c[s].y : b == 2 ? g.c[s].z : g.c[s].w;
            }
            ++k;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int32_t e = lane; e < total; e += 64) {
            qtet[base + e] = ti * kTetsPerTile + stage[0][e];
#pragma unroll
            for (int s = 0; s < MAXS; ++s)
                if (s < S) qcnt[s * h.qcap + base + e] = stage[1 + s][e];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// One period's scan by one wavefront over the tiles wave0, wave0 + n_waves,
// ...  Per wavefront LDS: glist, the tile's flagged groups, and stage, the
// queue entries of one chunk of 64 groups (at most 256 tets) staged at their
// ranks.
template <int MAXS, bool OWNED>
__device__ __forceinline__ void scan_tiles(const DevSim *__restrict__ sims, const Tile *__restrict__ tiles,
                                           int64_t iter, const Queue &q, int32_t qsel, int32_t wave0,
                                           int32_t n_waves, int32_t *__restrict__ glist,
                                           int32_t (*__restrict__ stage)[kTileGroups])
{
    const int lane = threadIdx.x & 63;
    const WorkHeader h = *q.hdr;
    // With a segment per tile and a wavefront per tile, each wavefront owns
    // its tile's segment: it places its entries by its own count and stores
    // the length once, instead of reserving room with a returning atomic per
    // chunk (one round trip off a small work list's period).  Compiled only
    // into the instances launched for small work lists (OWNED): the branch
    // costs the large work lists' instance 7% of its time.
    const bool own = OWNED && h.nseg == h.n_tiles && n_waves >= h.n_tiles;
    // one wavefront per tile; the tile index is uniform over the wavefront
    for (int32_t ti = __builtin_amdgcn_readfirstlane(wave0); ti < h.n_tiles; ti += n_waves) {
        const Tile tile = tiles[h.tile0 + ti];
        const DevSim &sm = sims[tile.sim];
        const int64_t period = sm.step0 + iter;
        if (period >= sm.step_end) continue;  // uniform over the wavefront
        const int32_t F = list_groups<MAXS>(sm, tile, period, glist);
        if (F == 0) continue;  // uniform over the wavefront
        const int S = sm.S;
        const int64_t Tp = ((int64_t)sm.T + 3) & ~(int64_t)3;
        int32_t *cur = sm.buf[period & 1] + (int64_t)tile.realization * S * Tp;
        // the realization's counts as a buffer resource (bounds-checked by
        // the hardware: loads past the block return zero)
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(cur, (short)0, (int32_t)(S * Tp * 4), kBufferWord3);
        const int32_t seg = ti % h.nseg;
        int32_t filled = 0;  // entries written to an owned segment
        // Chunks of 64 flagged groups, one per lane: the lane reads the
        // group's flagged count vectors, its occupied tets are ranked over the
        // wavefront, staged at their ranks and written to the queue with one
        // coalesced store per row; the vectors read are then cleared.
        for (int32_t c0 = 0; c0 < F; c0 += 64) {
            ChunkGroup<MAXS> g;
            read_chunk<MAXS>(sm, tile, rs, Tp, glist, c0, F, g);
            const int32_t total = g.total;
            if (total == 0) continue;  // uniform; every vector read was zero
            int32_t slot = filled;
            if (!OWNED || !own) {
                if (lane == 0) slot = atomicAdd(&q.len[(qsel * kMaxSegments + seg) * kLenStride], total);
                slot = __shfl(slot, 0);
            }
            if (slot + total > h.seg_cap) {  // cannot happen when len starts at 0; never write past
                if (lane == 0) atomicOr(sm.flags, 4);
                continue;
            }
            if (OWNED) filled = slot + total;
            write_chunk<MAXS>(rs, Tp, tile, ti, S, g, q, h, (int64_t)seg * h.seg_cap + slot, stage);
            clear_chunk<MAXS>(cur, tile, Tp, g);
        }
        if (OWNED && own && filled > 0 && lane == 0) q.len[(qsel * kMaxSegments + seg) * kLenStride] = filled;
        // the next tile's list must not overtake this tile's reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// The instances for more than 8 species get a register budget of four
// wavefronts per SIMD; left free, the 16-species one spreads over 250.
template <int MAXS, bool OWNED>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MAXS > 8 ? 4 : 1))) void scan_kernel(
    const DevSim *__restrict__ sims,
                                                      const Tile *__restrict__ tiles, int64_t iter, Queue q,
                                                      int32_t qsel)
{
    __shared__ int32_t glist[kScanWaves][kTileGroups];
    __shared__ int32_t stage[kScanWaves][stage_rows<MAXS>()][kTileGroups];
    const int wv = threadIdx.x >> 6;
    scan_tiles<MAXS, OWNED>(sims, tiles, iter, q, qsel, (int32_t)blockIdx.x * kScanWaves + wv,
                     (int32_t)gridDim.x * kScanWaves, glist[wv], stage[wv]);
}

// The work header's fields, uniform over the grid: held in scalar registers.
__device__ __forceinline__ WorkHeader read_header(const WorkHeader *p)
{
    WorkHeader h = *p;
    h.n_tiles = __builtin_amdgcn_readfirstlane(h.n_tiles);
    h.nseg = __builtin_amdgcn_readfirstlane(h.nseg);
    h.seg_cap = __builtin_amdgcn_readfirstlane(h.seg_cap);
    h.tile0 = __builtin_amdgcn_readfirstlane(h.tile0);
    h.qcap = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)h.qcap)) |
                       ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)((uint64_t)h.qcap >> 32)) << 32));
    return h;
}

// Steps 2-3 for the queued tet `entry` (tile index * kTetsPerTile + offset)
// of `tile`, its counts already in the lane's state.  Lanes of one
// simulation run together with a wavefront-uniform descriptor (one round
// when the wavefront holds one simulation); descriptors do not change during
// a launch, so they are read as constant memory, which lets the uniform
// reads be scalar loads.
template <bool ANY_SCALED, int KS>
__device__ __forceinline__ void update_entry(const DevSim *__restrict__ sims, const Tile &tile, int32_t entry,
                                             int64_t iter, int64_t partial, double tau_last, const LaneState &ls,
                                             unsigned long long *work)
{
    using ConstSim = const __attribute__((address_space(4))) DevSim;
    for (uint64_t todo = __ballot(1); todo;) {
        const int32_t first = __builtin_amdgcn_readlane(tile.sim, (int32_t)__builtin_ctzll(todo));
        // branch on the lane's ballot bit, not on the equality, so that the
        // compiler cannot put the lane's own index in place of `first`
        const uint64_t same = __ballot(tile.sim == first);
        todo &= ~same;
        if (!((same >> __lane_id()) & 1ull)) continue;
        const DevSim &sm = *(const DevSim *)((ConstSim *)sims + first);
        const int64_t period = sm.step0 + iter;
        const double tau_k = period == partial ? tau_last : sm.tau;
        const int64_t Tp = ((int64_t)sm.T + 3) & ~(int64_t)3;
        const int64_t base = (int64_t)tile.realization * sm.S * Tp;
        update_tet<ANY_SCALED, KS>(sm, tile.tet0 + entry % kTetsPerTile, period, tau_k,
                                   sm.key1 ^ (uint32_t)tile.realization, sm.buf[(period + 1) & 1] + base,
                                   (int32_t)Tp, sm.mask[(period + 1) & 1] + (int64_t)tile.realization * sm.S * sm.mstride,
                                   occupancy_tag(period + 1), ls, work);
    }
}

// One block's share (part of per_seg) of queue segment seg in one period:
// Steps 2-3 of Algorithm 1 for each queued tet, with its additions into the
// next buffer.
template <bool ANY_SCALED, int KS>
__device__ __forceinline__ void update_segment(const DevSim *__restrict__ sims, const Tile *__restrict__ tiles,
                                               const Queue &q, int32_t qsel, int64_t iter, int64_t partial,
                                               double tau_last, const WorkHeader &h, int32_t seg, int32_t part,
                                               int32_t per_seg, const LaneState &ls, unsigned long long *work)
{
    const int32_t n = min(q.len[(qsel * kMaxSegments + seg) * kLenStride], h.seg_cap);
    const int32_t stride = per_seg * kBlock;
    const int64_t seg0 = (int64_t)seg * h.seg_cap;
    // each lane's next queue entry is read one tet ahead, so that it arrives
    // with the loads of the tet before it instead of starting a round trip
    int32_t next = part * kBlock + (int32_t)threadIdx.x < n ? q.tet[seg0 + part * kBlock + threadIdx.x] : 0;
    for (int32_t i = part * kBlock + threadIdx.x; i < n; i += stride) {
        if (work) tally_count<KS>(work, 0);
        const int64_t idx = seg0 + i;
        const int32_t entry = next;
        // the entry's count rows are read with its tile and the next entry,
        // not after the simulation is known.  Every load is issued (slots past
        // the queue's rows repeat its last row), so none waits behind a
        // branch; slots past a simulation's S hold values it never reads.
        int32_t cn[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) cn[s] = q.counts[min(s, q.rows - 1) * h.qcap + idx];
        const Tile tile = tiles[h.tile0 + entry / kTetsPerTile];
        next = i + stride < n ? q.tet[idx + stride] : 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) ls.n(s) = cn[s];
        update_entry<ANY_SCALED, KS>(sims, tile, entry, iter, partial, tau_last, ls, work);
    }
}

// Per-lane state for up to KS species in LDS (20 KS bytes per lane).  With
// the default transfer form the kernel fits 128 VGPRs without spilling; for
// KS <= 8 the LDS allows four blocks per CU too (the 8-species instance fills
// a quarter of it to the byte, so it keeps no tallies there), so it runs four
// wavefronts per SIMD.  The transfer-form-1 instances and the 10-species one
// keep the register budget of three (the 10-species one, 50 KB of LDS per
// block, fits three blocks per CU: the paper's 10-species models run it); the
// 16-species one (80 KB) fits two blocks per CU.
template <bool ANY_SCALED, int KS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(KS <= 8 && !ANY_SCALED ? 4 : (KS <= 10 ? 3 : 2)))) void
update_kernel(const DevSim *__restrict__ sims, const Tile *__restrict__ tiles, Queue q, int32_t qsel, int64_t iter,
              int64_t partial, double tau_last, int32_t grid_segments)
{
    __shared__ double occ[KS * kBlock];
    __shared__ double last[KS * kBlock];
    __shared__ int32_t counts[KS * kBlock];
    const LaneState ls{counts + threadIdx.x, occ + threadIdx.x, last + threadIdx.x};
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < kMaxSegments; k += kBlock) q.len[((qsel ^ 1) * kMaxSegments + k) * kLenStride] = 0;
    const WorkHeader h = read_header(q.hdr);
    // The grid is grid_segments x blocks-per-segment; the host sizes
    // grid_segments to cover every segment a launch may find in use.  A
    // header with more segments than that is an internal error, reported
    // through the flags of the work list's first simulation (never silent).
    if (h.nseg > grid_segments) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(sims[tiles[h.tile0].sim].flags, 4);
        return;
    }
    // uniform over the block: kept in scalar registers
    const int32_t seg = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x % (uint32_t)grid_segments));
    const int32_t per_seg = __builtin_amdgcn_readfirstlane(max(1, (int32_t)(gridDim.x / (uint32_t)grid_segments)));
    const int32_t part = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x / (uint32_t)grid_segments));
    if (seg >= h.nseg || part >= per_seg) return;  // uniform over the block
    const bool tally = block_tallies<KS>() && q.work != nullptr;  // per-block tallies (see tally_count)
    if constexpr (block_tallies<KS>()) {
        if (tally) {
            if (threadIdx.x == 0) block_tets = block_adds = block_moves = 0;
            __syncthreads();
        }
    }
    update_segment<ANY_SCALED, KS>(sims, tiles, q, qsel, iter, partial, tau_last, h, seg, part, per_seg, ls, q.work);
    if constexpr (block_tallies<KS>()) {
        if (tally) {
            __syncthreads();
            if (threadIdx.x == 0) {
                atomicAdd(&q.work[0], (unsigned long long)block_tets);
                atomicAdd(&q.work[1], (unsigned long long)block_adds);
                atomicAdd(&q.work[2], (unsigned long long)block_moves);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Fused period: the scan and the update in one launch.  Within a period no
// tile's update touches what another tile's scan reads or writes (the scan
// reads and clears counts of buffer k and reads map k; updates add into
// buffer k + 1 and mark map k + 1), so each wavefront scans its tiles into a
// queue of its own in LDS, a ring, and updates the queued tets 64 at a time
// as they accumulate.  Only consecutive periods need the launch boundary
// between them.  No queue in device memory, one launch per period.
// ---------------------------------------------------------------------------
constexpr int kRing = 320;  // ring entries per wavefront: fewer than 64 waiting + one chunk's at most 256

// Steps 2-3 for the n (1..64) queued tets from ring position head on, one
// per lane.
template <bool ANY_SCALED, int KS>
__device__ __forceinline__ void ring_round(const DevSim *__restrict__ sims, const Tile *__restrict__ tiles,
                                           int32_t tile0, int64_t iter, int64_t partial, double tau_last,
                                           int32_t (*__restrict__ ring)[kRing], int32_t head, int32_t n,
                                           const LaneState &ls, unsigned long long *work)
{
    const int lane = threadIdx.x & 63;
    if (lane >= n) return;
    int32_t pos = head + lane;
    if (pos >= kRing) pos -= kRing;
    const int32_t entry = ring[0][pos];
    // rows past a simulation's S hold values it never reads
#pragma unroll
    for (int s = 0; s < KS; ++s) ls.n(s) = ring[1 + s][pos];
    const Tile tile = tiles[tile0 + entry / kTetsPerTile];
    if (work) tally_count<KS>(work, 0);
    update_entry<ANY_SCALED, KS>(sims, tile, entry, iter, partial, tau_last, ls, work);
}

// One period of the tiles wave0, wave0 + n_waves, ... by one wavefront.  LDS
// per wavefront: glist (the tile's flagged groups) and the ring, rows
// [0] entry (tile index * kTetsPerTile + offset) and [1 + s] its count of
// species s.
template <bool ANY_SCALED, int KS>
__device__ __forceinline__ void fused_tiles(const DevSim *__restrict__ sims, const Tile *__restrict__ tiles,
                                            const WorkHeader &h, int64_t iter, int64_t partial, double tau_last,
                                            int32_t wave0, int32_t n_waves, int32_t *__restrict__ glist,
                                            int32_t (*__restrict__ ring)[kRing], const LaneState &ls,
                                            unsigned long long *work)
{
    static_assert(KS <= kFusedSpecies, "the fused path keeps every count vector of a chunk in registers");
    int32_t head = 0, pending = 0;  // uniform over the wavefront
    for (int32_t ti = __builtin_amdgcn_readfirstlane(wave0); ti < h.n_tiles; ti += n_waves) {
        const Tile tile = tiles[h.tile0 + ti];
        const DevSim &sm = sims[tile.sim];
        const int64_t period = sm.step0 + iter;
        if (period >= sm.step_end) continue;  // uniform over the wavefront
        const int32_t F = list_groups<KS>(sm, tile, period, glist);
        if (F == 0) continue;  // uniform over the wavefront
        const int S = sm.S;
        const int64_t Tp = ((int64_t)sm.T + 3) & ~(int64_t)3;
        int32_t *cur = sm.buf[period & 1] + (int64_t)tile.realization * S * Tp;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(cur, (short)0, (int32_t)(S * Tp * 4), kBufferWord3);
        for (int32_t c0 = 0; c0 < F; c0 += 64) {
            ChunkGroup<KS> g;
            read_chunk<KS>(sm, tile, rs, Tp, glist, c0, F, g);
            if (g.total == 0) continue;  // uniform; every vector read was zero
            // append the chunk's occupied tets at the ring's tail, in rank order
            int32_t k = pending + g.before;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (!((g.bits >> b) & 1u)) continue;
                int32_t pos = head + k;
                if (pos >= kRing) pos -= kRing;
                ring[0][pos] = ti * kTetsPerTile + 4 * g.gid + b;
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    if (s >= S) break;
                    ring[1 + s][pos] = b == 0 ? g.c[s].x : b == 1 ? g.c[s].y : b == 2 ? g.c[s].z : g.c[s].w;
                }
                ++k;
            }
            pending += g.total;
            clear_chunk<KS>(cur, tile, Tp, g);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // whole rounds of 64 as soon as they are there
            while (pending >= 64) {
                ring_round<ANY_SCALED, KS>(sims, tiles, h.tile0, iter, partial, tau_last, ring, head, 64, ls, work);
                head += 64;
                if (head >= kRing) head -= kRing;
                pending -= 64;
                // the round's ring reads before the next chunk's writes
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        // the next tile's list must not overtake this tile's reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (pending > 0)
        ring_round<ANY_SCALED, KS>(sims, tiles, h.tile0, iter, partial, tau_last, ring, head, pending, ls, work);
}

template <bool ANY_SCALED, int KS>
__global__ __launch_bounds__(kBlock) void fused_kernel(const DevSim *__restrict__ sims,
                                                       const Tile *__restrict__ tiles, const WorkHeader *hdr,
                                                       int64_t iter, int64_t partial, double tau_last,
                                                       unsigned long long *work)
{
    __shared__ int32_t glist[kScanWaves][kTileGroups];
    __shared__ int32_t ring[kScanWaves][1 + KS][kRing];
    __shared__ double occ[KS * kBlock];
    __shared__ double last[KS * kBlock];
    __shared__ int32_t counts[KS * kBlock];
    const LaneState ls{counts + threadIdx.x, occ + threadIdx.x, last + threadIdx.x};
    const int wv = threadIdx.x >> 6;
    const WorkHeader h = read_header(hdr);
    const bool tally = block_tallies<KS>() && work != nullptr;  // per-block tallies (see tally_count)
    if constexpr (block_tallies<KS>()) {
        if (tally) {
            if (threadIdx.x == 0) block_tets = block_adds = block_moves = 0;
            __syncthreads();
        }
    }
    fused_tiles<ANY_SCALED, KS>(sims, tiles, h, iter, partial, tau_last, (int32_t)blockIdx.x * kScanWaves + wv,
                                (int32_t)gridDim.x * kScanWaves, glist[wv], ring[wv], ls, work);
    if constexpr (block_tallies<KS>()) {
        if (tally) {
            __syncthreads();
            if (threadIdx.x == 0) {
                atomicAdd(&work[0], (unsigned long long)block_tets);
                atomicAdd(&work[1], (unsigned long long)block_adds);
                atomicAdd(&work[2], (unsigned long long)block_moves);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Small work lists: all periods of a run in one cooperative launch.  Each
// period is the scan phase, a grid-wide barrier, the update phase and another
// barrier, in place of two kernel launches whose gaps dominate when a period
// holds little work (the 750-tet cube, served requests of a few hundred
// tiles).
// ---------------------------------------------------------------------------
constexpr uint32_t kBarrierSpins = 1u << 22;  // about half a second of waiting per barrier

// Grid-wide barrier of a cooperative launch (every block resident).  Block
// b arrives on counter b % 64 (one per 128-byte line, so that the arrivals,
// memory-side atomics, do not queue on one address) and the first
// wavefront waits until the 64 counters sum to the arrivals of this epoch,
// one counter per lane.  The agent-scope fences put each block's writes
// (stores and atomics) before its arrival and the reads after the wait
// behind every block's writes, as the boundary between two launches does.
// A wait past its bound raises `fail` and stops waiting, and every later
// barrier passes at once: a failure ends the kernel (with the simulations'
// flags raised) instead of hanging it.
constexpr int kBarrierLines = 64;
constexpr int kBarrierStride = 32;  // uint32 per 128-byte line
__device__ __forceinline__ void grid_barrier(uint32_t *bar, uint32_t nblocks, uint32_t &epoch, uint32_t *fail)
{
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t lane = threadIdx.x;
        if (lane == 0) {
            __threadfence();
            atomicAdd(&bar[(blockIdx.x % kBarrierLines) * kBarrierStride], 1u);
        }
        const uint64_t target = (uint64_t)(epoch + 1) * nblocks;
        uint32_t spins = 0;
        for (;;) {
            uint64_t sum = __hip_atomic_load(&bar[lane * kBarrierStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
            if (sum >= target) break;
            if (__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
            if (++spins > kBarrierSpins) {
                if (lane == 0) atomicOr(fail, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (lane == 0) __threadfence();
    }
    ++epoch;
    __syncthreads();
}

// n_periods periods of every tile: period i uses queue half (phase + i) & 1
// and the iteration index iter0 + i (period = step0 + iteration, the period
// equal to `partial` lasting tau_last).  Block b scans the tiles of its
// wavefronts (grid-stride) and updates the queue segments b, b + grid, ...
// sync holds the barrier counters (kBarrierLines lines, zero at launch) and,
// after them, the failure word.  Each queue segment is shared by
// max(1, grid / segments) blocks.
template <bool ANY_SCALED, int KS>
__global__ __launch_bounds__(kBlock) void persist_kernel(const DevSim *__restrict__ sims, const Tile *__restrict__ tiles,
                                                         Queue q, int32_t phase, int64_t iter0, int32_t n_periods,
                                                         int64_t partial, double tau_last, uint32_t *sync)
{
    __shared__ int32_t glist[kScanWaves][kTileGroups];
    __shared__ int32_t stage[kScanWaves][stage_rows<KS>()][kTileGroups];
    __shared__ double occ[KS * kBlock];
    __shared__ double last[KS * kBlock];
    __shared__ int32_t counts[KS * kBlock];
    const LaneState ls{counts + threadIdx.x, occ + threadIdx.x, last + threadIdx.x};
    const int wv = threadIdx.x >> 6;
    const uint32_t G = gridDim.x;
    uint32_t epoch = 0;
    const WorkHeader h = read_header(q.hdr);
    uint32_t *fail = sync + kBarrierLines * kBarrierStride;
    const int32_t per_seg = h.nseg > 0 ? max(1, (int32_t)G / h.nseg) : 1;
    for (int32_t p = 0; p < n_periods; ++p) {
        const int64_t iter = iter0 + p;
        const int32_t qsel = (phase + p) & 1;
        scan_tiles<KS, true>(sims, tiles, iter, q, qsel, (int32_t)blockIdx.x * kScanWaves + wv, (int32_t)G * kScanWaves,
                       glist[wv], stage[wv]);
        grid_barrier(sync, G, epoch, fail);
        if (blockIdx.x == 0)  // the other half serves the next period's scan
            for (int k = threadIdx.x; k < kMaxSegments; k += kBlock)
                q.len[((qsel ^ 1) * kMaxSegments + k) * kLenStride] = 0;
        if (per_seg > 1) {
            if ((int32_t)blockIdx.x < h.nseg * per_seg)
                update_segment<ANY_SCALED, KS>(sims, tiles, q, qsel, iter, partial, tau_last, h,
                                               (int32_t)blockIdx.x % h.nseg, (int32_t)blockIdx.x / h.nseg, per_seg,
                                               ls, nullptr);
        } else {
            for (int32_t seg = __builtin_amdgcn_readfirstlane((int32_t)blockIdx.x); seg < h.nseg; seg += (int32_t)G)
                update_segment<ANY_SCALED, KS>(sims, tiles, q, qsel, iter, partial, tau_last, h, seg, 0, 1, ls,
                                               nullptr);
        }
        grid_barrier(sync, G, epoch, fail);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
        for (int32_t i = 0; i < h.n_sims; ++i) atomicOr(sims[i].flags, 8);
}

__global__ void sync_reset_kernel(uint32_t *sync)
{
    for (int i = threadIdx.x; i < kPersistSyncWords; i += blockDim.x) sync[i] = 0u;
}

namespace {
template <bool ANY_SCALED, int KS>
const void *persist_entry()
{
    return reinterpret_cast<const void *>(&persist_kernel<ANY_SCALED, KS>);
}
const void *persist_pick(int32_t species, int32_t scaled)
{
    if (species <= 4) return scaled ? persist_entry<true, 4>() : persist_entry<false, 4>();
    if (species <= 6) return scaled ? persist_entry<true, 6>() : persist_entry<false, 6>();
    if (species <= 8) return scaled ? persist_entry<true, 8>() : persist_entry<false, 8>();
    return scaled ? persist_entry<true, kMaxSpecies>() : persist_entry<false, kMaxSpecies>();
}
}  // namespace

int32_t persist_grid_limit(const QueueView &qv)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_pick(qv.species, qv.scaled), kBlock, 0) !=
        hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_persist(const DevSim *sims, const Tile *tiles, int64_t iter0, int32_t n_periods, int32_t phase,
                          int64_t partial, double tau_last, const QueueView &qv, int32_t grid, uint32_t *sync,
                          hipStream_t st)
{
    if (n_periods <= 0) return hipSuccess;
    if (grid < 1 || !sync) return hipErrorInvalidValue;
    sync_reset_kernel<<<1, 256, 0, st>>>(sync);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    Queue q{qv.tet, qv.counts, qv.len, qv.hdr, nullptr, qv.species};
    void *args[] = {(void *)&sims, (void *)&tiles, (void *)&q, (void *)&phase, (void *)&iter0, (void *)&n_periods,
                    (void *)&partial, (void *)&tau_last, (void *)&sync};
    return hipLaunchCooperativeKernel(persist_pick(qv.species, qv.scaled), dim3(grid), dim3(kBlock), args, 0, st);
}

// Tile i belongs to the last unit whose first tile is at or before i.
__global__ __launch_bounds__(256) void expand_tiles_kernel(const WorkUnit *__restrict__ units, int32_t n_units,
                                                           int32_t n_tiles, Tile *__restrict__ tiles)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_tiles) return;
    int32_t lo = 0, hi = n_units - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (units[mid].first <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    const WorkUnit u = units[lo];
    const int32_t t0 = (i - u.first) * kTetsPerTile;
    tiles[i] = Tile{u.sim, u.realization, t0, min(kTetsPerTile, u.T - t0)};
}

hipError_t launch_expand_tiles(const WorkUnit *units, int32_t n_units, int32_t n_tiles, Tile *tiles, hipStream_t st)
{
    if (n_tiles <= 0) return hipSuccess;
    if (n_units <= 0) return hipErrorInvalidValue;
    expand_tiles_kernel<<<(n_tiles + 255) / 256, 256, 0, st>>>(units, n_units, n_tiles, tiles);
    return hipGetLastError();
}

template <bool OWNED>
static void scan_for_species(const DevSim *sims, const Tile *tiles, int64_t iter, const Queue &q, int32_t qsel,
                             int32_t species, int32_t scan_grid, hipStream_t st)
{
    // register arrays sized for the largest species count the queue holds
    if (species <= 2)
        scan_kernel<2, OWNED><<<scan_grid, kBlock, 0, st>>>(sims, tiles, iter, q, qsel);
    else if (species == 3)
        scan_kernel<3, OWNED><<<scan_grid, kBlock, 0, st>>>(sims, tiles, iter, q, qsel);
    else if (species <= 4)
        scan_kernel<4, OWNED><<<scan_grid, kBlock, 0, st>>>(sims, tiles, iter, q, qsel);
    else if (species <= 6)
        scan_kernel<6, OWNED><<<scan_grid, kBlock, 0, st>>>(sims, tiles, iter, q, qsel);
    else if (species <= 8)
        scan_kernel<8, OWNED><<<scan_grid, kBlock, 0, st>>>(sims, tiles, iter, q, qsel);
    else if (species <= 10)
        scan_kernel<10, OWNED><<<scan_grid, kBlock, 0, st>>>(sims, tiles, iter, q, qsel);
    else
        scan_kernel<kMaxSpecies, OWNED><<<scan_grid, kBlock, 0, st>>>(sims, tiles, iter, q, qsel);
}

hipError_t launch_scan(const DevSim *sims, const Tile *tiles, int64_t iter, const QueueView &qv, int32_t qsel,
                       int32_t scan_grid, hipStream_t st)
{
    if (scan_grid <= 0) return hipErrorInvalidValue;
    const Queue q{qv.tet, qv.counts, qv.len, qv.hdr, qv.work, qv.species};
    if (qv.owned)
        scan_for_species<true>(sims, tiles, iter, q, qsel, qv.species, scan_grid, st);
    else
        scan_for_species<false>(sims, tiles, iter, q, qsel, qv.species, scan_grid, st);
    return hipGetLastError();
}

hipError_t launch_update(const DevSim *sims, const Tile *tiles, int64_t iter, int64_t partial, double tau_last,
                         const QueueView &qv, int32_t qsel, int32_t blocks_per_segment, int32_t grid_segments,
                         hipStream_t st)
{
    if (grid_segments < 1 || grid_segments > kMaxSegments) return hipErrorInvalidValue;
    const Queue q{qv.tet, qv.counts, qv.len, qv.hdr, qv.work, qv.species};
    const int32_t bps = blocks_per_segment > 0 ? blocks_per_segment : 1;
    const dim3 grid(grid_segments * bps);
    // the queue's species rows bound the species of every simulation it serves
    if (qv.species <= 4) {
        if (qv.scaled)
            update_kernel<true, 4><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                grid_segments);
        else
            update_kernel<false, 4><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                grid_segments);
    } else if (qv.species <= 6) {
        if (qv.scaled)
            update_kernel<true, 6><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                grid_segments);
        else
            update_kernel<false, 6><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                grid_segments);
    } else if (qv.species <= 8) {
        if (qv.scaled)
            update_kernel<true, 8><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                grid_segments);
        else
            update_kernel<false, 8><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                grid_segments);
    } else if (qv.species <= 10) {
        if (qv.scaled)
            update_kernel<true, 10><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                 grid_segments);
        else
            update_kernel<false, 10><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                  grid_segments);
    } else {
        if (qv.scaled)
            update_kernel<true, kMaxSpecies><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                grid_segments);
        else
            update_kernel<false, kMaxSpecies><<<grid, kBlock, 0, st>>>(sims, tiles, q, qsel, iter, partial, tau_last,
                                                                grid_segments);
    }
    return hipGetLastError();
}

hipError_t launch_fused(const DevSim *sims, const Tile *tiles, int64_t iter, int64_t partial, double tau_last,
                        const QueueView &qv, int32_t grid, hipStream_t st)
{
    if (grid <= 0) return hipErrorInvalidValue;
    unsigned long long *work = qv.work;
    if (qv.species <= 4) {
        if (qv.scaled)
            fused_kernel<true, 4><<<grid, kBlock, 0, st>>>(sims, tiles, qv.hdr, iter, partial, tau_last, work);
        else
            fused_kernel<false, 4><<<grid, kBlock, 0, st>>>(sims, tiles, qv.hdr, iter, partial, tau_last, work);
    } else if (qv.species <= 6) {
        if (qv.scaled)
            fused_kernel<true, 6><<<grid, kBlock, 0, st>>>(sims, tiles, qv.hdr, iter, partial, tau_last, work);
        else
            fused_kernel<false, 6><<<grid, kBlock, 0, st>>>(sims, tiles, qv.hdr, iter, partial, tau_last, work);
    } else if (qv.species <= 8) {
        if (qv.scaled)
            fused_kernel<true, 8><<<grid, kBlock, 0, st>>>(sims, tiles, qv.hdr, iter, partial, tau_last, work);
        else
            fused_kernel<false, 8><<<grid, kBlock, 0, st>>>(sims, tiles, qv.hdr, iter, partial, tau_last, work);
    } else {
        return hipErrorInvalidValue;  // the rings and lane state of 16 species exceed the LDS
    }
    return hipGetLastError();
}

hipError_t launch_step(const DevSim *sims, const Tile *tiles, int64_t iter, int64_t partial, double tau_last,
                       const QueueView &qv, int32_t qsel, int32_t scan_grid, int32_t blocks_per_segment,
                       int32_t grid_segments, hipStream_t st)
{
    hipError_t e = launch_scan(sims, tiles, iter, qv, qsel, scan_grid, st);
    if (e != hipSuccess) return e;
    return launch_update(sims, tiles, iter, partial, tau_last, qv, qsel, blocks_per_segment, grid_segments, st);
}

// Streaming copy used to measure the device's achievable HBM bandwidth (and
// to calibrate byte counters): four independent 16-byte loads per lane in
// flight, then four stores, grid-stride.
__global__ __launch_bounds__(256) void bandwidth_copy_kernel(const int4 *__restrict__ src, int4 *__restrict__ dst,
                                                            int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const int4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st)
{
    const int64_t n = (int64_t)(bytes / sizeof(int4));
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 1023) / 1024;
    if (blocks > 16384) blocks = 16384;
    bandwidth_copy_kernel<<<(int)blocks, 256, 0, st>>>((const int4 *)src, (int4 *)dst, n);
    return hipGetLastError();
}

// Cost of splitting n molecules by each method of Sec. II.B (one categorical
// draw per molecule, or sequential binomials), for the tuner of the switch
// point: every lane splits n molecules `reps` times over a tet with four
// interior faces, each time from its own counter; the sink keeps the work.
template <bool ONE_BY_ONE>
__global__ __launch_bounds__(256) void split_cost_kernel(int64_t n, int32_t reps, int64_t *__restrict__ sink)
{
    const int32_t nbr[4] = {1, 2, 3, 4};
    const double w[4] = {0.3, 0.2, 0.2, 0.3};
    const uint32_t lane = blockIdx.x * blockDim.x + threadIdx.x;
    int64_t acc = 0;
    for (int32_t r = 0; r < reps; ++r) {
        Stream rng(0x2545F491u, 0x9E3779B9u, 0x80000001u, lane, (uint32_t)r);
        int32_t out[4];
        split_over_faces((int32_t)n, nbr, w, ONE_BY_ONE ? (int32_t)(n + 1) : 1, rng, out);
        acc += out[0] + 2 * out[1] + 3 * out[2] + 4 * out[3];
    }
    sink[lane] = acc;
}

hipError_t launch_split_cost(bool one_by_one, int64_t n, int32_t reps, int64_t *sink, int32_t blocks, hipStream_t st)
{
    if (one_by_one)
        split_cost_kernel<true><<<blocks, 256, 0, st>>>(n, reps, sink);
    else
        split_cost_kernel<false><<<blocks, 256, 0, st>>>(n, reps, sink);
    return hipGetLastError();
}

// One thread per occupancy byte: tets 4j .. 4j + 3 of one species of one
// realization (bytes of the row padding past Tp / 4 are zero).  The current
// map gets the current period's tag where the counts are non-zero.
__global__ __launch_bounds__(256) void mask_build_kernel(const int32_t *__restrict__ counts,
                                                         uint8_t *__restrict__ mask_cur,
                                                         uint8_t *__restrict__ mask_other, uint8_t tag, int64_t Tp,
                                                         int64_t stride, int64_t n_bytes)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_bytes) return;
    const int64_t row = i / stride;  // realization * S + species, as in the counts
    const int64_t t4 = (i % stride) * 4;
    int32_t any = 0;
    if (t4 < Tp) {
        const int4 c = *reinterpret_cast<const int4 *>(counts + row * Tp + t4);
        any = c.x | c.y | c.z | c.w;
    }
    mask_cur[i] = any != 0 ? tag : 0;
    mask_other[i] = 0;
}

hipError_t launch_mask_build(const int32_t *counts, uint8_t *mask_cur, uint8_t *mask_other, uint8_t tag, int32_t Rz,
                             int32_t S, int64_t Tp, hipStream_t st)
{
    const int64_t stride = mask_stride(Tp);
    const int64_t n = (int64_t)Rz * S * stride;
    if (n <= 0) return hipSuccess;
    mask_build_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(counts, mask_cur, mask_other, tag, Tp, stride,
                                                                    n);
    return hipGetLastError();
}

// After a chunk of periods: every simulation's period index moves on.
__global__ void advance_kernel(DevSim *sims, const WorkHeader *hdr, int64_t by)
{
    const int32_t n = hdr->n_sims;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        sims[i].step0 += by;
}

hipError_t launch_advance(DevSim *sims, const WorkHeader *hdr, int64_t by, hipStream_t st)
{
    advance_kernel<<<4, 256, 0, st>>>(sims, hdr, by);
    return hipGetLastError();
}

}  // namespace rdos
