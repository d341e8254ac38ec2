"""Seeded synthetic inputs: meshes, species/reaction sets and initial counts.

This module only builds inputs.  It holds none of the method's arithmetic
(no local rates, weights, period, sampling or stepping); both the GPU library
and the oracle receive exactly the arrays produced here.

Meshes are Kuhn (Freudenthal) lattices: an n x n x n grid of cubic cells of
edge ``a``, each cell cut into the 6 tetrahedra that share its main diagonal.
Numbering (fixed so every consumer sees the same mesh):

* vertex id   = i + (n+1) * (j + (n+1) * k), at (i a, j a, k a)
* tet id      = 6 * (ci + n * (cj + n * ck)) + p, where p indexes the axis
  permutations (pi0, pi1, pi2) of (0, 1, 2) in lexicographic order and tet p
  has the local vertices 0, e_pi0, e_pi0 + e_pi1, (1, 1, 1) of its cell.

The paper's own meshes (its spiny dendrite and its 1060-tet cylinder) are not
available; these lattices stand in for them (its Fig. 2 cube is 1 um on a
side, reused here for the small diffusion case).
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

N_A = 6.02214076e23  # Avogadro constant (SI 2019), for concentration -> count

_PERMS = list(itertools.permutations(range(3)))


@dataclasses.dataclass
class Model:
    """One simulation request: mesh, species, reactions, initial counts."""

    name: str
    xyz: np.ndarray                # [n_verts, 3] float64, metres
    tets: np.ndarray               # [n_tets, 4] int32
    D: List[float]                 # per species, m^2/s
    reactions: List[Tuple[List[int], List[int], float]]  # (reactants, products, k SI)
    init: np.ndarray               # [n_realizations, n_species, n_tets] int32
    t_end: float
    seed: int = 1
    tau_scale: float = 1.0
    species_names: Optional[List[str]] = None
    regions: Optional[dict] = None  # reaction id -> tets where it may fire

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_species(self) -> int:
        return len(self.D)

    @property
    def n_realizations(self) -> int:
        return int(self.init.shape[0])


def kuhn_lattice(n: int, a: float) -> Tuple[np.ndarray, np.ndarray]:
    """Vertices and tetrahedra of an n^3-cell Kuhn lattice with cell edge a."""
    return kuhn_box(n, n, n, a)


def kuhn_box(nx: int, ny: int, nz: int, a: float) -> Tuple[np.ndarray, np.ndarray]:
    """An nx x ny x nz-cell Kuhn lattice (vertex id i + (nx+1)(j + (ny+1)k),
    tet id 6 (ci + nx (cj + ny ck)) + p)."""
    mx, my, mz = nx + 1, ny + 1, nz + 1
    k, j, i = np.meshgrid(np.arange(mz), np.arange(my), np.arange(mx), indexing="ij")
    xyz = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * a

    def vid(ci, cj, ck):
        return ci + mx * (cj + my * ck)

    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    tets = np.empty((nx * ny * nz, 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        off = np.zeros(3, dtype=np.int64)
        corners = [off.copy()]
        for ax in perm:
            off[ax] += 1
            corners.append(off.copy())
        # corners: 0, e_pi0, e_pi0+e_pi1, (1,1,1)
        for v, cc in enumerate(corners):
            tets[:, p, v] = vid(ci + cc[0], cj + cc[1], ck + cc[2])
    return xyz, tets.reshape(-1, 4).astype(np.int32)


def jitter(xyz: np.ndarray, n: int, a: float, frac: float, seed: int) -> np.ndarray:
    """Move every interior vertex by a uniform offset in [-frac a, frac a]^3.

    Boundary vertices stay put, so the box volume is unchanged.  At frac=0.2 no
    tet can invert (largest height loss 0.69a < smallest Kuhn height 0.707a).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = xyz.copy()
    lim = n * a
    eps = 1e-9 * a
    interior = np.all((xyz > eps) & (xyz < lim - eps), axis=1)
    delta = rng.uniform(-frac * a, frac * a, size=(int(interior.sum()), 3))
    out[interior] += delta
    return out


def _tet_volumes(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Tet volumes for placing molecules (input recipe only)."""
    p0 = xyz[tets[:, 0]]
    a = xyz[tets[:, 1]] - p0
    b = xyz[tets[:, 2]] - p0
    c = xyz[tets[:, 3]] - p0
    return np.abs(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0


def _barycentres(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    return xyz[tets].mean(axis=1)


def count_for(conc_molar: float, volume_m3: float) -> int:
    """Molecules for a concentration in a volume, rounded half to even."""
    return int(round(conc_molar * N_A * volume_m3 * 1000.0))


def place_by_volume(xyz, tets, total: int, rng, mask: Optional[np.ndarray] = None,
                    vol: Optional[np.ndarray] = None) -> np.ndarray:
    """Scatter ``total`` molecules independently over tets, P(tet) ~ volume
    (inverse CDF of the volume prefix sum, one uniform per molecule)."""
    if vol is None:
        vol = _tet_volumes(xyz, tets)
    if mask is not None:
        vol = np.where(mask, vol, 0.0)
    cdf = np.cumsum(vol)
    u = rng.random(int(total)) * cdf[-1]
    idx = np.searchsorted(cdf, u, side="right")
    idx = np.minimum(idx, len(vol) - 1)
    return np.bincount(idx, minlength=len(vol)).astype(np.int32)


# ----------------------------------------------------------------------------
# The workloads
# ----------------------------------------------------------------------------

def diffusion_cube(seed: int = 1) -> Model:
    """1 um cube, 5x5x5 cells x 6 (750 tets), one species D=1e-12 m^2/s,
    1000 molecules in the first tet of the middle cell (2,2,2), 0.5 s."""
    n, a = 5, 0.2e-6
    xyz, tets = kuhn_lattice(n, a)
    init = np.zeros((1, 1, tets.shape[0]), dtype=np.int32)
    init[0, 0, 6 * (2 + n * (2 + n * 2))] = 1000
    return Model("diffusion_cube_750", xyz, tets, [1e-12], [], init, 0.5, seed)


def _abc_reactions():
    # A + B -> C at 1e6 /(M s); C -> A + B at 10 /s
    return [([0, 1], [2], 1e6), ([2], [0, 1], 10.0)]


def abc_lattice(n: int = 40, a: float = 0.1e-6, seed: int = 1, n_realizations: int = 1,
                conc: float = 100e-9, t_end: float = 0.1) -> Model:
    """A+B<->C on an n^3 x 6 Kuhn lattice: A and B at ``conc`` placed by
    volume, C empty; D_A = D_B = 1e-12, D_C = 0.5e-12 m^2/s."""
    xyz, tets = kuhn_lattice(n, a)
    vol_total = (n * a) ** 3
    total = count_for(conc, vol_total)
    rng = np.random.Generator(np.random.PCG64(seed))
    init = np.zeros((n_realizations, 3, tets.shape[0]), dtype=np.int32)
    vol = _tet_volumes(xyz, tets)
    for r in range(n_realizations):
        init[r, 0] = place_by_volume(xyz, tets, total, rng, vol=vol)
        init[r, 1] = place_by_volume(xyz, tets, total, rng, vol=vol)
    return Model(f"abc_{n}cube_{tets.shape[0]}", xyz, tets, [1e-12, 1e-12, 0.5e-12],
                 _abc_reactions(), init, t_end, seed, species_names=["A", "B", "C"])


def abcd_jittered(n: int = 40, a: float = 0.1e-6, seed: int = 1, t_end: float = 0.05) -> Model:
    """The A+B<->C lattice with interior vertices jittered by +-20% of the cell
    edge, plus species D (5e-12 m^2/s) decaying D -> 0 at 1/s, initialised at
    1 uM in the octant x, y, z < n a / 2 (by tet barycentre)."""
    xyz0, tets = kuhn_lattice(n, a)
    xyz = jitter(xyz0, n, a, 0.2, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    vol_total = (n * a) ** 3
    total = count_for(100e-9, vol_total)
    init = np.zeros((1, 4, tets.shape[0]), dtype=np.int32)
    init[0, 0] = place_by_volume(xyz, tets, total, rng)
    init[0, 1] = place_by_volume(xyz, tets, total, rng)
    bc = _barycentres(xyz, tets)
    half = n * a / 2
    octant = np.all(bc < half, axis=1)
    vol = _tet_volumes(xyz, tets)
    total_d = count_for(1e-6, float(vol[octant].sum()))
    init[0, 3] = place_by_volume(xyz, tets, total_d, rng, mask=octant)
    reactions = _abc_reactions() + [([3], [], 1.0)]
    return Model(f"abcd_jitter_{n}cube_{tets.shape[0]}", xyz, tets,
                 [1e-12, 1e-12, 0.5e-12, 5e-12], reactions, init, t_end, seed,
                 species_names=["A", "B", "C", "D"])


_LATTICES = {}


def _lattice_cached(n: int, a: float):
    key = (n, a)
    if key not in _LATTICES:
        if len(_LATTICES) > 64:
            _LATTICES.clear()
        _LATTICES[key] = kuhn_lattice(n, a)
    return _LATTICES[key]


def serving_request(rng: np.random.Generator, a: float = 0.1e-6, t_lo: float = 1e4,
                    t_hi: float = 1e6, max_species: int = 6) -> Model:
    """One request of the serving mix: jittered lattice with T log-uniform in
    [t_lo, t_hi] tets, 1..max_species species with D log-uniform in
    [1e-13, 1e-11] m^2/s, 0..2S random uni/bimolecular reactions (first order
    log-U [1, 1e3] /s, second order log-U [1e5, 1e8] /(M s)), each species
    initialised log-U [10 nM, 1 uM] placed by volume.  A reaction never has
    more products than reactants (conversions and degradations), so no
    request can grow without bound."""
    T = math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))
    n = max(2, int(round((T / 6.0) ** (1.0 / 3.0))))
    xyz0, tets = _lattice_cached(n, a)
    xyz = jitter(xyz0, n, a, 0.2, int(rng.integers(1, 2**31)))
    S = int(rng.integers(1, max_species + 1))
    D = [float(math.exp(rng.uniform(math.log(1e-13), math.log(1e-11)))) for _ in range(S)]
    n_reac = int(rng.integers(0, 2 * S + 1))
    reactions = []
    for _ in range(n_reac):
        if rng.random() < 0.5:
            r = [int(rng.integers(0, S))]
            k = float(math.exp(rng.uniform(math.log(1.0), math.log(1e3))))
        else:
            r = [int(rng.integers(0, S)), int(rng.integers(0, S))]
            k = float(math.exp(rng.uniform(math.log(1e5), math.log(1e8))))
        n_prod = int(rng.integers(0, len(r) + 1))
        p = [int(rng.integers(0, S)) for _ in range(n_prod)]
        reactions.append((r, p, k))
    vol_total = (n * a) ** 3
    init = np.zeros((1, S, tets.shape[0]), dtype=np.int32)
    vol = _tet_volumes(xyz, tets)
    for s in range(S):
        c = math.exp(rng.uniform(math.log(10e-9), math.log(1e-6)))
        init[0, s] = place_by_volume(xyz, tets, count_for(c, vol_total), rng, vol=vol)
    return Model(f"serve_{n}cube_S{S}_R{n_reac}", xyz, tets, D, reactions, init,
                 t_end=float("nan"), seed=int(rng.integers(1, 2**31)))


def tube_influx(nx: int = 40, ny: int = 2, nz: int = 2, a: float = 0.1e-6, D: float = 1e-12,
                kp: float = 2e-4, t_end: float = 0.05, n_realizations: int = 1, seed: int = 1) -> Model:
    """A bar of nx x ny x nz Kuhn cells (a tube along x) with a constant
    production 0 -> A restricted to the tets of the two end cell layers
    (constant influx at both ends, as in the validation of Sec. III.B),
    starting empty.  Model.regions maps the reaction to its tets."""
    xyz, tets = kuhn_box(nx, ny, nz, a)
    bc = _barycentres(xyz, tets)
    ends = np.nonzero((bc[:, 0] < a) | (bc[:, 0] > (nx - 1) * a))[0].astype(np.int32)
    init = np.zeros((n_realizations, 1, tets.shape[0]), dtype=np.int32)
    m = Model(f"tube_{nx}x{ny}x{nz}", xyz, tets, [D], [([], [0], kp)], init, t_end, seed,
              species_names=["A"])
    m.regions = {0: ends}
    return m


def production_annihilation(n: int = 5, a: float = 0.2e-6, D: float = 1e-11, k2: float = 1e8,
                            mean: float = 30.0, n_realizations: int = 1, seed: int = 1) -> Model:
    """Production and second-order degradation (the reaction-diffusion
    validation of Sec. III.B, Fig. 6): 0 -> A at k1 (M/s) and A + A -> 0 at
    k2 (1/(M s); 1e8 = 100 / (uM s)) on an n^3 x 6 Kuhn cube.  k1 is chosen
    so that the well-mixed stationary mean is close to `mean`
    (lambda = 2 mu mean^2 with mu = k2 / (N_A V), the pair rate of reading
    R9).  Each realization starts with `mean` molecules placed by volume."""
    xyz, tets = kuhn_lattice(n, a)
    vol = _tet_volumes(xyz, tets)
    nav = 6.02214076e23 * float(vol.sum()) * 1e3
    mu = k2 / nav
    k1 = 2.0 * mu * mean * mean / nav
    init = np.zeros((n_realizations, 1, tets.shape[0]), dtype=np.int32)
    for r in range(n_realizations):
        rng = np.random.default_rng([seed, r])
        init[r, 0] = place_by_volume(xyz, tets, int(round(mean)), rng, vol=vol)
    return Model(f"prod_annih_{n}cube", xyz, tets, [D], [([], [0], k1), ([0, 0], [], k2)], init, float("nan"),
                 seed, species_names=["A"])


def ten_species(nx: int = 20, ny: int = 3, nz: int = 3, a: float = 0.1e-6, seed: int = 1,
                n_realizations: int = 1, conc_lo: float = 0.1e-6, conc_hi: float = 1e-6) -> Model:
    """A stand-in for the reaction-diffusion model of Sec. III.C and Fig. 10
    (10 species, 8 reactions: 4 reversible pairs), whose exact species and
    constants the paper gives only as ranges: D log-uniform in [10, 100]
    um^2/s, the four bimolecular reactions log-uniform in [1, 1000] /(uM s),
    the four first-order reverses in [1, 100] /s.  Species pair up as
    S0 + S1 <-> S2, S2 + S3 <-> S4, S5 + S6 <-> S7, S7 + S8 <-> S9 in a bar of
    nx x ny x nz Kuhn cells (the paper's cylinder stands in as a square
    tube); each species starts log-uniform in [conc_lo, conc_hi] molar,
    placed by volume, independently per realization."""
    rng = np.random.default_rng([seed, 10])
    xyz, tets = kuhn_box(nx, ny, nz, a)
    D = [float(math.exp(rng.uniform(math.log(1e-11), math.log(1e-10)))) for _ in range(10)]
    reactions = []
    for x, y, z in ((0, 1, 2), (2, 3, 4), (5, 6, 7), (7, 8, 9)):
        kf = float(math.exp(rng.uniform(math.log(1e6), math.log(1e9))))   # 1..1000 /(uM s) in /(M s)
        kb = float(math.exp(rng.uniform(math.log(1.0), math.log(100.0))))
        reactions += [([x, y], [z], kf), ([z], [x, y], kb)]
    vol = _tet_volumes(xyz, tets)
    vol_total = float(vol.sum())
    conc = [math.exp(rng.uniform(math.log(conc_lo), math.log(conc_hi))) for _ in range(10)]
    init = np.zeros((n_realizations, 10, tets.shape[0]), dtype=np.int32)
    for r in range(n_realizations):
        for s_ in range(10):
            init[r, s_] = place_by_volume(xyz, tets, count_for(conc[s_], vol_total), rng, vol=vol)
    return Model(f"ten_species_{nx}x{ny}x{nz}", xyz, tets, D, reactions, init, t_end=float("nan"), seed=seed,
                 species_names=[f"S{i}" for i in range(10)])


def triangle_lattice(nx: int, ny: int, a: float, jitter_frac: float = 0.0, seed: int = 1) -> Tuple[np.ndarray, np.ndarray]:
    """A planar surface (z = 0) of nx x ny square cells of edge a, each cut
    into two right triangles along a diagonal that alternates like a
    checkerboard (so the walk has no preferred diagonal).  Interior vertices
    move uniformly within +-jitter_frac * a in x and y (numpy PCG64).
    Vertex i + (nx + 1) j; cell (i, j) gives triangles 2 (i + nx j) and + 1."""
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    xyz = np.stack([ii.ravel() * a, jj.ravel() * a, np.zeros(ii.size)], axis=1).astype(np.float64)
    tris = []
    for j in range(ny):
        for i in range(nx):
            v00, v10 = i + (nx + 1) * j, i + 1 + (nx + 1) * j
            v01, v11 = i + (nx + 1) * (j + 1), i + 1 + (nx + 1) * (j + 1)
            if (i + j) % 2 == 0:
                tris += [(v00, v10, v11), (v00, v11, v01)]
            else:
                tris += [(v00, v10, v01), (v10, v11, v01)]
    if jitter_frac > 0:
        rng = np.random.default_rng(seed)
        inner = (ii.ravel() > 0) & (ii.ravel() < nx) & (jj.ravel() > 0) & (jj.ravel() < ny)
        xyz[inner, :2] += rng.uniform(-jitter_frac * a, jitter_frac * a, size=(int(inner.sum()), 2))
    return xyz, np.array(tris, dtype=np.int32)


def box_surface(n: int, a: float) -> Tuple[np.ndarray, np.ndarray]:
    """The closed surface of the n^3 x 6 Kuhn cube: its boundary faces (faces
    on one tet only) as triangles, on the cube's vertices (unused ones
    dropped).  Every edge lies on exactly two triangles."""
    xyz, tets = kuhn_lattice(n, a)
    faces = {}
    for t in range(tets.shape[0]):
        for f in range(4):
            tri = tuple(sorted(int(v) for k, v in enumerate(tets[t]) if k != f))
            faces[tri] = faces.get(tri, 0) + 1
    tris = np.array([tri for tri, c in faces.items() if c == 1], dtype=np.int32)
    used, inv = np.unique(tris, return_inverse=True)
    return xyz[used].copy(), inv.reshape(tris.shape).astype(np.int32)


def tiny_lattice(n: int = 2, a: float = 0.2e-6, jitter_frac: float = 0.0, seed: int = 3) -> Tuple[np.ndarray, np.ndarray]:
    """Small meshes for exhaustive tests (n=1: 6 tets, n=2: 48 tets)."""
    xyz, tets = kuhn_lattice(n, a)
    if jitter_frac > 0:
        xyz = jitter(xyz, n, a, jitter_frac, seed)
    return xyz, tets


def reaction_arrays(reactions: Sequence[Tuple[Sequence[int], Sequence[int], float]]):
    """Flatten (reactants, products, k) triples into the fixed-width arrays the
    C interfaces take: reac_n[R], reac_ids[R][2], prod_n[R], prod_ids[R][3], k[R]."""
    R = len(reactions)
    rn = np.zeros(max(R, 1), dtype=np.int32)
    rid = np.full((max(R, 1), 2), -1, dtype=np.int32)
    pn = np.zeros(max(R, 1), dtype=np.int32)
    pid = np.full((max(R, 1), 3), -1, dtype=np.int32)
    k = np.zeros(max(R, 1), dtype=np.float64)
    for i, (re, pr, kk) in enumerate(reactions):
        rn[i] = len(re)
        rid[i, : len(re)] = re
        pn[i] = len(pr)
        pid[i, : len(pr)] = pr
        k[i] = kk
    return rn, rid, pn, pid, k
