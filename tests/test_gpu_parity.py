"""GPU path against the oracle, bit for bit (integer counts: tolerance 0).

Both sides receive the same seeded inputs (workloads) and draw from the same
Philox streams; every test compares whole count arrays.  Tests print the case
they are about to run so that a failing GPU step is named in the log.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_1512_03126_amd as P

    P.lib()
    return P


def make_pair(P, orc, xyz, tets, D, reactions, init, seed=1, tau_scale=1.0):
    """init: [Rz][S][T]"""
    init = np.asarray(init, np.int32)
    Rz = init.shape[0]
    g = P.Simulation(xyz, tets, D, reactions, seed=seed, n_realizations=Rz, tau_scale=tau_scale)
    os_ = []
    for r in range(Rz):
        o = orc.OracleSim(xyz, tets, D, reactions, tau_scale=tau_scale, seed=seed, realization=r)
        for s in range(len(D)):
            o.set_counts(s, init[r, s])
            g.set_counts(s, init[r, s], realization=r)
        os_.append(o)
    assert g.tau == os_[0].tau
    return g, os_


def assert_same(g, os_, where=""):
    for r, o in enumerate(os_):
        got = g.get_counts(None, realization=r)
        want = o.get_counts()
        if not np.array_equal(got, want):
            diff = np.argwhere(got != want)
            raise AssertionError(f"{where}: realization {r}: {len(diff)} counts differ, first at "
                                 f"(species, tet) {tuple(diff[0])}: gpu {got[tuple(diff[0])]} oracle "
                                 f"{want[tuple(diff[0])]}")


RICH_D = [1e-12, 1e-12, 0.5e-12, 0.0, 2e-12]
RICH_REACTIONS = [
    ([0, 1], [2], 3e8),        # A + B -> C
    ([2], [0, 1], 400.0),      # C -> A + B
    ([0, 0], [3], 5e7),        # 2A -> E   (homodimer)
    ([3], [0, 0], 80.0),       # E -> 2A   (E immobile)
    ([], [4], 2e-5),           # 0 -> F    (0th order, every tet active)
    ([4], [], 150.0),          # F -> 0
    ([1, 4], [1, 1, 4], 1e8),  # B + F -> 2B + F (three products)
]


def rich_init(T, Rz, seed, hi=25):
    rng = np.random.default_rng(seed)
    init = rng.integers(0, hi, size=(Rz, len(RICH_D), T)).astype(np.int32)
    init[:, 4] = 0
    return init


# ---------------------------------------------------------------------------
def test_geometry_and_tau_bit_exact(P, orc):
    cases = [("kuhn n=3", W.kuhn_lattice(3, 0.1e-6)),
             ("jittered n=4", (W.jitter(W.kuhn_lattice(4, 0.1e-6)[0], 4, 0.1e-6, 0.2, 2), W.kuhn_lattice(4, 0.1e-6)[1])),
             ("jittered n=40", (W.abcd_jittered().xyz, W.abcd_jittered().tets))]
    for name, (xyz, tets) in cases:
        note(f"geometry {name} T={tets.shape[0]}")
        for D, ts in [([1e-12, 0.5e-12], 1.0), ([3e-12, 0.0], 0.37)]:
            g = P.Simulation(xyz, tets, D, [], tau_scale=ts)
            o = orc.OracleSim(xyz, tets, D, [], tau_scale=ts)
            assert g.tau == o.tau, name
            gg, og = g.geometry(), o.geometry()
            np.testing.assert_array_equal(gg["nbr"], og["nbr"])
            for key in ("w", "g", "nav"):
                assert np.array_equal(gg[key].view(np.uint64), og[key].view(np.uint64)), (name, key)
            g.close()


def test_large_mesh_face_matching_paths(P, orc):
    """Meshes of at least 16,384 cells are matched on the device, in the
    set-up buffers.  A bad face there falls back to the host matching, which
    names it, and nothing is cached.  A fresh lattice matched on the device,
    the same lattice again from the cache, and the oracle agree on every
    neighbour, weight, g and N_A V, bit for bit."""
    n = 17   # 29,478 tets: a lattice no other test uses, so its first set-up is uncached
    xyz0, tets = W.kuhn_lattice(n, 0.1e-6)
    xyz = W.jitter(xyz0, n, 0.1e-6, 0.2, 5)
    note(f"face matching on the device: T={tets.shape[0]}, bad faces, then fresh and cached set-ups")
    bad = tets.copy()
    bad[100, 3] = bad[100, 2]
    with pytest.raises(P.RdosError, match="repeats a face"):
        P.Simulation(xyz, bad, [1e-12], [])
    with pytest.raises(P.RdosError, match="shared"):
        P.Simulation(xyz, np.concatenate([tets, tets[:1]]), [1e-12], [])
    o = orc.OracleSim(xyz, tets, [1e-12, 0.4e-12], [])
    og = o.geometry()
    for _ in range(2):   # matched on the device, then taken from the cache
        g = P.Simulation(xyz, tets, [1e-12, 0.4e-12], [])
        assert g.tau == o.tau
        gg = g.geometry()
        np.testing.assert_array_equal(gg["nbr"], og["nbr"])
        for key in ("w", "g", "nav"):
            assert np.array_equal(gg[key].view(np.uint64), og[key].view(np.uint64)), key
        g.close()


@pytest.mark.parametrize("n,jit,Rz,seed", [(1, 0.0, 3, 1), (2, 0.2, 2, 7), (3, 0.2, 1, 11)])
def test_rich_chemistry_every_period(P, orc, n, jit, Rz, seed):
    xyz, tets = W.tiny_lattice(n, 0.2e-6, jitter_frac=jit, seed=seed)
    T = tets.shape[0]
    note(f"rich chemistry n={n} T={T} Rz={Rz} seed={seed}")
    g, os_ = make_pair(P, orc, xyz, tets, RICH_D, RICH_REACTIONS, rich_init(T, Rz, seed), seed=seed)
    for k in range(40):
        g.step(1)
        for o in os_:
            o.step()
        assert_same(g, os_, f"period {k}")
    g.close()


def test_diffusion_cube_run_until(P, orc):
    m = W.diffusion_cube()
    note("diffusion cube 750 tets, run_until 0.5 s")
    g, os_ = make_pair(P, orc, m.xyz, m.tets, m.D, m.reactions, m.init, seed=m.seed)
    for t_end in (0.01, 0.1, 0.25, m.t_end):
        g.run_until(t_end)
        os_[0].run_until(t_end)
        assert g.time() == os_[0].time()
        assert_same(g, os_, f"t={t_end}")
    g.close()
    # one call: 422 full periods and one shortened to end at 0.5 s (Step 1)
    g, os_ = make_pair(P, orc, m.xyz, m.tets, m.D, m.reactions, m.init, seed=m.seed)
    g.run_until(m.t_end)
    os_[0].run_until(m.t_end)
    assert g.time() == (m.t_end, 423)
    assert_same(g, os_, "single run_until")
    g.close()


def test_abc_lattice_full_size(P, orc):
    m = W.abc_lattice()
    note(f"A+B<->C 40^3x6 T={m.n_tets}, 0.1 s")
    g, os_ = make_pair(P, orc, m.xyz, m.tets, m.D, m.reactions, m.init, seed=m.seed)
    g.run_until(0.02)
    os_[0].run_until(0.02)
    assert_same(g, os_, "t=0.02")
    g.run_until(m.t_end)
    os_[0].run_until(m.t_end)
    assert_same(g, os_, f"t={m.t_end}")
    c = g.get_counts()
    assert c[0].sum() + c[2].sum() == m.init[0, 0].sum()
    g.close()


def test_abcd_jittered_full_size(P, orc):
    """The jittered mesh with D decay at full size: every count against the
    oracle after 60 and 500 periods (the oracle takes about 10 ms a period
    here, the whole 0.05 s is about 5000 periods), then the GPU alone to the
    end with what holds at any length: A + C and B + C are conserved, and the
    first-order decay of D is exact under the splitting (each D molecule
    survives 0.05 s with probability exp(-0.05), whatever it diffuses), so the
    D total is Binomial(D0, exp(-0.05))."""
    m = W.abcd_jittered()
    note(f"A+B<->C + D decay, jittered 40^3x6 T={m.n_tets}: 500 periods against the oracle")
    g, os_ = make_pair(P, orc, m.xyz, m.tets, m.D, m.reactions, m.init, seed=m.seed)
    for n in (60, 440):
        g.step(n)
        os_[0].run_steps(n)
        assert_same(g, os_, "jittered")
    note(f"A+B<->C + D decay: to t = {m.t_end} on the GPU")
    g.run_until(m.t_end)
    c = g.get_counts()
    a0, b0, d0 = (int(m.init[0, q].sum()) for q in (0, 1, 3))
    assert c[0].sum() + c[2].sum() == a0 and c[1].sum() + c[2].sum() == b0
    p = math.exp(-1.0 * m.t_end)
    sd = math.sqrt(d0 * p * (1 - p))
    assert abs(int(c[3].sum()) - d0 * p) < 4 * sd, (int(c[3].sum()), d0 * p, sd)
    g.close()


def test_dense_counts_exercise_btrd(P, orc):
    xyz, tets = W.tiny_lattice(2, 0.2e-6, jitter_frac=0.2, seed=5)
    T = tets.shape[0]
    note(f"dense counts T={T}")
    rng = np.random.default_rng(3)
    init = np.zeros((2, 2, T), np.int32)
    init[:, 0] = rng.integers(0, 200000, size=(2, T))
    init[:, 1] = rng.integers(0, 40, size=(2, T))
    reactions = [([0], [1], 3000.0), ([1], [0], 1.0)]
    g, os_ = make_pair(P, orc, xyz, tets, [1e-12, 1e-12], reactions, init, seed=9, tau_scale=0.37)
    for k in range(6):
        g.step(1)
        for o in os_:
            o.step()
        assert_same(g, os_, f"dense period {k}")
    g.close()


@pytest.mark.parametrize("n", [6, 11])
def test_ragged_multi_tile_meshes(P, orc, n):
    xyz, tets = W.kuhn_lattice(n, 0.1e-6)
    T = tets.shape[0]
    note(f"ragged tiles T={T}")
    rng = np.random.default_rng(n)
    init = np.zeros((2, 2, T), np.int32)
    init[:, 0] = (rng.random((2, T)) < 0.3) * rng.integers(1, 40, size=(2, T))
    init[:, 1] = (rng.random((2, T)) < 0.05) * rng.integers(1, 4, size=(2, T))
    g, os_ = make_pair(P, orc, xyz, tets, [1e-12, 0.3e-12], [([0, 1], [1, 1], 1e9)], init, seed=n)
    for _ in range(4):
        g.step(5)
        for o in os_:
            o.run_steps(5)
        assert_same(g, os_, f"n={n}")
    g.close()


def test_zeroth_order_and_empty_start(P, orc):
    xyz, tets = W.kuhn_lattice(3, 0.1e-6)
    T = tets.shape[0]
    note("0th-order production from empty")
    init = np.zeros((1, 1, T), np.int32)
    g, os_ = make_pair(P, orc, xyz, tets, [1e-12], [([], [0], 1e-4), ([0], [], 10.0)], init, seed=4)
    for k in range(10):
        g.step(1)
        os_[0].step()
        assert_same(g, os_, f"period {k}")
    assert g.get_counts(0).sum() > 0
    g.close()
    note("empty state stays empty")
    g2, os2 = make_pair(P, orc, xyz, tets, [1e-12, 1e-12], [([0, 1], [], 1e6)], np.zeros((1, 2, T), np.int32))
    g2.step(7)
    assert g2.get_counts().sum() == 0
    g2.close()


def test_resume_is_bit_identical(P, orc):
    xyz, tets = W.tiny_lattice(2, 0.2e-6, jitter_frac=0.2, seed=8)
    T = tets.shape[0]
    note("resume")
    init = rich_init(T, 1, 21)
    g, os_ = make_pair(P, orc, xyz, tets, RICH_D, RICH_REACTIONS, init, seed=21)
    g.step(13)
    mid = g.get_counts()
    t_mid, k_mid = g.time()
    g.step(11)
    end = g.get_counts()
    h = P.Simulation(xyz, tets, RICH_D, RICH_REACTIONS, seed=21)
    for s in range(len(RICH_D)):
        h.set_counts(s, mid[s])
    h.set_state(k_mid, t_mid)
    h.step(11)
    np.testing.assert_array_equal(h.get_counts(), end)
    os_[0].run_steps(24)
    assert_same(g, os_, "continuous")
    g.close()
    h.close()


def test_set_state_alone_moves_the_period(P, orc):
    # set_state without new counts: the occupancy bytes carry the period's
    # tag, so the map is rebuilt for the new index (else no tet would be
    # queued and the molecules would be lost); the run then matches the
    # oracle moved to the same period index
    xyz, tets = W.tiny_lattice(2, 0.2e-6, jitter_frac=0.2, seed=8)
    T = tets.shape[0]
    note("set_state alone, to an index of the other parity and a new tag")
    init = rich_init(T, 1, 23)
    g, os_ = make_pair(P, orc, xyz, tets, RICH_D, RICH_REACTIONS, init, seed=23)
    g.step(5)
    os_[0].run_steps(5)
    assert_same(g, os_, "before set_state")
    t0 = g.time()[0]
    g.set_state(300, t0)
    os_[0].set_state(300, t0)
    g.step(9)
    os_[0].run_steps(9)
    assert_same(g, os_, "after set_state")
    g.close()


def test_counts_can_be_reset_between_periods(P, orc):
    xyz, tets = W.kuhn_lattice(2, 0.1e-6)
    T = tets.shape[0]
    note("set_counts between periods")
    init = np.zeros((1, 1, T), np.int32)
    init[0, 0, 3] = 50
    g, os_ = make_pair(P, orc, xyz, tets, [1e-12], [], init, seed=2)
    g.step(3)
    os_[0].run_steps(3)
    new = np.arange(T, dtype=np.int32) % 5
    g.set_counts(0, new)
    os_[0].set_counts(0, new)
    g.step(4)
    os_[0].run_steps(4)
    assert_same(g, os_, "after reset")
    g.close()


def test_torch_stream(P, orc):
    import torch

    xyz, tets = W.kuhn_lattice(2, 0.1e-6)
    T = tets.shape[0]
    note("torch stream")
    init = np.zeros((1, 1, T), np.int32)
    init[0, 0, 0] = 300
    g, os_ = make_pair(P, orc, xyz, tets, [1e-12], [], init, seed=6)
    st = torch.cuda.Stream()
    g.set_stream(st)
    g.step(9)
    g.synchronize()
    os_[0].run_steps(9)
    assert_same(g, os_, "torch stream")
    g.set_stream(None)
    g.step(2)
    os_[0].run_steps(2)
    assert_same(g, os_, "own stream again")
    g.close()


def test_device_counts_view(P, orc):
    """The zero-copy view reads what get_counts reads and writes like set_counts."""
    import torch

    xyz, tets = W.kuhn_lattice(2, 0.1e-6)
    T = tets.shape[0]
    note("device counts view")
    init = np.zeros((2, 2, T), np.int32)
    init[:, 0, 3] = 120
    init[1, 1, 40] = 17
    g, os_ = make_pair(P, orc, xyz, tets, [1e-12, 2e-12], [([0, 1], [], 1e9)], init, seed=8)
    g.step(5)
    g.synchronize()
    for o in os_:
        o.run_steps(5)
    for r in range(2):
        for s in range(2):
            v = g.device_counts(s, realization=r)
            assert v.dtype == torch.int32 and v.shape == (T,)
            assert np.array_equal(v.cpu().numpy(), os_[r].get_counts(s)), (r, s)
    # write through the view, then continue: same as set_counts on the oracle
    v = g.device_counts(1, realization=0)
    v[7] += 5
    torch.cuda.synchronize()
    c = os_[0].get_counts(1)
    c[7] += 5
    os_[0].set_counts(1, c)
    g.step(3)
    for o in os_:
        o.run_steps(3)
    assert_same(g, os_, "after writing through the view")
    with pytest.raises(P.RdosError):
        P.rdos_device_counts(g.h, 2, 0)
    g.close()


def test_invalid_inputs(P):
    note("invalid inputs")
    xyz, tets = W.kuhn_lattice(1, 0.1e-6)
    h = P.rdos_create(0, 1, 1)
    with pytest.raises(P.RdosError) as ei:
        P.rdos_set_counts(h, 0, 0, np.zeros(6, np.int32))
    assert ei.value.status == -4
    P.rdos_set_mesh(h, xyz, tets)
    with pytest.raises(P.RdosError):
        P.rdos_add_reaction(h, [0], [], 1.0)      # no species yet
    P.rdos_add_species(h, 1e-12)
    with pytest.raises(P.RdosError):
        P.rdos_set_counts(h, 0, 0, -np.ones(6, np.int32))
    with pytest.raises(P.RdosError):
        P.rdos_finalize(h, 1.5)
    P.rdos_destroy(h)
    bad = tets.copy()
    bad[0, 3] = bad[0, 2]
    with pytest.raises(P.RdosError, match="repeats a face"):
        P.Simulation(xyz, bad, [1e-12], [])
    flat = tets.copy()
    flat[0] = [0, 1, 2, 3]                    # four corners of the z = 0 face: zero volume
    with pytest.raises(P.RdosError, match="degenerate"):
        P.Simulation(xyz, flat, [1e-12], [])
    with pytest.raises(P.RdosError, match="shared"):
        P.Simulation(xyz, np.concatenate([tets, tets[:1]]), [1e-12], [])
    with pytest.raises(P.RdosError, match="tau"):
        P.Simulation(xyz, tets, [0.0], [])


def test_tiled_work_list_bound(P):
    # queue entries are int32 (tile * 1024 + offset): 1296 tets take two
    # 1024-tet tiles, so 1.2e6 realizations pass the realizations x tets bound
    # (1.56e9) but not the tiled one (2.46e9), and finalize refuses them
    # before allocating anything
    note("finalize: tiled work list over 2^31 tets")
    xyz, tets = W.kuhn_lattice(6, 0.1e-6)
    assert tets.shape[0] == 1296
    with pytest.raises(P.RdosError, match="tiled tets"):
        P.Simulation(xyz, tets, [1e-12], [], n_realizations=1_200_000)


EIGHT_D = [1e-12, 2e-12, 0.5e-12, 0.0, 1.5e-12, 1e-12, 0.2e-12, 2e-12]   # 8 species, one not diffusing
SIXTEEN_RX = [  # 16 reactions: every order, homodimers, up to three products
    ([], [0], 2e-3), ([], [4], 1e-3), ([0], [1], 20.0), ([1], [0], 5.0),
    ([0, 1], [2], 2e3), ([2], [0, 1], 30.0), ([3], [5], 8.0), ([5, 5], [6], 5e3),
    ([6], [5, 5], 12.0), ([4], [], 3.0), ([7, 0], [7, 1], 1e3), ([2, 2], [3], 4e3),
    ([6], [4, 5, 7], 2.0), ([1, 4], [], 1e3), ([7], [7, 7], 1.0), ([7, 7], [7], 3e3),
]
MAX_D = EIGHT_D + [0.8e-12, 3e-12, 0.0, 1.2e-12, 0.3e-12, 2.5e-12, 1e-12, 0.6e-12]   # 16 species, two immobile
MAX_REACTIONS = SIXTEEN_RX + [  # 16 more over species 8-15, among them a three-product and a 0th-order one
    ([], [8], 1e-3), ([8], [9], 15.0), ([9], [8], 6.0), ([8, 9], [10], 2e3),
    ([10], [8, 9], 25.0), ([11, 11], [12], 4e3), ([12], [11, 11], 10.0), ([13], [], 2.0),
    ([14, 2], [15], 1.5e3), ([15], [14, 2], 20.0), ([15], [13, 13, 14], 1.0), ([12, 13], [], 8e2),
    ([10], [11], 5.0), ([14, 14], [14], 2e3), ([9, 15], [9, 8], 1e3), ([3], [13], 4.0),
]


def run_every_twenty(P, orc, D, reactions, seed, what):
    xyz, tets = W.tiny_lattice(6, 0.2e-6, jitter_frac=0.2, seed=seed)   # 1296 tets: two tiles, ragged
    rng = np.random.default_rng(seed)
    init = rng.integers(0, 12, size=(2, len(D), tets.shape[0])).astype(np.int32)
    note(f"{what}: {len(D)} species, {len(reactions)} reactions, T={tets.shape[0]}, 2 realizations, 40 periods")
    g, os_ = make_pair(P, orc, xyz, tets, D, reactions, init, seed=seed)
    for _ in range(2):
        g.step(20)
        for o in os_:
            o.run_steps(20)
        assert_same(g, os_, what)
    g.close()
    return xyz, tets


def test_eight_species_sixteen_reactions(P, orc):
    """8 species and 16 reactions, every species present: the 8-species
    kernel instances, bit for bit."""
    assert len(EIGHT_D) == 8 and len(SIXTEEN_RX) == 16
    run_every_twenty(P, orc, EIGHT_D, SIXTEEN_RX, 21, "8 species")


def test_maximum_species_and_reactions(P, orc):
    """The limits of one simulation, 16 species and 32 reactions, every
    species present: the widest kernel instances, bit for bit; one more
    species or reaction, or a third reactant, is refused."""
    assert len(MAX_D) == P.MAX_SPECIES == 16 and len(MAX_REACTIONS) == P.MAX_REACTIONS == 32
    xyz, tets = run_every_twenty(P, orc, MAX_D, MAX_REACTIONS, 22, "maximum sizes")
    h = P.rdos_create(0, 1, 1)
    P.rdos_set_mesh(h, xyz, tets)
    for d in MAX_D:
        P.rdos_add_species(h, d)
    with pytest.raises(P.RdosError, match="at most 16 species"):
        P.rdos_add_species(h, 1e-12)
    for r, p_, k in MAX_REACTIONS:
        P.rdos_add_reaction(h, r, p_, k)
    with pytest.raises(P.RdosError, match="at most 32 reactions"):
        P.rdos_add_reaction(h, [0], [1], 1.0)
    with pytest.raises(P.RdosError, match="0..2 reactants"):
        P.rdos_add_reaction(h, [0, 1, 2], [], 1.0)
    P.rdos_destroy(h)


# ---------------------------------------------------------------------------
# Batching / serving engine
# ---------------------------------------------------------------------------
def test_engine_batched_equals_alone_and_oracle(P, orc):
    note("engine: three simulations in one batch")
    specs = []
    xyz1, tets1 = W.tiny_lattice(2, 0.2e-6, jitter_frac=0.2, seed=3)
    specs.append((xyz1, tets1, RICH_D, RICH_REACTIONS, rich_init(tets1.shape[0], 2, 5), 5, 37))
    m = W.diffusion_cube()
    specs.append((m.xyz, m.tets, m.D, [], m.init, 1, 50))
    xyz3, tets3 = W.kuhn_lattice(6, 0.1e-6)
    init3 = np.zeros((3, 2, tets3.shape[0]), np.int32)
    init3[:, 0, ::7] = 3
    init3[:, 1, ::11] = 2
    specs.append((xyz3, tets3, [1e-12, 0.3e-12], [([0, 1], [1, 1], 1e9)], init3, 8, 22))
    e = P.rdos_engine_create(0, 0)
    tickets = []
    for xyz, tets, D, rx, init, seed, n in specs:
        s = P.Simulation(xyz, tets, D, rx, seed=seed, n_realizations=init.shape[0], tau_scale=None)
        for r in range(init.shape[0]):
            for q in range(len(D)):
                s.set_counts(q, init[r, q], realization=r)
        tickets.append((P.rdos_engine_submit(e, s.h, n, 1.0), s))
    P.rdos_engine_drain(e)
    for (t, s), (xyz, tets, D, rx, init, seed, n) in zip(tickets, specs):
        done, lat = P.rdos_engine_poll(e, t)
        assert done and lat > 0
        P.rdos_engine_release(e, t)
        assert s.time()[1] == n
        for r in range(init.shape[0]):
            o = orc.OracleSim(xyz, tets, D, rx, seed=seed, realization=r)
            for q in range(len(D)):
                o.set_counts(q, init[r, q])
            o.run_steps(n)
            np.testing.assert_array_equal(s.get_counts(None, realization=r), o.get_counts())
        s.close()
    stats = P.rdos_engine_stats(e)
    assert stats["launches"] >= 50 and stats["updates"] > 0
    P.rdos_engine_destroy(e)


def test_engine_budget_admits_in_turn(P, orc):
    note("engine: budget admits one simulation at a time")
    xyz, tets = W.kuhn_lattice(4, 0.1e-6)
    T = tets.shape[0]
    sims = []
    for i in range(3):
        s = P.Simulation(xyz, tets, [1e-12], [], seed=40 + i, tau_scale=None)
        init = np.zeros(T, np.int32)
        init[i * 10] = 500
        s.set_counts(0, init)
        sims.append((s, init))
    need = sims[0][0].info()["device_bytes"]
    e = P.rdos_engine_create(0, int(need * 1.5))
    tks = [P.rdos_engine_submit(e, s.h, 12 + 2 * i, 1.0) for i, (s, _) in enumerate(sims)]
    # only one fits at a time: release each as it finishes
    for i, t in enumerate(tks):
        while True:
            done, _ = P.rdos_engine_poll(e, t)
            if done:
                break
        P.rdos_engine_release(e, t)
        s, init = sims[i]
        o = orc.OracleSim(xyz, tets, [1e-12], [], seed=40 + i)
        o.set_counts(0, init)
        o.run_steps(12 + 2 * i)
        np.testing.assert_array_equal(s.get_counts(0), o.get_counts(0))
        s.close()
    P.rdos_engine_destroy(e)


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_launch_modes_every_period(P, orc, mode):
    """The one-launch path (a cooperative kernel running every period, grid
    barriers between the scan and update phases), the two-launch path and
    the fused launch (scan and update of each period in one kernel) give the
    oracle's counts after every period and after a run to a t_end that
    shortens the last period (Algorithm 1, Step 1)."""
    xyz, tets = W.tiny_lattice(4, 0.2e-6, jitter_frac=0.2, seed=12)
    T = tets.shape[0]
    rng = np.random.default_rng(30 + mode)
    init = rng.integers(0, 20, size=(3, len(RICH_D), T)).astype(np.int32)
    init[:, 0, ::5] += 150
    note(f"launch mode {mode}: {T} tets x {len(RICH_D)} species x 3 realizations")
    g, os_ = make_pair(P, orc, xyz, tets, RICH_D, RICH_REACTIONS, init, seed=7)
    P.rdos_set_launch_mode(g.h, mode)
    for k in range(6):
        g.step(1 + k)
        for o in os_:
            o.run_steps(1 + k)
        assert_same(g, os_, f"mode {mode}, after {k + 1} runs")
    t_end = g.time()[0] + 17.5 * g.tau
    g.run_until(t_end)
    for o in os_:
        o.run_until(t_end)
    assert_same(g, os_, f"mode {mode}, run to t_end")
    assert g.time()[0] == t_end
    g.close()


def test_launch_modes_interleaved(P, orc):
    """Runs that switch between the fused, two-launch and one-launch paths on
    one simulation: the fused kernel leaves the queue's length halves alone,
    so the two-launch periods before and after it keep their parity; counts
    equal the oracle's after every run.  The fused runs cover a tile list of
    several tiles per wavefront's ring (3 realizations x 3 tiles)."""
    xyz, tets = W.tiny_lattice(6, 0.2e-6, jitter_frac=0.2, seed=14)   # 1296 tets: two tiles, ragged
    T = tets.shape[0]
    rng = np.random.default_rng(44)
    init = rng.integers(0, 20, size=(3, len(RICH_D), T)).astype(np.int32)
    init[:, 0, ::3] += 90   # A, not the autocatalytic B (B + F -> 2B + F would grow B several-fold per period)
    note(f"interleaved launch modes: {T} tets x {len(RICH_D)} species x 3 realizations")
    g, os_ = make_pair(P, orc, xyz, tets, RICH_D, RICH_REACTIONS, init, seed=9)
    for k, mode in enumerate([1, 3, 3, 1, 2, 3, 1, 1, 3, 2, 1]):
        P.rdos_set_launch_mode(g.h, mode)
        g.step(1 + k % 3)
        for o in os_:
            o.run_steps(1 + k % 3)
        assert_same(g, os_, f"run {k} (mode {mode})")
    g.close()


def test_one_launch_with_more_segments_than_blocks(P, orc):
    """The one-launch path forced on a work list larger than one cooperative
    grid can hold (three blocks per CU, 768 on 256 CUs): 48 realizations of a
    16^3 x 6 lattice (24 tiles each, 1152 tiles in 1024 queue segments), so
    blocks stride over the tiles and segments; counts equal to the oracle's
    after 12 periods."""
    xyz, tets = W.kuhn_lattice(16, 0.1e-6)
    T = tets.shape[0]
    rng = np.random.default_rng(5)
    Rz = 48
    init = np.zeros((Rz, 3, T), np.int32)
    for r in range(Rz):
        for q in range(2):
            np.add.at(init[r, q], rng.integers(0, T, 400), 1)
    note(f"one launch, strided: {T} tets x {Rz} realizations")
    g, os_ = make_pair(P, orc, xyz, tets, [1e-12, 1e-12, 0.5e-12], [([0, 1], [2], 1e8), ([2], [0, 1], 10.0)], init,
                       seed=9)
    P.rdos_set_launch_mode(g.h, 2)
    g.step(12)
    for o in os_:
        o.run_steps(12)
    assert_same(g, os_, "one launch, strided")
    g.close()
