"""Serving: requests that arrive while others run join the batch, and every
result is the same as the request run alone (bit for bit, checked against the
oracle and against a direct run on the GPU)."""
import sys
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def small_request(i):
    rng = np.random.default_rng([77, i])
    return W.serving_request(rng, t_lo=300, t_hi=4000, max_species=4)


def run_oracle(orc, m, periods):
    o = orc.OracleSim(m.xyz, m.tets, m.D, m.reactions, seed=m.seed)
    for q in range(m.n_species):
        o.set_counts(q, m.init[0, q])
    o.run_steps(periods)
    return o.get_counts()


def test_served_results_equal_alone(orc):
    import paper_1512_03126_amd as P

    reqs = [small_request(i) for i in range(8)]
    periods = [40 + 10 * i for i in range(8)]
    # simulations with fewer species than the queue has rows share it: the
    # update reads every row beside a queue entry and must use only its own
    assert len({m.n_species for m in reqs}) > 1
    note("serving: 8 requests arriving while others run")
    e = P.rdos_engine_create(0, 0)
    tickets = []
    for i, (m, n) in enumerate(zip(reqs, periods)):
        s = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, tau_scale=None)
        for q in range(m.n_species):
            s.set_counts(q, m.init[0, q])
        tickets.append((P.rdos_engine_submit(e, s.h, n, 1.0), s))
        time.sleep(0.002 * (i % 3))  # staggered arrivals: some join running chunks
    P.rdos_engine_drain(e)
    mixed = []
    for t, s in tickets:
        done, lat = P.rdos_engine_poll(e, t)
        assert done and lat > 0
        P.rdos_engine_release(e, t)
        mixed.append(s.get_counts())
        s.close()
    P.rdos_engine_destroy(e)
    note("serving: each request alone (direct stepping) and on the oracle")
    for m, n, got in zip(reqs, periods, mixed):
        alone = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed)
        for q in range(m.n_species):
            alone.set_counts(q, m.init[0, q])
        alone.step(n)
        np.testing.assert_array_equal(alone.get_counts(), got)
        alone.close()
        np.testing.assert_array_equal(run_oracle(orc, m, n), got)


def test_hold_starts_requests_together(orc):
    """Requests submitted while the engine is held are all admitted before
    it runs, then start from the same chunk: with the same number of
    periods their run times (first launch to completion) are identical; every
    result equals the oracle's, and the latency parts add up."""
    import paper_1512_03126_amd as P

    reqs = [small_request(60 + i) for i in range(3)]
    note("serving: three requests started together by rdos_engine_hold")
    e = P.rdos_engine_create(0, 0)
    P.rdos_engine_hold(e, True)
    tickets = []
    for m in reqs:
        s = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, tau_scale=None)
        for q in range(m.n_species):
            s.set_counts(q, m.init[0, q])
        tickets.append((P.rdos_engine_submit(e, s.h, 40, 1.0), s))
    time.sleep(0.05)
    assert not any(P.rdos_engine_poll(e, t)[0] for t, _ in tickets)  # held: nothing has run
    P.rdos_engine_hold(e, False)
    P.rdos_engine_drain(e)
    parts = [P.rdos_engine_ticket_times(e, t) for t, _ in tickets]
    assert len({p_["run_s"] for p_ in parts}) == 1, parts
    for (t, s), p_ in zip(tickets, parts):
        lat = P.rdos_engine_poll(e, t)[1]
        assert abs(sum(p_.values()) - lat) < 1e-6, (p_, lat)
        P.rdos_engine_release(e, t)
    for m, (t, s) in zip(reqs, tickets):
        np.testing.assert_array_equal(run_oracle(orc, m, 40), s.get_counts())
        s.close()
    P.rdos_engine_destroy(e)


def test_engine_stall_is_reported_not_hung():
    import paper_1512_03126_amd as P

    note("serving: budget held by an unreleased finished request")
    m = small_request(3)
    e = P.rdos_engine_create(0, 0)
    s1 = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, tau_scale=None)
    need = s1.info()["device_bytes"]
    P.rdos_engine_destroy(e)
    e = P.rdos_engine_create(0, int(need * 1.5))
    s2 = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed + 1, tau_scale=None)
    t1 = P.rdos_engine_submit(e, s1.h, 10, 1.0)
    t2 = P.rdos_engine_submit(e, s2.h, 10, 1.0)
    with pytest.raises(P.RdosError) as ei:
        P.rdos_engine_drain(e)        # t2 cannot start until t1 is released
    assert ei.value.status == -2
    P.rdos_engine_release(e, t1)
    P.rdos_engine_drain(e)
    assert P.rdos_engine_poll(e, t2)[0]
    P.rdos_engine_release(e, t2)
    s1.close()
    s2.close()
    P.rdos_engine_destroy(e)


@pytest.mark.parametrize("bps", [1, 0])
def test_two_chains_survive_slot_changes(orc, bps):
    """Two chains with requests joining and leaving mid-run: the second
    chain's place in the work list moves with every change of the slot set
    and must be read from the device header, not from the captured graph.
    With bps 0 every period is one fused launch per chain."""
    import paper_1512_03126_amd as P

    reqs = [small_request(20 + i) for i in range(10)]
    periods = [24 + 18 * (i % 4) for i in range(10)]
    note(f"serving: fixed two-chain shape (update blocks per segment {bps}), staggered arrivals and departures")
    e = P.rdos_engine_create(0, 0)
    P.rdos_engine_set_shape(e, 8, 64, bps, 2)
    tickets = []
    for i, (m, n) in enumerate(zip(reqs, periods)):
        s = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, tau_scale=None)
        for q in range(m.n_species):
            s.set_counts(q, m.init[0, q])
        tickets.append((P.rdos_engine_submit(e, s.h, n, 1.0), s))
        time.sleep(0.003 * (i % 4))
    P.rdos_engine_drain(e)
    assert P.rdos_engine_launch_shape(e)["chains"] == 2
    mixed = []
    for t, s in tickets:
        P.rdos_engine_release(e, t)
        mixed.append(s.get_counts())
        s.close()
    P.rdos_engine_destroy(e)
    for m, n, got in zip(reqs, periods, mixed):
        np.testing.assert_array_equal(run_oracle(orc, m, n), got)


def test_timing_pass_counts_work(orc):
    """The timing pass launches the kernels directly, tallies the update
    kernel's work on the device and leaves results unchanged: the tets it
    updated are, in every period, the tet-realizations holding molecules at
    the start of the period (all of them under a reaction without reactants),
    and every count that is non-zero at the end of a period came from at least
    one of its additions."""
    import paper_1512_03126_amd as P

    m = small_request(41)
    n = 24
    note(f"timing pass work counters: {m.n_tets} tets, {m.n_species} species, {n} periods")
    rn = W.reaction_arrays(m.reactions)[0]
    o = orc.OracleSim(m.xyz, m.tets, m.D, m.reactions, seed=m.seed)
    for q in range(m.n_species):
        o.set_counts(q, m.init[0, q])
    tets = nnz_end = 0
    for _ in range(n):
        c = o.get_counts()
        tets += m.n_tets if (rn == 0).any() else int((c != 0).any(axis=0).sum())
        o.run_steps(1)
        nnz_end += int((o.get_counts() != 0).sum())
    e = P.rdos_engine_create(0, 0)
    P.rdos_engine_set_profiling(e, True)
    s = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, tau_scale=None)
    for q in range(m.n_species):
        s.set_counts(q, m.init[0, q])
    t = P.rdos_engine_submit(e, s.h, n, 1.0)
    P.rdos_engine_drain(e)
    P.rdos_engine_release(e, t)
    kt = P.rdos_engine_kernel_times(e)
    work = P.rdos_engine_work_counts(e)
    got = s.get_counts()
    # timed without the tally: launches counted, the last tallies kept, results unchanged
    P.rdos_engine_set_profiling(e, True, tally=False)
    t = P.rdos_engine_submit(e, s.h, 6, 1.0)
    P.rdos_engine_drain(e)
    P.rdos_engine_release(e, t)
    kt2 = P.rdos_engine_kernel_times(e)
    assert kt2["update_launches"] == kt2["scan_launches"] == 6 and kt2["update_ms"] > 0
    assert P.rdos_engine_work_counts(e) == work
    o2 = orc.OracleSim(m.xyz, m.tets, m.D, m.reactions, seed=m.seed)
    for q in range(m.n_species):
        o2.set_counts(q, m.init[0, q])
    o2.run_steps(n + 6)
    np.testing.assert_array_equal(o2.get_counts(), s.get_counts())
    P.rdos_engine_destroy(e)
    s.close()
    np.testing.assert_array_equal(o.get_counts(), got)
    # a run's last periods, fewer than a chunk, are launched directly, as many
    # as are left: one launch pair per period and none idle
    assert kt["update_launches"] == kt["scan_launches"] == n
    assert work["tets"] == tets
    assert nnz_end <= work["additions"] <= 5 * m.n_species * tets
    assert 0 < work["transfers"] <= work["additions"]
    assert work["transfers"] <= 4 * m.n_species * tets


def test_ten_species_in_the_engine(orc):
    """A 10-species model of the shape of Sec. III.C served by the engine:
    once in the timing pass (its wide instances tally work per wavefront:
    the tets updated equal the tet-realizations holding molecules at the
    start of every period) and once as small work (every period of the run
    in one cooperative launch); both bit for bit against the oracle."""
    import paper_1512_03126_amd as P

    m = W.ten_species(seed=7)
    n = 30
    note(f"ten species in the engine: {m.n_tets} tets, {n} periods, timing pass then one launch")
    o = orc.OracleSim(m.xyz, m.tets, m.D, m.reactions, seed=m.seed)
    for q in range(10):
        o.set_counts(q, m.init[0, q])
    tets = 0
    for _ in range(n):
        tets += int((o.get_counts() != 0).any(axis=0).sum())
        o.run_steps(1)
    want = o.get_counts()
    for profiling in (True, False):
        e = P.rdos_engine_create(0, 0)
        P.rdos_engine_set_profiling(e, profiling)
        s = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, tau_scale=None)
        for q in range(10):
            s.set_counts(q, m.init[0, q])
        t = P.rdos_engine_submit(e, s.h, n, 1.0)
        P.rdos_engine_drain(e)
        P.rdos_engine_release(e, t)
        if profiling:
            work = P.rdos_engine_work_counts(e)
            assert work["tets"] == tets
            assert 0 < work["transfers"] <= work["additions"]
        P.rdos_engine_destroy(e)
        np.testing.assert_array_equal(want, s.get_counts())
        s.close()


def serving_size_request(i, species=6, t_lo=1e5, t_hi=2.5e5):
    """A request of the serving mix's middle sizes (jittered lattice of
    1e5-2.5e5 tets) with `species` species and at least two reactions: the
    first seed of a fixed sequence that draws one."""
    for j in range(1000):
        m = W.serving_request(np.random.default_rng([91, i, j]), t_lo=t_lo, t_hi=t_hi, max_species=species)
        if m.n_species == species and len(m.reactions) >= 2:
            return m
    raise AssertionError("no request of that shape in the first 1000 seeds")


def test_serving_size_request_in_a_mix(orc):
    """One request at the serving mix's sizes (>= 1e5 tets, 6 species, random
    reactions) batched with small ones of 1-4 species in one engine: every
    count of every request equals the oracle's after its periods."""
    import paper_1512_03126_amd as P

    big = serving_size_request(0)
    assert big.n_tets >= 100000 and big.n_species == 6
    reqs = [big] + [small_request(50 + i) for i in range(4)]
    periods = [48, 30, 48, 62, 20]
    note(f"serving-size mix: {big.n_tets} tets x 6 species + 4 small requests")
    e = P.rdos_engine_create(0, 0)
    tickets = []
    for m, n in zip(reqs, periods):
        s = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, tau_scale=None)
        for q in range(m.n_species):
            s.set_counts(q, m.init[0, q])
        tickets.append((P.rdos_engine_submit(e, s.h, n, 1.0), s))
    P.rdos_engine_drain(e)
    mixed = []
    for t, s in tickets:
        P.rdos_engine_release(e, t)
        mixed.append(s.get_counts())
        s.close()
    P.rdos_engine_destroy(e)
    for k, (m, n, got) in enumerate(zip(reqs, periods, mixed)):
        want = run_oracle(orc, m, n)
        assert np.array_equal(want, got), (k, m.n_tets, m.n_species, int((want != got).sum()))
    assert int(mixed[0].sum()) > 0


def test_tuner_scores_and_shape_independence(orc):
    """A work list large enough to be tuned (48 realizations x 48,000 tets,
    2256 tiles): every candidate shape is scored in both passes, the kept
    shape has the lowest mean time per period, and the counts equal a run
    with a fixed shape, a run from the cached shape (no scores of its own)
    and, for one realization, the oracle."""
    import paper_1512_03126_amd as P

    m = W.abc_lattice(n=20, a=0.1e-6, seed=3, n_realizations=48)
    n = 320
    note(f"tuner: {m.n_realizations} x {m.n_tets} tets, {n} periods, tuned against a fixed shape")
    out = []
    for fixed in (None, (16, 1024, 1, 1), "cached"):
        e = P.rdos_engine_create(0, 0)
        if isinstance(fixed, tuple):
            P.rdos_engine_set_shape(e, *fixed)
        s = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, n_realizations=m.n_realizations)
        for r in range(m.n_realizations):
            for q in range(m.n_species):
                s.set_counts(q, m.init[r, q], realization=r)
        t = P.rdos_engine_submit(e, s.h, n, 1.0)
        P.rdos_engine_drain(e)
        P.rdos_engine_release(e, t)
        shape = P.rdos_engine_launch_shape(e)
        scores = P.rdos_engine_tuner_scores(e)
        P.rdos_engine_destroy(e)
        out.append([s.get_counts(None, realization=r) for r in range(m.n_realizations)])
        s.close()
        if fixed == "cached":   # a second engine on the same size bucket starts from the tuned shape
            assert shape["source"] == "cached", shape
            assert all(c["ms_first"] == 0 and c["ms_second"] == 0 for c in scores), scores
            continue
        if fixed:
            assert shape["source"] == "fixed"
            continue
        assert shape["source"] == "tuned", shape
        assert len(scores) >= 2
        assert all(c["ms_first"] > 0 and c["ms_second"] > 0 for c in scores), scores
        mean = [0.5 * (c["ms_first"] + c["ms_second"]) for c in scores]
        best = scores[int(np.argmin(mean))]
        assert (best["scan_grid"], best["update_blocks_per_segment"], best["chains"]) == \
            (shape["scan_grid"], shape["update_blocks_per_segment"], shape["chains"]), (shape, scores)
    for r in range(m.n_realizations):
        np.testing.assert_array_equal(out[0][r], out[1][r])
        np.testing.assert_array_equal(out[0][r], out[2][r])
    o = orc.OracleSim(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, realization=7)
    for q in range(m.n_species):
        o.set_counts(q, m.init[7, q])
    o.run_steps(n)
    np.testing.assert_array_equal(o.get_counts(), out[0][7])


@pytest.mark.parametrize("shape", [None, (8, 64, 1, 2), (8, 64, 0, 2)])
def test_zeroth_order_reaction_in_the_engine(orc, shape):
    """A reaction without reactants (0 -> A, Sec. III.A's production) makes
    every tet of its simulation run each period, whatever the occupancy map
    holds.  Two such simulations (one production everywhere, one restricted
    to a region) batched with one without, through the one-launch path for
    small work lists, two chains of two launches, and two fused chains:
    every count of every realization against the oracle."""
    import paper_1512_03126_amd as P

    xyz, tets = W.tiny_lattice(4, 0.2e-6, jitter_frac=0.2, seed=12)
    T = tets.shape[0]
    D = [1e-12, 0.6e-12, 0.3e-12]
    base = [([0, 1], [2], 3e8), ([2], [0, 1], 400.0)]
    models = [(base + [([], [0], 3e-5)], None, 2, 31), (base + [([], [1], 8e-5)], {2: np.arange(0, T, 7)}, 2, 32),
              (base, None, 3, 33)]
    periods = 60
    note(f"zeroth-order production in the engine: {T} tets, shape {shape}")
    e = P.rdos_engine_create(0, 0)
    if shape is not None:
        P.rdos_engine_set_shape(e, *shape)
    rng = np.random.default_rng(5)
    runs = []
    P.rdos_engine_hold(e, True)
    for rx, regions, rz, seed in models:
        init = rng.integers(0, 4, size=(rz, 3, T)).astype(np.int32)
        init[:, :, rng.random(T) < 0.7] = 0   # sparse: the map, not the production, decides most tets
        s = P.Simulation(xyz, tets, D, rx, seed=seed, n_realizations=rz, tau_scale=None, regions=regions)
        for r in range(rz):
            for q in range(3):
                s.set_counts(q, init[r, q], realization=r)
        runs.append((s, rx, regions, rz, seed, init, P.rdos_engine_submit(e, s.h, periods, 1.0)))
    P.rdos_engine_hold(e, False)
    P.rdos_engine_drain(e)
    if shape is not None:
        assert P.rdos_engine_launch_shape(e)["chains"] == 2
    for s, rx, regions, rz, seed, init, t in runs:
        P.rdos_engine_release(e, t)
        for r in range(rz):
            o = orc.OracleSim(xyz, tets, D, rx, seed=seed, realization=r)
            for rid, tl in (regions or {}).items():
                o.set_reaction_region(rid, tl)
            for q in range(3):
                o.set_counts(q, init[r, q])
            o.run_steps(periods)
            np.testing.assert_array_equal(o.get_counts(), s.get_counts(None, realization=r))
        s.close()
    P.rdos_engine_destroy(e)


@pytest.mark.parametrize("shape", [None, (8, 64, 1, 2), (8, 64, 0, 2)])
def test_method_options_mixed_in_the_engine(orc, shape):
    """Simulations with different method options in one work list: transfer
    form 1 (the closing alternative of Sec. II.B) beside form 0 makes the
    whole list run the scaled update instance, in which each simulation must
    still follow its own form; first-order splitting, a split threshold of 2
    and outlier relaxation ride along.  Through the one-launch path, two
    chains of two launches and two fused chains, every count of every
    realization against the oracle."""
    import paper_1512_03126_amd as P

    xyz, tets = W.tiny_lattice(4, 0.2e-6, jitter_frac=0.2, seed=13)
    T = tets.shape[0]
    D = [1e-12, 0.6e-12, 0.3e-12]
    rx = [([0, 1], [2], 3e8), ([2], [0, 1], 400.0), ([0], [], 20.0)]
    opts = [dict(transfer_form=1), dict(), dict(occupancy_correction=False, split_threshold=2),
            dict(tau_outliers=5, transfer_form=1)]
    periods = 50
    note(f"method options mixed in the engine: {T} tets, shape {shape}")
    e = P.rdos_engine_create(0, 0)
    if shape is not None:
        P.rdos_engine_set_shape(e, *shape)
    rng = np.random.default_rng(8)
    runs = []
    P.rdos_engine_hold(e, True)
    for k, o in enumerate(opts):
        rz = 2
        init = rng.integers(0, 40, size=(rz, 3, T)).astype(np.int32)
        init[:, 0, ::5] += 60   # some tets with many molecules: the sequential-binomial branch
        s = P.Simulation(xyz, tets, D, rx, seed=40 + k, n_realizations=rz, tau_scale=None, **o)
        for r in range(rz):
            for q in range(3):
                s.set_counts(q, init[r, q], realization=r)
        runs.append((s, o, rz, 40 + k, init, P.rdos_engine_submit(e, s.h, periods, 1.0)))
    P.rdos_engine_hold(e, False)
    P.rdos_engine_drain(e)
    for s, o, rz, seed, init, t in runs:
        P.rdos_engine_release(e, t)
        for r in range(rz):
            orc_sim = orc.OracleSim(xyz, tets, D, rx, seed=seed, realization=r)
            orc_sim.set_first_order(not o.get("occupancy_correction", True))
            orc_sim.set_split_threshold(o.get("split_threshold", 10))
            orc_sim.set_transfer_form(o.get("transfer_form", 0))
            orc_sim.set_tau_outliers(o.get("tau_outliers", 0))
            for q in range(3):
                orc_sim.set_counts(q, init[r, q])
            orc_sim.run_steps(periods)
            np.testing.assert_array_equal(orc_sim.get_counts(), s.get_counts(None, realization=r), str(o))
        s.close()
    P.rdos_engine_destroy(e)
