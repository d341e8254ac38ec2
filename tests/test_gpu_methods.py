"""Method options on the GPU against the oracle, bit for bit: first-order
splitting, the split threshold, tau outlier relaxation, localized reactions
(the building blocks of the tube-with-influx validation) and the
one-multinomial transfer form."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

RX = [([0, 1], [2], 3e8), ([2], [0, 1], 400.0), ([], [1], 3e-5), ([0], [], 50.0)]
D = [1e-12, 2e-12, 0.5e-12]


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def pair(P, orc, xyz, tets, init, seed, occ=True, thr=10, k=0, regions=None, form=0):
    T = tets.shape[0]
    g = P.Simulation(xyz, tets, D, RX, seed=seed, n_realizations=init.shape[0], occupancy_correction=occ,
                     split_threshold=thr, tau_outliers=k, regions=regions, transfer_form=form)
    os_ = []
    for r in range(init.shape[0]):
        o = orc.OracleSim(xyz, tets, D, RX, seed=seed, realization=r)
        o.set_first_order(not occ)
        o.set_split_threshold(thr)
        o.set_transfer_form(form)
        o.set_tau_outliers(k)
        for rid, tl in (regions or {}).items():
            o.set_reaction_region(rid, tl)
        for s in range(len(D)):
            o.set_counts(s, init[r, s])
            g.set_counts(s, init[r, s], realization=r)
        os_.append(o)
    assert g.tau == os_[0].tau
    return g, os_


@pytest.mark.parametrize("occ,thr,k,use_region,form", [(False, 10, 0, False, 0), (True, 1, 0, False, 0),
                                                       (True, 40, 0, True, 0), (True, 10, 9, False, 0),
                                                       (False, 3, 25, True, 0), (True, 10, 0, False, 1),
                                                       (True, 2, 0, True, 1), (False, 60, 7, False, 1)])
def test_method_options_every_period(orc, occ, thr, k, use_region, form):
    import paper_1512_03126_amd as P

    xyz, tets = W.tiny_lattice(3, 0.2e-6, jitter_frac=0.2, seed=6)
    T = tets.shape[0]
    rng = np.random.default_rng(thr + 7 * k)
    init = rng.integers(0, 30, size=(2, len(D), T)).astype(np.int32)
    init[:, 0, ::3] += 200          # some tets with many molecules: the sequential-binomial branch
    regions = {2: np.arange(0, T, 5, dtype=np.int32), 3: np.arange(T // 2, T, dtype=np.int32)} if use_region else None
    note(f"method options occ={occ} threshold={thr} outliers={k} regions={use_region} transfer form={form}")
    g, os_ = pair(P, orc, xyz, tets, init, seed=5 + k, occ=occ, thr=thr, k=k, regions=regions, form=form)
    for period in range(30):
        g.step(1)
        for r, o in enumerate(os_):
            o.step()
            got, want = g.get_counts(None, realization=r), o.get_counts()
            assert np.array_equal(got, want), (period, r, int((got != want).sum()))
    g.close()


def test_split_threshold_tuner():
    """The measured switch point of the split (Sec. II.B): from the returned
    threshold on, the sequential binomials are never slower than one draw
    per molecule, whose cost grows with n."""
    import paper_1512_03126_amd as P

    note("split threshold tuner")
    n_max = 160
    r = P.rdos_tune_split_threshold(0, n_max)
    one, seq, t = r["ms_one_by_one"], r["ms_sequential"], r["threshold"]
    note(f"switch point {t}; n=1,10,{n_max}: one-by-one {one[[0, 9, n_max - 1]]} ms, "
         f"sequential {seq[[0, 9, n_max - 1]]} ms")
    assert 1 <= t <= n_max + 1
    assert (one > 0).all() and (seq > 0).all()
    assert (seq[t - 1:] <= one[t - 1:]).all()
    if t > 1:
        assert seq[t - 2] > one[t - 2]
    assert one[n_max - 1] > 4 * one[3]    # one draw per molecule: cost grows with n
    with pytest.raises(P.RdosError):
        P.rdos_tune_split_threshold(0, 1)


# Wider chemistries for the kernel instances sized for 5-6 and 7-8 species
# (per-lane LDS and register budget depend on the species bound): A+B<->C,
# a conversion chain, a pair that consumes and a homodimer that produces.
WIDE_RX = {
    6: [([0, 1], [2], 3e8), ([2], [0, 1], 400.0), ([3], [4], 60.0), ([4, 5], [3], 2e8), ([5, 5], [1], 1e8),
        ([1], [5], 20.0)],
    8: [([0, 1], [2], 3e8), ([2], [0, 1], 400.0), ([3], [4], 60.0), ([4, 5], [3], 2e8), ([5, 5], [1], 1e8),
        ([6], [7], 30.0), ([7], [6], 25.0), ([6, 7], [], 1e8), ([1], [5], 20.0)],
    16: [([0, 1], [2], 3e8), ([2], [0, 1], 400.0), ([3], [4], 60.0), ([4, 5], [3], 2e8), ([5, 5], [1], 1e8),
         ([6], [7], 30.0), ([7], [6], 25.0), ([6, 7], [], 1e8), ([1], [5], 20.0), ([8, 9], [10], 2e8),
         ([10], [8, 9], 300.0), ([11], [12], 40.0), ([12, 12], [11], 1e8), ([13, 14], [15], 3e8),
         ([15], [13, 14, 9], 50.0), ([9], [], 10.0)],
}


@pytest.mark.parametrize("S,form,occ,thr", [(5, 1, True, 10), (6, 1, True, 3), (6, 0, True, 10),
                                            (7, 1, False, 10), (8, 1, True, 40), (8, 0, True, 2),
                                            (10, 1, True, 10), (12, 0, True, 10), (16, 1, True, 4),
                                            (16, 0, False, 10)])
def test_wide_chemistry_every_period(orc, S, form, occ, thr):
    """Transfer form 1 (the closing alternative of Sec. II.B) and form 0 with
    5-16 species: the update instances for the 6-, 8-, 10- and 16-species bounds
    and the matching scan instances, bit for bit against the oracle after
    every one of 32 periods (Algorithm 1, Steps 2-3)."""
    import paper_1512_03126_amd as P

    bound = 6 if S <= 6 else (8 if S <= 8 else 16)
    rx = [r for r in WIDE_RX[bound] if max(r[0] + r[1] + [0]) < S]
    Ds = [1e-12, 2e-12, 0.5e-12, 3e-12, 1.5e-12, 0.0, 4e-12, 1e-12,
          2e-12, 0.7e-12, 1e-12, 0.0, 3e-12, 1.2e-12, 0.4e-12, 2.2e-12][:S]
    xyz, tets = W.tiny_lattice(3, 0.2e-6, jitter_frac=0.2, seed=11 + S)
    T = tets.shape[0]
    rng = np.random.default_rng(100 * S + thr)
    init = rng.integers(0, 25, size=(2, S, T)).astype(np.int32)
    init[:, 0, ::4] += 150           # the sequential-binomial branch
    init[:, S - 1, 1::5] += 60
    note(f"wide chemistry: {S} species, {len(rx)} reactions, transfer form {form}, occ={occ}, threshold {thr}")
    g = P.Simulation(xyz, tets, Ds, rx, seed=21 + S, n_realizations=2, occupancy_correction=occ,
                     split_threshold=thr, transfer_form=form)
    os_ = []
    for r in range(2):
        o = orc.OracleSim(xyz, tets, Ds, rx, seed=21 + S, realization=r)
        o.set_first_order(not occ)
        o.set_split_threshold(thr)
        o.set_transfer_form(form)
        for q in range(S):
            o.set_counts(q, init[r, q])
            g.set_counts(q, init[r, q], realization=r)
        os_.append(o)
    assert g.tau == os_[0].tau
    for period in range(32):
        g.step(1)
        for r, o in enumerate(os_):
            o.step()
            got, want = g.get_counts(None, realization=r), o.get_counts()
            assert np.array_equal(got, want), (period, r, int((got != want).sum()))
    g.close()


def test_tags_wrap_without_a_zeroth_order_reaction(orc):
    """The occupancy bytes hold a tag of the period they mark, repeating every
    255 periods, and each map serves every other period, so a byte untouched
    for a multiple of 510 periods matches again.  A+B<->C (no reaction without
    reactants, so the map decides which tets run) for 1100 periods, compared
    with the oracle at checkpoints on both sides of 510 and 1020."""
    import paper_1512_03126_amd as P

    xyz, tets = W.tiny_lattice(4, 0.2e-6, jitter_frac=0.2, seed=8)
    T = tets.shape[0]
    rx = [([0, 1], [2], 3e8), ([2], [0, 1], 400.0)]
    Ds = [1e-12, 1e-12, 0.5e-12]
    rng = np.random.default_rng(9)
    init = np.zeros((3, T), np.int32)
    for q in range(2):
        np.add.at(init[q], rng.integers(0, T, 12), 1)   # sparse: most groups stay empty for long spells
    note(f"tag wrap: {T} tets, 1100 periods")
    g = P.Simulation(xyz, tets, Ds, rx, seed=4)
    o = orc.OracleSim(xyz, tets, Ds, rx, seed=4)
    for q in range(3):
        g.set_counts(q, init[q])
        o.set_counts(q, init[q])
    done = 0
    for stop in (250, 509, 510, 511, 765, 1019, 1020, 1021, 1100):
        g.step(stop - done)
        o.run_steps(stop - done)
        done = stop
        got, want = g.get_counts(), o.get_counts()
        assert np.array_equal(got, want), (stop, int((got != want).sum()))
    assert int(got.sum()) > 0
    g.close()


def test_ten_species_model_every_period(orc):
    """A model of the shape of Sec. III.C (10 species, 4 reversible
    reactions, D of 10-100 um^2/s) in three realizations: the 16-species
    kernel instances, bit for bit against the oracle after every one of 40
    periods."""
    import paper_1512_03126_amd as P

    m = W.ten_species(n_realizations=3, seed=5)
    note(f"ten species: {m.n_tets} tets, {len(m.reactions)} reactions, 3 realizations, 40 periods")
    g = P.Simulation(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, n_realizations=3)
    os_ = []
    for r in range(3):
        o = orc.OracleSim(m.xyz, m.tets, m.D, m.reactions, seed=m.seed, realization=r)
        for q in range(10):
            o.set_counts(q, m.init[r, q])
            g.set_counts(q, m.init[r, q], realization=r)
        os_.append(o)
    assert g.tau == os_[0].tau
    fired = 0
    for period in range(40):
        g.step(1)
        for r, o in enumerate(os_):
            o.step()
            got, want = g.get_counts(None, realization=r), o.get_counts()
            assert np.array_equal(got, want), (period, r, int((got != want).sum()))
        fired += int((got[2] + got[4] + got[7] + got[9]).sum() != (m.init[2, [2, 4, 7, 9]]).sum())
    assert fired > 0   # the reactions ran
    g.close()


def test_atomic_probe_rate():
    """The random-atomic probe that prices the update's count additions: a
    positive, plausible rate, and the same order of magnitude for a buffer
    16 times smaller."""
    import paper_1512_03126_amd as P

    note("random-atomic probe: 2^22 additions into 1 GiB and into 64 MiB")
    big = P.rdos_atomic_probe(0, 1 << 30, 1 << 22, 3)
    small = P.rdos_atomic_probe(0, 64 << 20, 1 << 22, 3)
    note(f"random atomics: {big:.3e}/s into 1 GiB, {small:.3e}/s into 64 MiB")
    assert 1e9 < big < 1e13 and 1e9 < small < 1e13
    assert small > 0.5 * big
    with pytest.raises(P.RdosError):
        P.rdos_atomic_probe(0, 1 << 20, 0, 1)
