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
