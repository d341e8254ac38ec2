"""The reaction-diffusion validation models of Sec. III.B on the GPU.

Tube with constant influx at both ends (Fig. 7).

A production reaction restricted to the two end cell layers of a bar feeds
molecules that diffuse towards the middle.  The network is linear, so the mean
of the exact process solves dM/dt = Q^T M + s on the mesh (Q the hop
generator), computed here with a matrix exponential.  Thousands of
realizations of the splitting method, with and without the occupancy
correction (Sec. II.C), are averaged per cell layer and compared with it: the
first-order variant (diffusion from the count at the end of the period) must
err more than the occupancy method, whose error must stay at the level of the
sampling noise, as in Fig. 7(c)-(d).  A few realizations are also compared
with the oracle bit for bit.

Production and second-order degradation (Fig. 6): stationary totals against
an exact SSA of the same master equation, and the apparent second-order rate
from a fit of the well-mixed law.
"""
import sys

import numpy as np
import pytest

import workloads as W
from tests.helpers import exact_mean_linear

pytestmark = pytest.mark.gpu

N_REALIZATIONS = 8000
KP = 2e-3          # molecules per (s m^3) scaled: about 480 molecules in the bar at t_end


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def layer_matrix(model, a=0.1e-6):
    bc = model.xyz[model.tets].mean(axis=1)
    layer = (bc[:, 0] / a).astype(int)
    P = np.zeros((model.n_tets, layer.max() + 1))
    P[np.arange(model.n_tets), layer] = 1.0
    return P


def run_profiles(P_mod, model, occupancy):
    g = P_mod.Simulation.from_model(model, n_realizations=N_REALIZATIONS, occupancy_correction=occupancy)
    g.run_until(model.t_end)
    g.synchronize()
    counts = np.stack([g.get_counts(0, realization=r) for r in range(N_REALIZATIONS)])
    tau = g.tau
    g.close()
    return counts, tau


def test_tube_influx_occupancy_beats_first_order(orc):
    import paper_1512_03126_amd as P_mod

    model = W.tube_influx(kp=KP)
    P = layer_matrix(model)
    o = orc.OracleSim.from_model(model)
    geo = o.geometry()
    prod = np.zeros(model.n_tets)
    ends = model.regions[0]
    prod[ends] = KP * geo["nav"][ends]
    exact = exact_mean_linear(geo, model.D[0], prod, model.t_end) @ P
    err, se = {}, {}
    for occupancy in (True, False):
        note(f"tube influx occupancy={occupancy} realizations={N_REALIZATIONS}")
        counts, tau = run_profiles(P_mod, model, occupancy)
        assert tau == o.tau
        # sampled realizations against the oracle, bit for bit
        for r in (0, 4321, N_REALIZATIONS - 1):
            ref = orc.OracleSim.from_model(model, realization=r)
            ref.set_first_order(not occupancy)
            ref.run_until(model.t_end)
            assert np.array_equal(counts[r], ref.get_counts(0)), (occupancy, r)
        prof = counts.astype(np.float64) @ P
        mean = prof.mean(axis=0)
        err[occupancy] = float(np.abs(mean - exact).mean())
        se[occupancy] = float((prof.std(axis=0) / np.sqrt(N_REALIZATIONS)).mean())
        # production does not depend on the method: the total is Poisson
        total = prof.sum(axis=1)
        assert abs(total.mean() - exact.sum()) < 4 * np.sqrt(exact.sum() / N_REALIZATIONS)
    note(f"mean |error| per layer: occupancy {err[True]:.4f} first-order {err[False]:.4f} "
         f"(standard error {se[True]:.4f})")
    assert err[True] < 4 * se[True]
    assert err[False] > 1.3 * err[True]


# ---------------------------------------------------------------------------
# Production and second-order degradation (Sec. III.B, Fig. 6)
# ---------------------------------------------------------------------------
FIG6_R = 4096
FIG6_TIMES = (0.4, 0.7, 1.0)      # s; relaxation takes about 0.05 s, so the samples are independent
FIG6_ISSA_SAMPLES = 3000          # per exact run, sampled every 0.3 s after 1 s
FIG6_ISSA_SEEDS = (1, 2, 3, 4)    # four independent exact runs (in threads: the C call drops the GIL)


def fit_k2(samples, model):
    """Apparent second-order rate: maximum-likelihood fit of the well-mixed
    stationary law (births lam, pair annihilation mu n (n - 1)) with lam
    known, as in Fig. 6(a)-(c)."""
    import math

    from scipy.optimize import minimize_scalar

    from tests.helpers import annihilation_pmf

    nav = 6.02214076e23 * float(np.abs(np.linalg.det(
        model.xyz[model.tets[:, 1:]] - model.xyz[model.tets[:, :1]])).sum() / 6.0) * 1e3
    lam = model.reactions[0][2] * nav
    mu = model.reactions[1][2] / nav
    counts = np.bincount(np.asarray(samples, np.int64))

    def nll(log_a):
        p = annihilation_pmf(math.exp(log_a), len(counts) - 1)
        return -(counts * np.log(np.maximum(p, 1e-300))).sum()

    a0 = math.log(lam / mu)
    r = minimize_scalar(nll, bounds=(a0 - 2.0, a0 + 2.0), method="bounded")
    return lam / math.exp(r.x) * nav


def test_production_annihilation_matches_exact_issa(orc):
    """Stationary totals of the splitting method against an exact SSA of the
    same master equation on the same mesh: the same law (KS) and the same
    apparent second-order rate within 2% of k2 (Fig. 6(c)-(d): the error of
    the splitting method is comparable to that of the ISSA).  On this mesh
    both sit about 4% below the well-mixed rate (the spatial effect of the
    master equation itself); the fit's sampling spread is about 1%."""
    import paper_1512_03126_amd as P
    from scipy import stats

    from tests.helpers import issa_run

    m = W.production_annihilation(n_realizations=FIG6_R)
    note(f"production + annihilation: {FIG6_R} realizations on the GPU")
    g = P.Simulation.from_model(m)
    totals = np.zeros((FIG6_R, len(FIG6_TIMES)), np.int64)
    for j, t in enumerate(FIG6_TIMES):
        g.run_until(t)
        g.synchronize()
        for r in range(FIG6_R):
            totals[r, j] = int(g.get_counts(0, realization=r).sum())
        if j == 0:
            for r in (0, FIG6_R - 1):
                o = orc.OracleSim.from_model(m, realization=r)
                o.run_until(t)
                assert np.array_equal(g.get_counts(0, realization=r), o.get_counts(0)), r
    g.close()
    note("production + annihilation: exact SSA on the CPU")
    from concurrent.futures import ThreadPoolExecutor

    geo = orc.OracleSim.from_model(m).geometry()
    ts = 1.0 + 0.3 * np.arange(FIG6_ISSA_SAMPLES)
    with ThreadPoolExecutor(len(FIG6_ISSA_SEEDS)) as pool:
        runs = list(pool.map(lambda sd: issa_run(geo, m.D, m.reactions, m.init[0], ts, seed=sd, tree=True),
                             FIG6_ISSA_SEEDS))
    exact = np.concatenate([x.sum(axis=(1, 2)) for x in runs])
    split = totals.reshape(-1)
    k2 = m.reactions[1][2]
    ks = stats.ks_2samp(split, exact)
    k_split, k_exact = fit_k2(split, m) / k2, fit_k2(exact, m) / k2
    note(f"apparent k2 / k2: splitting {k_split:.4f}, exact SSA {k_exact:.4f}; KS p {ks.pvalue:.3g}")
    assert ks.pvalue > 1e-3
    assert abs(k_split - k_exact) < 0.02
    assert abs(k_split - 1.0) < 0.1 and abs(k_exact - 1.0) < 0.1
