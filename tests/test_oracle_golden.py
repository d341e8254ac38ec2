"""The oracle against numbers the paper prints (tests/golden/paper_values.txt)."""
import math
import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.txt")


def golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                name, value = line.split()[:2]
                vals[name] = float(value)
    return vals


def _one_interior_tet(orc, tau_scale, n_molecules, seed=1):
    """A 4^3 Kuhn lattice, one species, all molecules in one tet whose four
    faces are interior; returns (molecules that left after one period, zeta
    of that tet)."""
    xyz, tets = W.kuhn_lattice(4, 0.1e-6)
    o = orc.OracleSim(xyz, tets, [1e-12], [], tau_scale=tau_scale, seed=seed)
    geo = o.geometry()
    t = int(np.nonzero((geo["nbr"] >= 0).all(axis=1))[0][0])
    c = np.zeros(tets.shape[0], np.int32)
    c[t] = n_molecules
    o.set_counts(0, c)
    o.run_steps(1)
    zeta = min(1.0, (o.tau * 1e-12) * geo["g"][t])
    return n_molecules - int(o.get_counts(0)[t]), zeta


def test_leave_probability_is_zeta_not_the_exact_cdf(orc):
    """At zeta = 1 the exact method would move 63.2% of the molecules in the
    mean transfer time; the splitting method compensates the delay and moves
    each with probability zeta, so all of them."""
    g = golden()
    assert round(1.0 - math.exp(-1.0), 3) == g["issa_leave_probability_zeta1"]
    n = 100000
    left, zeta = _one_interior_tet(orc, 1.0, n)
    assert zeta > 1.0 - 1e-12
    assert left == n  # not 0.632 n
    for scale in (0.5, 0.1):
        left, zeta = _one_interior_tet(orc, scale, n)
        sd = math.sqrt(n * zeta * (1.0 - zeta))
        assert abs(left - n * zeta) < 4.0 * sd, (scale, left, n * zeta, sd)


def test_default_split_threshold_is_the_papers(orc):
    """Ten molecules leave a tet at zeta = 1: the default run is the run with
    the paper's threshold set explicitly, and not the one with 11 (whose
    one-by-one draws differ)."""
    thr = int(golden()["split_threshold"])

    def run(threshold):
        xyz, tets = W.kuhn_lattice(4, 0.1e-6)
        o = orc.OracleSim(xyz, tets, [1e-12], [], tau_scale=1.0, seed=4)
        t = int(np.nonzero((o.geometry()["nbr"] >= 0).all(axis=1))[0][0])
        if threshold is not None:
            o.set_split_threshold(threshold)
        c = np.zeros(tets.shape[0], np.int32)
        c[t] = thr
        o.set_counts(0, c)
        o.run_steps(1)
        return o.get_counts(0)

    default = run(None)
    assert np.array_equal(default, run(thr))
    assert not np.array_equal(default, run(thr + 1))


def test_fig6_model_uses_the_printed_rate():
    g = golden()
    m = W.production_annihilation()
    k2 = m.reactions[1][2]  # 1/(M s)
    assert m.reactions[1][0] == [0, 0]
    assert abs(k2 * 1e-6 - g["fig6_k2_per_uM_s"]) < 1e-9
