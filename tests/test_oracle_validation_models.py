"""Pins of the validation-model machinery (Sec. III.B) on the CPU.

* The well-mixed stationary law of production and pair annihilation (the
  analytic form fitted in Fig. 6) against a direct solve of the truncated
  master equation.
* The sum-tree exact SSA against the plain direct-method ISSA (same process,
  different bookkeeping) in law.
* The oracle's splitting method on the production / annihilation model
  against the exact SSA on a small mesh: same stationary law of the total.
"""
import numpy as np
import pytest
from scipy import stats

import workloads as W
from tests.helpers import annihilation_pmf, issa_run


@pytest.mark.parametrize("a", [0.3, 2.0, 40.0, 1800.0])
def test_annihilation_law_is_the_master_equation_solution(a):
    n_max = int(6 * a ** 0.5 + 40)
    p = annihilation_pmf(a, n_max)
    Q = np.zeros((n_max + 1, n_max + 1))
    for n in range(n_max + 1):
        if n < n_max:
            Q[n, n + 1] += a               # births (time in units of 1 / mu)
        if n >= 2:
            Q[n, n - 2] += n * (n - 1.0)   # one pair annihilates
        Q[n, n] = -Q[n].sum()
    A = Q.T.copy()
    A[-1, :] = 1.0
    rhs = np.zeros(n_max + 1)
    rhs[-1] = 1.0
    exact = np.linalg.solve(A, rhs)
    assert abs(p.sum() - 1.0) < 1e-12
    assert np.abs(p - exact).max() < 1e-12


def _tiny_model(D=1e-11, mean=12.0, n_realizations=1):
    return W.production_annihilation(n=2, D=D, mean=mean, n_realizations=n_realizations, seed=3)


def test_tree_ssa_matches_direct_ssa(orc):
    m = _tiny_model(D=1e-12)
    geo = orc.OracleSim.from_model(m).geometry()
    ts = 0.5 + 0.25 * np.arange(1500)
    a = issa_run(geo, m.D, m.reactions, m.init[0], ts, seed=11).sum(axis=(1, 2))
    b = issa_run(geo, m.D, m.reactions, m.init[0], ts, seed=12, tree=True).sum(axis=(1, 2))
    assert stats.ks_2samp(a, b).pvalue > 1e-3
    assert abs(a.mean() - b.mean()) < 4 * np.sqrt((a.var() + b.var()) / len(a))


def test_splitting_matches_exact_ssa_production_annihilation(orc):
    R = 400
    m = _tiny_model(n_realizations=R)
    times = (0.4, 0.7, 1.0)
    split = []
    for r in range(R):
        o = orc.OracleSim.from_model(m, realization=r)
        for t in times:
            o.run_until(t)
            split.append(int(o.get_counts(0).sum()))
    split = np.array(split)
    geo = orc.OracleSim.from_model(m).geometry()
    exact = issa_run(geo, m.D, m.reactions, m.init[0], 1.0 + 0.3 * np.arange(1500), seed=21,
                     tree=True).sum(axis=(1, 2))
    assert stats.ks_2samp(split, exact).pvalue > 1e-3
    assert abs(split.mean() - exact.mean()) < 4 * np.sqrt(split.var() / len(split) + exact.var() / len(exact))
