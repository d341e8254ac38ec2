"""Pins of the oracle's binomial sampler and multinomial split (Sec. II.A-B).

The binomial draws are compared with the exact probability mass function
(scipy) by a chi-square test over a grid that reaches every branch: BINV
(n p < 10), BTRD (n p >= 10), the reflection p > 1/2 and the trivial cases.
The split is compared with the multinomial law it must produce: exhaustively
for the one-by-one branch, through marginals and covariances for the
sequential-binomial branch.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

ALPHA = 1e-3  # per case; every case is a fixed seeded draw, so the outcome is fixed


def _chi2_pvalue(observed, expected, min_expected=5.0):
    """Chi-square goodness of fit after merging bins with low expectation."""
    obs, exp = [], []
    acc_o = acc_e = 0.0
    for o, e in zip(observed, expected):
        acc_o += o
        acc_e += e
        if acc_e >= min_expected:
            obs.append(acc_o)
            exp.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0:
        if exp:
            obs[-1] += acc_o
            exp[-1] += acc_e
        else:
            obs.append(acc_o)
            exp.append(acc_e)
    obs, exp = np.array(obs), np.array(exp)
    if len(obs) < 2:
        return 1.0
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    return float(stats.chi2.sf(chi2, len(obs) - 1))


BINOMIAL_GRID = [
    (1, 0.3), (3, 0.5), (7, 0.05), (9, 0.999),        # tiny n
    (30, 0.2), (60, 0.16),                              # BINV, n p = 6, 9.6
    (50, 0.2), (100, 0.3), (400, 0.45),                 # BTRD, n p >= 10
    (40, 0.7), (2000, 0.93),                            # reflected into BTRD / BINV
    (1000, 0.5), (100000, 0.25),                        # BTRD, large
    (1000000, 5e-6), (50000, 1e-4),                     # BINV, large n small p
    (12, 0.9999999),                                    # reflected, p close to 1
]


@pytest.mark.parametrize("n,p", BINOMIAL_GRID)
def test_binomial_law(orc, n, p):
    count = 60000
    x = orc.binomial_many(n, p, seed=1000 + n, count=count)
    assert x.min() >= 0 and x.max() <= n
    lo, hi = int(x.min()), int(x.max())
    lo = max(0, min(lo, int(stats.binom.ppf(1e-9, n, p))))
    hi = min(n, max(hi, int(stats.binom.isf(1e-9, n, p))))
    ks = np.arange(lo, hi + 1)
    observed = np.bincount(x - lo, minlength=hi - lo + 1)[: hi - lo + 1]
    pmf = stats.binom.pmf(ks, n, p)
    # mass outside [lo, hi] goes to the end bins
    pmf[0] += stats.binom.cdf(lo - 1, n, p) if lo > 0 else 0.0
    pmf[-1] += stats.binom.sf(hi, n, p)
    pv = _chi2_pvalue(observed, pmf * count)
    assert pv > ALPHA, (n, p, pv)
    # the mean to within 4 standard errors
    sd = math.sqrt(n * p * (1 - p) / count)
    assert abs(x.mean() - n * p) <= 4 * sd + 1e-12


def test_binomial_trivial_cases(orc):
    assert (orc.binomial_many(0, 0.3, 1, 100) == 0).all()
    assert (orc.binomial_many(17, 0.0, 1, 100) == 0).all()
    assert (orc.binomial_many(17, 1.0, 1, 100) == 17).all()
    assert (orc.binomial_many(17, 1.5, 1, 100) == 17).all()
    assert (orc.binomial_many(5, -0.1, 1, 100) == 0).all()


def test_binomial_draw_accounting(orc):
    """Trivial cases consume no draws; the others consume at least one."""
    import ctypes as C

    j = C.c_uint32(0)
    assert orc.lib().orc_binomial(10, 1.0, 1, 0, 0, 0, 0, C.byref(j)) == 10 and j.value == 0
    assert orc.lib().orc_binomial(0, 0.4, 1, 0, 0, 0, 0, C.byref(j)) == 0 and j.value == 0
    orc.lib().orc_binomial(10, 0.4, 1, 0, 0, 0, 0, C.byref(j))
    assert j.value >= 1
    j2 = C.c_uint32(3)
    orc.lib().orc_binomial(1000, 0.4, 1, 0, 0, 0, 0, C.byref(j2))
    assert j2.value >= 4


def _multinomial_pmf(counts, probs):
    n = sum(counts)
    lp = math.lgamma(n + 1)
    for c, p in zip(counts, probs):
        if p == 0:
            if c:
                return 0.0
            continue
        lp += c * math.log(p) - math.lgamma(c + 1)
    return math.exp(lp)


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_split_one_by_one_is_multinomial(orc, n):
    w = np.array([0.1, 0.0, 0.35, 0.55])       # face 1 is a boundary face
    nbr = np.array([4, -1, 7, 9], dtype=np.int32)
    count = 40000
    out = orc.split_many(n, w, nbr, seed=77 + n, count=count)
    assert (out.sum(axis=1) == n).all()
    assert (out[:, 1] == 0).all()
    outcomes = [c for c in itertools.product(range(n + 1), repeat=3) if sum(c) == n]
    keys = {c: i for i, c in enumerate(outcomes)}
    obs = np.zeros(len(outcomes))
    for row in out[:, [0, 2, 3]]:
        obs[keys[tuple(int(v) for v in row)]] += 1
    pmf = np.array([_multinomial_pmf(c, [0.1, 0.35, 0.55]) for c in outcomes])
    assert abs(pmf.sum() - 1) < 1e-12
    assert _chi2_pvalue(obs, pmf * count) > ALPHA


@pytest.mark.parametrize("n", [10, 37, 500, 20000])
def test_split_sequential_binomials_is_multinomial(orc, n):
    w = np.array([0.2, 0.3, 0.05, 0.45])
    nbr = np.array([1, 2, 3, 4], dtype=np.int32)
    count = 30000
    out = orc.split_many(n, w, nbr, seed=991 + n, count=count).astype(np.float64)
    assert (out.sum(axis=1) == n).all()
    for f in range(4):
        # each face count is Binomial(n, w_f)
        x = out[:, f].astype(np.int64)
        lo, hi = int(x.min()), int(x.max())
        ks = np.arange(lo, hi + 1)
        pmf = stats.binom.pmf(ks, n, w[f])
        pmf[0] += stats.binom.cdf(lo - 1, n, w[f]) if lo > 0 else 0.0
        pmf[-1] += stats.binom.sf(hi, n, w[f])
        obs = np.bincount(x - lo, minlength=hi - lo + 1)
        assert _chi2_pvalue(obs, pmf * count) > ALPHA, (n, f)
    # covariances -n w_i w_j
    cov = np.cov(out.T)
    for i in range(4):
        for j in range(i + 1, 4):
            want = -n * w[i] * w[j]
            se = n * math.sqrt((w[i] * w[j]) * (1 + w[i] * w[j]) / count) * 1.2 + 1e-9
            assert abs(cov[i, j] - want) < 5 * se, (i, j, cov[i, j], want)


def test_split_single_interior_face_takes_all(orc):
    w = np.array([0.0, 1.0, 0.0, 0.0])
    nbr = np.array([-1, 3, -1, -1], dtype=np.int32)
    for n in (1, 9, 10, 12345):
        out = orc.split_many(n, w, nbr, seed=5, count=20)
        assert (out[:, 1] == n).all() and (out.sum(axis=1) == n).all()


def test_split_threshold_is_ten(orc):
    """Below 10 molecules one draw per molecule; at 10 the binomial chain."""
    import ctypes as C

    w = np.array([0.25, 0.25, 0.25, 0.25])
    nbr = np.array([1, 2, 3, 4], dtype=np.int32)
    o = np.zeros(4, np.int64)
    L = orc.lib()
    P = C.POINTER
    j9 = L.orc_split(9, w.ctypes.data_as(P(C.c_double)), nbr.ctypes.data_as(P(C.c_int32)), 1, 0, 0, 0, 0, 0,
                     o.ctypes.data_as(P(C.c_int64)))
    assert j9 == 9
    j10 = L.orc_split(10, w.ctypes.data_as(P(C.c_double)), nbr.ctypes.data_as(P(C.c_int32)), 1, 0, 0, 0, 0, 0,
                      o.ctypes.data_as(P(C.c_int64)))
    assert j10 <= 8  # at most 3 binomials of n p < 10 (BINV: one draw each unless it restarts)


@pytest.mark.parametrize("threshold,n", [(1, 7), (4, 7), (50, 30), (2, 120)])
def test_split_law_at_any_threshold(orc, threshold, n):
    """The switch point between one-by-one and the multinomial function only
    changes which draws are used (Sec. II.B): every face count stays
    Binomial(n, w_f)."""
    w = np.array([0.15, 0.35, 0.0, 0.5])
    nbr = np.array([2, 5, -1, 9], dtype=np.int32)
    count = 30000
    out = orc.split_many(n, w, nbr, seed=313 + threshold, count=count, threshold=threshold)
    assert (out.sum(axis=1) == n).all() and (out[:, 2] == 0).all()
    for f in (0, 1, 3):
        x = out[:, f]
        lo, hi = int(x.min()), int(x.max())
        ks = np.arange(lo, hi + 1)
        pmf = stats.binom.pmf(ks, n, w[f])
        pmf[0] += stats.binom.cdf(lo - 1, n, w[f]) if lo > 0 else 0.0
        pmf[-1] += stats.binom.sf(hi, n, w[f])
        obs = np.bincount(x - lo, minlength=hi - lo + 1)
        assert _chi2_pvalue(obs, pmf * count) > ALPHA, (threshold, n, f)


@pytest.mark.parametrize("n,zeta,threshold", [(7, 0.4, 10), (9, 1.0, 10), (60, 0.25, 10), (500, 0.8, 10),
                                               (30, 0.6, 50), (12, 0.9, 1)])
def test_split_scaled_is_the_same_law(orc, n, zeta, threshold):
    """The one-multinomial transfer form (Sec. II.B, last sentences): face f
    receives Binomial(n, zeta w_f), the total leaving is Binomial(n, zeta),
    and face counts have covariance -n zeta^2 w_i w_j -- the law of
    binomial(n, zeta) followed by the multinomial split."""
    w = np.array([0.15, 0.35, 0.0, 0.5])
    nbr = np.array([2, 5, -1, 9], dtype=np.int32)
    count = 30000
    out = orc.split_scaled_many(n, zeta, w, nbr, seed=4242 + n, count=count, threshold=threshold)
    assert (out[:, 2] == 0).all() and (out.sum(axis=1) <= n).all()

    def check(x, p):
        lo, hi = int(x.min()), int(x.max())
        ks = np.arange(lo, hi + 1)
        pmf = stats.binom.pmf(ks, n, p)
        pmf[0] += stats.binom.cdf(lo - 1, n, p) if lo > 0 else 0.0
        pmf[-1] += stats.binom.sf(hi, n, p)
        obs = np.bincount(x - lo, minlength=hi - lo + 1)
        return _chi2_pvalue(obs, pmf * count)

    for f in (0, 1, 3):
        assert check(out[:, f], zeta * w[f]) > ALPHA, (n, zeta, f)
    if zeta < 1.0:
        assert check(out.sum(axis=1), zeta) > ALPHA
    else:
        assert (out.sum(axis=1) == n).all() or (out.sum(axis=1) >= n - 1).mean() > 0.999
    cov = np.cov(out.astype(np.float64).T)
    for i, j in ((0, 1), (0, 3), (1, 3)):
        want = -n * zeta * zeta * w[i] * w[j]
        se = n * np.sqrt(zeta * w[i] * zeta * w[j] * (1 + zeta * w[i] * zeta * w[j]) / count) * 1.2 + 1e-9
        assert abs(cov[i, j] - want) < 5 * se, (i, j, cov[i, j], want)
