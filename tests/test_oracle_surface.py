"""Pins of the oracle's surface diffusion (transfer between surface
triangles, Sec. III.A, Fig. 5(c)-(d)) and surface reactions.

A triangle is the 2D subvolume: neighbours across edges, r_e = L_e/(A d_e)
(edge length over area times the distance between barycentres), g = sum r_e,
w_e = r_e / g, amounts in N_A A.  Checked against formulas computed here
independently, the exact law of a point source, the mean-square displacement
of the exact chain and 4 D t, and the well-mixed A+B<->C law.
"""
import math

import numpy as np
import pytest
from scipy import sparse, stats

import workloads as W

N_A = 6.02214076e23


def _independent_geometry(xyz, tris):
    """Areas by Heron's formula, barycentres, neighbours by an edge
    dictionary, r_e = L_e / (A d_e); no code shared with the oracle."""
    T = tris.shape[0]
    P = xyz[tris]                                      # [T, 3, 3]
    L = np.stack([np.linalg.norm(P[:, (e + 2) % 3] - P[:, (e + 1) % 3], axis=1) for e in range(3)], axis=1)
    s = L.sum(axis=1) / 2
    area = np.sqrt(np.maximum(s * (s - L[:, 0]) * (s - L[:, 1]) * (s - L[:, 2]), 0.0))
    bc = P.mean(axis=1)
    owners = {}
    for t in range(T):
        for e in range(3):
            key = tuple(sorted(int(tris[t, k]) for k in range(3) if k != e))
            owners.setdefault(key, []).append((t, e))
    nbr = -np.ones((T, 4), dtype=np.int64)
    for lst in owners.values():
        if len(lst) == 2:
            (t0, e0), (t1, e1) = lst
            nbr[t0, e0], nbr[t1, e1] = t1, t0
    r = np.zeros((T, 4))
    for t in range(T):
        for e in range(3):
            u = nbr[t, e]
            if u >= 0:
                r[t, e] = L[t, e] / (area[t] * np.linalg.norm(bc[u] - bc[t]))
    return area, nbr, r


def _transition_matrix(geo, D, tau):
    nbr, w, g = geo["nbr"], geo["w"], geo["g"]
    T = nbr.shape[0]
    zeta = np.minimum(1.0, (tau * D) * g)
    rows, cols, vals = [], [], []
    for t in range(T):
        rows.append(t)
        cols.append(t)
        vals.append(1.0 - zeta[t])
        for f in range(4):
            if nbr[t, f] >= 0:
                rows.append(t)
                cols.append(nbr[t, f])
                vals.append(zeta[t] * w[t, f])
    return sparse.csr_matrix((vals, (rows, cols)), shape=(T, T))


def test_surface_geometry_against_independent_formulas(orc):
    xyz, tris = W.triangle_lattice(7, 5, 0.1e-6, jitter_frac=0.25, seed=4)
    geo = orc.OracleSim(xyz, tris, [1e-12], []).geometry()
    area, nbr, r = _independent_geometry(xyz, tris)
    np.testing.assert_allclose(geo["vol"], area, rtol=1e-11)
    assert np.array_equal(geo["nbr"], nbr)
    g = r.sum(axis=1)
    np.testing.assert_allclose(geo["g"], g, rtol=1e-11)
    np.testing.assert_allclose(geo["w"], r / g[:, None], rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(geo["nav"], N_A * area, rtol=1e-11)
    # detailed balance of the walk: A_t r_te = A_u r_ue' (the edge's L / d)
    for t in range(tris.shape[0]):
        for e in range(3):
            u = geo["nbr"][t, e]
            if u >= 0:
                e2 = int(np.nonzero(geo["nbr"][u] == t)[0][0])
                a = geo["vol"][t] * geo["g"][t] * geo["w"][t, e]
                b = geo["vol"][u] * geo["g"][u] * geo["w"][u, e2]
                assert abs(a - b) <= 1e-9 * abs(a)


def test_surface_lattice_closed_forms_and_closed_box(orc):
    a = 0.1e-6
    xyz, tris = W.triangle_lattice(6, 6, a)
    o = orc.OracleSim(xyz, tris, [2e-12], [])
    geo = o.geometry()
    np.testing.assert_allclose(geo["vol"], a * a / 2, rtol=1e-12)
    # an interior right isosceles triangle: its two legs (length a) face
    # neighbours at barycentre distance a * sqrt(2) / 3 ... and the hypotenuse
    # (length a sqrt 2) one at distance a sqrt(2) / 3; so r = 3/a^2 * (1 + 1 + ...)
    interior = (geo["nbr"][:, :3] >= 0).all(axis=1)
    g_int = geo["g"][interior]
    assert np.allclose(g_int, g_int[0], rtol=1e-12)
    assert o.tau == pytest.approx(1.0 / (2e-12 * geo["g"].max()), rel=1e-14)
    bx, bt = W.box_surface(3, a)
    gb = orc.OracleSim(bx, bt, [1e-12], []).geometry()
    assert (gb["nbr"][:, :3] >= 0).all() and (gb["nbr"][:, 3] == -1).all()
    assert gb["vol"].sum() == pytest.approx(6 * (3 * a) ** 2, rel=1e-12)


def test_surface_invalid_meshes(orc):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [2, 0, 0]], float) * 1e-7
    fan = np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4]], np.int32)       # edge (0,1) on three triangles
    with pytest.raises(ValueError, match="three|more than two"):
        orc.OracleSim(xyz, fan, [1e-12], [])
    flat = np.array([[0, 1, 5], [0, 1, 2]], np.int32)                 # 0, 1, 5 are collinear
    with pytest.raises(ValueError, match="degenerate"):
        orc.OracleSim(xyz, flat, [1e-12], [])


@pytest.mark.parametrize("N0,tau_scale", [(5, 1.0), (200, 0.7)])
def test_surface_point_source_is_exactly_multinomial(orc, N0, tau_scale):
    xyz, tris = W.triangle_lattice(5, 5, 0.1e-6, jitter_frac=0.2, seed=8)
    T, D, src, k_steps, runs = tris.shape[0], 1e-12, 24, 3, 1500
    agg = np.zeros(T)
    for r in range(runs):
        sim = orc.OracleSim(xyz, tris, [D], [], tau_scale=tau_scale, seed=41, realization=r)
        init = np.zeros(T, np.int32)
        init[src] = N0
        sim.set_counts(0, init)
        sim.run_steps(k_steps)
        c = sim.get_counts(0)
        assert c.sum() == N0
        agg += c
    P = _transition_matrix(sim.geometry(), D, sim.tau)
    pi = np.zeros(T)
    pi[src] = 1.0
    for _ in range(k_steps):
        pi = P.T @ pi
    expected = pi * runs * N0
    keep = expected >= 5
    other = np.array([agg[~keep].sum(), expected[~keep].sum()])
    obs = np.append(agg[keep], other[0])
    exp = np.append(expected[keep], other[1])
    chi2 = float(((obs - exp) ** 2 / np.maximum(exp, 1e-300)).sum())
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-3


def test_surface_msd_against_exact_chain_and_4Dt(orc):
    n, a, D = 40, 0.1e-6, 1e-12
    xyz, tris = W.triangle_lattice(n, n, a)
    T = tris.shape[0]
    bc = xyz[tris].mean(axis=1)
    src = 2 * ((n // 2) + n * (n // 2))
    d2 = ((bc - bc[src]) ** 2).sum(axis=1)
    N0, seeds, k = 1000, 4, 30
    tot = 0.0
    for sd in range(seeds):
        sim = orc.OracleSim(xyz, tris, [D], [], seed=300 + sd)
        init = np.zeros(T, np.int32)
        init[src] = N0
        sim.set_counts(0, init)
        sim.run_steps(k)
        tot += float((sim.get_counts(0) * d2).sum())
    msd = tot / (N0 * seeds)
    P = _transition_matrix(sim.geometry(), D, sim.tau)
    pi = np.zeros(T)
    pi[src] = 1.0
    for _ in range(k):
        pi = P.T @ pi
    exact = float((pi * d2).sum())
    se = math.sqrt(float((pi * d2 ** 2).sum()) - exact ** 2) / math.sqrt(N0 * seeds)
    assert abs(msd - exact) < 3 * se, (msd, exact, se)
    # the finite-volume walk on this lattice against continuum 2D diffusion
    ratio = exact / (4 * D * k * sim.tau)
    assert 0.9 < ratio < 1.1, ratio


def test_surface_abc_equilibrium_mean(orc):
    """A + B <-> C on the closed surface of a box: the stationary mean of C
    against the well-mixed law with the area unit N_A A."""
    a = 0.1e-6
    xyz, tris = W.box_surface(3, a)
    area = 6 * (3 * a) ** 2
    nav = N_A * area
    kb, A0 = 10.0, 30
    kf = 0.5 * nav                        # 0.5 per pair per second, in m^2/(mol s)
    kappa = kf / (nav * kb)
    c = np.arange(0, A0 + 1)
    from scipy.special import gammaln

    lp = c * math.log(kappa) - 2 * gammaln(A0 - c + 1) - gammaln(c + 1)
    p = np.exp(lp - lp.max())
    p /= p.sum()
    mean_c = float((c * p).sum())
    runs, burn, keep = 8, 300, 2500
    rng = np.random.default_rng(12)
    means = []
    for r in range(runs):
        sim = orc.OracleSim(xyz, tris, [1e-12, 1e-12, 0.5e-12], [([0, 1], [2], kf), ([2], [0, 1], kb)],
                            tau_scale=0.5, seed=500 + r)
        for q in (0, 1):
            init = np.bincount(rng.integers(0, tris.shape[0], A0), minlength=tris.shape[0]).astype(np.int32)
            sim.set_counts(q, init)
        sim.run_steps(burn)
        acc = 0.0
        for _ in range(keep):
            sim.step()
            acc += sim.get_counts(2).sum()
        means.append(acc / keep)
    means = np.array(means)
    se = means.std(ddof=1) / math.sqrt(runs)
    assert abs(means.mean() - mean_c) < 3 * se + 0.01 * mean_c, (means.mean(), mean_c, se)
