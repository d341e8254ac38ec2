"""Pins of the oracle's mesh set-up (Sec. II.A, Algorithm 1 "precompute tau").

Regular Kuhn lattice: every quantity has a closed form in the cell edge a
(volumes a^3/6; cell-face triangles a^2/2, diagonal triangles a^2/sqrt 2;
barycentre distances a sqrt(3/8) across cell faces and a sqrt(2)/4 inside a
cell).  Jittered lattice: volumes by the Cayley-Menger determinant, areas by
Heron's formula (formulas the oracle does not use), plus exact invariants.
"""
import math

import numpy as np
import pytest

import workloads as W


def test_kuhn_closed_forms(orc):
    n, a, D = 4, 0.1e-6, 1e-12
    xyz, tets = W.kuhn_lattice(n, a)
    sim = orc.OracleSim(xyz, tets, [D], [])
    geo = sim.geometry()
    T = tets.shape[0]
    assert T == 6 * n**3
    np.testing.assert_allclose(geo["vol"], a**3 / 6, rtol=1e-13)
    # faces 0 and 3 lie on cell faces, faces 1 and 2 contain the cell diagonal
    np.testing.assert_allclose(geo["area"][:, [0, 3]], a**2 / 2, rtol=1e-13)
    np.testing.assert_allclose(geo["area"][:, [1, 2]], a**2 / math.sqrt(2), rtol=1e-13)
    r_outer = math.sqrt(24.0) / a**2   # (a^2/2) / (a^3/6 * a sqrt(3/8))
    r_inner = 12.0 / a**2              # (a^2/sqrt2) / (a^3/6 * a sqrt2/4)
    nbr = geo["nbr"]
    expect_g = np.where(nbr[:, 0] >= 0, r_outer, 0) + np.where(nbr[:, 3] >= 0, r_outer, 0) \
        + np.where(nbr[:, 1] >= 0, r_inner, 0) + np.where(nbr[:, 2] >= 0, r_inner, 0)
    assert (nbr[:, 1] >= 0).all() and (nbr[:, 2] >= 0).all()   # inner faces never on the boundary
    np.testing.assert_allclose(geo["g"], expect_g, rtol=1e-13)
    interior = (nbr >= 0).all(axis=1)
    assert interior.any()
    np.testing.assert_allclose(geo["g"][interior], (24 + 2 * math.sqrt(24)) / a**2, rtol=1e-13)
    np.testing.assert_allclose(geo["w"][interior][:, 1], 12 / (24 + 2 * math.sqrt(24)), rtol=1e-13)
    np.testing.assert_allclose(geo["w"][interior][:, 0], math.sqrt(24) / (24 + 2 * math.sqrt(24)), rtol=1e-13)
    # tau = 1 / (D g_max): zeta = 1 in the fastest tet
    assert sim.tau == pytest.approx(a**2 / (D * (24 + 2 * math.sqrt(24))), rel=1e-14)
    # 12 n^2 boundary triangles on the cube's surface
    assert int((nbr < 0).sum()) == 12 * n * n
    nav = geo["nav"]
    np.testing.assert_allclose(nav, 6.02214076e23 * a**3 / 6 * 1000, rtol=1e-13)


def test_tau_of_the_paper_cube_and_lattice(orc):
    """The 1 um cube with 0.2 um cells and the 4 um lattice with 0.1 um cells."""
    for n, a in [(5, 0.2e-6), (10, 0.1e-6)]:
        xyz, tets = W.kuhn_lattice(n, a)
        sim = orc.OracleSim(xyz, tets, [1e-12, 0.5e-12], [])
        assert sim.tau == pytest.approx(a**2 / (1e-12 * (24 + 2 * math.sqrt(24))), rel=1e-14)
        sim2 = orc.OracleSim(xyz, tets, [1e-12], [], tau_scale=0.25)
        assert sim2.tau == pytest.approx(0.25 * sim.tau, rel=1e-15)


def _cayley_menger_volume(P):
    d2 = np.array([[np.sum((P[i] - P[j]) ** 2) for j in range(4)] for i in range(4)])
    M = np.ones((5, 5))
    M[0, 0] = 0
    M[1:, 1:] = d2
    return math.sqrt(np.linalg.det(M) / 288.0)


def _heron(A, B, C):
    x, y, z = sorted([np.linalg.norm(A - B), np.linalg.norm(B - C), np.linalg.norm(C - A)], reverse=True)
    # Kahan's numerically stable form of Heron's formula
    return 0.25 * math.sqrt((x + (y + z)) * (z - (x - y)) * (z + (x - y)) * (x + (y - z)))


def test_jittered_geometry_independent_formulas(orc):
    n, a = 3, 0.1e-6
    xyz0, tets = W.kuhn_lattice(n, a)
    xyz = W.jitter(xyz0, n, a, 0.2, seed=4)
    sim = orc.OracleSim(xyz, tets, [1e-12], [])
    geo = sim.geometry()
    for t in range(tets.shape[0]):
        P = xyz[tets[t]]
        assert geo["vol"][t] == pytest.approx(_cayley_menger_volume(P), rel=1e-9)
        for f in range(4):
            Q = [P[v] for v in range(4) if v != f]
            assert geo["area"][t, f] == pytest.approx(_heron(*Q), rel=1e-10)
    assert geo["vol"].sum() == pytest.approx((n * a) ** 3, rel=1e-13)
    vmax, vmin = geo["vol"].max(), geo["vol"].min()
    assert vmax / vmin > 2.0


def test_neighbour_symmetry_and_detailed_balance(orc):
    """nbr is an involution over shared faces; V_t r_tf = V_u r_uf' (the
    diffusive flux through a face is the same seen from both sides), so the
    one-molecule chain is reversible with stationary law proportional to V."""
    n, a = 3, 0.1e-6
    xyz0, tets = W.kuhn_lattice(n, a)
    xyz = W.jitter(xyz0, n, a, 0.2, seed=9)
    sim = orc.OracleSim(xyz, tets, [1e-12], [])
    geo = sim.geometry()
    nbr, w, g, vol = geo["nbr"], geo["w"], geo["g"], geo["vol"]
    for t in range(tets.shape[0]):
        assert abs(w[t][nbr[t] >= 0].sum() - 1.0) < 1e-14
        assert (w[t][nbr[t] < 0] == 0).all()
        for f in range(4):
            u = nbr[t, f]
            if u < 0:
                continue
            back = [ff for ff in range(4) if nbr[u, ff] == t]
            assert len(back) == 1
            fb = back[0]
            assert set(tets[t][[v for v in range(4) if v != f]]) == set(tets[u][[v for v in range(4) if v != fb]])
            assert geo["area"][t, f] == geo["area"][u, fb]
            assert vol[t] * g[t] * w[t, f] == pytest.approx(vol[u] * g[u] * w[u, fb], rel=1e-13)


def test_invalid_meshes_are_rejected(orc):
    xyz, tets = W.kuhn_lattice(1, 1e-7)
    bad = tets.copy()
    bad[0, 3] = bad[0, 2]                     # repeated vertex: zero volume
    with pytest.raises(ValueError, match="degenerate"):
        orc.OracleSim(xyz, bad, [1e-12], [])
    three = np.concatenate([tets, tets[:1]])  # one tet listed twice: its faces shared by three
    with pytest.raises(ValueError, match="shared"):
        orc.OracleSim(xyz, three, [1e-12], [])
    with pytest.raises(ValueError, match="tau"):
        orc.OracleSim(xyz, tets, [0.0], [])
    with pytest.raises(ValueError, match="tau_scale"):
        orc.OracleSim(xyz, tets, [1e-12], [], tau_scale=1.5)
