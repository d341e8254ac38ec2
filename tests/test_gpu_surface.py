"""Surface diffusion and surface reactions (the transfer between surface
triangles, Sec. III.A, Fig. 5(c)-(d)) on the GPU: geometry and every period
bit for bit against the oracle, surfaces and volumes in one engine, and the
spread of a point source and of a line source against 2D diffusion."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N_A = 6.02214076e23
D_S = [1e-12, 2e-12, 0.5e-12]
# per-area rates: a triangle of ~5e-15 m^2 has N_A A ~ 3e9
RX_S = [([0, 1], [2], 3e11), ([2], [0, 1], 40.0), ([], [1], 3e-10), ([0], [], 30.0)]


@pytest.fixture(scope="module")
def P():
    import paper_1512_03126_amd as P

    P.lib()
    return P


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def surfaces():
    return {"jittered plane": W.triangle_lattice(8, 6, 0.1e-6, jitter_frac=0.25, seed=9),
            "box surface": W.box_surface(3, 0.1e-6)}


@pytest.mark.parametrize("name", ["jittered plane", "box surface"])
def test_surface_geometry_and_tau_bit_exact(P, orc, name):
    xyz, tris = surfaces()[name]
    note(f"surface geometry: {name}")
    g = P.Simulation(xyz, tris, D_S, RX_S, seed=3)
    o = orc.OracleSim(xyz, tris, D_S, RX_S, seed=3)
    assert g.tau == o.tau
    gg, og = g.geometry(), o.geometry()
    for key in ("nbr", "w", "g", "nav"):
        assert np.array_equal(gg[key], og[key]), key
    g.close()


@pytest.mark.parametrize("name", ["jittered plane", "box surface"])
def test_surface_every_period(P, orc, name):
    xyz, tris = surfaces()[name]
    T = tris.shape[0]
    rng = np.random.default_rng(17)
    init = rng.integers(0, 6, size=(2, len(D_S), T)).astype(np.int32)
    init[:, 0, ::5] += 60                      # the sequential-binomial branch of the split
    note(f"surface every period: {name}")
    g = P.Simulation(xyz, tris, D_S, RX_S, seed=21, n_realizations=2, tau_scale=0.8)
    os_ = []
    for r in range(2):
        o = orc.OracleSim(xyz, tris, D_S, RX_S, tau_scale=0.8, seed=21, realization=r)
        for s in range(len(D_S)):
            o.set_counts(s, init[r, s])
            g.set_counts(s, init[r, s], realization=r)
        os_.append(o)
    for period in range(40):
        g.step(1)
        for r, o in enumerate(os_):
            o.step()
            got, want = g.get_counts(None, realization=r), o.get_counts()
            assert np.array_equal(got, want), (period, r, int((got != want).sum()))
    g.close()


def test_surfaces_and_volumes_in_one_engine(P, orc):
    """A volume request and two surface requests batched together: each
    result equals the oracle's."""
    xyz_v, tets = W.tiny_lattice(3, 0.2e-6, jitter_frac=0.2, seed=2)
    rx_v = [([0, 1], [2], 5e8), ([2], [0, 1], 30.0)]
    reqs = [(xyz_v, tets, [1e-12, 1e-12, 0.5e-12], rx_v, 40),
            (*surfaces()["jittered plane"], D_S, RX_S, 56),
            (*surfaces()["box surface"], D_S[:2], [([0], [1], 20.0)], 32)]
    note("engine: volume and surface requests together")
    e = P.rdos_engine_create(0, 0)
    P.rdos_engine_set_shape(e, 8, 64, 1, 2)
    rng = np.random.default_rng(5)
    runs = []
    for i, (xyz, cells, D, rx, n) in enumerate(reqs):
        init = rng.integers(0, 8, size=(len(D), cells.shape[0])).astype(np.int32)
        s = P.Simulation(xyz, cells, D, rx, seed=40 + i, tau_scale=None)
        for q in range(len(D)):
            s.set_counts(q, init[q])
        runs.append((P.rdos_engine_submit(e, s.h, n, 1.0), s, init))
    P.rdos_engine_drain(e)
    for i, ((t, s, init), (xyz, cells, D, rx, n)) in enumerate(zip(runs, reqs)):
        P.rdos_engine_release(e, t)
        got = s.get_counts()
        s.close()
        o = orc.OracleSim(xyz, cells, D, rx, seed=40 + i)
        for q in range(len(D)):
            o.set_counts(q, init[q])
        o.run_steps(n)
        assert np.array_equal(got, o.get_counts())
    P.rdos_engine_destroy(e)


def _spread(P, orc, xyz, tris, init, periods, realizations, coord):
    """Run `realizations` copies of a surface diffusion from `init` and
    return the mean over molecules of the squared displacement measure
    `coord(bc)` after `periods`, with its standard error, plus the exact
    chain's prediction."""
    from scipy import sparse

    D = 1e-12
    T = tris.shape[0]
    g = P.Simulation(xyz, tris, [D], [], seed=77, n_realizations=realizations)
    for r in range(realizations):
        g.set_counts(0, init, realization=r)
    g.step(periods)
    g.synchronize()
    bc = xyz[tris].mean(axis=1)
    m = coord(bc)
    per_molecule = np.concatenate([np.repeat(m, g.get_counts(0, realization=r)) for r in range(realizations)])
    o = orc.OracleSim(xyz, tris, [D], [], seed=77, realization=realizations - 1)
    o.set_counts(0, init)
    o.run_steps(periods)
    assert np.array_equal(g.get_counts(0, realization=realizations - 1), o.get_counts(0))
    geo = o.geometry()
    zeta = np.minimum(1.0, (o.tau * D) * geo["g"])
    rows, cols, vals = [], [], []
    for t in range(T):
        rows.append(t), cols.append(t), vals.append(1.0 - zeta[t])
        for f in range(4):
            if geo["nbr"][t, f] >= 0:
                rows.append(t), cols.append(geo["nbr"][t, f]), vals.append(zeta[t] * geo["w"][t, f])
    Pm = sparse.csr_matrix((vals, (rows, cols)), shape=(T, T))
    pi = init / init.sum()
    for _ in range(periods):
        pi = Pm.T @ pi
    g.close()
    return per_molecule.mean(), per_molecule.std() / np.sqrt(per_molecule.size), float((pi * m).sum()), o.tau


def test_surface_point_source_spreads_as_2d_diffusion(P, orc):
    """Fig. 5(c): unbounded surface diffusion from a point source; the mean
    squared distance is the exact chain's and 4 D t on this lattice."""
    n, a = 40, 0.1e-6
    xyz, tris = W.triangle_lattice(n, n, a)
    src = 2 * ((n // 2) + n * (n // 2))
    init = np.zeros(tris.shape[0], np.int32)
    init[src] = 400
    bc0 = xyz[tris[src]].mean(axis=0)
    note("surface point source, 64 realizations")
    k = 30
    msd, se, exact, tau = _spread(P, orc, xyz, tris, init, k, 64, lambda bc: ((bc - bc0) ** 2).sum(axis=1))
    note(f"point source: msd {msd:.4e} +- {se:.1e}, exact chain {exact:.4e}, 4Dt {4e-12 * k * tau:.4e}")
    assert abs(msd - exact) < 4 * se
    assert abs(exact / (4e-12 * k * tau) - 1.0) < 0.02


def test_surface_line_source_spreads_as_1d_diffusion(P, orc):
    """Fig. 5(d): a line source across the plane; the variance of x grows
    as 2 D t (the exact chain's prediction on this lattice)."""
    n, a = 40, 0.1e-6
    xyz, tris = W.triangle_lattice(n, n, a)
    bc = xyz[tris].mean(axis=1)
    x0 = (n // 2 + 0.5) * a
    line = np.abs(bc[:, 0] - x0) < 0.5 * a          # the triangles of the middle cell column
    init = np.where(line, 10, 0).astype(np.int32)
    note("surface line source, 32 realizations")
    k = 30
    var0 = float((init * (bc[:, 0] - x0) ** 2).sum() / init.sum())
    msx, se, exact, tau = _spread(P, orc, xyz, tris, init, k, 32, lambda b: (b[:, 0] - x0) ** 2)
    note(f"line source: <dx^2> {msx:.4e} +- {se:.1e}, exact chain {exact:.4e}, start + 2Dt {var0 + 2e-12 * k * tau:.4e}")
    assert abs(msx - exact) < 4 * se
    assert abs((exact - var0) / (2e-12 * k * tau) - 1.0) < 0.03
