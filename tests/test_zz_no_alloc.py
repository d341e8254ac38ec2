"""The entry point that allocates nothing (rdos_step_static: the step
kernels' queue in the library's static device array) against rdos_step, bit
for bit, on two calls in a row, the second on a smaller simulation."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


RX = [([0, 1], [2], 3e8), ([2], [0, 1], 400.0), ([0], [], 20.0)]
D = [1e-12, 2e-12, 0.5e-12]


def pair(P, n_cells, realizations, seed):
    xyz, tets = W.tiny_lattice(n_cells, 0.2e-6, jitter_frac=0.2, seed=seed)
    T = tets.shape[0]
    rng = np.random.default_rng(seed)
    init = rng.integers(0, 12, size=(realizations, len(D), T)).astype(np.int32)
    init[:, 0, ::7] += 60
    sims = []
    for _ in range(2):
        s = P.Simulation(xyz, tets, D, RX, seed=seed, n_realizations=realizations)
        for r in range(realizations):
            for q in range(len(D)):
                s.set_counts(q, init[r, q], realization=r)
        sims.append(s)
    return sims, T


def test_static_queue_step_equals_step():
    import paper_1512_03126_amd as P

    # first call: 9 x 9 x 9 cells (4374 tets) x 3 realizations, 5 tiles per
    # realization; second: 4 x 4 x 4 cells (384 tets) x 2 realizations, so the
    # static queue keeps stale entries and lengths from the first call
    for n_cells, Rz, periods, seed in ((9, 3, 40, 3), (4, 2, 25, 4)):
        note(f"static queue: {n_cells}^3 x 6 tets, {Rz} realizations, {periods} periods")
        (a, b), T = pair(P, n_cells, Rz, seed)
        a.step(periods)
        P.rdos_step_static(b.h, periods)
        for r in range(Rz):
            got, want = b.get_counts(None, realization=r), a.get_counts(None, realization=r)
            assert np.array_equal(got, want), (n_cells, r, int((got != want).sum()))
        assert a.time() == b.time()
        # the two entry points interleave on one handle: its own queue is untouched
        a.step(3)
        P.rdos_step_static(a.h, 2)
        b.step(5)
        for r in range(Rz):
            assert np.array_equal(a.get_counts(None, realization=r), b.get_counts(None, realization=r))
        a.close()
        b.close()


def test_static_queue_refuses_large_work_lists():
    import paper_1512_03126_amd as P

    xyz, tets = W.kuhn_lattice(20, 0.1e-6)  # 48,000 tets: 47 tiles per realization
    s = P.Simulation(xyz, tets, [1e-12] * 8, [], n_realizations=8)
    note("static queue: a work list past its size is refused before any launch")
    with pytest.raises(P.RdosError) as ei:
        P.rdos_step_static(s.h, 1)
    assert ei.value.status == -1 and "static queue" in str(ei.value)
    s.close()
