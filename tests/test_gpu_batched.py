"""The batched A+B<->C workload at full size, in the launch configuration the
benchmark times: 256 realizations of the 40^3x6 Kuhn lattice (384,000 tets)
and 64 of the 20^3x6 one (48,000 tets), advanced together by the engine
(captured chunks, the tuner's launch shapes, two chains) for 0.1 s.

The oracle cannot run all 320 realizations in a test's time, but each
realization is an independent computation: sampled realizations are compared
with the oracle element by element (tolerance 0), and every realization is
checked for the invariants of the chemistry (A + C and B + C are conserved)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_batched_full_size_sampled_realizations(orc):
    import bench
    import paper_1512_03126_amd as P

    from concurrent.futures import ThreadPoolExecutor

    models = bench.build_batched()
    periods = 338
    samples = {0: [0, 131, 255], 1: [0, 63]}

    def oracle_run(kr):
        k, r = kr
        o = orc.OracleSim.from_model(models[k], realization=r)
        o.run_steps(periods)
        return o.get_counts()

    # the sampled realizations on the oracle run on host threads meanwhile
    keys = [(k, r) for k in samples for r in samples[k]]
    pool = ThreadPoolExecutor(max_workers=len(keys))
    futures = {kr: pool.submit(oracle_run, kr) for kr in keys}
    note("batched A+B<->C: 256 x 384000 + 64 x 48000 tets, 3 species, 338 periods through the engine")
    sims = bench.make_sims(P, models)
    e = P.rdos_engine_create(0, 0)
    bench.run_engine(P, e, sims, periods)
    P.rdos_engine_destroy(e)
    for k, (sim, m) in enumerate(zip(sims, models)):
        for r in range(m.n_realizations):
            got = sim.get_counts(None, realization=r)
            a0, b0 = m.init[r, 0].sum(), m.init[r, 1].sum()
            assert got[0].sum() + got[2].sum() == a0, (k, r)
            assert got[1].sum() + got[2].sum() == b0, (k, r)
            if r in samples[k]:
                note(f"compare with the oracle: model {k} ({m.n_tets} tets) realization {r}")
                want = futures[(k, r)].result()
                if not np.array_equal(got, want):
                    diff = np.argwhere(got != want)
                    raise AssertionError(f"model {k} realization {r}: {len(diff)} counts differ, first at "
                                         f"(species, tet) {tuple(diff[0])}")
    pool.shutdown()
    for s in sims:
        s.close()
