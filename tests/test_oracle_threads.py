"""The OpenMP build of the oracle (the CPU baseline on all host cores) gives
the single-threaded oracle's results bit for bit: its threads share only the
integer deposit sums and every order-dependent step (tallies, ionisation
products, compaction, births) stays in particle order."""
import numpy as np

from paper_2605_07083_amd import presets


def test_openmp_build_equals_single_thread(O):
    cfg = presets.scaled(presets.tiny(), gamma_emit=1e21, Te0=25.0, ng=3.2e22)
    a, b = O.Sim(cfg), O.Sim(cfg, omp=True)
    assert O.threads() == 1
    a.load()
    b.load()
    a.step(40)
    b.step(40)
    for sp in range(3):
        pa, pb = a.particles(sp), b.particles(sp)
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), (sp, k)
        assert np.array_equal(a.hist(sp), b.hist(sp))
        ma, mb = a.last_moves(sp), b.last_moves(sp)
        for k in ma:
            assert np.array_equal(ma[k], mb[k]), (sp, k)
    ta, tb = a.tally(), b.tally()
    for k in ta:
        assert np.array_equal(ta[k], tb[k]), k
    assert ta["coll"][2] > 0 and ta["n_emit"] > 0
    assert np.array_equal(a.phi(), b.phi())
