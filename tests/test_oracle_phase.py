"""Pins of the oracle's phase-space histogram (the (z, v_z) counts behind the
kinetic diagnostics of "Phase-space and velocity-distribution
characteristics"): bin edges and the under/overflow columns by hand, the
interior bins against numpy's histogram2d, conservation of the count."""
import numpy as np


def test_edges_by_hand(O):
    L, nz, nv, vmin, vmax = 1.0, 4, 8, -4.0, 4.0          # unit-wide velocity bins
    z = np.array([0.0, 0.25, 0.5 - 1e-12, np.nextafter(1.0, 0.0), 0.6, 0.6, 0.6, 0.6, 0.6, -1.0])
    v = np.array([-4.0, 0.0, 3.999, 4.0, np.nextafter(-4.0, -5.0), -1e30, 1e30, 3.0, -0.5, 0.0])
    H = O.phase_space(z, v, L, nz, nv, vmin, vmax)
    want = np.zeros((nz, nv + 2), dtype=np.int64)
    want[0, 1] += 1          # z = 0, v = vmin: first row, first inside column
    want[1, 5] += 1          # z on the row edge, v = 0 on a column edge: the upper bins
    want[1, 8] += 1          # just below z = L/2 and v = vmax
    want[3, 9] += 1          # last row; v = vmax is overflow
    want[2, 0] += 1          # one ulp below vmin: underflow
    want[2, 0] += 1
    want[2, 9] += 1
    want[2, 8] += 1          # v = 3 opens the last inside column
    want[2, 4] += 1          # v = -0.5 in [-1, 0)
    assert np.array_equal(H, want)                     # the hole (z < 0) is not counted
    assert H.sum() == 9


def test_interior_matches_histogram2d(O):
    rng = np.random.default_rng(17)
    L, nz, nv, vmin, vmax = 5e-3, 16, 40, -2e6, 2e6
    n = 200000
    z = rng.uniform(0.0, L, n)
    v = rng.normal(0.0, 8e5, n).astype(np.float32)
    H = O.phase_space(z, v, L, nz, nv, vmin, vmax)
    vd = v.astype(np.float64)
    ref, _, _ = np.histogram2d(z, vd, bins=[np.linspace(0.0, L, nz + 1), np.linspace(vmin, vmax, nv + 1)])
    assert np.array_equal(H[:, 1:nv + 1], ref.astype(np.int64))
    # under- and overflow per row
    rows = np.minimum(nz - 1, np.floor(z * (nz / L)).astype(int))
    for r in range(nz):
        sel = rows == r
        assert H[r, 0] == np.count_nonzero(vd[sel] < vmin)
        assert H[r, nv + 1] == np.count_nonzero(vd[sel] >= vmax)
    assert H.sum() == n
