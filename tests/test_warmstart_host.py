"""Host-side pieces of the warm start that run without a GPU: the per-cell
velocity quantiles of the training targets (checked against numpy's
quantile, cell by cell) and the conversion of targets into the loader's
state (the host counterpart of sur_state)."""
import math

import numpy as np

from paper_2605_07083_amd import pic, presets, warmstart as WS


def test_cell_quantiles_match_numpy_per_cell():
    cfg = presets.scaled(presets.tiny(), N=40)
    rng = np.random.default_rng(4)
    z = rng.random(3000) * cfg["L"]
    v = rng.standard_cauchy(3000)
    z[:7] = 0.999 * cfg["L"]                 # a crowded last cell
    z = z[(z < 3 * cfg["L"] / 40) | (z > 5 * cfg["L"] / 40)]   # empty cells 3 and 4
    v = v[:len(z)]
    q = WS.cell_quantiles(cfg, z, v)
    cell = np.clip((z * (40 / cfg["L"])).astype(int), 0, 39)
    for c in range(40):
        sel = v[cell == c]
        if len(sel):
            assert np.allclose(q[:, c], np.quantile(sel, pic.STATE_LEVELS), rtol=0, atol=1e-12)
        else:
            assert np.all(q[:, c] == 0.0)


def test_state_from_targets_units():
    cfg = presets.surrogate_cases(2, presets.SURROGATE_TRAIN_SEED)[1]
    t = np.random.default_rng(5).normal(size=(pic.STATE_ROWS, cfg["N"]))
    st = WS.state_from_targets(cfg, t)
    q, me, mhe = 1.602176634e-19, 9.1093837015e-31, 6.6464731e-27
    assert np.allclose(st[0], cfg["n0"] * np.exp(t[1])) and np.allclose(st[1], cfg["n0"] * np.exp(t[2]))
    assert np.allclose(st[2], cfg["V"] * t[0])
    assert np.allclose(st[3:21], t[3:21] * math.sqrt(q / me))
    assert np.allclose(st[21:], t[21:] * math.sqrt(q / (mhe - me)))
