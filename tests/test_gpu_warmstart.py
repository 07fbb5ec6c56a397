"""What the trained surrogate gains over the method without it.

The network in paper_2605_07083_amd/data/surrogate_w512.npz was trained by the
library's own kernels (sur_train_step) on the steady states of 512 diodes the
PIC itself produced (python -m paper_2605_07083_amd.warmstart generate /
train).  On the first 8 held-out diodes (a seed never used in training), each
run is taken to steady state twice -- from the uniform Maxwellian load (the
paper's cold start) and from the state the surrogate predicts
(pic_init_from_state) -- under the same detector (blocks of 2500 steps,
backflow within 1 pp over three blocks, live count within 2.5e-4 per block).
The warm start must reach steady sooner on every diode, land within 1 pp of
the cold run's steady backflow ratio (the cold start is the judge of the
warm start's error), and halve the median steps to steady.
"""
import os

import numpy as np
import pytest

from paper_2605_07083_amd import presets

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2605_07083_amd", "data",
                       "surrogate_w512.npz")


def test_warm_start_beats_cold_start_on_heldout_diodes():
    import torch
    assert torch.cuda.is_available()
    from paper_2605_07083_amd import warmstart
    from paper_2605_07083_amd.surrogate import Surrogate
    cfgs = presets.surrogate_cases(64, presets.SURROGATE_HELDOUT_SEED)[:8]
    print("case: 8 held-out diodes, cold start", flush=True)
    cold = warmstart.run_to_steady(cfgs, label="cold")
    W, b = warmstart.load_weights(WEIGHTS)
    net = Surrogate(len(cfgs), cfgs[0]["N"])
    net.set_weights(W, b)
    p = torch.tensor([warmstart.params_of(c) for c in cfgs], dtype=torch.float32, device="cuda:0")
    n0 = torch.tensor([c["n0"] for c in cfgs], dtype=torch.float64, device="cuda:0")
    st = net.state(p, n0).contiguous()
    print("case: the same diodes from the surrogate's state", flush=True)
    warm = warmstart.run_to_steady(cfgs, state=st, label="warm")
    ratios = []
    for d, (c, w) in enumerate(zip(cold, warm)):
        print("  diode %d: cold %d steps, warm %d steps; backflow %.2f %% vs %.2f %%" % (
            d, c["steady_step"], w["steady_step"], c["backflow_pct"], w["backflow_pct"]), flush=True)
        assert c["steady_step"] > 0 and w["steady_step"] > 0, d
        assert w["steady_step"] < c["steady_step"], d
        assert abs(w["backflow_pct"] - c["backflow_pct"]) <= 1.0, d
        ratios.append(c["steady_step"] / w["steady_step"])
    assert np.median(ratios) >= 2.0
