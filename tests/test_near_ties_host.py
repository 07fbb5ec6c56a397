"""The parity helpers' near-tie classification (no GPU): a particle whose
wall decision differs between the two sides counts as a legitimate near-tie
only when the oracle's pushed position lies within 1e-9 L of the electrode;
a differing collision outcome only when the channel-choice uniform lay
within 1e-6 of nu_max from a cumulative boundary."""
import numpy as np

from _helpers import NEVER, empty, quiet_cfg, set_species
from gpu_compare import CHANNEL_TIE, WALL_TIE, near_ties


def test_wall_near_tie_classification(O):
    L = 5e-3
    cfg = quiet_cfg(L=L, V=0.0, dt=1e-12)
    s = O.Sim(cfg)
    s.load()
    for q in range(3):
        empty(s, q)
    # one electron landing a hair inside the anode, one in mid-gap
    v = 1e5
    z_edge = L * (1 - 1e-13) - v * cfg["dt"]
    set_species(s, 0, [z_edge, L / 2], np.array([[0.0, 0.0, v], [0.0, 0.0, v]]), [0, 1], NEVER)
    s.refield()
    s.step()
    after = {sp: s.particles(sp) for sp in range(3)}
    assert len(after[0]["id"]) == 2
    # a GPU that absorbed the edge particle: a near-tie
    gpu = dict(after)
    gpu[0] = {k: v[after[0]["id"] != 0] for k, v in after[0].items()}
    t = near_ties(cfg, s, gpu)
    assert len(t) == 1 and t[0][1] == 0 and t[0][2] == "wall" and t[0][4] and t[0][3] < WALL_TIE
    # a GPU that absorbed the mid-gap particle: a real disagreement
    gpu[0] = {k: v[after[0]["id"] != 1] for k, v in after[0].items()}
    t = near_ties(cfg, s, gpu)
    assert len(t) == 1 and t[0][1] == 1 and not t[0][4]
    # identical outcomes: nothing to explain
    assert near_ties(cfg, s, after) == []


def test_channel_margin_recorded(O):
    from paper_2605_07083_amd import presets
    cfg = presets.scaled(presets.tiny(), ng=3.2e23)
    s = O.Sim(cfg)
    s.load()
    s.step()
    m = s.last_moves(0)
    cand = m["ch"] >= -1
    assert cand.sum() > 100
    assert np.all(np.isfinite(m["margin"][cand])) and np.all(m["margin"][cand] >= 0)
    assert np.all(np.isinf(m["margin"][~cand]))
    # uniform draws: the share within the tie band is of order the band itself
    assert np.mean(m["margin"][cand] < CHANNEL_TIE) < 1e-3
    # a velocity flip on a candidate with a wide margin is a real disagreement
    after = {sp: s.particles(sp) for sp in range(3)}
    k = int(np.argmax(np.where(cand, m["margin"], -1)))
    pid = m["id"][k]
    gpu = {sp: {a: v.copy() for a, v in after[sp].items()} for sp in range(3)}
    j = int(np.nonzero(gpu[0]["id"] == pid)[0][0])
    gpu[0]["vz"][j] = -gpu[0]["vz"][j] + 1e5
    t = near_ties(cfg, s, gpu)
    assert len(t) == 1 and t[0][2] == "channel" and not t[0][4]
