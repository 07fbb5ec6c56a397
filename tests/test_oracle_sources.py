"""Pins of the oracle's particle sources ("Model", "Emission and collisions").

* Thermionic emission: N_emit = Gamma dt / w0 with a Bernoulli draw for the
  fractional part; velocities from the flux-weighted half-Maxwellian whose
  mean kinetic energy is 2 T_c (the value eq. 1 uses); placement z = v_z dt.
* Pair replenishment: as many electron-ion pairs as ions were lost, sharing a
  uniform position, Maxwellian at the initial temperatures.
* Child-Langmuir: a collisionless vacuum diode transmits the emitted flux below
  the space-charge limit and saturates at
  Gamma_CL = (4 eps0 / 9) sqrt(2 e / m) V^1.5 / (e L^2) above it.
* Restart: a run saved and resumed from its state is bit identical.
"""
import numpy as np
import pytest
from scipy import stats

from _helpers import EPS0, M_E, M_I, Q_E, by_id, empty, quiet_cfg, set_species
from paper_2605_07083_amd import presets


def test_emission_count_is_bernoulli_fraction(O):
    cfg = quiet_cfg(gamma_emit=1.0, n_load=1)
    w0 = O.derive(cfg)["w0"]
    x = 2.37
    cfg["gamma_emit"] = x * w0 / cfg["dt"]
    s = O.Sim(cfg)
    s.load()
    for q in range(3):
        empty(s, q)
    s.set_counters(0, 10)
    s.refield()
    counts = []
    prev = 0
    for _ in range(2000):
        s.step()
        ne = s.tally()["n_emit"]
        counts.append(ne - prev)
        prev = ne
    counts = np.array(counts)
    assert set(np.unique(counts)) <= {2, 3}
    frac = (counts == 3).mean()
    assert abs(frac - 0.37) < 4 * np.sqrt(0.37 * 0.63 / len(counts))


def test_emission_distribution(O):
    Tc = 2000.0 * presets.KB_OVER_E
    cfg = quiet_cfg(n_load=1, Tc=Tc, L=1.0)
    w0 = O.derive(cfg)["w0"]
    cfg["gamma_emit"] = 40000.5 * w0 / cfg["dt"]
    s = O.Sim(cfg)
    s.load()
    for q in range(3):
        empty(s, q)
    s.set_counters(0, 10)
    s.refield()
    s.step()
    p = s.particles(1)
    n = len(p["z"])
    assert n in (40000, 40001)
    sc = np.sqrt(Q_E * Tc / M_E)
    # z = v_z dt exactly; all inward
    assert np.array_equal(p["z"], p["vz"] * cfg["dt"])
    assert (p["vz"] > 0).all()
    # v_z is Rayleigh(sc): flux-weighted half-Maxwellian; v_x, v_y Gaussian
    assert stats.kstest(p["vz"] / sc, "rayleigh").pvalue > 1e-3
    assert stats.kstest(p["vx"] / sc, "norm").pvalue > 1e-3
    assert stats.kstest(p["vy"] / sc, "norm").pvalue > 1e-3
    ke = 0.5 * M_E * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2) / Q_E
    # mean energy of the flux-weighted half-Maxwellian is 2 T_c (eq. 1)
    assert ke.mean() == pytest.approx(2 * Tc, rel=0.015)
    # ids are consecutive from next_id
    assert np.array_equal(np.sort(p["id"]), 10 + np.arange(n))


def test_replenishment_pairs(O):
    cfg = presets.tiny()
    cfg.update(gamma_emit=0.0, ng=0.0, Ti0=2.0)          # hot ions reach the walls quickly
    s = O.Sim(cfg)
    s.load()
    nid0 = s.next_id
    ids_before = set(by_id(s.particles(2))["id"].tolist())
    s.step(30)
    t = s.tally()
    lost = t["abs_count"][2].sum()
    assert lost > 0 and t["n_repl"] == lost
    # ion count restored
    assert s.count(2) == cfg["n_load"]
    pe, pi = by_id(s.particles(0)), by_id(s.particles(2))
    new_i = pi["id"][pi["id"] >= nid0]
    assert len(new_i) == lost
    # pair ids are (k, k+1) with the electron first, and share the birth position
    assert np.all((new_i - nid0) % 2 == 1)
    assert not ids_before & set(new_i.tolist())
    ek = new_i - 1
    sel = np.isin(pe["id"], ek)
    assert sel.sum() == len(ek)


def test_child_langmuir(O):
    L, V, N = 5e-3, 10.0, 128
    gcl = (4 * EPS0 / 9) * np.sqrt(2 * Q_E / M_E) * V**1.5 / (Q_E * L * L)
    res = {}
    for mult in (0.5, 3.0):
        cfg = presets.tiny()
        cfg.update(L=L, V=V, N=N, ng=0.0, replenish=0, Tc=1e-4, n_load=2000,
                   gamma_emit=mult * gcl, dt=5e-12)
        w0 = O.derive(cfg)["w0"]
        cfg["n0"] = cfg["n0"] * (mult * gcl * cfg["dt"] / w0) / 15.0   # ~15 emitted per step
        s = O.Sim(cfg)
        s.load()
        for q in range(3):
            empty(s, q)
        s.refield()
        s.step(5000)
        t0 = s.tally()
        s.step(5000)
        t1 = s.tally()
        w0 = s.derived()["w0"]
        T = 5000 * cfg["dt"]
        res[mult] = (t1["abs_count"][1][1] - t0["abs_count"][1][1]) * w0 / T
    assert res[0.5] == pytest.approx(0.5 * gcl, rel=0.03)
    assert res[3.0] == pytest.approx(gcl, rel=0.05)


def test_restart_bit_identical(O):
    cfg = presets.tiny()
    cfg.update(gamma_emit=2e21)
    a = O.Sim(cfg)
    a.load()
    a.step(40)
    b = O.Sim(cfg)
    b.load()
    b.step(20)
    state = {sp: b.particles(sp) for sp in range(3)}
    step, nid = b.stepno, b.next_id
    t20 = b.tally()
    c = O.Sim(cfg)
    c.load()
    for sp in range(3):
        c.set_particles(sp, state[sp])
    c.set_counters(step, nid)
    c.refield()
    c.step(20)
    for sp in range(3):
        pa, pc = by_id(a.particles(sp)), by_id(c.particles(sp))
        for k in pa:
            assert np.array_equal(pa[k], pc[k]), (sp, k)
        assert np.array_equal(a.hist(sp), c.hist(sp))
    assert np.array_equal(a.phi(), c.phi())
    ta, tc = a.tally(), c.tally()
    assert np.array_equal(ta["abs_count"] - t20["abs_count"], tc["abs_count"])
    assert np.array_equal(ta["coll"] - t20["coll"], tc["coll"])
    assert ta["n_emit"] - t20["n_emit"] == tc["n_emit"]
