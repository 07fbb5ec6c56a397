"""Pins of the oracle's boundary tallies, initial load and pair replenishment.

* Absorbed energy ("Boundary energy diagnostics", eqs. 3-8 rest on it): a
  single particle in the vacuum diode reaches the electrode at the step the
  closed form gives, and its tallied energy is the full 3V kinetic energy
  1/2 m (v_x^2 + v_y^2 + v_z^2) at the crossing velocity v_z^{n+1/2} =
  v^{-1/2} + (n + 1) a dt -- for an electron at the anode and an ion at the
  cathode.
* A thermionic electron placed at z = v_z dt >= L is absorbed at once at the
  anode and tallied with its birth energy: over many such electrons the
  count equals the emitted count and the mean energy is 2 T_c (the
  flux-weighted half-Maxwellian, eq. 1).
* Initial load ("Model": uniform positions, Maxwellian velocities at T_e0,
  T_i0, no drift): z is uniform on [0, L) (KS), every velocity component is
  normal with variance k T / m (KS and a 4-sigma variance bound).
* Pair replenishment ("Model"): in the step of birth every new electron-ion
  pair shares one position bit for bit, the pair count equals the ions lost
  at both walls in that step, the positions are uniform on [0, L) and the
  pair's velocities are Maxwellian at T_e0 (electron) and T_i0 (ion).

Each test fails on the oracle with the corresponding mistake planted in a
copy of its source (tests/test_oracle_mutants.py).
"""
import numpy as np
import pytest
from scipy import stats

from _helpers import M_E, M_I, NEVER, Q_E, by_id, empty, quiet_cfg, set_species
from paper_2605_07083_amd import presets


def _closed_form_arrival(z0, v0, a, dt, L, kmax=20000):
    k = np.arange(1, kmax)
    zk = z0 + v0 * dt * k + a * dt * dt * k * (k + 1) / 2
    return int(k[(zk >= L) | (zk <= 0)][0])


@pytest.mark.parametrize("sp,wall,z0,v0,vperp,dt", [
    (0, 1, 2.2e-3, -2e5, (3.0e5, -4.0e5), 5e-12),     # electron reaching the anode
    (2, 0, 2e-5, 1e3, (1.0e3, -2.0e3), 2e-10),        # ion reaching the cathode
])
def test_absorbed_energy_is_full_3v_energy_at_crossing(O, sp, wall, z0, v0, vperp, dt):
    L, V = 5e-3, 10.0
    s = O.Sim(quiet_cfg(V=V, L=L, dt=dt))
    s.load()
    for q in range(3):
        empty(s, q)
    vx, vy = vperp
    set_species(s, sp, [z0], np.array([[vx, vy, v0]]), [0], NEVER)
    s.refield()
    m = M_E if sp == 0 else M_I
    a = (-Q_E if sp == 0 else Q_E) / m * (-V / L)
    n_arr = _closed_form_arrival(z0, v0, a, dt, L)
    s.step(n_arr - 1)
    assert s.count(sp) == 1 and s.tally()["abs_count"].sum() == 0
    s.step()
    t = s.tally()
    assert s.count(sp) == 0
    assert t["abs_count"][sp][wall] == 1 and t["abs_count"].sum() == 1
    # v_z at the crossing step: the half-step velocity after n_arr kicks
    vz = v0 + n_arr * a * dt
    want = 0.5 * m * (vx * vx + vy * vy + vz * vz)
    assert t["abs_energy"][sp][wall] == pytest.approx(want, rel=1e-10, abs=0.0)
    assert t["abs_energy"].sum() == t["abs_energy"][sp][wall]
    # the kick of one step changes the energy by far more than the tolerance,
    # so the velocity of the step before would not pass
    assert abs(0.5 * m * ((vz - a * dt) ** 2 - vz * vz)) > 1e-4 * want


def test_newborn_beyond_the_anode_is_absorbed_at_once(O):
    Tc = 2000.0 * presets.KB_OVER_E
    # a gap far shorter than one step of the slowest emitted electron
    cfg = quiet_cfg(n_load=1, Tc=Tc, L=1e-11, N=2)
    w0 = O.derive(cfg)["w0"]
    cfg["gamma_emit"] = 20000.5 * w0 / cfg["dt"]
    s = O.Sim(cfg)
    s.load()
    for q in range(3):
        empty(s, q)
    s.set_counters(0, 10)
    s.refield()
    s.step(2)
    t = s.tally()
    n = t["n_emit"]
    assert n in (40000, 40001, 40002)
    # P(v_z dt < L) ~ 1e-10: every electron crosses at birth
    assert s.count(1) == 0
    assert t["abs_count"][1][1] == n and t["abs_count"].sum() == n
    kT = Q_E * Tc
    mean = t["abs_energy"][1][1] / n
    # KE = kT (chi2_1 / 2 + chi2_1 / 2 + Exp(1)): mean 2 kT, variance 2 (kT)^2
    assert abs(mean - 2 * kT) < 4 * np.sqrt(2.0 / n) * kT


def _maxwellian_ok(v, T, m):
    """Each component normal with variance k T / m: KS p-value and a 4-sigma
    bound on the sample variance."""
    sig = np.sqrt(Q_E * T / m)
    n = len(v)
    for c in range(3):
        x = v[:, c] / sig
        assert stats.kstest(x, "norm").pvalue > 1e-4, c
        assert abs(x.var() - 1.0) < 4 * np.sqrt(2.0 / n), c
        assert abs(x.mean()) < 4 / np.sqrt(n), c


def test_initial_load_uniform_and_maxwellian(O):
    cfg = presets.tiny()
    s = O.Sim(cfg)
    s.load()
    L = cfg["L"]
    for sp, T, m in ((0, cfg["Te0"], M_E), (2, cfg["Ti0"], M_I)):
        p = s.particles(sp)
        assert len(p["z"]) == cfg["n_load"]
        assert (p["z"] >= 0).all() and (p["z"] < L).all()
        assert stats.kstest(p["z"] / L, "uniform").pvalue > 1e-4
        _maxwellian_ok(np.stack([p["vx"], p["vy"], p["vz"]], 1), T, m)
    assert s.count(1) == 0
    # electrons and ions are drawn independently (not paired): the positions
    # of electron k and ion k are uncorrelated
    pe, pi = by_id(s.particles(0)), by_id(s.particles(2))
    assert abs(np.corrcoef(pe["z"], pi["z"])[0, 1]) < 4 / np.sqrt(len(pe["z"]))


def test_replenished_pairs_share_position_and_are_maxwellian(O):
    # hot ions in a short gap with a long step: hundreds lost per step; a
    # negligible macro-weight keeps the field off
    cfg = quiet_cfg(L=1e-4, N=16, n_load=40000, Te0=2.0, Ti0=0.5, dt=1e-9, replenish=1)
    s = O.Sim(cfg)
    s.load()
    L = cfg["L"]
    ze, ve, vi = [], [], []
    pairs_total = 0
    for _ in range(12):
        nid0 = s.next_id
        t0 = s.tally()
        s.step()
        t1 = s.tally()
        lost = int((t1["abs_count"][2] - t0["abs_count"][2]).sum())
        pe, pi = by_id(s.particles(0)), by_id(s.particles(2))
        new_e = pe["id"] >= nid0
        new_i = pi["id"] >= nid0
        # one pair per ion lost at either wall, ids (k, k + 1) electron first
        assert new_e.sum() == new_i.sum() == lost == t1["n_repl"] - t0["n_repl"]
        assert s.next_id == nid0 + 2 * lost
        assert np.array_equal(pe["id"][new_e] + 1, pi["id"][new_i])
        # the pair shares its birth position bit for bit
        assert np.array_equal(pe["z"][new_e], pi["z"][new_i])
        ze.append(pe["z"][new_e])
        ve.append(np.stack([pe["vx"][new_e], pe["vy"][new_e], pe["vz"][new_e]], 1))
        vi.append(np.stack([pi["vx"][new_i], pi["vy"][new_i], pi["vz"][new_i]], 1))
        pairs_total += lost
    assert pairs_total > 3000
    z = np.concatenate(ze)
    assert (z > 0).all() and (z < L).all()
    assert stats.kstest(z / L, "uniform").pvalue > 1e-4
    _maxwellian_ok(np.concatenate(ve), cfg["Te0"], M_E)
    _maxwellian_ok(np.concatenate(vi), cfg["Ti0"], M_I)
