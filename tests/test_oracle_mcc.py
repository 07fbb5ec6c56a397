"""Pins of the oracle's null-collision MCC ("Emission and collisions").

* Collision frequency: per-channel counts of a mono-energetic beam on a cold
  target match n_g sigma_k(eps) g against the null-collision bound (binomial,
  4 sigma), both for forced candidates and for the free-flight countdown.
* Kinematics: elastic keeps |g|; excitation removes exactly E_x in the
  centre-of-mass frame; ionisation removes exactly E_iz and shares the rest
  between two electrons; the mean fractional energy loss of electron-He
  elastic scattering on a cold target is 2 m M / (m + M)^2.
* Charge exchange and ion elastic scattering relax an ion population to a
  Maxwellian at the neutral temperature (stationary by detailed balance).
* The null-collision bound is never exceeded.
"""
import numpy as np
import pytest

from _helpers import M_E, M_HE, M_I, NEVER, Q_E, by_id, empty, iso_beam, quiet_cfg, set_species
from paper_2605_07083_amd import presets

E_EXC, E_ION = 19.82, 24.59


def _beam_sim(O, sp, n, speed, channels, ng=3.2e21, Tn=0.0, dt=5e-12, tc=0, seed=1, L=1.0):
    cfg = quiet_cfg(ng=ng, channels=channels, Tne=Tn, Tni=Tn, dt=dt, L=L, N=64)
    s = O.Sim(cfg)
    s.load()
    for q in range(3):
        empty(s, q)
    rng = np.random.default_rng(seed)
    v = iso_beam(n, speed, rng)
    z = rng.uniform(0.3 * L, 0.7 * L, n)
    set_species(s, sp, z, v, np.arange(n), tc)
    s.set_counters(0, n)
    s.refield()
    return s, cfg, v


def _within(count, n, p, k=4.0):
    mu, sd = n * p, np.sqrt(n * p * (1 - p))
    return abs(count - mu) <= k * sd + 1


def test_sigma_special_values(O):
    p = presets.tiny()
    assert O.sigma(p, 0, 3.0) == presets.SIG_EL
    assert O.sigma(p, 3, 1.0) == presets.SIG_CX
    assert O.sigma(p, 1, E_EXC) == 0.0 and O.sigma(p, 2, E_ION) == 0.0
    # ln(x)/x peaks at x = e with value 1/e
    assert O.sigma(p, 1, np.e * E_EXC) == pytest.approx(presets.SIG_X0 / np.e, rel=1e-12, abs=0.0)
    # Lotz: a q ln(eps/E)/(eps E) at eps = e E_iz is a q / (e E_iz^2)
    assert O.sigma(p, 2, np.e * E_ION) == pytest.approx(presets.LOTZ_A * 2 / (np.e * E_ION**2), rel=1e-12, abs=0.0)
    q = dict(p, channels=presets.CH_EEL)
    assert O.sigma(q, 1, 60.0) == 0.0


@pytest.mark.parametrize("eps_eV", [5.0, 60.0, 85.0])
def test_forced_candidates_channel_frequencies(O, eps_eV):
    n = 100000
    mu = M_E * M_HE / (M_E + M_HE)
    g = np.sqrt(2 * Q_E * eps_eV / mu)
    chans = presets.CH_EEL | presets.CH_EXC | presets.CH_IZ
    s, cfg, _ = _beam_sim(O, 0, n, g, chans)
    numax = s.derived()["numax"][0]
    s.step()
    t = s.tally()
    assert t["cand"][0] == n
    assert t["nullcoll_exceed"] == 0
    for ch in range(3):
        p = cfg["ng"] * O.sigma(cfg, ch, eps_eV) * g / numax
        assert _within(t["coll"][ch], n, p), (ch, t["coll"][ch], n * p)


def test_countdown_rate(O):
    # free flight: candidates arrive as a Bernoulli(1 - exp(-lam)) process per
    # step and real collisions with probability nu/numax among them
    n, steps, speed = 20000, 200, 1.0e6
    s, cfg, _ = _beam_sim(O, 0, n, speed, presets.CH_EEL, tc=NEVER)
    # draw the initial free flights the way a fresh load does
    s2 = O.Sim(dict(cfg, n_load=n))
    s2.load()
    tc0 = by_id(s2.particles(0))["tc"]
    p = by_id(s.particles(0))
    p["tc"] = tc0
    s.set_particles(0, p)
    s.refield()
    live = 0
    for _ in range(steps):
        live += s.count(0)
        s.step()
    lam = s.derived()["lam"][0]
    numax = s.derived()["numax"][0]
    t = s.tally()
    pc = 1 - np.exp(-lam)
    assert _within(t["cand"][0], live, pc)
    assert _within(t["coll"][0], live, pc * cfg["ng"] * presets.SIG_EL * speed / numax)


def _one_collision_step(O, channels, eps_eV, n=4000, sp=0):
    m = M_E if sp == 0 else M_I
    mu = m * M_HE / (m + M_HE)
    g = np.sqrt(2 * Q_E * eps_eV / mu)
    s, cfg, v = _beam_sim(O, sp, n, g, channels, ng=1e24)
    nid = s.next_id
    s.step()
    after = by_id(s.particles(sp))
    keep = after["id"] < n
    after = {k: a[keep] for k, a in after.items()}
    va = np.stack([after["vx"], after["vy"], after["vz"]], 1)
    fr = M_HE / (m + M_HE)
    vcm = m * v / (m + M_HE)              # cold target: v_n = 0
    return s, cfg, v, va, vcm, fr, mu, g, nid


def test_elastic_keeps_relative_speed(O):
    s, cfg, v, va, vcm, fr, mu, g, _ = _one_collision_step(O, presets.CH_EEL, 10.0)
    moved = np.linalg.norm(va - v, axis=1) > 1e-6 * g
    assert moved.sum() == s.tally()["coll"][0] > 100
    r = np.linalg.norm(va[moved] - vcm[moved], axis=1)
    assert np.allclose(r, fr * g, rtol=1e-12)


def test_excitation_removes_threshold_energy(O):
    s, cfg, v, va, vcm, fr, mu, g, _ = _one_collision_step(O, presets.CH_EXC, 60.0)
    moved = np.linalg.norm(va - v, axis=1) > 1e-6 * g
    assert moved.sum() == s.tally()["coll"][1] > 50
    gp = np.linalg.norm(va[moved] - vcm[moved], axis=1) / fr
    eps_after = 0.5 * mu * gp**2 / Q_E
    assert np.allclose(eps_after, 60.0 - E_EXC, rtol=1e-11)


def test_ionisation_energy_balance_and_ids(O):
    s, cfg, v, va, vcm, fr, mu, g, nid = _one_collision_step(O, presets.CH_IZ, 80.0)
    t = s.tally()
    niz = t["coll"][2]
    assert niz > 50 and t["n_iz"] == niz
    moved = np.nonzero(np.linalg.norm(va - v, axis=1) > 1e-6 * g)[0]
    assert len(moved) == niz
    pe = by_id(s.particles(0))
    pi = by_id(s.particles(2))
    # children: secondary electron id next_id + 2r, ion next_id + 2r + 1, r by parent id
    sec_ids = nid + 2 * np.arange(niz)
    ion_ids = sec_ids + 1
    assert np.array_equal(pi["id"], ion_ids)
    sel = np.isin(pe["id"], sec_ids)
    assert sel.sum() == niz
    vs = np.stack([pe["vx"][sel], pe["vy"][sel], pe["vz"][sel]], 1)
    # parents sorted by id pair with secondaries in id order
    e1 = 0.5 * mu * (np.linalg.norm(va[moved] - vcm[moved], axis=1) / fr) ** 2 / Q_E
    e2 = 0.5 * mu * (np.linalg.norm(vs - vcm[moved], axis=1) / fr) ** 2 / Q_E
    assert np.allclose(e1 + e2, 80.0 - E_ION, rtol=1e-10)
    # children sit at the parent's position; the new ion has the (cold) neutral's velocity
    assert np.allclose(pe["z"][sel], pe["z"][moved], rtol=0, atol=0)
    assert np.all(pi["vx"] == 0) and np.all(pi["vz"] == 0)


def test_elastic_mean_energy_loss(O):
    n = 60000
    s, cfg, v, va, vcm, fr, mu, g, _ = _one_collision_step(O, presets.CH_EEL, 10.0, n=n)
    moved = np.linalg.norm(va - v, axis=1) > 1e-6 * g
    e0 = (v[moved] ** 2).sum(1)
    e1 = (va[moved] ** 2).sum(1)
    loss = ((e0 - e1) / e0)
    expect = 2 * M_E * M_HE / (M_E + M_HE) ** 2
    assert loss.mean() == pytest.approx(expect, rel=0.03)


def test_ion_relaxation_to_neutral_maxwellian(O):
    n = 20000
    Tn = 300.0 * presets.KB_OVER_E
    cfg = quiet_cfg(ng=3.2e23, channels=presets.CH_CX | presets.CH_IEL, Tni=Tn, Tne=Tn,
                    dt=1e-9, L=1.0, N=64, Ti0=1.0)
    s = O.Sim(cfg)
    s.load()
    for q in range(3):
        empty(s, q)
    rng = np.random.default_rng(4)
    vi = rng.normal(0, np.sqrt(Q_E * 1.0 / M_I), (n, 3))
    s2 = O.Sim(dict(cfg, n_load=n))
    s2.load()
    tc0 = by_id(s2.particles(2))["tc"]
    set_species(s, 2, rng.uniform(0.4, 0.6, n), vi, np.arange(n), tc0)
    s.refield()
    s.step(1000)
    t = s.tally()
    assert t["coll"][3] > 5 * n and t["coll"][4] > 5 * n
    p = s.particles(2)
    ke = 0.5 * M_I * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2) / Q_E
    assert ke.mean() == pytest.approx(1.5 * Tn, rel=0.03)
    # each component is Gaussian with variance e Tn / M
    from scipy import stats
    sig = np.sqrt(Q_E * Tn / M_HE)
    assert stats.kstest(p["vx"] / sig, "norm").pvalue > 1e-3


def test_numax_bounds_rate(O):
    p = presets.tiny()
    d = O.derive(p)
    for sp, m, idx in ((0, M_E, 0), (2, M_I, 1)):
        mu = m * M_HE / (m + M_HE)
        ecap = abs(p["V"]) + (40 * p["Te0"] + 40 * p["Tc"] if sp == 0 else 40 * p["Ti0"])
        Tn = p["Tne"] if sp == 0 else p["Tni"]
        gcap = np.sqrt(2 * Q_E * ecap / m) + 6 * np.sqrt(Q_E * Tn / M_HE)
        g = np.linspace(1.0, gcap, 20001)
        eps = 0.5 * mu * g**2 / Q_E
        chans = (0, 1, 2) if sp == 0 else (3, 4)
        nu = np.array([p["ng"] * sum(O.sigma(p, c, e) for c in chans) * gg for e, gg in zip(eps, g)])
        assert nu.max() <= d["numax"][idx]
        assert nu.max() >= d["numax"][idx] / 1.01
