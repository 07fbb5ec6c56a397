"""Pins of the oracle's gather + leapfrog push and of its periodic test mode.

* Single particle in a vacuum diode: the field is the Laplace field -V/L and
  leapfrog reproduces the closed form z_m = z_0 + m v dt + a dt^2 m(m+1)/2;
  the step at which it reaches the electrode is exact.
* Periodic plasma: charge is conserved exactly, momentum to rounding, a cold
  plasma oscillates at the frequency of the discrete dispersion relation
  (CIC shape, central-difference field, leapfrog), total energy is bounded.
"""
import numpy as np
import pytest

from _helpers import EPS0, M_E, M_I, NEVER, Q_E, empty, quiet_cfg, set_species


@pytest.mark.parametrize("sp,sign,z0,v0,dt", [(0, +1, 2.2e-3, -2e5, 5e-12),
                                               (2, -1, 2e-5, 1e3, 2e-10)])
def test_single_particle_closed_form(O, sp, sign, z0, v0, dt):
    L, V = 5e-3, 10.0
    cfg = quiet_cfg(V=V, L=L, dt=dt)
    s = O.Sim(cfg)
    s.load()
    for q in range(3):
        empty(s, q)
    set_species(s, sp, [z0], np.array([[3.0, -4.0, v0]]), [0], NEVER)
    s.refield()
    m = M_E if sp == 0 else M_I
    q = -Q_E if sp == 0 else Q_E
    a = q / m * (-V / L)
    arrived = None
    for k in range(1, 3000):
        s.step()
        zk = v0 * dt * k + a * dt * dt * k * (k + 1) / 2 + z0
        if s.count(sp) == 0:
            arrived = k
            break
        got = s.particles(sp)["z"][0]
        assert got == pytest.approx(zk, rel=1e-11, abs=1e-12 * L)
        assert s.particles(sp)["vx"][0] == 3.0
    # first step at which the closed form crosses the electrode
    k = np.arange(1, 3000)
    zk = z0 + v0 * dt * k + a * dt * dt * k * (k + 1) / 2
    cross = k[(zk >= L) | (zk <= 0)][0]
    assert arrived == cross
    t = s.tally()
    wall = 1 if sign > 0 else 0
    assert t["abs_count"][sp][wall] == 1


def _periodic(O, N=64, ppc=64, L=1e-2, n0=1e14, wdt=0.1, Te=0.0, seed=5):
    wpe = np.sqrt(n0 * Q_E**2 / (M_E * EPS0))
    cfg = quiet_cfg(periodic=1, N=N, L=L, n0=n0, n_load=N * ppc, dt=wdt / wpe)
    s = O.Sim(cfg)
    s.load()
    n = N * ppc
    z0 = (np.arange(n) + 0.5) * L / n
    return s, cfg, wpe, z0


def test_periodic_cold_oscillation_frequency(O):
    s, cfg, wpe, z0 = _periodic(O, N=8, ppc=512, wdt=0.3)
    L, N, n = cfg["L"], cfg["N"], len(z0)
    k = 2 * np.pi / L
    amp = 1e-3 * L / n
    ze = z0 + amp * np.sin(k * z0)
    set_species(s, 0, ze, np.zeros((n, 3)), np.arange(n), NEVER)
    set_species(s, 2, z0, np.zeros((n, 3)), np.arange(n, 2 * n), NEVER)
    s.refield()
    x1 = []
    for _ in range(200):
        s.step()
        p = s.particles(0)
        o = np.argsort(p["id"])
        dzp = (p["z"][o] - z0 + L / 2) % L - L / 2
        x1.append((dzp * np.sin(k * z0)).sum())
    x1 = np.array(x1)
    # zero crossings with linear interpolation
    idx = np.where(np.sign(x1[:-1]) != np.sign(x1[1:]))[0]
    tz = idx + x1[idx] / (x1[idx] - x1[idx + 1])
    half = np.diff(tz).mean()
    w_meas = np.pi / (half * cfg["dt"])
    x = k * (L / N) / 2
    w_grid = wpe * np.sqrt((np.sin(x) / x) ** 3 * np.cos(x))
    w_exp = 2.0 / cfg["dt"] * np.arcsin(w_grid * cfg["dt"] / 2)
    assert w_meas == pytest.approx(w_exp, rel=3e-3)
    # and clearly distinct from the undiscretised value
    assert abs(w_exp / wpe - 1) > 0.05


def test_periodic_conservation(O):
    s, cfg, wpe, z0 = _periodic(O, N=32, ppc=100, L=32 * 1.05e-4, n0=1e16, wdt=0.05)
    rng = np.random.default_rng(2)
    n = len(z0)
    L = cfg["L"]
    ze = rng.uniform(0, L, n)
    ve = rng.normal(0, np.sqrt(Q_E * 2.0 / M_E), (n, 3))
    zi = rng.uniform(0, L, n)
    vi = rng.normal(0, np.sqrt(Q_E * 0.05 / M_I), (n, 3))
    set_species(s, 0, ze, ve, np.arange(n), NEVER)
    set_species(s, 2, zi, vi, np.arange(n, 2 * n), NEVER)
    s.refield()
    w0 = s.derived()["w0"]
    dz = L / cfg["N"]

    def totals():
        pe, pi = s.particles(0), s.particles(2)
        P = M_E * pe["vz"].sum() + M_I * pi["vz"].sum()
        Pabs = M_E * np.abs(pe["vz"]).sum() + M_I * np.abs(pi["vz"]).sum()
        q = (s.hist(2) - s.hist(0) - s.hist(1))[: cfg["N"]].sum()
        return P, Pabs, q

    P0, Pabs, q0 = totals()

    def energy():
        pe = s.particles(0)
        ke = 0.5 * M_E * (pe["vx"] ** 2 + pe["vy"] ** 2 + pe["vz"] ** 2).sum() * w0
        E = s.E()[: cfg["N"]]
        return ke + 0.5 * EPS0 * (E ** 2).sum() * dz

    W = []
    for _ in range(300):
        s.step()
        W.append(energy())
        P, _, q = totals()
        assert q == q0                          # exact charge conservation
    assert abs(P - P0) < 1e-8 * Pabs            # momentum to rounding
    W = np.array(W)
    assert np.ptp(W) < 0.02 * W.mean()          # bounded energy error
