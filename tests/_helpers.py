"""Shared helpers for the oracle pins (test-side input construction only)."""
import numpy as np

from paper_2605_07083_amd import presets

Q_E = 1.602176634e-19
M_E = 9.1093837015e-31
M_HE = 6.6464731e-27
M_I = M_HE - M_E
EPS0 = 8.8541878128e-12
NEVER = 0xFFFFFFFF


def quiet_cfg(**kw):
    """A diode with negligible self-field: tiny density so each macro-particle
    carries almost no charge, no emission, no replenishment."""
    base = presets.tiny()
    base.update(n0=1e-6, V=0.0, gamma_emit=0.0, replenish=0, ng=0.0, n_load=1)
    base.update(kw)
    return base


def set_species(sim, sp, z, v, ids, tc):
    n = len(z)
    sim.set_particles(sp, {"z": np.asarray(z, float), "vx": np.asarray(v[:, 0], float),
                           "vy": np.asarray(v[:, 1], float), "vz": np.asarray(v[:, 2], float),
                           "id": np.asarray(ids, np.uint32), "tc": np.full(n, tc, np.uint32)
                           if np.isscalar(tc) else np.asarray(tc, np.uint32)})


def empty(sim, sp):
    set_species(sim, sp, [], np.zeros((0, 3)), [], 0)


def iso_beam(n, speed, rng):
    ct = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    st = np.sqrt(1 - ct * ct)
    return speed * np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)


def by_id(d):
    o = np.argsort(d["id"])
    return {k: v[o] for k, v in d.items()}
