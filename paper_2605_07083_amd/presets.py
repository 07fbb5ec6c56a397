"""Seeded synthetic diode configurations (input recipes only).

Both the HIP library's binding and the CPU oracle's wrapper take these plain
dictionaries.  The module holds inputs and unit conversions of inputs only;
none of the method's arithmetic lives here.

Temperatures are in eV; Kelvin values given by a workload are converted with
k_B / e.  Channel bits: 1 e-He elastic, 2 excitation, 4 ionisation,
8 He+-He charge exchange, 16 He+-He elastic.
"""
import math

KB_OVER_E = 1.380649e-23 / 1.602176634e-19   # eV per kelvin

CH_EEL, CH_EXC, CH_IZ, CH_CX, CH_IEL = 1, 2, 4, 8, 16
CH_ALL = CH_EEL | CH_EXC | CH_IZ | CH_CX | CH_IEL

# Effective helium cross sections of the paper's benchmark (fixed sigma_e for
# e-He elastic, sigma_i for He+-He charge exchange), plus project-chosen
# analytic forms for the channels whose data the paper does not print.
SIG_EL = 6.8877e-20
SIG_CX = 1.7241e-20
SIG_IEL = 1.7241e-20
SIG_X0 = 1.0e-21          # excitation scale: peak 3.7e-22 m^2 near 54 eV
LOTZ_A = 4.0e-18          # Lotz constant for He 1s^2 (4.0e-14 cm^2 eV^2)


def _base(**kw):
    d = dict(L=5e-3, N=256, periodic=0, V=10.0, n0=1e16, Te0=2.0, Ti0=0.05,
             n_load=25600, gamma_emit=1e19, Tc=2000.0 * KB_OVER_E, ng=3.2e21,
             Tne=300.0 * KB_OVER_E, Tni=300.0 * KB_OVER_E, dt=5e-12,
             sig_el=SIG_EL, sig_x0=SIG_X0, lotz_a=LOTZ_A, sig_cx=SIG_CX, sig_iel=SIG_IEL,
             channels=CH_ALL, replenish=1, seed=0x5EED0000, diode=0,
             tally_period=100, nsteps=2000)
    d.update(kw)
    return d


def tiny():
    """Tiny diode: 5 mm gap, 256 cells, 100 particles/cell/species, 2000 steps."""
    return _base()


def bench():
    """Benchmark-scale diode: 2048 cells, 200 particles/cell/species,
    emission 7.25e19 m^-2 s^-1, 50k steps, tallies every 100 steps."""
    return _base(N=2048, n_load=409600, gamma_emit=7.25e19, seed=0x5EED0001, nsteps=50000)


def sweep(n_diodes=32):
    """Batched emission sweep: diodes of the benchmark geometry, fluxes
    log-uniform in [1e19, 1.2e20], cathode temperatures 1800-2200 K
    (decorrelated from the flux by a fixed permutation), 100-600k particles
    per species per diode."""
    out = []
    for d in range(n_diodes):
        frac = d / (n_diodes - 1) if n_diodes > 1 else 0.0
        gamma = 1e19 * 12.0 ** frac
        pt = (d * 7) % n_diodes
        pn = (d * 13) % n_diodes
        den = max(n_diodes - 1, 1)
        Tk = 1800.0 + 400.0 * pt / den
        nl = int(100000 + 500000 * pn / den)
        out.append(_base(N=2048, n_load=nl, gamma_emit=gamma, Tc=Tk * KB_OVER_E,
                         seed=0x5EED0002, diode=d, nsteps=50000))
    return out


def large():
    """Large collisional diode: 20 mm, 16384 cells, 1000 particles/cell/species,
    n_g = 3.2e22, emission 7.5e19, dt = 2e-12 s, 20k steps."""
    return _base(L=20e-3, N=16384, n_load=16384000, ng=3.2e22, gamma_emit=7.5e19,
                 dt=2e-12, seed=0x5EED0003, nsteps=20000)


def paper():
    """The paper's own benchmark diode (helium, 10 cm, 40 V, elastic + CX only,
    neutral targets 300 K / 1740 K)."""
    return _base(L=0.1, N=4096, V=40.0, n0=5e14, Te0=3.0, Ti0=0.15, n_load=4096000,
                 gamma_emit=7.25e19, Tc=0.2, ng=2.9e21, Tne=300.0 * KB_OVER_E,
                 Tni=1740.0 * KB_OVER_E, dt=6.722e-12, channels=CH_EEL | CH_CX,
                 seed=0x5EED00FF, nsteps=4500000)


def scaled(cfg, **kw):
    d = dict(cfg)
    d.update(kw)
    return d


def surrogate_params(n, seed):
    """Warm-start training / evaluation draws: flux, cathode temperature (K),
    bias, neutral density, uniform over the stated ranges."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return dict(gamma_emit=rng.uniform(1e19, 1.2e20, n), T_K=rng.uniform(1800.0, 2200.0, n),
                V=rng.uniform(5.0, 20.0, n), ng=rng.uniform(1e21, 1e22, n))


SURROGATE_TRAIN_SEED = 0x5EED0004
SURROGATE_HELDOUT_SEED = 0x5EED0104


def surrogate_cases(n, seed):
    """Warm-start dataset diodes: the benchmark geometry (5 mm, 2048 cells,
    200 particles per cell and species, dt 5 ps) with flux, cathode
    temperature, bias and neutral density drawn uniformly (surrogate_params).
    Tallies every 500 steps so that the snapshot ring spans 512k steps."""
    import numpy as np
    q = surrogate_params(n, seed)
    out = []
    for d in range(n):
        out.append(_base(N=2048, n_load=409600, gamma_emit=float(q["gamma_emit"][d]),
                         Tc=float(q["T_K"][d]) * KB_OVER_E, V=float(q["V"][d]), ng=float(q["ng"][d]),
                         seed=seed & 0xFFFFFFFF, diode=d, tally_period=500, nsteps=400000,
                         T_K=float(q["T_K"][d])))
    return out


SURROGATE_LAYERS = [(16, 64), (64, 64), (64, 64), (64, 64), (64, 64), (64, 39)]


def surrogate_test_weights(seed, scale=1.0):
    """Seeded FP32 weights W_l [Cout][Cin][5] ~ N(0, scale^2 / (5 Cin)) and
    biases ~ N(0, 0.01^2) for the six surrogate layers (test inputs)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    W, b = [], []
    for cin, cout in SURROGATE_LAYERS:
        W.append((scale * rng.normal(0.0, math.sqrt(1.0 / (5 * cin)), (cout, cin, 5))).astype(np.float32))
        b.append(rng.normal(0.0, 0.01, cout).astype(np.float32))
    return W, b


__all__ = ["tiny", "bench", "sweep", "large", "paper", "scaled", "surrogate_params", "surrogate_cases", "SURROGATE_TRAIN_SEED", "SURROGATE_HELDOUT_SEED", "surrogate_test_weights", "SURROGATE_LAYERS",
           "KB_OVER_E", "CH_ALL", "CH_EEL", "CH_EXC", "CH_IZ", "CH_CX", "CH_IEL", "math"]
