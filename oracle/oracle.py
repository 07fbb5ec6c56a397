"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this module.
"""
import ctypes as C
import os

import numpy as np

from . import build_oracle

NSP = 3
# warm-start state rows and quantile levels (pic_oracle.h, o_load_state)
STATE_ROWS = 39
STATE_LEVELS = (0.0, 0.02, 0.1, 0.25, 0.5, 0.75, 0.9, 0.98, 1.0)
_lib = None


class OCfg(C.Structure):
    _fields_ = [("L", C.c_double), ("N", C.c_int32), ("periodic", C.c_int32), ("V", C.c_double),
                ("n0", C.c_double), ("Te0", C.c_double), ("Ti0", C.c_double),
                ("n_load", C.c_int64), ("gamma_emit", C.c_double), ("Tc", C.c_double),
                ("ng", C.c_double), ("Tne", C.c_double), ("Tni", C.c_double), ("dt", C.c_double),
                ("sig_el", C.c_double), ("sig_x0", C.c_double), ("lotz_a", C.c_double),
                ("sig_cx", C.c_double), ("sig_iel", C.c_double), ("channels", C.c_uint32),
                ("replenish", C.c_int32), ("seed", C.c_uint32), ("diode", C.c_uint32)]


class ODerived(C.Structure):
    _fields_ = [("dz", C.c_double), ("invdz", C.c_double), ("w0", C.c_double),
                ("qm", C.c_double * 3), ("mass", C.c_double * 3), ("numax", C.c_double * 2),
                ("lam", C.c_double * 2), ("sig_n", C.c_double * 2)]


class OTally(C.Structure):
    _fields_ = [("abs_count", (C.c_int64 * 2) * 3), ("abs_energy", (C.c_double * 2) * 3),
                ("n_emit", C.c_int64), ("n_repl", C.c_int64), ("n_iz", C.c_int64),
                ("cand", C.c_int64 * 2), ("coll", C.c_int64 * 5), ("nullcoll_exceed", C.c_int64)]


class ODiag(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("gamma_emit", "gamma_emit_meas", "gamma_ref", "gamma_net",
                                          "gamma_anode", "backflow_pct", "eta_net", "eta_anode")] + [
        ("gamma_abs", (C.c_double * 2) * 3), ("q_abs", (C.c_double * 2) * 3)] + [
        (n, C.c_double) for n in ("wf_eff", "q_emit_theory", "q_ion_cath_recomb", "q_cool1", "q_cool2",
                                  "q_ion_anode_recomb", "q_anode1", "q_anode2", "phi_vc_eff")]


_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        # PIC_ORACLE_LIB: another build of the oracle source (the tests that
        # plant a mistake in a copy of the source load the copy this way)
        path = os.environ.get("PIC_ORACLE_LIB") or build_oracle.LIB
        if path == build_oracle.LIB and not os.path.exists(path):
            build_oracle.build()
        _lib = _setup(C.CDLL(path))
    return _lib


def lib_omp():
    """The same oracle built with OpenMP over its per-particle loops."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(build_oracle.LIB_OMP):
            build_oracle.build()
        _lib_omp = _setup(C.CDLL(build_oracle.LIB_OMP))
    return _lib_omp


def threads(omp=False):
    return (lib_omp() if omp else lib()).o_threads()


def _setup(L):
    P = C.c_void_p
    d, i64, u32, i32 = C.c_double, C.c_int64, C.c_uint32, C.c_int32
    L.o_create.restype = P
    L.o_create.argtypes = [C.POINTER(OCfg)]
    L.o_destroy.argtypes = [P]
    for f in ("o_load", "o_step", "o_refield"):
        getattr(L, f).argtypes = [P]
        getattr(L, f).restype = C.c_int
    L.o_load_profiles.argtypes = [P, P, P]
    L.o_load_profiles.restype = C.c_int
    L.o_load_state.argtypes = [P, P]
    L.o_load_state.restype = C.c_int
    L.o_count.argtypes = [P, C.c_int]
    L.o_count.restype = i64
    L.o_stepno.argtypes = [P]
    L.o_stepno.restype = i64
    L.o_next_id.argtypes = [P]
    L.o_next_id.restype = u32
    L.o_set_counters.argtypes = [P, i64, u32]
    L.o_get_particles.argtypes = [P, C.c_int] + [P] * 6
    L.o_set_particles.argtypes = [P, C.c_int, i64] + [P] * 6
    L.o_set_particles.restype = C.c_int
    for f in ("o_get_hist",):
        getattr(L, f).argtypes = [P, C.c_int, P]
    L.o_get_phi.argtypes = [P, P]
    L.o_get_E.argtypes = [P, P]
    L.o_get_tally.argtypes = [P, C.POINTER(OTally)]
    L.o_get_derived.argtypes = [P, C.POINTER(ODerived)]
    L.o_philox4x32_10.argtypes = [P, P, P]
    L.o_u24.argtypes = [u32]
    L.o_u24.restype = d
    L.o_u32.argtypes = [u32]
    L.o_u32.restype = d
    L.o_u53.argtypes = [u32, u32]
    L.o_u53.restype = d
    L.o_sigma.argtypes = [C.POINTER(OCfg), C.c_int, d]
    L.o_sigma.restype = d
    L.o_derive.argtypes = [C.POINTER(OCfg), C.POINTER(ODerived)]
    L.o_derive.restype = C.c_int
    L.o_deposit.argtypes = [i64, P, i32, d, P]
    L.o_solve.argtypes = [i32, d, d, P, P]
    L.o_solve.restype = C.c_int
    L.o_efield.argtypes = [i32, d, P, P]
    L.o_diag.argtypes = [d, d, d, d, P, P, d, C.POINTER(ODiag)]
    L.o_eta_vc.argtypes = [d, d, d]
    L.o_eta_vc.restype = d
    L.o_threads.argtypes = []
    L.o_threads.restype = C.c_int
    L.o_last_moves.argtypes = [P, C.c_int] + [P] * 5
    L.o_last_moves.restype = i64
    L.o_last_moves_count.argtypes = [P, C.c_int]
    L.o_last_moves_count.restype = i64
    return L


def make_cfg(p: dict) -> OCfg:
    c = OCfg()
    for name, _ in OCfg._fields_:
        setattr(c, name, p[name])
    return c


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().o_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def derive(p: dict) -> dict:
    c = make_cfg(p)
    d = ODerived()
    if lib().o_derive(C.byref(c), C.byref(d)) != 0:
        raise ValueError("invalid configuration")
    return {"dz": d.dz, "invdz": d.invdz, "w0": d.w0, "qm": list(d.qm), "mass": list(d.mass),
            "numax": list(d.numax), "lam": list(d.lam), "sig_n": list(d.sig_n)}


def sigma(p: dict, channel: int, eps_eV: float) -> float:
    c = make_cfg(p)
    return lib().o_sigma(C.byref(c), channel, float(eps_eV))


def deposit(z, N, invdz):
    z = np.ascontiguousarray(z, dtype=np.float64)
    H = np.zeros(N + 1, dtype=np.int64)
    lib().o_deposit(len(z), _ptr(z), N, invdz, _ptr(H))
    return H


def solve(N, dz, V, rho):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.zeros(N + 1, dtype=np.float64)
    lib().o_solve(N, dz, V, _ptr(rho), _ptr(phi))
    return phi


Q_E = 1.602176634e-19
EPS0 = 8.8541878128e-12


def solve_exact(N, dz, V, R, w0):
    """The Dirichlet Poisson system of the model section (phi_0 = 0,
    phi_N = V, phi_{j-1} - 2 phi_j + phi_{j+1} = -rho_j dz^2 / eps0 on the
    interior nodes) for the charge of the fixed-point deposit,
    rho_j = e w0 R_j / (2^32 dz) with integer R_j, eliminated in exact
    rational arithmetic and rounded to FP64 once per node.  Slow and exact:
    the reference for grids where the FP64 sweep of ``solve`` loses digits
    to rounding."""
    from fractions import Fraction
    N = int(N)
    phi = np.zeros(N + 1, dtype=np.float64)
    phi[N] = V
    k = Fraction(Q_E) * Fraction(w0) / (Fraction(2**32) * Fraction(dz))
    alpha = k * Fraction(dz) * Fraction(dz) / Fraction(EPS0)
    psi = solve_exact_psi(N, R)
    Vf = Fraction(V)
    for j in range(1, N):
        phi[j] = float(Vf * j / N + alpha * psi[j])
    return phi


def solve_exact_psi(N, R):
    """psi with psi_{j-1} - 2 psi_j + psi_{j+1} = -R_j (j = 1..N-1),
    psi_0 = psi_N = 0, as exact Fractions: the Thomas forward sweep and back
    substitution on rationals (so phi_j = V j / N + alpha psi_j with
    alpha = e w0 dz / (2^32 eps0))."""
    from fractions import Fraction
    N = int(N)
    n = N - 1
    psi = [Fraction(0)] * (N + 1)
    if n <= 0:
        return psi
    cp = [Fraction(0)] * n
    dp = [Fraction(0)] * n
    for i in range(n):
        rhs = Fraction(-int(R[i + 1]))
        cc = 1 if i < n - 1 else 0
        if i == 0:
            cp[i] = Fraction(cc, -2)
            dp[i] = rhs / -2
        else:
            m = -2 - cp[i - 1]
            cp[i] = cc / m
            dp[i] = (rhs - dp[i - 1]) / m
    psi[n] = dp[n - 1]
    for i in range(n - 2, -1, -1):
        psi[i + 1] = dp[i] - cp[i] * psi[i + 2]
    return psi


def phase_space(z, vz, L, nz, nv, vmin, vmax):
    """Counts of particles per (z, v_z) bin (the kinetic diagnostics of
    "Phase-space and velocity-distribution characteristics"), in FP64: row
    min(nz - 1, floor(z nz / L)); with x = (v_z - vmin) nv / (vmax - vmin),
    column 0 below vmin, 1 + floor(x) inside, nv + 1 at or above vmax.
    Holes (z < 0) are skipped."""
    z = np.asarray(z, dtype=np.float64)
    v = np.asarray(vz, dtype=np.float64)
    live = z >= 0.0
    z, v = z[live], v[live]
    sz = nz / L
    sv = nv / (vmax - vmin)
    iz = np.minimum(nz - 1, np.floor(z * sz).astype(np.int64))
    x = (v - vmin) * sv
    inside = 1 + np.floor(np.clip(x, 0.0, nv - 1)).astype(np.int64)
    iv = np.where(x >= nv, nv + 1, np.where(x >= 0.0, inside, 0))
    H = np.zeros((nz, nv + 2), dtype=np.int64)
    np.add.at(H, (iz, iv), 1)
    return H


def efield(N, dz, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    E = np.zeros(N + 1, dtype=np.float64)
    lib().o_efield(N, dz, _ptr(phi), _ptr(E))
    return E


def diag(gamma_emit, Tc, w0, window_s, count, energy, n_emit):
    cnt = np.ascontiguousarray(count, dtype=np.float64).reshape(3, 2)
    en = np.ascontiguousarray(energy, dtype=np.float64).reshape(3, 2)
    out = ODiag()
    lib().o_diag(gamma_emit, Tc, w0, window_s, _ptr(cnt), _ptr(en), n_emit, C.byref(out))
    res = {}
    for name, typ in ODiag._fields_:
        v = getattr(out, name)
        res[name] = np.array([[v[s][w] for w in range(2)] for s in range(3)]) if name in (
            "gamma_abs", "q_abs") else v
    return res


class Sim:
    """One oracle diode."""

    def __init__(self, p: dict, omp=False):
        """omp: run on the OpenMP build (identical results, all host cores)."""
        self.p = dict(p)
        self._cfg = make_cfg(p)
        self.L = lib_omp() if omp else lib()
        self.h = self.L.o_create(C.byref(self._cfg))
        if not self.h:
            raise ValueError("oracle: invalid configuration")
        self.N = p["N"]

    def __del__(self):
        if getattr(self, "h", None):
            self.L.o_destroy(self.h)
            self.h = None

    def load(self):
        if self.L.o_load(self.h) != 0:
            raise RuntimeError("oracle load failed")

    def load_profiles(self, ne, ni):
        """Warm start from cell-centre densities (N values each, m^-3)."""
        ne = np.ascontiguousarray(ne, dtype=np.float64)
        ni = np.ascontiguousarray(ni, dtype=np.float64)
        assert ne.shape == (self.N,) and ni.shape == (self.N,)
        rc = self.L.o_load_profiles(self.h, _ptr(ne), _ptr(ni))
        if rc == -2:
            raise ValueError("oracle: negative or non-finite density")
        if rc != 0:
            raise RuntimeError("oracle profile load failed")

    def load_state(self, prof):
        """Warm start from a late-time state prof [39][N]: n_e, n_i (m^-3),
        phi (V), then per species (electrons, ions) nine quantiles of v_z and
        nine of |v_perp| (m/s) at the levels STATE_LEVELS."""
        prof = np.ascontiguousarray(prof, dtype=np.float64)
        assert prof.shape == (STATE_ROWS, self.N)
        rc = self.L.o_load_state(self.h, _ptr(prof))
        if rc == -2:
            raise ValueError("oracle: negative density or non-finite state entry")
        if rc != 0:
            raise RuntimeError("oracle state load failed")

    def step(self, n=1):
        for _ in range(n):
            if self.L.o_step(self.h) != 0:
                raise RuntimeError("oracle step failed")

    def refield(self):
        self.L.o_refield(self.h)

    @property
    def stepno(self):
        return self.L.o_stepno(self.h)

    @property
    def next_id(self):
        return self.L.o_next_id(self.h)

    def set_counters(self, step, next_id):
        self.L.o_set_counters(self.h, int(step), int(next_id))

    def count(self, sp):
        return self.L.o_count(self.h, sp)

    def particles(self, sp):
        n = self.count(sp)
        z, vx, vy, vz = (np.zeros(n) for _ in range(4))
        pid, tc = np.zeros(n, np.uint32), np.zeros(n, np.uint32)
        self.L.o_get_particles(self.h, sp, _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(pid), _ptr(tc))
        return {"z": z, "vx": vx, "vy": vy, "vz": vz, "id": pid, "tc": tc}

    def set_particles(self, sp, d):
        n = len(d["z"])
        arrs = [np.ascontiguousarray(d[k], dtype=np.float64) for k in ("z", "vx", "vy", "vz")]
        arrs += [np.ascontiguousarray(d[k], dtype=np.uint32) for k in ("id", "tc")]
        if self.L.o_set_particles(self.h, sp, n, *[_ptr(a) for a in arrs]) != 0:
            raise MemoryError
        self._keep = getattr(self, "_keep", []) + [arrs]

    def last_moves(self, sp):
        """The last step's moves of species sp in that step's particle order:
        id, z after the push, fate (0 stays, 1 cathode, 2 anode), channel (-1
        none, -2 not a candidate) and channel-choice margin (relative to
        nu_max) of the candidates."""
        n = self.L.o_last_moves_count(self.h, sp)
        m = {"id": np.zeros(n, np.uint32), "z": np.zeros(n), "fate": np.zeros(n, np.int32),
             "ch": np.zeros(n, np.int32), "margin": np.zeros(n)}
        self.L.o_last_moves(self.h, sp, _ptr(m["id"]), _ptr(m["z"]), _ptr(m["fate"]), _ptr(m["ch"]),
                            _ptr(m["margin"]))
        return m

    def hist(self, sp):
        H = np.zeros(self.N + 1, np.int64)
        self.L.o_get_hist(self.h, sp, _ptr(H))
        return H

    def phi(self):
        a = np.zeros(self.N + 1)
        self.L.o_get_phi(self.h, _ptr(a))
        return a

    def E(self):
        a = np.zeros(self.N + 1)
        self.L.o_get_E(self.h, _ptr(a))
        return a

    def tally(self):
        t = OTally()
        self.L.o_get_tally(self.h, C.byref(t))
        return {"abs_count": np.array([[t.abs_count[s][w] for w in range(2)] for s in range(3)]),
                "abs_energy": np.array([[t.abs_energy[s][w] for w in range(2)] for s in range(3)]),
                "n_emit": t.n_emit, "n_repl": t.n_repl, "n_iz": t.n_iz,
                "cand": np.array(list(t.cand)), "coll": np.array(list(t.coll)),
                "nullcoll_exceed": t.nullcoll_exceed}

    def derived(self):
        d = ODerived()
        self.L.o_get_derived(self.h, C.byref(d))
        return {"dz": d.dz, "invdz": d.invdz, "w0": d.w0, "numax": list(d.numax), "lam": list(d.lam)}
