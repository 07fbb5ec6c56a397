"""Thin ctypes binding of the gfx950 PIC-MCC library (``libpic.so``).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides the device workspace and the stream.  Importing
works without a GPU (for the host-only calls); creating a ``Handle`` needs the
built library and a ROCm device and fails loudly otherwise.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOSPACE, PIC_EHIP, PIC_ENULLCOLL, PIC_ENAN, PIC_ERANGE = 0, -1, -2, -3, -4, -5, -6
# warm-start state: rows per diode and quantile levels (include/pic.h, pic_init_from_state)
STATE_ROWS = 39
STATE_LEVELS = (0.0, 0.02, 0.1, 0.25, 0.5, 0.75, 0.9, 0.98, 1.0)
NSP, NCH = 3, 5


class PicConfig(C.Structure):
    _fields_ = [("L", C.c_double), ("N", C.c_int32), ("flags", C.c_int32), ("V", C.c_double),
                ("n0", C.c_double), ("Te0", C.c_double), ("Ti0", C.c_double), ("n_load", C.c_int64),
                ("gamma_emit", C.c_double), ("Tc", C.c_double), ("ng", C.c_double),
                ("Tne", C.c_double), ("Tni", C.c_double), ("dt", C.c_double),
                ("sig_el", C.c_double), ("sig_x0", C.c_double), ("lotz_a", C.c_double),
                ("sig_cx", C.c_double), ("sig_iel", C.c_double), ("channels", C.c_uint32),
                ("replenish", C.c_int32), ("seed", C.c_uint32), ("diode", C.c_uint32),
                ("tally_period", C.c_int32), ("sort_period", C.c_int32),
                ("capacity_factor", C.c_double)]


class PicTally(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_live", C.c_int64 * 3), ("abs_count", (C.c_int64 * 2) * 3),
                ("abs_energy", (C.c_double * 2) * 3), ("n_emit", C.c_int64), ("n_repl", C.c_int64),
                ("n_iz", C.c_int64), ("cand", C.c_int64 * 2), ("coll", C.c_int64 * 5),
                ("next_id", C.c_uint32), ("err_bits", C.c_uint32), ("rare_spill", C.c_int64),
                ("resorts", C.c_int64), ("resorts_ions_kept", C.c_int64)]


_DIAG_SCALARS = ("gamma_emit", "gamma_emit_meas", "gamma_ref", "gamma_net", "gamma_anode",
                 "backflow_pct", "eta_net", "eta_anode")
_DIAG_SCALARS2 = ("wf_eff", "q_emit_theory", "q_ion_cath_recomb", "q_cool1", "q_cool2",
                  "q_ion_anode_recomb", "q_anode1", "q_anode2", "phi_vc_eff")


class PicDiag(C.Structure):
    _fields_ = ([("step_begin", C.c_int64), ("step_end", C.c_int64)]
                + [(n, C.c_double) for n in _DIAG_SCALARS]
                + [("gamma_abs", (C.c_double * 2) * 3), ("q_abs", (C.c_double * 2) * 3)]
                + [(n, C.c_double) for n in _DIAG_SCALARS2]
                + [("n_live", C.c_double * 3)])


class PicSteady(C.Structure):
    _fields_ = [("steady", C.c_int32), ("blocks", C.c_int32), ("block_steps", C.c_int64),
                ("steady_step", C.c_int64), ("backflow_pct", C.c_double), ("blocks_averaged", C.c_int32),
                ("pad", C.c_int32), ("last_backflow_pct", C.c_double)]


class PicDerived(C.Structure):
    _fields_ = [("dz", C.c_double), ("invdz", C.c_double), ("w0", C.c_double),
                ("numax", C.c_double * 2), ("lam", C.c_double * 2),
                ("emit_per_step", C.c_double), ("capacity", C.c_int64 * 3)]


SYMBOLS = ["pic_derive", "pic_workspace_size", "pic_init", "pic_init_from_profiles", "pic_init_from_state", "pic_step", "pic_sync", "pic_get_tally", "pic_get_snapshot",
           "pic_diagnostics", "pic_get_fields", "pic_avg_reset", "pic_avg_control", "pic_get_hist", "pic_get_efield", "pic_phase_space",
           "pic_get_particles", "pic_set_particles", "pic_set_counters", "pic_refield",
           "pic_step_timed", "pic_set_tuning", "pic_get_tuning", "pic_autotune", "pic_steady_state", "pic_steady_from_series", "pic_checkpoint_size", "pic_save", "pic_load", "pic_last_error",
           "pic_destroy"]

_lib = None


def lib():
    """Load libpic.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpic.so is not built: run __graft_entry__.build() (hipcc, gfx950)")
    # PyTorch ships its own HIP runtime: load it first, so that this library
    # binds to the same one (a library loaded before torch would bind to the
    # system runtime, and the two would not share kernels or memory)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, i, i64, d = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "pic_derive": ([C.POINTER(PicConfig), C.POINTER(PicDerived)], i),
        "pic_workspace_size": ([C.POINTER(PicConfig), i, C.POINTER(C.c_size_t)], i),
        "pic_init": ([C.POINTER(PicConfig), i, P, C.c_size_t, P, C.POINTER(P)], i),
        "pic_init_from_profiles": ([C.POINTER(PicConfig), i, P, C.c_size_t, P, P, C.POINTER(P)], i),
        "pic_init_from_state": ([C.POINTER(PicConfig), i, P, C.c_size_t, P, P, C.POINTER(P)], i),
        "pic_step": ([P, i64], i),
        "pic_sync": ([P], i),
        "pic_get_tally": ([P, i, C.POINTER(PicTally)], i),
        "pic_get_snapshot": ([P, i, i64, C.POINTER(PicTally)], i),
        "pic_diagnostics": ([P, i, i64, C.POINTER(PicDiag)], i),
        "pic_get_fields": ([P, i, P, P, P, i], i),
        "pic_avg_reset": ([P, i], i),
        "pic_avg_control": ([P, i, i], i),
        "pic_get_hist": ([P, i, i, P], i),
        "pic_get_efield": ([P, i, P], i),
        "pic_phase_space": ([P, i, i, i, i, d, d, P], i),
        "pic_get_particles": ([P, i, i, i64, C.POINTER(i64), P, P, P, P, P, P], i),
        "pic_set_particles": ([P, i, i, i64, P, P, P, P, P, P], i),
        "pic_set_counters": ([P, i, i64, C.c_uint32], i),
        "pic_refield": ([P], i),
        "pic_step_timed": ([P, i64, C.POINTER(d), C.POINTER(d)], i),
        "pic_set_tuning": ([P, i, i, i, i], i),
        "pic_get_tuning": ([P, C.POINTER(i), C.POINTER(i), C.POINTER(i), C.POINTER(i)], i),
        "pic_autotune": ([P, i64, C.POINTER(i), C.POINTER(i), C.POINTER(i), C.POINTER(i), C.POINTER(d)], i),
        "pic_steady_state": ([P, i, i, d, d, C.POINTER(PicSteady)], i),
        "pic_steady_from_series": ([P, P, i, d, d, C.POINTER(i), C.POINTER(d), C.POINTER(i)], i),
        "pic_checkpoint_size": ([P, C.POINTER(C.c_size_t)], i),
        "pic_save": ([P, P, C.c_size_t, C.POINTER(C.c_size_t)], i),
        "pic_load": ([P, P, C.c_size_t], i),
        "pic_last_error": ([], C.c_char_p),
        "pic_destroy": ([P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pic error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != PIC_OK:
        raise PicError(rc, lib().pic_last_error().decode(errors="replace"))


def make_config(p: dict) -> PicConfig:
    c = PicConfig()
    for name, _ in PicConfig._fields_:
        if name in ("flags",):
            continue
        if name == "sort_period":
            c.sort_period = int(p.get("sort_period", 0))
        elif name == "capacity_factor":
            c.capacity_factor = float(p.get("capacity_factor", 0.0))
        elif name == "tally_period":
            c.tally_period = int(p.get("tally_period", 100))
        else:
            setattr(c, name, p[name])
    return c


def _cfg_array(cfgs):
    arr = (PicConfig * len(cfgs))()
    for k, p in enumerate(cfgs):
        arr[k] = make_config(p)
    return arr


def pic_derive(p: dict) -> dict:
    c = make_config(p)
    out = PicDerived()
    _check(lib().pic_derive(C.byref(c), C.byref(out)))
    return {"dz": out.dz, "invdz": out.invdz, "w0": out.w0, "numax": list(out.numax),
            "lam": list(out.lam), "emit_per_step": out.emit_per_step, "capacity": list(out.capacity)}


def pic_workspace_size(cfgs) -> int:
    arr = _cfg_array(cfgs)
    n = C.c_size_t()
    _check(lib().pic_workspace_size(arr, len(cfgs), C.byref(n)))
    return n.value


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def steady_from_series(br, n_live, tol_pp=1.0, tol_rel=0.01):
    """Host-only steady-state criterion on per-block series (see pic.h)."""
    br = np.ascontiguousarray(br, np.float64)
    nl = np.ascontiguousarray(n_live, np.float64)
    b, m = C.c_int(), C.c_int()
    v = C.c_double()
    _check(lib().pic_steady_from_series(_ptr(br), _ptr(nl), len(br), tol_pp, tol_rel, C.byref(b), C.byref(v),
                                        C.byref(m)))
    return {"steady_block": b.value, "backflow_pct": v.value, "blocks_averaged": m.value}


def _tally_dict(t):
    return {"step": t.step, "n_live": np.array(list(t.n_live)),
            "abs_count": np.array([[t.abs_count[s][w] for w in range(2)] for s in range(3)]),
            "abs_energy": np.array([[t.abs_energy[s][w] for w in range(2)] for s in range(3)]),
            "n_emit": t.n_emit, "n_repl": t.n_repl, "n_iz": t.n_iz,
            "cand": np.array(list(t.cand)), "coll": np.array(list(t.coll)),
            "next_id": t.next_id, "err_bits": t.err_bits, "rare_spill": t.rare_spill,
            "resorts": t.resorts, "resorts_ions_kept": t.resorts_ions_kept}


class Handle:
    """One or more diodes advanced together on one GPU."""

    def __init__(self, cfgs, device="cuda:0", ppt=None, grid=None, densities=None, state=None):
        """densities: optional device tensor [n_diodes][2][max N] float64 of
        cell-centre electron and ion densities (m^-3) for the warm start;
        state: optional device tensor [n_diodes][STATE_ROWS][max N] float64,
        densities, potential and velocity quantiles (pic_init_from_state)."""
        import torch
        if isinstance(cfgs, dict):
            cfgs = [cfgs]
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm GPU visible: the PIC library runs only on the GPU")
        self.cfgs = [dict(c) for c in cfgs]
        self.nd = len(cfgs)
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self._arr = _cfg_array(cfgs)
        nbytes = pic_workspace_size(cfgs)
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        if densities is not None and state is not None:
            raise ValueError("give densities or state, not both")
        if state is not None:
            nmax = max(c["N"] for c in cfgs)
            if (state.device != self.device or state.dtype != torch.float64
                    or tuple(state.shape) != (self.nd, STATE_ROWS, nmax) or not state.is_contiguous()):
                raise ValueError("state must be a contiguous float64 [%d, %d, %d] tensor on %s"
                                 % (self.nd, STATE_ROWS, nmax, self.device))
            _check(lib().pic_init_from_state(self._arr, self.nd, C.c_void_p(self.ws.data_ptr()), nbytes,
                                             C.c_void_p(self.stream.cuda_stream),
                                             C.c_void_p(state.data_ptr()), C.byref(h)))
        elif densities is None:
            _check(lib().pic_init(self._arr, self.nd, C.c_void_p(self.ws.data_ptr()), nbytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        else:
            nmax = max(c["N"] for c in cfgs)
            if (densities.device != self.device or densities.dtype != torch.float64
                    or tuple(densities.shape) != (self.nd, 2, nmax) or not densities.is_contiguous()):
                raise ValueError("densities must be a contiguous float64 [%d, 2, %d] tensor on %s"
                                 % (self.nd, nmax, self.device))
            _check(lib().pic_init_from_profiles(self._arr, self.nd, C.c_void_p(self.ws.data_ptr()), nbytes,
                                                C.c_void_p(self.stream.cuda_stream),
                                                C.c_void_p(densities.data_ptr()), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().pic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- stepping -------------------------------------------------------
    def step(self, n=1):
        _check(lib().pic_step(self.h, int(n)))

    def sync(self):
        _check(lib().pic_sync(self.h))

    def refield(self):
        _check(lib().pic_refield(self.h))

    def live_total(self):
        """Live particles summed over every diode and species (synchronises)."""
        return int(sum(self.tally(d)["n_live"].sum() for d in range(self.nd)))

    def step_timed(self, n):
        """pic_step_timed: mean particle-kernel duration and the events' total
        (ms).  Nothing is read from the device inside; the caller reads live
        counts before and after (live_total)."""
        k, tot = C.c_double(), C.c_double()
        _check(lib().pic_step_timed(self.h, int(n), C.byref(k), C.byref(tot)))
        return {"particle_kernel_ms": k.value, "total_ms": tot.value}

    # --- state access ---------------------------------------------------
    def tally(self, d=0):
        t = PicTally()
        _check(lib().pic_get_tally(self.h, d, C.byref(t)))
        return _tally_dict(t)

    def snapshot(self, d, step):
        """Tallies of diode d at the end of tally step `step` (pic_get_snapshot)."""
        t = PicTally()
        _check(lib().pic_get_snapshot(self.h, d, int(step), C.byref(t)))
        return _tally_dict(t)

    def diagnostics(self, d=0, window_steps=0):
        o = PicDiag()
        _check(lib().pic_diagnostics(self.h, d, int(window_steps), C.byref(o)))
        res = {"step_begin": o.step_begin, "step_end": o.step_end}
        for n in _DIAG_SCALARS + _DIAG_SCALARS2:
            res[n] = getattr(o, n)
        for n in ("gamma_abs", "q_abs"):
            v = getattr(o, n)
            res[n] = np.array([[v[s][w] for w in range(2)] for s in range(3)])
        res["n_live"] = np.array(list(o.n_live))
        return res

    def fields(self, d=0, time_avg=False):
        nn = self.cfgs[d]["N"] + 1
        phi, ne, ni = np.zeros(nn), np.zeros(nn), np.zeros(nn)
        _check(lib().pic_get_fields(self.h, d, _ptr(phi), _ptr(ne), _ptr(ni), 1 if time_avg else 0))
        return {"phi": phi, "n_e": ne, "n_i": ni}

    def avg_reset(self, on=True):
        _check(lib().pic_avg_reset(self.h, 1 if on else 0))

    def avg_control(self, d, on=True):
        """Clear diode d's time averages and switch its averaging on or off."""
        _check(lib().pic_avg_control(self.h, int(d), 1 if on else 0))

    def hist(self, d=0, sp=0):
        H = np.zeros(self.cfgs[d]["N"] + 1, np.int64)
        _check(lib().pic_get_hist(self.h, d, sp, _ptr(H)))
        return H

    def phase_space(self, d, sp, nz, nv, vmin, vmax, out=None):
        """(z, v_z) counts of species sp of diode d, nz rows of nv + 2 columns
        (under- and overflow of v_z at the ends); added to `out` (a device
        int64 tensor of that shape) when given, else to a new zeroed one.
        Stream-ordered: read it after sync()."""
        import torch
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.zeros((nz, nv + 2), dtype=torch.int64, device=self.device)
        if (out.dtype != torch.int64 or tuple(out.shape) != (nz, nv + 2) or not out.is_contiguous()
                or out.device != self.device):
            raise ValueError("out must be a contiguous int64 tensor of shape (nz, nv + 2) on the handle's device")
        _check(lib().pic_phase_space(self.h, int(d), int(sp), int(nz), int(nv), float(vmin), float(vmax),
                                     C.c_void_p(out.data_ptr())))
        return out

    def efield(self, d=0):
        E = np.zeros(self.cfgs[d]["N"] + 1)
        _check(lib().pic_get_efield(self.h, d, _ptr(E)))
        return E

    def particles(self, d=0, sp=0):
        cap = int(pic_derive(self.cfgs[d])["capacity"][sp])
        z = np.zeros(cap)
        vx, vy, vz = (np.zeros(cap, np.float32) for _ in range(3))
        pid, tc = np.zeros(cap, np.uint32), np.zeros(cap, np.uint32)
        n = C.c_int64()
        _check(lib().pic_get_particles(self.h, d, sp, cap, C.byref(n), _ptr(z), _ptr(vx), _ptr(vy),
                                       _ptr(vz), _ptr(pid), _ptr(tc)))
        k = n.value
        return {"z": z[:k].copy(), "vx": vx[:k].copy(), "vy": vy[:k].copy(), "vz": vz[:k].copy(),
                "id": pid[:k].copy(), "tc": tc[:k].copy()}

    def set_particles(self, d, sp, p):
        z = np.ascontiguousarray(p["z"], np.float64)
        arrs = [z] + [np.ascontiguousarray(p[k], np.float32) for k in ("vx", "vy", "vz")]
        arrs += [np.ascontiguousarray(p[k], np.uint32) for k in ("id", "tc")]
        _check(lib().pic_set_particles(self.h, d, sp, len(z), *[_ptr(a) for a in arrs]))

    def set_tuning(self, ppt=0, grid=0, sort_period=0, use_graph=-1):
        _check(lib().pic_set_tuning(self.h, int(ppt), int(grid), int(sort_period), int(use_graph)))

    def autotune(self, trial_steps=64):
        v = [C.c_int() for _ in range(4)]
        ms = C.c_double()
        _check(lib().pic_autotune(self.h, int(trial_steps), *[C.byref(x) for x in v], C.byref(ms)))
        return dict(zip(("ppt", "grid", "sort_period", "use_graph"), [x.value for x in v]), ms_per_step=ms.value)

    def steady_state(self, d=0, block_tallies=50, tol_pp=1.0, tol_rel=0.01):
        o = PicSteady()
        _check(lib().pic_steady_state(self.h, d, int(block_tallies), float(tol_pp), float(tol_rel), C.byref(o)))
        return {"steady": bool(o.steady), "blocks": o.blocks, "block_steps": o.block_steps,
                "steady_step": o.steady_step, "backflow_pct": o.backflow_pct,
                "blocks_averaged": o.blocks_averaged, "last_backflow_pct": o.last_backflow_pct}

    def tuning(self):
        v = [C.c_int() for _ in range(4)]
        _check(lib().pic_get_tuning(self.h, *[C.byref(x) for x in v]))
        return dict(zip(("ppt", "grid", "sort_period", "use_graph"), [x.value for x in v]))

    def save(self):
        """Checkpoint image of every diode (numpy uint8 array, host memory)."""
        n = C.c_size_t()
        _check(lib().pic_checkpoint_size(self.h, C.byref(n)))
        buf = np.empty(n.value, np.uint8)
        w = C.c_size_t()
        _check(lib().pic_save(self.h, _ptr(buf), buf.size, C.byref(w)))
        return buf[:w.value]

    def load(self, image):
        """Restore a checkpoint image written by save() of a handle with the same configurations."""
        buf = np.ascontiguousarray(image, np.uint8)
        _check(lib().pic_load(self.h, _ptr(buf), buf.size))

    def set_counters(self, d, step, next_id):
        _check(lib().pic_set_counters(self.h, d, int(step), int(next_id)))
