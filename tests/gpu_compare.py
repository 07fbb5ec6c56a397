"""GPU-vs-oracle comparison helpers used by the GPU parity tests and the smoke check.

Tolerances (derived from the arithmetic, see the design notes):
  * deposits, ids, free-flight counters and all integer tallies: bit exact;
  * positions: |dz| <= 1e-5 max(|z|, dz_cell); velocities:
    |dv| <= 1e-5 max(|v|, v_th) per species (FP32 velocities against FP64);
  * absorbed-energy sums: relative 1e-5;
  * phi and E after a solve from identical deposits: 1e-10 of max |phi| / max |E|.
"""
import numpy as np

Q_E = 1.602176634e-19
M_E = 9.1093837015e-31
M_I = 6.6464731e-27 - M_E
REL = 1e-5


def by_id(d):
    o = np.argsort(d["id"], kind="stable")
    return {k: np.asarray(v)[o] for k, v in d.items()}


def vth(cfg, sp):
    if sp == 2:
        return np.sqrt(Q_E * max(cfg["Ti0"], 1e-3) / M_I)
    T = cfg["Te0"] if sp == 0 else cfg["Tc"]
    return np.sqrt(Q_E * max(T, 1e-3) / M_E)


def gpu_state(h, d=0):
    st = {sp: h.particles(d, sp) for sp in range(3)}
    t = h.tally(d)
    return st, t


def oracle_from_gpu(O, cfg, st, t):
    """An oracle diode holding exactly the GPU's particle state and counters."""
    s = O.Sim(cfg)
    s.load()
    for sp in range(3):
        p = st[sp]
        s.set_particles(sp, {"z": p["z"], "vx": p["vx"].astype(np.float64),
                             "vy": p["vy"].astype(np.float64), "vz": p["vz"].astype(np.float64),
                             "id": p["id"], "tc": p["tc"]})
    s.set_counters(t["step"], t["next_id"])
    s.refield()
    return s


def compare_particles(cfg, gp, op, sp, rel=REL):
    """Return a list of problems (empty if the species agree)."""
    probs = []
    g, o = by_id(gp), by_id(op)
    if len(g["id"]) != len(o["id"]) or not np.array_equal(g["id"], o["id"]):
        extra = np.setxor1d(g["id"], o["id"])
        probs.append("species %d: id sets differ (%d vs %d, e.g. %s)" % (sp, len(g["id"]), len(o["id"]),
                                                                         extra[:5]))
        common = np.intersect1d(g["id"], o["id"])
        g = {k: v[np.isin(g["id"], common)] for k, v in g.items()}
        o = {k: v[np.isin(o["id"], common)] for k, v in o.items()}
    if len(g["id"]) == 0:
        return probs
    dzc = cfg["L"] / cfg["N"]
    ez = np.abs(g["z"] - o["z"]) / np.maximum(np.abs(o["z"]), dzc)
    if ez.max() > rel:
        k = int(np.argmax(ez))
        probs.append("species %d: z rel err %.3g at id %d" % (sp, ez.max(), g["id"][k]))
    vt = vth(cfg, sp)
    for c in ("vx", "vy", "vz"):
        ev = np.abs(g[c].astype(np.float64) - o[c]) / np.maximum(np.abs(o[c]), vt)
        if ev.max() > rel:
            k = int(np.argmax(ev))
            probs.append("species %d: %s rel err %.3g at id %d (gpu %r oracle %r)" % (
                sp, c, ev.max(), g["id"][k], float(g[c][k]), float(o[c][k])))
    bad = np.nonzero(g["tc"] != o["tc"])[0]
    if len(bad):
        probs.append("species %d: %d free-flight counters differ, e.g. id %d" % (sp, len(bad), g["id"][bad[0]]))
    return probs


def compare_tallies(gt0, gt1, ot0, ot1, rel=REL, slack=0):
    """Counts must agree exactly; with slack > 0 (a step with that many
    near-ties) each count may differ by up to slack and the energies are not
    compared."""
    probs = []
    for k in ("abs_count", "cand", "coll"):
        dg = np.asarray(gt1[k]) - np.asarray(gt0[k])
        do = np.asarray(ot1[k]) - np.asarray(ot0[k])
        if np.abs(dg - do).max() > slack:
            probs.append("%s: gpu %s oracle %s" % (k, dg.tolist(), do.tolist()))
    for k in ("n_emit", "n_repl", "n_iz"):
        dg, do = gt1[k] - gt0[k], ot1[k] - ot0[k]
        if abs(dg - do) > slack:
            probs.append("%s: gpu %d oracle %d" % (k, dg, do))
    if slack:
        return probs
    eg = np.asarray(gt1["abs_energy"]) - np.asarray(gt0["abs_energy"])
    eo = np.asarray(ot1["abs_energy"]) - np.asarray(ot0["abs_energy"])
    scale = np.maximum(np.abs(eo), 1e-30)
    if (np.abs(eg - eo) / scale > rel).any():
        probs.append("abs_energy: gpu %s oracle %s" % (eg.tolist(), eo.tolist()))
    return probs


# A decision taken in FP32 on the GPU and in FP64 by the oracle may fall on
# different sides when the particle sat within rounding of it: a wall
# crossing within WALL_TIE of the electrode, or a channel choice whose uniform
# lay within CHANNEL_TIE (relative to nu_max) of a cumulative boundary.
WALL_TIE = 1e-9       # of L
CHANNEL_TIE = 1e-6


def near_ties(cfg, s, gpu_after, rel=REL):
    """Particles whose outcome in the oracle's last step differs from the
    GPU's: (species, id, kind, margin, tie).  tie is True when the margin is
    within the rounding band of the decision (a legitimate near-tie)."""
    L = cfg["L"]
    out = []
    for sp in range(3):
        m = s.last_moves(sp)
        g, o = gpu_after[sp], s.particles(sp)
        gi = {int(i): k for k, i in enumerate(g["id"])}
        oi = {int(i): k for k, i in enumerate(o["id"])}
        vt = vth(cfg, sp)
        for k in range(len(m["id"])):
            pid = int(m["id"][k])
            ig, io = gi.get(pid), oi.get(pid)
            if (ig is None) != (io is None):
                z = m["z"][k]
                margin = min(abs(z), abs(L - z)) / L
                out.append((sp, pid, "wall", margin, margin < WALL_TIE))
            elif ig is not None and m["ch"][k] >= -1:
                dv = max(abs(float(g[c][ig]) - o[c][io]) / max(abs(o[c][io]), vt) for c in ("vx", "vy", "vz"))
                if dv > rel:
                    out.append((sp, pid, "channel", m["margin"][k], m["margin"][k] < CHANNEL_TIE))
    return out


def _without(p, ids, newborn_from):
    keep = ~np.isin(p["id"], list(ids)) & (p["id"] < newborn_from)
    return {k: np.asarray(v)[keep] for k, v in p.items()}


def deposit_matches(O, cfg, h, st, d=0):
    """The GPU deposit of the last step equals the oracle's deposit of the same particles."""
    probs = []
    invdz = cfg["N"] / cfg["L"]
    for sp in range(3):
        ref = O.deposit(st[sp]["z"], cfg["N"], invdz)
        got = h.hist(d, sp)
        if not np.array_equal(ref, got):
            k = int(np.argmax(ref != got))
            probs.append("deposit species %d differs at node %d: %d vs %d" % (sp, k, got[k], ref[k]))
    return probs


def field_matches(O, cfg, h, s, d=0, tol=1e-10, exact=False):
    """phi and E of the GPU against the oracle's, within tol of their maxima.
    exact: the reference potential is the exact rational solve of the
    oracle's deposit (the FP64 sweep's own rounding reaches ~1e-10 on the
    largest grids); the GPU rounds its exact integer solution once per term,
    so phi is held to 1e-12 there, E (a difference over one cell) to tol."""
    probs = []
    if exact:
        N = cfg["N"]
        der = O.derive(cfg)
        R = s.hist(2).astype(np.int64) - s.hist(0).astype(np.int64) - s.hist(1).astype(np.int64)
        R[0] = R[N] = 0
        phi_o = O.solve_exact(N, der["dz"], cfg["V"], R, der["w0"])
        E_o = O.efield(N, der["dz"], phi_o)
        tol_phi = 1e-12
    else:
        phi_o = s.phi()
        E_o = s.E()
        tol_phi = tol
    phi_g = h.fields(d)["phi"]
    E_g = h.efield(d)
    sp = max(np.max(np.abs(phi_o)), 1e-30)
    se = max(np.max(np.abs(E_o)), 1e-30)
    if np.max(np.abs(phi_g - phi_o)) > tol_phi * sp:
        probs.append("phi differs by %.3g of max" % (np.max(np.abs(phi_g - phi_o)) / sp))
    if np.max(np.abs(E_g - E_o)) > tol * se:
        probs.append("E differs by %.3g of max" % (np.max(np.abs(E_g - E_o)) / se))
    return probs


def restart_step_check(O, cfg, h, nsteps, d=0, check_every=1, exact_field=False, max_ties=1, ties=None):
    """Advance GPU and oracle from the same state one step at a time; collect
    problems.  A step whose disagreement is fully explained by near-ties
    (near_ties) passes and is reported, up to max_ties over the run; a
    near-tie step's newborns are not compared (their ids may shift).  The
    near-ties found are appended to `ties` when given."""
    probs = []
    n_ties = 0
    for k in range(nsteps):
        st, gt0 = gpu_state(h, d)
        if k % check_every == 0:
            s = oracle_from_gpu(O, cfg, st, gt0)
            for p in deposit_matches(O, cfg, h, st, d) + field_matches(O, cfg, h, s, d, exact=exact_field):
                probs.append("step %d (before): %s" % (gt0["step"], p))
            ot0 = s.tally()
            s.step()
            ot1 = s.tally()
        h.step(1)
        if k % check_every == 0:
            st1, gt1 = gpu_state(h, d)
            step_probs = []
            for sp in range(3):
                step_probs += compare_particles(cfg, st1[sp], s.particles(sp), sp)
            step_probs += compare_tallies(gt0, gt1, ot0, ot1)
            if gt1["next_id"] != s.next_id:
                step_probs.append("next_id gpu %d oracle %d" % (gt1["next_id"], s.next_id))
            if step_probs:
                found = near_ties(cfg, s, st1)
                real = [t for t in found if not t[4]]
                if found and not real and n_ties + len(found) <= max_ties:
                    ids = {t[1] for t in found}
                    nb = int(gt0["next_id"])
                    again = []
                    for sp in range(3):
                        again += compare_particles(cfg, _without(st1[sp], ids, nb), _without(s.particles(sp), ids, nb),
                                                   sp)
                    again += compare_tallies(gt0, gt1, ot0, ot1, slack=len(found))
                    if not again:
                        n_ties += len(found)
                        for t in found:
                            print("near-tie at step %d: species %d id %d, %s margin %.3g" % (
                                gt0["step"], t[0], t[1], t[2], t[3]), flush=True)
                        if ties is not None:
                            ties.extend(found)
                        step_probs = []
                if step_probs and found:
                    step_probs.append("decisions that differ: %s" % (found[:5],))
            probs += ["step %d: %s" % (gt0["step"], p) for p in step_probs]
        if len(probs) > 20:
            break
    return probs
