"""Baseline emission-flux scan of the paper's benchmark diode.

The eleven imposed fluxes of the paper's benchmark suite ("Benchmark cases";
results in "Flux-scan results", Table 2 for the emitted-electron transport
and Table 4 for the boundary energy terms) run as one batch of diodes on the
paper's preset (10 cm helium gap, 40 V, elastic and charge-exchange
collisions only).  Reported per flux: late-time averages of the backflow,
net and anode fluxes, the backflow ratio and efficiencies, the boundary
energy terms, the depth and position of the potential minimum in front of
the cathode (time-averaged potential), and the backflow ratio's time series.

Host orchestration only: the steps are the library's graph-replayed step,
the averages come from pic_diagnostics over the tally snapshot ring and from
the device's time-averaged potential.

    python -m paper_2605_07083_amd.fluxscan --ppc 100 --steps 4500000 --out scan.json
    python -m paper_2605_07083_amd.fluxscan --ppc 1000 --fluxes 7.0e19 7.25e19 --out transition.json
    python -m paper_2605_07083_amd.fluxscan --ppc 100 --sensitivity --out sensitivity.json
    python -m paper_2605_07083_amd.fluxscan --ppc 100 --phase --out phase.json
"""
import argparse
import json
import sys
import time

import numpy as np

from . import pic, presets

FLUXES = (1.5e19, 2.0e19, 4.5e19, 5.0e19, 6.0e19, 7.0e19, 7.25e19, 7.5e19, 8.0e19, 1.0e20, 1.2e20)
# the three transport states of the paper's phase-space figure
PHASE_FLUXES = (1.5e19, 7.0e19, 1.0e20)
Q_E, M_E = 1.602176634e-19, 9.1093837015e-31
PHASE_NZ = 50                 # 2 mm rows over the 10 cm gap
PHASE_NV = 160                # v_z over [-8, 8) v_te, v_te = (e T_e0 / m_e)^(1/2)
PHASE_VMAX = 8.0
REGION_ROWS = 10              # 2 cm regions, as in the paper's regional distributions
PHASE_EARLY = (100000, 1000000)   # steps of the gap-integrated snapshots
TALLY_PERIOD = 1000
RING = 1024                   # snapshots the device keeps
NEAR_CATHODE = 0.1            # fraction of the gap searched for the potential minimum


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def configs(ppc, fluxes=FLUXES):
    """One diode per flux on the paper's preset, ppc particles per cell and
    species (the paper loads 1000)."""
    base = presets.paper()
    return [presets.scaled(base, gamma_emit=float(g), diode=d, n_load=int(ppc) * base["N"],
                           tally_period=TALLY_PERIOD) for d, g in enumerate(fluxes)]


# The paper's selected sensitivity cases ("Selected sensitivity to collisional
# modeling details", Table 3, cases 1-7): label, flux, changes to the preset.
SENSITIVITY = (
    ("excitation on", 1.5e19, {"exc": True}),
    ("excitation on", 4.5e19, {"exc": True}),
    ("excitation on", 5.0e19, {"exc": True}),
    ("excitation on", 8.0e19, {"exc": True}),
    ("excitation on", 1.0e20, {"exc": True}),
    ("electron-side neutral target 1740 K", 7.0e19, {"Tne_K": 1740.0}),
    ("charge exchange off", 1.0e20, {"cx": False}),
)


def sensitivity_configs(ppc, cases=None):
    """The SENSITIVITY cases (all, or the listed indices) as one batch."""
    base = presets.paper()
    out = []
    for d, (label, g, ch) in enumerate(SENSITIVITY):
        if cases is not None and d not in cases:
            continue
        kw = dict(gamma_emit=float(g), diode=d, n_load=int(ppc) * base["N"], tally_period=TALLY_PERIOD)
        channels = base["channels"]
        if ch.get("exc"):
            channels |= presets.CH_EXC
        if ch.get("cx") is False:
            channels &= ~presets.CH_CX
        kw["channels"] = channels
        if "Tne_K" in ch:
            kw["Tne"] = ch["Tne_K"] * presets.KB_OVER_E
        out.append(presets.scaled(base, **kw))
    return out


def check_windows(steps, window, chunk):
    """The averaging window and the series' chunk are whole tally periods
    that the snapshot ring still holds, and the window is whole chunks."""
    if window <= 0 or chunk <= 0 or steps <= window:
        raise ValueError("need 0 < window < steps and chunk > 0")
    if window % TALLY_PERIOD or chunk % TALLY_PERIOD:
        raise ValueError("window and chunk must be multiples of %d steps" % TALLY_PERIOD)
    if window > RING * TALLY_PERIOD or chunk > RING * TALLY_PERIOD:
        raise ValueError("window and chunk must be at most %d steps" % (RING * TALLY_PERIOD))
    if window % chunk:
        raise ValueError("window must be a multiple of chunk")


def potential_minimum(cfg, phi):
    """Depth (V, relative to the cathode) and position (m) of the lowest
    potential within NEAR_CATHODE of the gap from the cathode."""
    n = max(2, int(NEAR_CATHODE * cfg["N"]))
    j = int(np.argmin(phi[:n + 1]))
    return float(phi[j]), j * cfg["L"] / cfg["N"]


def run(ppc=100, steps=4500000, window=1000000, chunk=250000, max_seconds=0.0, fluxes=FLUXES, tune_steps=256,
        cfgs=None, labels=None, phase_every=0):
    """phase_every > 0: electron phase space summed over samples every
    phase_every steps of the late-time window, plus single snapshots at the
    PHASE_EARLY steps (both electron populations, device histograms)."""
    check_windows(steps, window, chunk)
    if phase_every and (chunk % phase_every or window % phase_every):
        raise ValueError("phase_every must divide chunk and window")
    if cfgs is None:
        cfgs = configs(ppc, fluxes)
    h = pic.Handle(cfgs)
    tuning = h.autotune(trial_steps=tune_steps)
    step = h.diagnostics(0, 0)["step_end"]
    phase = early = None
    if phase_every:
        import torch
        vte = [(Q_E * c["Te0"] / M_E) ** 0.5 for c in cfgs]
        lim = [(-PHASE_VMAX * v, PHASE_VMAX * v) for v in vte]
        with torch.cuda.stream(h.stream):
            phase = [[torch.zeros((PHASE_NZ, PHASE_NV + 2), dtype=torch.int64, device=h.device) for _ in range(2)]
                     for _ in cfgs]
        early = {t: None for t in PHASE_EARLY}

    def sample(into):
        for d in range(len(cfgs)):
            for sp in range(2):
                h.phase_space(d, sp, PHASE_NZ, PHASE_NV, lim[d][0], lim[d][1], out=into[d][sp])

    def advance(step, end):
        """Step to `end`, taking the early snapshots on the way."""
        if phase_every:
            for t in sorted(early):
                if early[t] is None and step < t <= end:
                    h.step(t - step)
                    step = t
                    with torch.cuda.stream(h.stream):
                        early[t] = [[torch.zeros_like(phase[0][0]) for _ in range(2)] for _ in cfgs]
                    sample(early[t])
        return step

    target = step + (-step % chunk)            # the series starts on a chunk boundary
    step = advance(step, target)
    if target > step:
        h.step(target - step)
        step = target
    series = [[] for _ in cfgs]
    averaging = False
    _log("fluxscan: %d diodes, %d particles per species each, schedule %s, from step %d"
         % (len(cfgs), cfgs[0]["n_load"], {k: tuning[k] for k in ("ppt", "grid", "sort_period", "use_graph")},
            step))
    t0 = time.time()
    step0 = step
    stopped_early = False
    while step < steps:
        if not averaging and steps - step <= window:
            h.avg_control(-1, True)
            averaging = True
            avg_from = step
        n = min(chunk, steps - step)
        end = step + n
        step = advance(step, end)
        rest = end - step
        if phase_every and averaging:
            for _ in range(rest // phase_every):
                h.step(phase_every)
                sample(phase)
            if rest % phase_every:
                h.step(rest % phase_every)
        elif rest:
            h.step(rest)
        h.sync()
        step = end
        for d in range(len(cfgs)):
            g = h.diagnostics(d, n)
            series[d].append([step, g["backflow_pct"], g["gamma_net"], float(np.sum(g["n_live"]))])
        el = time.time() - t0
        _log("fluxscan: step %d of %d, %.0f s, %.1f us per step; backflow %% %s"
             % (step, steps, el, 1e6 * el / (step - step0),
                " ".join("%.1f" % series[d][-1][1] for d in range(len(cfgs)))))
        if max_seconds and el > max_seconds and step < steps:
            stopped_early = True
            break
    wall = time.time() - t0
    # late-time window: the requested one, or what the run reached
    win = window if not stopped_early else min(window, step - step0)
    out = {"ppc": ppc, "steps": step, "steps_requested": steps, "window": win, "stopped_early": stopped_early,
           "wall_s": wall, "schedule": tuning, "diodes": []}
    for d, cfg in enumerate(cfgs):
        g = h.diagnostics(d, win)
        rec = {k: g[k] for k in pic._DIAG_SCALARS + pic._DIAG_SCALARS2}
        rec["label"] = labels[d] if labels else "baseline"
        rec["channels"] = cfg["channels"]
        rec["Tne_eV"] = cfg["Tne"]
        rec["q_back_em_cath"] = float(g["q_abs"][1][0])
        rec["q_back_p_cath"] = float(g["q_abs"][0][0])
        rec["q_ion_cath"] = float(g["q_abs"][2][0])
        rec["n_live"] = [float(x) for x in g["n_live"]]
        if averaging:
            phi = h.fields(d, time_avg=True)["phi"]
            rec["phi_min_V"], rec["phi_min_z_m"] = potential_minimum(cfg, phi)
            rec["avg_from_step"] = avg_from
        rec["series"] = series[d]
        if phase_every:
            rec["phase_vlim"] = list(lim[d])
            rec["phase_late"] = [phase[d][sp].cpu().numpy().tolist() for sp in range(2)]
            rec["phase_early"] = {str(t): [e[d][sp].cpu().numpy().tolist() for sp in range(2)]
                                  for t, e in early.items() if e is not None}
            rec["kinetics"] = kinetic_summary(np.array(rec["phase_late"]))
        out["diodes"].append(rec)
    h.close()
    return out


def kinetic_summary(ph):
    """Figures of the electron velocity distributions from summed phase-space
    counts ph[species][row][column] (plasma, emitted): per 2 cm region and
    over the gap, the emitted share of the electrons, the share moving toward
    the cathode (v_z < 0), the share with |v_z| < v_te / 5 (a Maxwellian at
    T_e0 puts 0.159 there), and the half L1 distance of the gap-integrated
    v_z distribution from the T_e0 Maxwellian (0 identical, 1 disjoint)."""
    from math import erf, sqrt
    ph = np.asarray(ph, dtype=np.float64)
    nz, w = ph.shape[1], ph.shape[2]
    nv = w - 2
    edges = np.linspace(-PHASE_VMAX, PHASE_VMAX, nv + 1)          # in units of v_te
    centre = 0.5 * (edges[:-1] + edges[1:])
    slow = np.abs(centre) < 0.2
    back = centre < 0.0
    cdf = np.array([0.5 * (1.0 + erf(x / sqrt(2.0))) for x in edges])
    maxw = np.diff(cdf)
    out = {"regions": []}

    def figures(block):
        tot = block.sum()
        if tot == 0:
            return None
        allv = block.sum(axis=0)                # both species
        inside = allv[1:nv + 1]
        return {"n": float(tot), "emitted_share": float(block[1].sum() / tot),
                "toward_cathode": float((inside[back].sum() + allv[0]) / tot),
                "slow_share": float(inside[slow].sum() / tot)}

    for r0 in range(0, nz, REGION_ROWS):
        out["regions"].append(figures(ph[:, r0:r0 + REGION_ROWS, :].sum(axis=1)))
    gap = ph.sum(axis=1)
    out["gap"] = figures(gap)
    f = gap.sum(axis=0)[1:nv + 1]
    if f.sum() > 0:
        out["gap"]["l1_from_maxwellian"] = float(0.5 * np.abs(f / f.sum() - maxw / maxw.sum()).sum())
    return out


def table(res):
    rows = ["| case | Γ_emit (1e19) | Γ_ref | Γ_net | Γ_anode | backflow % | q_cool1 | q_cool2 | q_anode1 | φ_min (V) |",
            "|---|---|---|---|---|---|---|---|---|---|"]
    for r in res["diodes"]:
        rows.append("| %s | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f | %s |" % (
            r["label"], r["gamma_emit"] / 1e19, r["gamma_ref"] / 1e19, r["gamma_net"] / 1e19, r["gamma_anode"] / 1e19,
            r["backflow_pct"], r["q_cool1"], r["q_cool2"], r["q_anode1"],
            "%.3f" % r["phi_min_V"] if "phi_min_V" in r else "—"))
    return "\n".join(rows)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--ppc", type=int, default=100, help="particles per cell and species (paper: 1000)")
    ap.add_argument("--steps", type=int, default=4500000)
    ap.add_argument("--window", type=int, default=1000000, help="late-time averaging window (steps)")
    ap.add_argument("--chunk", type=int, default=250000, help="steps per series point")
    ap.add_argument("--max-seconds", type=float, default=0.0, help="stop stepping after this wall time")
    ap.add_argument("--fluxes", type=float, nargs="+", default=list(FLUXES), help="imposed fluxes (m^-2 s^-1)")
    ap.add_argument("--sensitivity", action="store_true", help="the paper's sensitivity cases instead of the scan")
    ap.add_argument("--cases", type=int, nargs="+", default=None, help="with --sensitivity: case indices 0-6 (the paper's cases 1-7)")
    ap.add_argument("--phase", action="store_true",
                    help="the three states of the paper's phase-space figure, with electron phase space")
    ap.add_argument("--phase-every", type=int, default=10000, help="steps between phase-space samples")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.phase:
        res = run(a.ppc, a.steps, a.window, a.chunk, a.max_seconds, fluxes=list(PHASE_FLUXES),
                  phase_every=a.phase_every)
    elif a.sensitivity:
        picked = [i for i in range(len(SENSITIVITY)) if a.cases is None or i in a.cases]
        res = run(a.ppc, a.steps, a.window, a.chunk, a.max_seconds, cfgs=sensitivity_configs(a.ppc, picked),
                  labels=[SENSITIVITY[i][0] for i in picked])
    else:
        res = run(a.ppc, a.steps, a.window, a.chunk, a.max_seconds, fluxes=a.fluxes)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    print(table(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
