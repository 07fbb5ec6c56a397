"""GPU parity on the paths and configurations the basic parity cases do not
reach, and the library's error reporting, through the C ABI.

* The particle kernel's spill of rare items (collision candidates, absorbed
  particles) to the global lists when a wave's LDS queue fills, worked off by
  the sources kernel: forced with a strongly collisional diode on a tiny grid.
* The paper's benchmark diode ("Model": numerical setup; "Emission and
  collisions": elastic + charge exchange only, electron- and ion-side
  neutral targets at 300 K and 1740 K, 40 V, 4096 cells -- the tiled field
  kernel, nine tiles, the last of one node) and two of its sensitivity cases (Table 3: charge exchange off; the
  electron-side neutral target at 1740 K), at 20 particles per cell.
* Thermionic newborns placed beyond the anode (a gap shorter than one
  step): every step's snapshot holds the record block's tallies of them.
* The largest batch (256 diodes, one on the tiled field grid), through
  re-sorts with graph replay, then restart parity on three of them.
* The 32-diode emission sweep (100k-600k particles per species per diode):
  one restart step against the oracle on three diodes of different sizes.
* Graph replay of runs shorter than a re-sort period equals plain launches,
  and the live timing covers them.
* The steady-state verdict on the device ring equals the host criterion on
  the same snapshots.
* Re-sorts that leave the ions in their buffer while the diode's buffer
  parity flips: restart parity through them, phase-space counts and a
  checkpoint read through the kept buffer.
* Error reporting: the null-collision bound, non-finite particle input, a
  node deposit reaching 2^53.
"""
import numpy as np
import pytest

from _helpers import empty, quiet_cfg
from gpu_compare import by_id, gpu_state, oracle_from_gpu, restart_step_check
from paper_2605_07083_amd import presets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2605_07083_amd import pic as P
    P.lib()
    return P


def _say(msg):
    print(msg, flush=True)


def test_rare_queue_spill_parity(pic, O):
    """A collision candidate rate near 1 - e^-1 per step and a grid of 8
    blocks (each wave streams ~16k particles per run) overflow the waves'
    LDS queues; the spilled items go through the sources kernel's pass."""
    cfg = presets.scaled(presets.tiny(), ng=3.2e23, Te0=5.0, gamma_emit=1e21)
    _say("case: rare-item spill, n_g = 3.2e23, grid 8, 4 particles per thread")
    h = pic.Handle(cfg)
    lam = pic.pic_derive(cfg)["lam"][0]
    assert lam > 0.5
    h.set_tuning(ppt=4, grid=8, sort_period=16, use_graph=0)
    h.step(3)
    s0 = h.tally()["rare_spill"]
    probs = restart_step_check(O, cfg, h, 20)
    assert probs == [], "\n".join(probs[:20])
    t = h.tally()
    _say("  spilled items over 20 steps: %d, candidates %d" % (t["rare_spill"] - s0, t["cand"][0]))
    assert t["rare_spill"] - s0 > 1000
    assert t["coll"][0] > 0 and t["abs_count"].sum() > 0


@pytest.mark.parametrize("cells", [2048, 8192])
def test_rare_queue_spill_parity_tiled_field(pic, O, cells):
    """The spill on a grid of several field tiles.  2048 cells: the record
    block of the single field kernel works the spilled items off and the tile
    blocks wait for it before they read the counters those items change.
    8192 cells: the record block of the tiled field kernel does, and its
    tile blocks wait for it the same way."""
    cfg = presets.scaled(presets.tiny(), N=cells, L=5e-3 * cells / 256, n_load=40 * cells, ng=3.2e23, Te0=5.0,
                         gamma_emit=1e21)
    _say("case: rare-item spill on %d cells, grid 8" % cells)
    h = pic.Handle(cfg)
    h.set_tuning(ppt=4, grid=8, sort_period=16, use_graph=0)
    h.step(3)
    s0 = h.tally()["rare_spill"]
    probs = restart_step_check(O, cfg, h, 6)
    assert probs == [], "\n".join(probs[:20])
    assert h.tally()["rare_spill"] - s0 > 1000


PAPER_CASES = [
    ("baseline: elastic + charge exchange, T_n 300 / 1740 K", {}),
    ("Table 3: charge exchange off", dict(channels=presets.CH_EEL)),
    ("Table 3: electron-side neutral target at 1740 K", dict(Tne=1740.0 * presets.KB_OVER_E)),
]


@pytest.mark.parametrize("name,over", PAPER_CASES)
def test_paper_preset_parity(pic, O, name, over):
    cfg = presets.scaled(presets.paper(), n_load=20 * 4096, gamma_emit=1.0e20, **over)
    _say("case: the paper's diode at 20 per cell, %s: 200 steps, then 20 restart steps" % name)
    h = pic.Handle(cfg)
    h.step(200)
    probs = restart_step_check(O, cfg, h, 20)
    assert probs == [], "\n".join(probs[:20])
    t = h.tally()
    assert t["n_emit"] > 100 and t["cand"][0] > 0 and t["coll"][0] > 0
    assert t["coll"][1] == t["coll"][2] == t["coll"][4] == 0     # excitation, ionisation, ion elastic off
    if "channels" in over:
        assert t["cand"][1] == 0 and t["coll"][3] == 0           # no ion channel: no ion candidates
    else:
        assert t["cand"][1] > 0 and t["coll"][3] > 0


def test_sweep_32_diodes_parity(pic, O):
    cfgs = presets.sweep()
    sizes = [c["n_load"] for c in cfgs]
    picks = [int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), int(np.argmax(sizes))]
    _say("case: 32-diode sweep, 4 steps, then one restart step on diodes %s (%s per species)"
         % (picks, [sizes[d] for d in picks]))
    h = pic.Handle(cfgs)
    h.step(4)
    for d in picks:
        probs = restart_step_check(O, cfgs[d], h, 1, d=d)
        assert probs == [], "diode %d:\n%s" % (d, "\n".join(probs[:20]))


def test_maximum_batch_of_diodes(pic, O):
    """The largest batch a handle takes (256 diodes), one of them on a grid of
    the tiled field kernel so that every diode's field step runs there: 64
    steps through four re-sorts (three of them leaving the ions in place),
    with graph replay; every diode's field step waits only on blocks
    dispatched before it, so a batch that cannot be resident at once still
    completes.  Then restart parity on the first, a middle and the last
    diode."""
    base = presets.scaled(presets.tiny(), n_load=2560)
    cfgs = [presets.scaled(base, gamma_emit=1e20 * (1 + d % 7), diode=d) for d in range(255)]
    cfgs.append(presets.scaled(presets.tiny(), N=5000, L=5e-3 * 5000 / 256, n_load=50000, gamma_emit=3e21,
                               diode=255))
    _say("case: 256 diodes in one handle (255 x 256 cells, 1 x 5000 cells), 64 steps")
    h = pic.Handle(cfgs)
    h.set_tuning(sort_period=16, use_graph=1)
    h.step(64)
    h.sync()
    t = h.tally(0)
    assert t["step"] == 64 and t["err_bits"] == 0 and t["resorts"] >= 4
    for d in range(256):
        assert h.tally(d)["step"] == 64 and h.tally(d)["err_bits"] == 0, d
    for d in (0, 127, 255):
        # each check steps the whole handle on from the state it finds
        probs = restart_step_check(O, cfgs[d], h, 2, d=d)
        assert probs == [], "diode %d:\n%s" % (d, "\n".join(probs[:20]))


def test_snapshots_hold_newborns_beyond_the_anode(pic, O):
    """On a gap far shorter than one step of the slowest emitted electron,
    every thermionic newborn crosses at birth: the record block tallies it,
    absorbed at the anode with its birth energy, and releases those tallies
    to the tail block, which waits for them on a step that takes a snapshot.
    With a snapshot every step, each step's snapshot equals the oracle's
    tallies after that step (counts exactly, the energy within 1e-5)."""
    Tc = 2000.0 * presets.KB_OVER_E
    cfg = quiet_cfg(n_load=1, Tc=Tc, L=1e-11, N=2, tally_period=1)
    cfg["gamma_emit"] = 500.5 * O.derive(cfg)["w0"] / cfg["dt"]
    _say("case: every newborn beyond the anode, a snapshot every step")
    h = pic.Handle(cfg)
    s = O.Sim(cfg)
    s.load()
    none = {"z": np.zeros(0), "vx": np.zeros(0), "vy": np.zeros(0), "vz": np.zeros(0),
            "id": np.zeros(0, np.uint32), "tc": np.zeros(0, np.uint32)}
    for sp in range(3):
        h.set_particles(0, sp, none)
        empty(s, sp)
    h.set_counters(0, 0, 10)
    s.set_counters(0, 10)
    h.refield()
    s.refield()
    for k in range(1, 7):
        h.step(1)
        s.step()
        snap, ot = h.snapshot(0, k), s.tally()
        # 500.5 newborns per step: 500 or 501 each
        assert snap["n_emit"] == ot["n_emit"] and 500 * k <= ot["n_emit"] <= 501 * k, k
        assert snap["abs_count"][1][1] == ot["abs_count"][1][1] == ot["n_emit"], k
        assert snap["abs_count"].sum() == ot["n_emit"], k
        # velocities are FP32 on the device: energies agree to the parity tests' 1e-5
        assert np.isclose(snap["abs_energy"][1][1], ot["abs_energy"][1][1], rtol=1e-5, atol=0.0), k


def test_graph_runs_equal_plain_stream(pic):
    """Runs shorter than a re-sort period, replayed from captured graphs,
    give the plain launches' result bit for bit."""
    cfg = presets.scaled(presets.tiny(), gamma_emit=1e21, Te0=10.0, ng=3.2e22)
    _say("case: partial-period graph replay vs plain launches")
    a, b = pic.Handle(cfg), pic.Handle(cfg)
    a.set_tuning(ppt=2, grid=0, sort_period=16, use_graph=0)
    b.set_tuning(ppt=2, grid=0, sort_period=16, use_graph=1)
    for n in (5, 20, 1, 13, 40, 3):
        a.step(n)
        b.step(n)
    ta, tb = a.tally(), b.tally()
    assert ta["step"] == tb["step"] == 82
    for k in ("abs_count", "cand", "coll", "n_live"):
        assert np.array_equal(ta[k], tb[k]), k
    for sp in range(3):
        pa, pb = by_id(a.particles(0, sp)), by_id(b.particles(0, sp))
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), (sp, k)
        assert np.array_equal(a.hist(0, sp), b.hist(0, sp))


@pytest.mark.parametrize("use_graph", [0, 1])
def test_step_timed_shorter_than_a_period(pic, use_graph):
    """Fewer steps than one re-sort period, from the middle of a period: the
    particle kernel is still timed (finite, below the whole step)."""
    cfg = presets.scaled(presets.tiny(), N=2048, L=5e-3 * 8, n_load=200 * 2048)
    _say("case: step_timed(20) with a 32-step re-sort period, graph %d" % use_graph)
    h = pic.Handle(cfg)
    h.set_tuning(ppt=2, grid=0, sort_period=32, use_graph=use_graph)
    h.step(5)
    r = h.step_timed(20)
    assert np.isfinite(r["particle_kernel_ms"])
    assert 0.0 < r["particle_kernel_ms"] < r["total_ms"] / 20
    assert h.tally()["step"] == 25


def test_steady_verdict_matches_series(pic):
    """pic_steady_state's verdict on the device ring equals
    pic_steady_from_series on block series rebuilt from the ring's
    snapshots (backflow ratio of each block and live count at its end)."""
    cfg = presets.scaled(presets.tiny(), gamma_emit=2e21, tally_period=10)
    _say("case: steady-state verdict against the series criterion")
    h = pic.Handle(cfg)
    h.step(3000)
    w0 = pic.pic_derive(cfg)["w0"]
    bt, D = 20, cfg["tally_period"]
    blk = bt * D
    snaps = [h.snapshot(0, k * blk) for k in range(3000 // blk + 1)]
    win = blk * cfg["dt"]
    br = np.array([100.0 * (float(b["abs_count"][1][0] - a["abs_count"][1][0]) * w0 / win) / cfg["gamma_emit"]
                   for a, b in zip(snaps[:-1], snaps[1:])])
    nl = np.array([float(b["n_live"].sum()) for b in snaps[1:]])
    seen = set()
    for tol_pp, tol_rel in ((5.0, 0.05), (2.0, 0.02), (0.01, 1e-6)):
        dev = h.steady_state(0, block_tallies=bt, tol_pp=tol_pp, tol_rel=tol_rel)
        ref = pic.steady_from_series(br, nl, tol_pp, tol_rel)
        assert dev["blocks"] == len(br)
        assert dev["steady"] == (ref["steady_block"] >= 0)
        seen.add(dev["steady"])
        if dev["steady"]:
            assert dev["steady_step"] == (ref["steady_block"] + 1) * blk
            assert dev["blocks_averaged"] == ref["blocks_averaged"]
            assert dev["backflow_pct"] == pytest.approx(ref["backflow_pct"], rel=1e-12, abs=1e-12)
        assert dev["last_backflow_pct"] == pytest.approx(br[-1], rel=1e-12, abs=1e-12)
    assert seen == {True, False}, "the tolerances should give both verdicts"


def test_ions_kept_in_place_across_resorts(pic, O):
    """The ions move a small fraction of a cell per re-sort period, so most
    re-sorts leave them in their buffer (the diode's parity flips, the
    ions' buffer does not) with the ions born since appended to their tail.
    Restart parity runs through kept and sorting re-sorts; the phase-space
    counts and a checkpoint taken while the ions sit in the other buffer than
    the electrons read them from there."""
    cfg = presets.scaled(presets.tiny(), gamma_emit=1e21, Te0=10.0, ng=3.2e22)
    _say("case: ions kept in place across re-sorts, re-sort every 8 steps")
    h = pic.Handle(cfg)
    h.set_tuning(sort_period=8, use_graph=0)
    h.step(12)
    t0 = h.tally()
    _say("  after 12 steps: %d re-sorts, %d kept the ions; live %s"
         % (t0["resorts"], t0["resorts_ions_kept"], t0["n_live"].tolist()))
    assert t0["resorts"] >= 2 and t0["resorts_ions_kept"] >= 1
    out = h.phase_space(0, 2, 16, 40, -3e4, 3e4)
    h.sync()
    p = h.particles(0, 2)
    assert np.array_equal(out.cpu().numpy(), O.phase_space(p["z"], p["vz"], cfg["L"], 16, 40, -3e4, 3e4))
    img = h.save()
    probs = restart_step_check(O, cfg, h, 30)
    assert probs == [], "\n".join(probs[:20])
    t1 = h.tally()
    kept = t1["resorts_ions_kept"] - t0["resorts_ions_kept"]
    _say("  30 more steps: %d re-sorts, %d kept the ions; %d ionisations"
         % (t1["resorts"] - t0["resorts"], kept, t1["n_iz"] - t0["n_iz"]))
    assert kept >= 1 and t1["resorts"] - t0["resorts"] - kept >= 1 and t1["n_iz"] > t0["n_iz"]
    b = pic.Handle(cfg)
    b.set_tuning(sort_period=8, use_graph=0)
    b.load(img)
    b.step(30)
    ta, tb = h.tally(), b.tally()
    assert ta["step"] == tb["step"] and np.array_equal(ta["n_live"], tb["n_live"])
    for sp in range(3):
        pa, pb = by_id(h.particles(0, sp)), by_id(b.particles(0, sp))
        for k in ("id", "z", "vx", "vy", "vz", "tc"):
            assert np.array_equal(pa[k], pb[k]), (sp, k)
    assert np.array_equal(h.fields(0)["phi"], b.fields(0)["phi"])


def test_nullcoll_bound_reported(pic, O):
    """A candidate whose collision frequency exceeds nu_max sets the sticky
    PIC_ENULLCOLL bit (the oracle counts the same event)."""
    cfg = presets.tiny()
    _say("case: null-collision bound exceeded")
    h = pic.Handle(cfg)
    h.step(5)
    p = h.particles(0, 0)
    step = h.tally()["step"]
    fast = {"z": [cfg["L"] / 2], "vx": [1.0e8], "vy": [0.0], "vz": [0.0],
            "id": [h.tally()["next_id"]], "tc": [step]}
    q = {k: np.concatenate([np.asarray(p[k]), np.asarray(fast[k], dtype=np.asarray(p[k]).dtype)]) for k in p}
    h.set_particles(0, 0, q)
    h.set_counters(0, step, int(fast["id"][0]) + 1)
    st, t = gpu_state(h)
    s = oracle_from_gpu(O, cfg, st, t)
    s.step()
    assert s.tally()["nullcoll_exceed"] == 1
    h.step(1)
    with pytest.raises(pic.PicError) as e:
        h.sync()
    assert e.value.code == pic.PIC_ENULLCOLL


def test_nonfinite_particles_rejected(pic):
    cfg = presets.tiny()
    _say("case: non-finite particle input")
    h = pic.Handle(cfg)
    h.step(2)
    p = h.particles(0, 2)
    n = len(p["z"])
    for key in ("vx", "vy", "vz"):
        for bad in (np.nan, np.inf):
            q = {k: v.copy() for k, v in p.items()}
            q[key][n // 2] = bad
            with pytest.raises(pic.PicError) as e:
                h.set_particles(0, 2, q)
            assert e.value.code == pic.PIC_ENAN
    q = {k: v.copy() for k, v in p.items()}
    q["z"][0] = np.nan
    with pytest.raises(pic.PicError) as e:
        h.set_particles(0, 2, q)
    assert e.value.code == pic.PIC_EINVAL
    # nothing changed: the diode steps on
    assert np.array_equal(by_id(h.particles(0, 2))["id"], by_id(p)["id"])
    h.step(2)
    h.sync()
    # a checkpoint image with a non-finite velocity is refused before any copy
    marker = np.float32(12345.678)
    q = {k: v.copy() for k, v in h.particles(0, 2).items()}
    q["vz"][3] = marker
    h.set_particles(0, 2, q)
    img = h.save()
    raw = img.tobytes()
    at = raw.find(marker.tobytes())
    assert at > 0 and raw.find(marker.tobytes(), at + 1) < 0
    bad = np.frombuffer(raw[:at] + np.float32(np.nan).tobytes() + raw[at + 4:], np.uint8)
    with pytest.raises(pic.PicError) as e:
        h.load(bad)
    assert e.value.code == pic.PIC_ENAN
    h.load(img)
    h.step(1)
    h.sync()


@pytest.mark.parametrize("N", [256, 4500])
def test_deposit_range_reported(pic, N):
    """2^21 + 10% particles of one species on one node push its fixed-point
    deposit past 2^53: the field step sets PIC_ERANGE (single-block and tiled
    field kernels)."""
    n = 2_300_000
    cfg = presets.scaled(presets.tiny(), N=N, L=5e-3 * N / 256, n_load=n, gamma_emit=0.0, ng=0.0)
    _say("case: deposit range, %d electrons on one node, N = %d" % (n, N))
    h = pic.Handle(cfg)
    h.sync()
    z = np.full(n, cfg["L"] / N * (N // 2))
    zero = np.zeros(n, np.float32)
    h.set_particles(0, 0, {"z": z, "vx": zero, "vy": zero, "vz": zero,
                           "id": np.arange(n, dtype=np.uint32), "tc": np.full(n, 0xFFFFFFFF, np.uint32)})
    h.refield()
    with pytest.raises(pic.PicError) as e:
        h.sync()
    assert e.value.code == pic.PIC_ERANGE
    assert int(h.hist(0, 0)[N // 2]) == n << 32
