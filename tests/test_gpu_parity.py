"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Bit-exact: deposits (as a function of the particle array), ids, free-flight
counters, absorbed / collision / birth counts.  Floating point: positions and
velocities within 1e-5 relative (FP32 velocities), phi and E within 1e-10 of
their maxima.
"""
import numpy as np
import pytest

from gpu_compare import (by_id, compare_particles, compare_tallies, deposit_matches, field_matches,
                         gpu_state, oracle_from_gpu, restart_step_check)
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


def test_load_matches_oracle(pic, O):
    cfg = presets.tiny()
    _say("case: load, tiny diode")
    h = pic.Handle(cfg)
    st, t = gpu_state(h)
    s = O.Sim(cfg)
    s.load()
    for sp in (0, 2):
        g, o = by_id(st[sp]), by_id(s.particles(sp))
        assert np.array_equal(g["id"], o["id"])
        assert np.array_equal(g["z"], o["z"])            # same FP64 expression: bit exact
        assert np.array_equal(g["tc"], o["tc"])
        for c in ("vx", "vy", "vz"):
            # FP64 Box-Muller on both sides, rounded once to FP32 on the GPU
            assert np.max(np.abs(g[c] - o[c].astype(np.float32)) / np.abs(o[c]).max()) < 1e-6
    assert len(st[1]["id"]) == 0
    assert deposit_matches(O, cfg, h, st) == []
    s2 = oracle_from_gpu(O, cfg, st, t)
    assert field_matches(O, cfg, h, s2) == []


@pytest.mark.parametrize("name,over", [
    ("tiny, emission x100", dict(gamma_emit=1e21)),
    ("hot electrons: excitation and ionisation", dict(Te0=25.0, gamma_emit=1e21, ng=3.2e22)),
    ("ions: charge exchange and elastic", dict(Ti0=1.0, ng=3.2e22, gamma_emit=0.0)),
])
def test_restart_parity_per_step(pic, O, name, over):
    cfg = presets.scaled(presets.tiny(), **over)
    _say("case: restart parity, " + name)
    h = pic.Handle(cfg)
    probs = restart_step_check(O, cfg, h, 100)
    assert probs == [], "\n".join(probs[:20])
    t = h.tally()
    assert t["cand"].sum() > 0 and t["coll"].sum() > 0
    if over.get("Te0", 0) > 20:
        assert t["coll"][1] > 0 and t["coll"][2] > 0 and t["n_iz"] > 0
    if over.get("Ti0", 0) >= 1.0:
        assert t["coll"][3] > 0 and t["coll"][4] > 0
    if over.get("gamma_emit", 0) > 0:
        assert t["n_emit"] > 100


def test_free_run_100_steps(pic, O):
    cfg = presets.scaled(presets.tiny(), gamma_emit=1e21)
    _say("case: free-running 100 steps, tiny")
    h = pic.Handle(cfg)
    s = O.Sim(cfg)
    s.load()
    t0g, t0o = h.tally(), s.tally()
    h.step(100)
    s.step(100)
    st, t1g = gpu_state(h)
    probs = []
    for sp in range(3):
        probs += compare_particles(cfg, st[sp], s.particles(sp), sp)
    probs += compare_tallies(t0g, t1g, t0o, s.tally())
    probs += deposit_matches(O, cfg, h, st)
    assert probs == [], "\n".join(probs[:20])


def test_batched_equals_single(pic, O):
    base = presets.tiny()
    cfgs = [presets.scaled(base, diode=d, gamma_emit=g, Tc=T * presets.KB_OVER_E, n_load=nl)
            for d, (g, T, nl) in enumerate([(1e21, 1800, 20000), (3e21, 2200, 31000), (5e20, 2000, 9000)])]
    _say("case: batched 3 diodes vs single")
    hb = pic.Handle(cfgs)
    hs = [pic.Handle(c) for c in cfgs]
    hb.step(60)
    for h in hs:
        h.step(60)
    for d, h in enumerate(hs):
        tb, ts = hb.tally(d), h.tally()
        for k in ("abs_count", "cand", "coll", "n_live"):
            assert np.array_equal(tb[k], ts[k]), (d, k)
        for k in ("n_emit", "n_repl", "n_iz", "next_id"):
            assert tb[k] == ts[k]
        for sp in range(3):
            assert np.array_equal(hb.hist(d, sp), h.hist(0, sp))
            pb, ps = hb.particles(d, sp), h.particles(0, sp)
            for k in pb:
                assert np.array_equal(pb[k], ps[k]), (d, sp, k)


def test_bench_scale_parity(pic, O):
    cfg = presets.bench()
    _say("case: benchmark diode (2048 cells, 409.6k per species), 40 steps then restart parity")
    h = pic.Handle(cfg)
    h.step(40)
    probs = restart_step_check(O, cfg, h, 2)
    assert probs == [], "\n".join(probs[:20])


def test_large_scale_parity(pic, O):
    cfg = presets.large()
    _say("case: large diode (16384 cells, 16.4M per species), 3 steps then one restart step")
    h = pic.Handle(cfg)
    h.step(3)
    probs = restart_step_check(O, cfg, h, 1)
    assert probs == [], "\n".join(probs[:20])
    _say("  phase space of the plasma electrons, all 16.4M")
    out = h.phase_space(0, 0, 64, 100, -4e6, 4e6)
    h.sync()
    p = h.particles(0, 0)
    assert np.array_equal(out.cpu().numpy(), O.phase_space(p["z"], p["vz"], cfg["L"], 64, 100, -4e6, 4e6))


def test_phase_space_matches_oracle(pic, O):
    """(z, v_z) counts of every species against the oracle's on the GPU's own
    particles, bit for bit, with wide and narrow velocity ranges (the under-
    and overflow columns); a second call into the same buffer accumulates;
    bad arguments are rejected."""
    cfg = presets.scaled(presets.tiny(), gamma_emit=1e21, Te0=10.0, ng=3.2e22)
    _say("case: phase space, tiny diode after 60 steps")
    h = pic.Handle(cfg)
    h.step(60)
    cases = [(0, 16, 40, -4e6, 4e6), (1, 16, 40, -4e6, 4e6), (2, 16, 40, -3e4, 3e4),
             (0, 7, 9, -1e5, 2e5), (2, 1, 1, -1.0, 1.0), (0, 256, 126, -4e6, 4e6)]
    for sp, nz, nv, lo, hi in cases:
        out = h.phase_space(0, sp, nz, nv, lo, hi)
        h.sync()
        p = h.particles(0, sp)
        ref = O.phase_space(p["z"], p["vz"], cfg["L"], nz, nv, lo, hi)
        g = out.cpu().numpy()
        assert np.array_equal(g, ref), (sp, nz, nv)
        assert g.sum() == np.count_nonzero(p["z"] >= 0) > 0
        h.phase_space(0, sp, nz, nv, lo, hi, out=out)
        h.sync()
        assert np.array_equal(out.cpu().numpy(), 2 * ref)
    # the narrow ranges put counts in the under- and overflow columns
    ref = O.phase_space(h.particles(0, 0)["z"], h.particles(0, 0)["vz"], cfg["L"], 7, 9, -1e5, 2e5)
    assert ref[:, 0].sum() > 0 and ref[:, -1].sum() > 0
    for bad in [(0, 0, 200, 200, -1.0, 1.0), (0, 0, 4, 4, 1.0, 1.0), (0, 3, 4, 4, -1.0, 1.0),
                (1, 0, 4, 4, -1.0, 1.0), (0, 0, 0, 4, -1.0, 1.0), (0, 0, 4, 4, float("nan"), 1.0)]:
        with pytest.raises(pic.PicError):
            h.phase_space(*bad)
    # host memory is refused by the library, a tensor on another device by the binding
    import ctypes
    import torch
    host = np.zeros((4, 6), dtype=np.int64)
    assert pic.lib().pic_phase_space(h.h, 0, 0, 4, 4, -1.0, 1.0, host.ctypes.data_as(ctypes.c_void_p)) == pic.PIC_EINVAL
    with pytest.raises(ValueError):
        h.phase_space(0, 0, 4, 4, -1.0, 1.0, out=torch.zeros((4, 6), dtype=torch.int64))


def test_edge_cases(pic, O):
    _say("case: edge cases")
    # smallest grid, no emission: the emitted population stays empty
    cfg = presets.scaled(presets.tiny(), N=2, n_load=500, gamma_emit=0.0)
    h = pic.Handle(cfg)
    assert restart_step_check(O, cfg, h, 20) == []
    assert len(h.particles(0, 1)["id"]) == 0
    # particles exactly on nodes, in the last ulp below L, and an empty species
    cfg = presets.scaled(presets.tiny(), n_load=64, gamma_emit=0.0, ng=0.0)
    h = pic.Handle(cfg)
    L, N = cfg["L"], cfg["N"]
    z = np.array([L / N * k for k in range(1, 9)] + [np.nextafter(L, 0), L * 0.5])
    n = len(z)
    p = {"z": z, "vx": np.zeros(n, np.float32), "vy": np.zeros(n, np.float32),
         "vz": np.zeros(n, np.float32), "id": np.arange(n, dtype=np.uint32),
         "tc": np.full(n, 0xFFFFFFFF, np.uint32)}
    h.set_particles(0, 0, p)
    h.set_particles(0, 2, {k: v[:0] for k, v in p.items()})
    h.set_counters(0, 0, n)
    h.refield()
    st, t = gpu_state(h)
    assert deposit_matches(O, cfg, h, st) == []
    assert restart_step_check(O, cfg, h, 5) == []
    # rejected inputs
    with pytest.raises(pic.PicError) as e:
        h.set_particles(0, 0, dict(p, z=np.full(n, 2 * L)))
    assert e.value.code == pic.PIC_EINVAL
    with pytest.raises(pic.PicError):
        pic.Handle(presets.scaled(presets.tiny(), N=1))


def test_capacity_overflow_reported(pic):
    _say("case: capacity overflow")
    cfg = presets.scaled(presets.tiny(), n_load=1000, capacity_factor=0.001, gamma_emit=2e25)
    h = pic.Handle(cfg)
    h.step(50)
    with pytest.raises(pic.PicError) as e:
        h.sync()
    assert e.value.code == pic.PIC_ENOSPACE


def test_diagnostics_window(pic, O):
    cfg = presets.scaled(presets.tiny(), gamma_emit=3e21, tally_period=50)
    _say("case: diagnostics windows")
    h = pic.Handle(cfg)
    h.step(300)
    t = h.tally()
    w0 = pic.pic_derive(cfg)["w0"]
    whole = h.diagnostics(0, 0)
    ref = O.diag(cfg["gamma_emit"], cfg["Tc"], w0, 300 * cfg["dt"], t["abs_count"], t["abs_energy"],
                 t["n_emit"])
    for k in ("gamma_ref", "gamma_net", "gamma_anode", "backflow_pct", "eta_net", "eta_anode",
              "wf_eff", "q_emit_theory", "q_cool1", "q_cool2", "q_anode1", "q_anode2"):
        assert whole[k] == pytest.approx(ref[k], rel=1e-12, abs=1e-12), k
    win = h.diagnostics(0, 100)
    assert (win["step_begin"], win["step_end"]) == (200, 300)
    assert np.array_equal(win["n_live"], t["n_live"])


def test_time_average_fields(pic, O):
    """The time-averaged potential and densities are the mean of the
    instantaneous ones over the averaging window, and every instantaneous
    field that enters the mean matches the oracle: each step is a restart
    step against the oracle (deposit bit for bit, potential of the oracle's
    solve, particles and tallies after the step), and so is the last state."""
    cfg = presets.tiny()
    _say("case: time-averaged fields")
    h = pic.Handle(cfg)
    h.step(5)
    h.avg_reset(True)
    acc = None
    probs = []
    for _ in range(8):
        probs += restart_step_check(O, cfg, h, 1)        # one GPU step, checked
        f = h.fields(0)
        acc = {k: v.copy() for k, v in f.items()} if acc is None else {k: acc[k] + f[k] for k in f}
    st, gt = gpu_state(h)
    s = oracle_from_gpu(O, cfg, st, gt)
    probs += deposit_matches(O, cfg, h, st) + field_matches(O, cfg, h, s)
    assert probs == [], "\n".join(probs[:20])
    avg = h.fields(0, time_avg=True)
    for k in acc:
        assert np.allclose(avg[k], acc[k] / 8, rtol=1e-12, atol=1e-9 * np.abs(acc[k]).max())


def test_autotune_keeps_parity(pic, O):
    cfg = presets.scaled(presets.bench(), n_load=204800)
    _say("case: autotune then restart parity")
    h = pic.Handle(cfg)
    h.step(10)
    t = h.autotune(trial_steps=16)
    # the schedule is one of the searched ones (pic_autotune in include/pic.h)
    assert t["ppt"] in (1, 2, 4) and t["sort_period"] in (16, 32, 64, 128) and t["ms_per_step"] > 0
    # a listed grid, or the one giving each block eight chunks (a multiple of 8, 256..65536)
    assert t["grid"] in (2048, 3072, 4096, 6144, 8192, 12288, 16384) or (
        t["grid"] % 8 == 0 and 256 <= t["grid"] <= 65536)
    assert t["use_graph"] in (0, 1)
    probs = restart_step_check(O, cfg, h, 3)
    assert probs == [], "\n".join(probs[:20])


def test_steady_state_on_device(pic):
    cfg = presets.scaled(presets.tiny(), gamma_emit=2e21, tally_period=10)
    _say("case: steady-state detector on device tallies")
    h = pic.Handle(cfg)
    h.step(3000)
    st = h.steady_state(0, block_tallies=20, tol_pp=5.0, tol_rel=0.05)
    assert st["blocks"] == 3000 // 200
    assert st["block_steps"] == 200
    if st["steady"]:
        assert st["steady_step"] % 200 == 0 and st["steady_step"] <= 3000


def test_tiled_field_path_ragged(pic, O):
    """Grids above 2049 nodes take the multi-block field solve (births, tile
    aggregates, tiled solve): a ragged 9001-node diode batched with a 257-node
    one, field and deposit against the oracle, then restart parity."""
    _say("case: tiled field path, N = 9000 with N = 256 in one batch")
    big = presets.scaled(presets.tiny(), N=9000, L=5e-3 * 9000 / 256, n_load=180000, gamma_emit=3e21, diode=0)
    small = presets.scaled(presets.tiny(), gamma_emit=1e21, diode=1)
    h = pic.Handle([big, small])
    for d, cfg in enumerate((big, small)):
        st, t = gpu_state(h, d)
        assert deposit_matches(O, cfg, h, st, d) == []
        s = oracle_from_gpu(O, cfg, st, t)
        assert field_matches(O, cfg, h, s, d) == []
    assert restart_step_check(O, big, h, 8, d=0) == []
    assert restart_step_check(O, small, h, 4, d=1) == []


def test_tiled_field_path_maximum_grid(pic, O):
    """The largest grid the library accepts (32767 cells: 64 tiles of the
    field solve, combined by one wave): load field and deposit, then restart
    parity over steps with births.  The potential is checked against the
    exact rational solve of the oracle's deposit, since the oracle's FP64
    sweep rounds by ~1e-10 of the maximum at this size."""
    _say("case: tiled field path, N = 32767")
    cfg = presets.scaled(presets.tiny(), N=32767, L=5e-3 * 32767 / 256, n_load=131068, gamma_emit=3e22)
    h = pic.Handle(cfg)
    st, t = gpu_state(h)
    assert deposit_matches(O, cfg, h, st) == []
    s = oracle_from_gpu(O, cfg, st, t)
    assert field_matches(O, cfg, h, s, exact=True) == []
    probs = restart_step_check(O, cfg, h, 4, exact_field=True)
    assert probs == [], "\n".join(probs[:20])


def test_particles_outside_the_window(pic, O):
    """With no re-sort for 800 steps, electrons drift past the 160-cell margin
    of their run's LDS window and births sit unsorted at the end of the
    store: those particles take the particle kernel's slow path (field read
    from global memory, deposit through global atomics).  One-step parity
    against the oracle from that state."""
    _say("case: 4096-cell diode, 800 steps without re-sort, then restart parity")
    cfg = presets.scaled(presets.tiny(), N=4096, L=5e-3 * 4096 / 256, n_load=100 * 4096, gamma_emit=3e21, Te0=8.0)
    h = pic.Handle(cfg)
    h.set_tuning(sort_period=1000000, use_graph=0)
    h.step(800)
    probs = restart_step_check(O, cfg, h, 2)
    assert probs == [], "\n".join(probs[:20])


@pytest.mark.parametrize("N", [2048, 9000])
def test_step_timed_measures_the_particle_kernel(pic, N):
    """The live timing of the particle kernel (events spliced around it in the
    replayed graph) agrees with the plain-stream timing, on the single-block
    and the tiled field paths, and stays below the whole step."""
    _say("case: step_timed, N = %d" % N)
    cfg = presets.scaled(presets.tiny(), N=N, L=5e-3 * N / 256, n_load=200 * N)
    h = pic.Handle(cfg)
    res = {}
    for g in (0, 1):
        h.set_tuning(ppt=2, grid=0, sort_period=16, use_graph=g)
        h.step(32)
        r = h.step_timed(64)
        res[g] = r
        assert 0.0 < r["particle_kernel_ms"] < r["total_ms"] / 64
    a, b = res[0]["particle_kernel_ms"], res[1]["particle_kernel_ms"]
    _say("  particle kernel: stream %.1f us, graph %.1f us" % (a * 1e3, b * 1e3))
    assert abs(a - b) < 0.35 * max(a, b)


def test_checkpoint_restart_is_exact(pic):
    """A run restored from a checkpoint continues as the saved run does:
    particles, deposits, fields and integer tallies identical; the FP64
    absorbed-energy sums to rounding.  Two diodes, one batch."""
    _say("case: checkpoint / restart")
    cfgs = [presets.scaled(presets.tiny(), gamma_emit=1e21, diode=0),
            presets.scaled(presets.tiny(), gamma_emit=3e21, Te0=10.0, ng=3.2e22, diode=1)]
    a = pic.Handle(cfgs)
    a.step(40)
    img = a.save()
    a.step(30)
    b = pic.Handle(cfgs)
    b.step(3)                      # a different state, overwritten by the image
    b.load(img)
    b.step(30)
    for d in range(2):
        ta, tb = a.tally(d), b.tally(d)
        assert ta["step"] == tb["step"] == 70 and ta["next_id"] == tb["next_id"]
        for k in ("abs_count", "cand", "coll", "n_live"):
            assert np.array_equal(ta[k], tb[k]), k
        for k in ("n_emit", "n_repl", "n_iz"):
            assert ta[k] == tb[k], k
        assert np.allclose(ta["abs_energy"], tb["abs_energy"], rtol=1e-12, atol=0)
        for sp in range(3):
            pa, pb = by_id(a.particles(d, sp)), by_id(b.particles(d, sp))
            for k in ("id", "z", "vx", "vy", "vz", "tc"):
                assert np.array_equal(pa[k], pb[k]), (d, sp, k)
            assert np.array_equal(a.hist(d, sp), b.hist(d, sp))
        assert np.array_equal(a.fields(d)["phi"], b.fields(d)["phi"])
    # a handle of another configuration refuses the image
    c = pic.Handle([presets.scaled(cfgs[0], V=5.0), cfgs[1]])
    with pytest.raises(pic.PicError) as e:
        c.load(img)
    assert e.value.code == pic.PIC_EINVAL
    with pytest.raises(pic.PicError):
        b.load(img[:100])
