"""GPU parity of the warm start: the BF16 matrix-core surrogate and the
profile loader, through the C ABI, against the FP64 oracle.

Surrogate tolerances.  The oracle's quantised mode rounds weights, layer
inputs and pre-activation gradients to bfloat16 at the same points as the
kernels.  What remains is FP32 accumulation order and FP32 tanh / features,
and those are not small at the output: an FP32 difference of one unit in the
last place flips a bfloat16 rounding with probability |delta| / ulp_bf16, a
flip moves that activation by 2^-8 relative, and every activation feeds
5 x 64 pre-activations of the next layer, so flips cascade.  Emulating the
kernels' arithmetic in numpy float32 against the FP64 oracle gives relative
L2 errors from 1e-7 (no flip) up to 2e-3 on these shapes.  The bars are
therefore:
  * forward outputs: relative L2 <= 1e-2 per sample and max error <= 2e-2 of
    the sample's max (a wrong border tap or a dropped bias exceeds both at
    X = 64);
  * gradients of every layer (weights and biases): relative L2 <= 1e-2;
  * Adam: the closed-form update of the kernel's own gradients to 1e-6 of lr;
  * a short training run: losses within 2 % of the oracle's trajectory.
Profile loader: counts, ids, positions and free-flight counters bit-exact,
velocities to FP32 rounding, deposit and field as in the uniform load.
"""
import math

import numpy as np
import pytest

from gpu_compare import by_id, deposit_matches, field_matches, gpu_state, oracle_from_gpu, restart_step_check
from oracle import surrogate_oracle as SO
from paper_2605_07083_amd import presets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a ROCm device"
    return T


@pytest.fixture(scope="module")
def sur(torch):
    from paper_2605_07083_amd import surrogate as S
    S.lib()
    return S


def _say(msg):
    print(msg, flush=True)


def _params(n, seed):
    d = presets.surrogate_params(n, seed)
    return np.stack([d["gamma_emit"], d["T_K"], d["V"], d["ng"]], axis=1)


def _target39(u, k):
    """Smooth targets for all output channels: the three profiles, then
    quantile-like channels increasing with the channel index."""
    rows = [u * (1 + 0.1 * k), np.log(0.2 + u), np.log(1.2 - u)]
    for c in range(3, SO.N_OUT):
        j = (c - 3) % 9
        rows.append(0.3 * (j - 4) + 0.2 * np.sin(3 * u + c + k))
    return np.stack(rows)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("B,X", [(1, 64), (3, 192), (2, 2048), (32, 2048)])
def test_forward_matches_oracle(sur, torch, B, X):
    _say("case: surrogate forward B=%d X=%d" % (B, X))
    W, b = presets.surrogate_test_weights(11)
    p = _params(B, 21)
    net = sur.Surrogate(B, X, device="cuda:0")
    net.set_weights(W, b)
    got = net.forward(p).cpu().numpy()
    p32 = p.astype(np.float32).astype(np.float64)     # the kernel receives FP32 parameters
    ref = SO.forward(W, b, SO.features(p32, X), quantize=True)
    for k in range(B):
        e = _rel(got[k], ref[k])
        m = np.max(np.abs(got[k] - ref[k])) / np.max(np.abs(ref[k]))
        _say("  sample %d rel L2 %.3g, max err / max %.3g" % (k, e, m))
        assert e <= 1e-2 and m <= 2e-2
    # weights round-trip through the packed layout
    W2, b2 = net.weights()
    assert all(np.array_equal(x, y) for x, y in zip(W, W2)) and all(np.array_equal(x, y) for x, y in zip(b, b2))


# X = 256: one whole slice of the backward kernel; 320: a second slice of 64
# positions (a part shorter than the LDS part); 64: one short part with the
# sample's zero padding on both sides; 2048: eight slices per sample
@pytest.mark.parametrize("B,X", [(2, 256), (3, 320), (1, 64), (2, 2048)])
def test_gradients_and_adam_match_oracle(sur, torch, B, X):
    lr = 1e-3
    _say("case: surrogate gradients B=%d X=%d" % (B, X))
    W, b = presets.surrogate_test_weights(12)
    p = _params(B, 22)
    rng = np.random.default_rng(5)
    u = (np.arange(X) + 0.5) / X
    target = np.stack([_target39(u, k) for k in range(B)])
    target = (target + 0.01 * rng.normal(size=target.shape)).astype(np.float32)
    net = sur.Surrogate(B, X, device="cuda:0")
    net.set_weights(W, b)
    loss = net.train_step(p, target, lr)
    gW, gb = net.grads()
    p32 = p.astype(np.float32).astype(np.float64)
    f = SO.features(p32, X)
    lo, oW, ob = SO.loss_and_grads(W, b, f, target.astype(np.float64), quantize=True)
    _say("  loss gpu %.9g oracle %.9g" % (loss, lo))
    assert loss == pytest.approx(lo, rel=1e-4)
    for l in range(6):
        ew, eb = _rel(gW[l], oW[l]), _rel(gb[l], ob[l])
        _say("  layer %d grad rel L2: W %.3g b %.3g" % (l, ew, eb))
        assert ew <= 1e-2 and eb <= 1e-2
    # Adam step 1 from zero moments on the kernel's own gradients:
    # w1 = w0 - lr g / (|g| + eps)
    W1, b1 = net.weights()
    for l in range(6):
        for w0, w1, g in ((W[l], W1[l], gW[l]), (b[l], b1[l], gb[l])):
            exp = w0.astype(np.float64) - lr * g / (np.abs(g.astype(np.float64)) + 1e-8)
            assert np.max(np.abs(w1 - exp)) <= 1e-6 * lr + 1e-7 * np.abs(exp).max()


def test_training_trajectory_matches_oracle(sur, torch):
    B, X, lr, steps = 2, 128, 2e-3, 12
    _say("case: surrogate training trajectory, %d steps" % steps)
    W, b = presets.surrogate_test_weights(13)
    p = _params(B, 23)
    u = (np.arange(X) + 0.5) / X
    target = np.stack([_target39(u, 0) for _ in range(B)]).astype(np.float32)
    net = sur.Surrogate(B, X, device="cuda:0")
    net.set_weights(W, b)
    f = SO.features(p.astype(np.float32).astype(np.float64), X)
    oW = [w.astype(np.float64) for w in W]
    ob = [v.astype(np.float64) for v in b]
    mW = [np.zeros_like(w) for w in oW]; vW = [np.zeros_like(w) for w in oW]
    mb = [np.zeros_like(v) for v in ob]; vb = [np.zeros_like(v) for v in ob]
    lg, lo = [], []
    for t in range(1, steps + 1):
        lg.append(net.train_step(p, target, lr))
        r = SO.train_step(oW, ob, mW, vW, mb, vb, t, f, target.astype(np.float64), lr)
        lo.append(r[0])
        oW, ob, mW, vW, mb, vb = r[3], r[4], r[5], r[6], r[7], r[8]
    _say("  gpu    %s" % np.array2string(np.array(lg), precision=5))
    _say("  oracle %s" % np.array2string(np.array(lo), precision=5))
    assert np.allclose(lg, lo, rtol=2e-2)
    assert lg[-1] < 0.8 * lg[0]


def test_densities_are_exp_of_forward(sur, torch):
    B, X = 3, 128
    W, b = presets.surrogate_test_weights(14, scale=0.5)
    p = _params(B, 24)
    net = sur.Surrogate(B, X, device="cuda:0")
    net.set_weights(W, b)
    out = net.forward(p).cpu().numpy().astype(np.float64)
    n0 = np.array([1e16, 2e16, 5e15])
    d = net.densities(p, n0).cpu().numpy()
    assert np.allclose(d[:, 0, :], n0[:, None] * np.exp(out[:, 1, :]), rtol=1e-12)
    assert np.allclose(d[:, 1, :], n0[:, None] * np.exp(out[:, 2, :]), rtol=1e-12)
    # the loader's state: densities, V phi/V, quantile channels times the 1 eV speeds
    st = net.state(p, n0).cpu().numpy()
    q_e, m_e, m_i = 1.602176634e-19, 9.1093837015e-31, 6.6464731e-27 - 9.1093837015e-31
    V = p[:, 2].astype(np.float32).astype(np.float64)
    assert np.allclose(st[:, 0:2, :], d, rtol=1e-12)
    assert np.allclose(st[:, 2, :], V[:, None] * out[:, 0, :], rtol=1e-12)
    assert np.allclose(st[:, 3:21, :], out[:, 3:21, :] * np.sqrt(q_e / m_e), rtol=1e-12)
    assert np.allclose(st[:, 21:39, :], out[:, 21:39, :] * np.sqrt(q_e / m_i), rtol=1e-12)


def test_surrogate_rejects_bad_shapes(sur, torch):
    net = sur.Surrogate(2, 64, device="cuda:0")
    with pytest.raises(ValueError):
        net.forward(_params(3, 1))
    from paper_2605_07083_amd import pic
    with pytest.raises(pic.PicError) as e:
        sur.Surrogate(2, 100, device="cuda:0")
    assert e.value.code == pic.PIC_EINVAL


# ---------------------------------------------------------------------------
# warm-start loader
# ---------------------------------------------------------------------------
def _profiles(cfg, seed, scale=1.0):
    """A sheath-like synthetic profile pair with fractional counts per cell."""
    rng = np.random.default_rng(seed)
    N = cfg["N"]
    u = (np.arange(N) + 0.5) / N
    ne = cfg["n0"] * scale * (0.15 + 0.85 * np.sin(np.pi * u) ** 0.5) * (1 + 0.05 * rng.normal(size=N))
    ni = cfg["n0"] * scale * (0.4 + 0.6 * np.sin(np.pi * u) ** 0.3) * (1 + 0.05 * rng.normal(size=N))
    return ne, ni


def _check_load(O, cfg, h, ne, ni, d=0):
    st, t = gpu_state(h, d)
    s = O.Sim(cfg)
    s.load_profiles(ne, ni)
    for sp in (0, 2):
        g, o = by_id(st[sp]), by_id(s.particles(sp))
        assert np.array_equal(g["id"], o["id"])
        assert np.array_equal(g["z"], o["z"])
        assert np.array_equal(g["tc"], o["tc"])
        for c in ("vx", "vy", "vz"):
            assert np.max(np.abs(g[c] - o[c].astype(np.float32)) / np.abs(o[c]).max()) < 1e-6
    assert len(st[1]["id"]) == 0
    assert t["next_id"] == s.next_id
    assert list(t["n_live"]) == [s.count(0), 0, s.count(2)]
    assert deposit_matches(O, cfg, h, st, d) == []
    s2 = oracle_from_gpu(O, cfg, st, t)
    assert field_matches(O, cfg, h, s2, d) == []


def test_profile_load_matches_oracle(torch, O):
    from paper_2605_07083_amd import pic
    cfg = presets.scaled(presets.tiny(), gamma_emit=1e21)
    ne, ni = _profiles(cfg, 1)
    _say("case: profile load, tiny diode")
    dens = torch.tensor(np.stack([ne, ni])[None], dtype=torch.float64, device="cuda:0")
    h = pic.Handle(cfg, densities=dens)
    _check_load(O, cfg, h, ne, ni)
    _say("case: restart parity from the profile load, 30 steps")
    assert restart_step_check(O, cfg, h, 30) == []


def test_profile_load_batched(torch, O):
    from paper_2605_07083_amd import pic
    cfgs = [presets.scaled(presets.tiny(), diode=d, gamma_emit=1e21) for d in range(3)]
    cfgs[1]["N"] = 128
    prof = [_profiles(c, 10 + d, scale=0.5 + 0.3 * d) for d, c in enumerate(cfgs)]
    nmax = 256
    arr = np.zeros((3, 2, nmax))
    for d, (ne, ni) in enumerate(prof):
        arr[d, 0, :len(ne)] = ne
        arr[d, 1, :len(ni)] = ni
    _say("case: profile load, 3 diodes (N 256/128/256)")
    h = pic.Handle(cfgs, densities=torch.tensor(arr, device="cuda:0"))
    for d in range(3):
        _check_load(O, cfgs[d], h, *prof[d], d=d)


def test_profile_load_errors(torch):
    from paper_2605_07083_amd import pic
    cfg = presets.tiny()
    N = cfg["N"]
    bad = np.ones((1, 2, N)) * cfg["n0"]
    bad[0, 1, 7] = -1.0
    with pytest.raises(pic.PicError) as e:
        pic.Handle(cfg, densities=torch.tensor(bad, device="cuda:0"))
    assert e.value.code == pic.PIC_ENAN
    big = np.ones((1, 2, N)) * cfg["n0"] * 3.0
    with pytest.raises(pic.PicError) as e:
        pic.Handle(cfg, densities=torch.tensor(big, device="cuda:0"))
    assert e.value.code == pic.PIC_ENOSPACE
    zero = np.zeros((1, 2, N))
    h = pic.Handle(cfg, densities=torch.tensor(zero, device="cuda:0"))
    t = h.tally(0)
    assert list(t["n_live"]) == [0, 0, 0]
    h.step(5)
    h.sync()
    with pytest.raises(ValueError):
        pic.Handle(cfg, densities=torch.zeros((1, 2, N + 1), dtype=torch.float64, device="cuda:0"))


# ---------------------------------------------------------------------------
# warm-start state loader (densities, potential, velocity quantiles)
# ---------------------------------------------------------------------------
def _state(cfg, seed, scale=1.0):
    """Densities as _profiles, a sheath-like potential and per-cell quantile
    vectors of a skewed, drifting distribution (unsorted in some cells), with
    a few cells above the energy limit so the clamp is exercised."""
    from paper_2605_07083_amd import pic
    rng = np.random.default_rng(seed + 100)
    N = cfg["N"]
    ne, ni = _profiles(cfg, seed, scale)
    u = (np.arange(N) + 0.5) / N
    L = np.array(pic.STATE_LEVELS)
    st = np.zeros((pic.STATE_ROWS, N))
    st[0], st[1] = ne, ni
    st[2] = cfg["V"] * u ** 0.7
    for q, (vth, drift) in enumerate(((6e5, 2e5), (2.5e3, -8e3))):
        base_z = drift * (1 - u)[None, :] + vth * (L[:, None] - 0.5) * (1 + 0.3 * rng.random((9, N)))
        base_p = vth * (0.2 + L[:, None]) * (1 + 0.2 * rng.random((9, N)))
        base_z[:, ::17] = base_z[::-1, ::17]           # unordered quantiles in some cells
        base_z[8, ::31] *= 40.0                         # some far above the energy limit
        st[3 + 18 * q:12 + 18 * q] = base_z
        st[12 + 18 * q:21 + 18 * q] = base_p
    return st


def test_state_load_matches_oracle(torch, O):
    from paper_2605_07083_amd import pic
    cfg = presets.scaled(presets.tiny(), gamma_emit=1e21)
    st = _state(cfg, 3)
    _say("case: state load, tiny diode")
    h = pic.Handle(cfg, state=torch.tensor(st[None], dtype=torch.float64, device="cuda:0"))
    g, t = gpu_state(h, 0)
    s = O.Sim(cfg)
    s.load_state(st)
    for sp in (0, 2):
        a, o = by_id(g[sp]), by_id(s.particles(sp))
        assert np.array_equal(a["id"], o["id"])
        assert np.array_equal(a["z"], o["z"])
        assert np.array_equal(a["tc"], o["tc"])
        for c in ("vx", "vy", "vz"):
            assert np.max(np.abs(a[c] - o[c].astype(np.float32)) / np.abs(o[c]).max()) < 1e-6, (sp, c)
    assert t["next_id"] == s.next_id
    assert deposit_matches(O, cfg, h, g, 0) == []
    assert field_matches(O, cfg, h, oracle_from_gpu(O, cfg, g, t), 0) == []
    _say("case: restart parity from the state load, 20 steps")
    assert restart_step_check(O, cfg, h, 20) == []


def test_state_load_batched_and_errors(torch, O):
    from paper_2605_07083_amd import pic
    cfgs = [presets.scaled(presets.tiny(), diode=d, gamma_emit=1e21) for d in range(2)]
    cfgs[1]["N"] = 128
    nmax = 256
    arr = np.zeros((2, pic.STATE_ROWS, nmax))
    sts = [_state(c, 20 + d, 0.7 + 0.3 * d) for d, c in enumerate(cfgs)]
    for d, st in enumerate(sts):
        arr[d, :, :st.shape[1]] = st
    _say("case: state load, 2 diodes (N 256/128)")
    h = pic.Handle(cfgs, state=torch.tensor(arr, device="cuda:0"))
    for d in range(2):
        g, t = gpu_state(h, d)
        s = O.Sim(cfgs[d])
        s.load_state(sts[d])
        for sp in (0, 2):
            a, o = by_id(g[sp]), by_id(s.particles(sp))
            assert np.array_equal(a["z"], o["z"]) and np.array_equal(a["id"], o["id"])
            assert np.max(np.abs(a["vz"] - o["vz"].astype(np.float32)) / np.abs(o["vz"]).max()) < 1e-6
    bad = arr[:1].copy()
    bad[0, 25, 7] = np.nan
    with pytest.raises(pic.PicError) as e:
        pic.Handle(cfgs[0], state=torch.tensor(bad, device="cuda:0"))
    assert e.value.code == pic.PIC_ENAN
    with pytest.raises(ValueError):
        pic.Handle(cfgs[0], state=torch.zeros((1, 3, 256), dtype=torch.float64, device="cuda:0"))
