"""Pins of the warm-start oracle: the surrogate network and the profile loader.

Surrogate (a reading; the paper has no surrogate, it fixes only what the
profiles are: late-time potential and densities, "Results"):
* one layer equals a brute-force shifted-sum convolution (orientation,
  padding side, bias);
* the FP64 backward equals central finite differences of the loss along
  random directions and along single coordinates of every layer;
* the quantised mode equals bfloat16 rounding defined bit-wise (round to
  nearest even on the float32 pattern) and stays within bfloat16 noise of the
  plain network;
* Adam's first two steps under a constant gradient move every weight by
  lr * sign(g) (closed form of the bias-corrected moments);
* the input features take their closed-form values at the centre cell.

Profile loader ("Model": macro-particles loaded from a density; the warm start
replaces the uniform n0 by a given n(z)):
* an integer number of particles per cell is reproduced exactly, every
  particle inside its cell, ids in cell order;
* fractional expectations give counts floor(x) or floor(x) + 1 with mean x;
* a particle with a given id has the same velocity and free-flight counter as
  the uniform load's particle with that id (the same keyed draws);
* negative densities are rejected, zero densities load nothing.
"""
import math

import numpy as np
import pytest
import torch

from oracle import surrogate_oracle as S
from paper_2605_07083_amd import presets

from _helpers import M_E, M_I, Q_E


def _brute_conv(a, w, bias):
    # y[b][co][x] = bias[co] + sum_{ci,t} w[co][ci][t] a[b][ci][x+t-2], by shifted copies
    B, Cin, X = a.shape
    Cout = w.shape[0]
    y = np.zeros((B, Cout, X)) + bias[None, :, None]
    for t in range(5):
        sh = np.zeros_like(a)
        d = t - 2
        for x in range(X):
            xs = x + d
            if 0 <= xs < X:
                sh[:, :, x] = a[:, :, xs]
        for co in range(Cout):
            for ci in range(Cin):
                y[:, co, :] += w[co, ci, t] * sh[:, ci, :]
    return y


def test_conv_layer_is_shifted_sum():
    rng = np.random.default_rng(3)
    a = rng.normal(size=(2, 3, 9))
    w = rng.normal(size=(4, 3, 5))
    bias = rng.normal(size=4)
    y = S.conv(torch.tensor(a), torch.tensor(w), torch.tensor(bias)).numpy()
    assert np.allclose(y, _brute_conv(a, w, bias), rtol=1e-13, atol=1e-13)
    # a delta input at x=4 in channel 1 reads back the kernel reversed in x
    a = np.zeros((1, 3, 9)); a[0, 1, 4] = 1.0
    y = S.conv(torch.tensor(a), torch.tensor(w), torch.tensor(np.zeros(4))).numpy()
    for t in range(5):
        assert np.allclose(y[0, :, 4 - (t - 2)], w[:, 1, t])


def test_network_matches_brute_force_stack():
    W, b = presets.surrogate_test_weights(5)
    p = np.array([[3e19, 1900.0, 8.0, 2e21]])
    f = S.features(p, 6)
    a = f.copy()
    for l, (w, bb) in enumerate(zip(W, b)):
        a = _brute_conv(a, w.astype(np.float64), bb.astype(np.float64))
        if l < 5:
            a = np.tanh(a)
    assert np.allclose(S.forward(W, b, f, quantize=False), a, rtol=1e-12, atol=1e-12)


def _loss(W, b, f, t):
    return float(((torch.tensor(S.forward(W, b, f, quantize=False)) - torch.tensor(t)) ** 2).mean())


def test_backward_matches_finite_differences():
    W, b = presets.surrogate_test_weights(7)
    W = [w.astype(np.float64) for w in W]
    b = [v.astype(np.float64) for v in b]
    rng = np.random.default_rng(8)
    p = np.array([[2e19, 2100.0, 15.0, 5e21], [9e19, 1850.0, 6.0, 1.5e21]])
    f = S.features(p, 12)
    t = rng.normal(size=(2, S.N_OUT, 12))
    loss, gW, gb = S.loss_and_grads(W, b, f, t, quantize=False)
    assert loss == pytest.approx(_loss(W, b, f, t), rel=1e-14)
    h = 1e-5
    # random directions through all parameters
    for k in range(3):
        dW = [rng.normal(size=w.shape) for w in W]
        db = [rng.normal(size=v.shape) for v in b]
        lp = _loss([w + h * d for w, d in zip(W, dW)], [v + h * d for v, d in zip(b, db)], f, t)
        lm = _loss([w - h * d for w, d in zip(W, dW)], [v - h * d for v, d in zip(b, db)], f, t)
        fd = (lp - lm) / (2 * h)
        an = sum((g * d).sum() for g, d in zip(gW, dW)) + sum((g * d).sum() for g, d in zip(gb, db))
        assert fd == pytest.approx(an, rel=1e-6)
    # single coordinates of every layer
    for l in range(6):
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in W[l].shape)
            Wp = [w.copy() for w in W]; Wm = [w.copy() for w in W]
            Wp[l][idx] += h; Wm[l][idx] -= h
            fd = (_loss(Wp, b, f, t) - _loss(Wm, b, f, t)) / (2 * h)
            assert fd == pytest.approx(gW[l][idx], rel=1e-5, abs=1e-11)
        j = int(rng.integers(0, b[l].shape[0]))
        bp = [v.copy() for v in b]; bm = [v.copy() for v in b]
        bp[l][j] += h; bm[l][j] -= h
        fd = (_loss(W, bp, f, t) - _loss(W, bm, f, t)) / (2 * h)
        assert fd == pytest.approx(gb[l][j], rel=1e-5, abs=1e-11)


def _bf16_bits(x):
    # round-to-nearest-even of the float32 pattern to its top 16 bits
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_rounding_definition():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=1000).astype(np.float32),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0], np.float32)])
    got = S.bf16(torch.tensor(x.astype(np.float64))).numpy()
    assert np.array_equal(got, _bf16_bits(x))
    # ties go to even: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6
    assert got[1000] == 1.0 and got[1001] == 1.0 + 2 ** -6


def test_quantised_network_within_bf16_noise():
    W, b = presets.surrogate_test_weights(2)
    p = np.array([[5e19, 2000.0, 10.0, 3e21]])
    f = S.features(p, 64)
    q = S.forward(W, b, f, quantize=True)
    e = S.forward(W, b, f, quantize=False)
    rel = np.linalg.norm(q - e) / np.linalg.norm(e)
    assert 1e-4 < rel < 3e-2
    # the quantised gradients are those of the same loss up to bf16 noise
    t = np.zeros_like(e)
    _, gq, bq = S.loss_and_grads(W, b, f, t, quantize=True)
    _, ge, be = S.loss_and_grads(W, b, f, t, quantize=False)
    for l in range(6):
        assert np.linalg.norm(gq[l] - ge[l]) < 5e-2 * np.linalg.norm(ge[l])


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(4)
    g = rng.normal(size=100) * 10.0 ** rng.uniform(-3, 3, 100)
    w0 = rng.normal(size=100)
    lr = 1e-3
    w1, m1, v1 = S.adam(w0, np.zeros(100), np.zeros(100), g, 1, lr)
    # bias-corrected moments at t = 1 are g and g^2
    assert np.allclose(w1, w0 - lr * g / (np.abs(g) + S.ADAM_EPS), rtol=0, atol=1e-15)
    w2, m2, v2 = S.adam(w1, m1, v1, g, 2, lr)
    assert np.allclose(m2 / (1 - 0.9 ** 2), g, rtol=1e-12)
    assert np.allclose(v2 / (1 - 0.999 ** 2), g * g, rtol=1e-12)
    assert np.allclose(w2, w0 - 2 * lr * g / (np.abs(g) + S.ADAM_EPS), rtol=0, atol=1e-14)
    big = np.abs(g) > 1e-2          # there eps is negligible: two steps of lr sign(g)
    assert np.allclose(w2[big], w0[big] - 2 * lr * np.sign(g[big]), rtol=0, atol=1e-8)


def test_features_at_centre_and_corners():
    p = np.array([[1e19, 1800.0, 5.0, 1e21], [1.2e20, 2200.0, 20.0, 1e22]])
    f = S.features(p, 1)         # one cell: u = 1/2
    assert np.allclose(f[0, :4, 0], -1.0) and np.allclose(f[1, :4, 0], 1.0)
    c = f[0, 4:, 0]
    exp = [0, 0, 1, 0, 0, -1, 0, 1, math.exp(-32), math.exp(-32), math.exp(-8), math.exp(-8)]
    assert np.allclose(c, exp, atol=1e-15)
    f = S.features(p[:1], 4)
    assert np.allclose(f[0, 4, :], [-0.75, -0.25, 0.25, 0.75])


# ---------------------------------------------------------------------------
# profile loader
# ---------------------------------------------------------------------------
def _cfg(**kw):
    c = presets.scaled(presets.tiny(), gamma_emit=0.0, replenish=0)
    c.update(kw)
    return c


def _ppc(O, c):
    d = O.derive(c)
    return d["dz"] / d["w0"]


def test_profile_integer_counts_exact(O):
    c = _cfg()
    d = O.derive(c)
    N = c["N"]
    k = c["n_load"] // N                       # 100 per cell
    n = np.full(N, k * d["w0"] / d["dz"])
    assert np.all(n * d["dz"] / d["w0"] == k)
    s = O.Sim(c)
    s.load_profiles(n, n)
    for sp, base in ((0, 0), (2, N * k)):
        P = s.particles(sp)
        assert len(P["z"]) == N * k
        cell = np.floor(P["z"] / d["dz"]).astype(int)
        assert np.array_equal(cell, np.repeat(np.arange(N), k))
        assert np.array_equal(P["id"], base + np.arange(N * k))
    assert s.next_id == 2 * N * k
    assert s.count(1) == 0


def test_profile_fractional_counts(O):
    c = _cfg()
    d = O.derive(c)
    N = c["N"]
    x = 0.3 + 2.0 * (np.arange(N) % 7) / 7.0      # 0.3 .. 2.01 per cell
    ne = x * d["w0"] / d["dz"]
    ni = np.zeros(N)
    ni[N // 2:] = 1.5 * d["w0"] / d["dz"]
    s = O.Sim(c)
    s.load_profiles(ne, ni)
    P = s.particles(0)
    cnt = np.bincount(np.floor(P["z"] / d["dz"]).astype(int), minlength=N)
    xe = ne * d["dz"] / d["w0"]
    assert np.all((cnt == np.floor(xe)) | (cnt == np.floor(xe) + 1))
    assert abs(cnt.sum() - xe.sum()) < 4 * math.sqrt(np.sum(xe % 1 * (1 - xe % 1)))
    I = s.particles(2)
    ci = np.floor(I["z"] / d["dz"]).astype(int)
    assert ci.min() >= N // 2
    # uniform inside the cells
    fr = I["z"] / d["dz"] - ci
    assert abs(fr.mean() - 0.5) < 4 * math.sqrt(1 / 12 / len(fr))


def test_profile_draws_match_uniform_load_by_id(O):
    c = _cfg()
    d = O.derive(c)
    N = c["N"]
    u = O.Sim(c)
    u.load()
    w = O.Sim(c)
    k = c["n_load"] // N
    w.load_profiles(np.full(N, k * d["w0"] / d["dz"]), np.full(N, k * d["w0"] / d["dz"]))
    for sp in (0, 2):
        A, B = u.particles(sp), w.particles(sp)
        assert np.array_equal(A["id"], B["id"])
        for key in ("vx", "vy", "vz", "tc"):
            assert np.array_equal(A[key], B[key]), key
    # Maxwellian electrons at Te0
    v = u.particles(0)["vz"]
    sig = math.sqrt(Q_E * c["Te0"] / M_E)
    assert np.std(v) == pytest.approx(sig, rel=0.02)


def test_profile_rejects_negative_and_loads_nothing_for_zero(O):
    c = _cfg()
    N = c["N"]
    s = O.Sim(c)
    with pytest.raises(ValueError):
        s.load_profiles(np.full(N, -1.0), np.zeros(N))
    s.load_profiles(np.zeros(N), np.zeros(N))
    assert s.count(0) == 0 and s.count(2) == 0


# ---------------------------------------------------------------------------
# warm start with velocity quantiles (o_load_state)
# ---------------------------------------------------------------------------
def _state(O, c, nper, qz_e, qp_e, qz_i, qp_i, phi=None):
    """State rows for densities of `nper` particles per cell and the given
    nine-level quantile vectors (the same in every cell)."""
    d = O.derive(c)
    N = c["N"]
    prof = np.zeros((O.STATE_ROWS, N))
    prof[0] = prof[1] = nper * d["w0"] / d["dz"]
    prof[2] = 0.5 * c["V"] if phi is None else phi
    for r0, q in ((3, qz_e), (12, qp_e), (21, qz_i), (30, qp_i)):
        prof[r0:r0 + 9] = np.asarray(q, float)[:, None]
    return prof


def test_state_uniform_quantiles_give_uniform_speeds(O):
    """Quantiles of U[a, b] at any levels are a + level (b - a), and the
    piecewise-linear inverse of that quantile function is exact: v_z must be
    uniform on [a, b] (mean, variance, KS) and the azimuth uniform."""
    from scipy import stats
    c = _cfg()
    L = np.array(O.STATE_LEVELS)
    a, b = -5.0e3, 1.2e4          # ions below the load's energy limit (12 eV here)
    qz = a + L * (b - a)
    qp = 1.0e3 + L * 2.0e3
    s = O.Sim(c)
    s.load_state(_state(O, c, 100, qz * 30, qp * 30, qz, qp))
    I = s.particles(2)
    v = I["vz"]
    assert stats.kstest((v - a) / (b - a), "uniform").pvalue > 1e-3
    vp = np.hypot(I["vx"], I["vy"])
    assert stats.kstest((vp - 1.0e3) / 2.0e3, "uniform").pvalue > 1e-3
    az = np.arctan2(I["vy"], I["vx"])
    assert stats.kstest((az + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3
    E = s.particles(0)["vz"]
    assert stats.kstest((E / 30 - a) / (b - a), "uniform").pvalue > 1e-3


def test_state_degenerate_quantiles_and_rearrangement(O):
    """Equal quantiles give that value for every particle; reversed quantile
    vectors load exactly what the sorted ones do."""
    c = _cfg()
    L = np.array(O.STATE_LEVELS)
    s = O.Sim(c)
    s.load_state(_state(O, c, 20, np.full(9, 1.0e5), np.full(9, 3.0e4), np.full(9, -2.0e3), np.full(9, 500.0)))
    P, I = s.particles(0), s.particles(2)
    assert np.all(P["vz"] == 1.0e5) and np.all(I["vz"] == -2.0e3)
    assert np.allclose(np.hypot(P["vx"], P["vy"]), 3.0e4, rtol=1e-12)
    assert np.allclose(np.hypot(I["vx"], I["vy"]), 500.0, rtol=1e-12)
    q = 1.0e4 * (L - 0.3) ** 3
    s1, s2 = O.Sim(c), O.Sim(c)
    s1.load_state(_state(O, c, 20, q, np.abs(q), q / 50, np.abs(q) / 50))
    s2.load_state(_state(O, c, 20, q[::-1], np.abs(q)[::-1], q[::-1] / 50, np.abs(q)[::-1] / 50))
    for sp in (0, 2):
        A, B = s1.particles(sp), s2.particles(sp)
        for k in ("z", "vx", "vy", "vz", "id", "tc"):
            assert np.array_equal(A[k], B[k]), k


def test_state_positions_ids_and_flights_match_profile_load(O):
    """Counts, ids, positions and free flights use the draws of the profile
    loader, so they are identical to it for the same densities."""
    c = _cfg()
    d = O.derive(c)
    N = c["N"]
    x = 0.3 + 2.0 * (np.arange(N) % 7) / 7.0
    ne = x * d["w0"] / d["dz"]
    ni = ne[::-1].copy()
    L = np.array(O.STATE_LEVELS)
    prof = _state(O, c, 1, 1e5 * (L - 0.5), 1e5 * L, 1e3 * (L - 0.5), 1e3 * L)
    prof[0], prof[1] = ne, ni
    a, b = O.Sim(c), O.Sim(c)
    a.load_profiles(ne, ni)
    b.load_state(prof)
    for sp in (0, 2):
        A, B = a.particles(sp), b.particles(sp)
        for k in ("z", "id", "tc"):
            assert np.array_equal(A[k], B[k]), k
    assert a.next_id == b.next_id


def test_state_energy_clamp(O):
    """Kinetic energy at load is scaled down to the null-collision bound's
    energy cap, e (|V| + 40 T0) with T0 = Te0 + Tc for electrons and Ti0 for
    ions (the range the bound was scanned over); the potential row does not
    enter."""
    c = _cfg()
    N = c["N"]
    huge = np.full(9, 5.0e7)
    s1, s2 = O.Sim(c), O.Sim(c)
    s1.load_state(_state(O, c, 20, huge, huge, huge / 1e3, huge / 1e3, phi=np.linspace(0.0, c["V"], N)))
    s2.load_state(_state(O, c, 20, huge, huge, huge / 1e3, huge / 1e3, phi=np.zeros(N)))
    for sp, m, T0 in ((0, M_E, c["Te0"] + c["Tc"]), (2, M_I, c["Ti0"])):
        P = s1.particles(sp)
        ke = 0.5 * m * (P["vx"] ** 2 + P["vy"] ** 2 + P["vz"] ** 2) / Q_E
        cap = abs(c["V"]) + 40.0 * T0
        assert np.all(ke <= cap * (1 + 1e-12))
        assert np.all(ke >= cap * (1 - 1e-9))       # every particle was above it
        for k in ("vx", "vy", "vz"):
            assert np.array_equal(P[k], s2.particles(sp)[k])


def test_state_rejects_non_finite(O):
    c = _cfg()
    L = np.array(O.STATE_LEVELS)
    prof = _state(O, c, 5, L, L, L, L)
    prof[25, 3] = np.nan
    with pytest.raises(ValueError):
        O.Sim(c).load_state(prof)
