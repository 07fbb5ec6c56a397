"""Host-side checks of the C-ABI library (no GPU needed).

* libpic.so loads and exports every function declared in include/pic.h.
* Host derivation (dz, w0, null-collision bounds, emission per step) equals the
  oracle's bit for bit: both follow the same reading with independent code.
* Configuration errors are rejected with PIC_EINVAL.
* The steady-state criterion on synthetic block series.
"""
import os
import re

import numpy as np
import pytest

from paper_2605_07083_amd import pic, presets

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="pic.h", prefix="pic"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(%s_[a-z_]+)\s*\(" % prefix, src)))


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(pic.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(pic.SYMBOLS)
    from paper_2605_07083_amd import surrogate
    names = _declared("surrogate.h", "sur")
    assert len(names) == 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(surrogate.SYMBOLS)


def test_surrogate_workspace_and_shapes():
    from paper_2605_07083_amd import surrogate
    assert surrogate.N_WEIGHTS == 99520 and surrogate.N_BIASES == 359 and surrogate.N_OUT == 39
    a = surrogate.workspace_size(1, 2048)
    b = surrogate.workspace_size(32, 2048)
    # per position: features 16 bf16, outputs 5 x 64 + 48 FP32 (39 channels
    # padded to 48), hidden bf16 copies 5 x 64, two gradient buffers 2 x 64
    # bf16 = 2400 bytes; per sample, the partial weight and bias gradients of
    # one layer over its slices of 256 positions
    per_pos = 16 * 2 + (5 * 64 + 48) * 4 + 5 * 64 * 2 + 2 * 64 * 2
    per_sample = (2048 // 256) * (64 * 320 + 64) * 4
    assert abs((b - a) - (per_pos * 2048 + per_sample) * 31) < 64 * 1024
    for bad in ((0, 2048), (4, 100), (4, 0)):
        with pytest.raises(pic.PicError) as e:
            surrogate.workspace_size(*bad)
        assert e.value.code == pic.PIC_EINVAL
    W = [np.arange(ci * co * 5, dtype=np.float32).reshape(co, ci, 5) for ci, co in surrogate.LAYERS]
    B = [np.arange(co, dtype=np.float32) for _, co in surrogate.LAYERS]
    w, b = surrogate.pack(W, B)
    W2, B2 = surrogate.unpack(w, b)
    assert all(np.array_equal(x, y) for x, y in zip(W, W2)) and all(np.array_equal(x, y) for x, y in zip(B, B2))


@pytest.mark.parametrize("name", ["tiny", "bench", "large", "paper"])
def test_derived_match_oracle(O, name):
    p = getattr(presets, name)()
    a, b = pic.pic_derive(p), O.derive(p)
    for k in ("dz", "invdz", "w0"):
        assert a[k] == b[k], k
    assert a["numax"] == b["numax"] and a["lam"] == b["lam"]
    assert a["emit_per_step"] == p["gamma_emit"] * p["dt"] / b["w0"]
    assert all(c % 2048 == 0 and c >= p["n_load"] for c in a["capacity"])


def test_sweep_derived_and_workspace():
    cfgs = presets.sweep()
    assert len(cfgs) == 32
    w = [pic.pic_derive(c)["w0"] for c in cfgs]
    assert min(w) > 0
    g = [c["gamma_emit"] for c in cfgs]
    assert g[0] == pytest.approx(1e19) and g[-1] == pytest.approx(1.2e20)
    T = sorted(c["Tc"] / presets.KB_OVER_E for c in cfgs)
    assert T[0] == pytest.approx(1800) and T[-1] == pytest.approx(2200)
    n = [c["n_load"] for c in cfgs]
    assert min(n) == 100000 and max(n) == 600000
    one = pic.pic_workspace_size([cfgs[0]])
    all_ = pic.pic_workspace_size(cfgs)
    assert all_ > 20 * one


@pytest.mark.parametrize("bad", [dict(N=1), dict(L=0.0), dict(dt=-1.0), dict(n_load=0), dict(ng=-1.0),
                                 dict(tally_period=0)])
def test_bad_config_rejected(bad):
    p = presets.scaled(presets.tiny(), **bad)
    with pytest.raises(pic.PicError) as e:
        pic.pic_derive(p)
    assert e.value.code == pic.PIC_EINVAL


def test_steady_state_criterion():
    rng = np.random.default_rng(0)
    # a relaxation towards 40 % with noise, live count settling
    b = np.arange(30)
    br = 40 + 30 * np.exp(-b / 4.0) + rng.normal(0, 0.1, len(b))
    nl = 1e6 * (1 + 0.2 * np.exp(-b / 3.0))
    r = pic.steady_from_series(br, nl, tol_pp=1.0, tol_rel=0.01)
    k = r["steady_block"]
    assert k > 0
    # first block meeting both conditions, computed directly
    ok = [i for i in range(2, len(b)) if abs(br[i] - br[i - 1]) < 1 and abs(br[i] - br[i - 2]) < 1
          and abs(nl[i] - nl[i - 1]) / nl[i] < 0.01]
    assert k == ok[0]
    assert r["blocks_averaged"] == 4
    assert r["backflow_pct"] == pytest.approx(br[k + 1:k + 5].mean())
    # never steady
    r = pic.steady_from_series(np.arange(10) * 5.0, np.ones(10), 1.0, 0.01)
    assert r["steady_block"] == -1 and np.isnan(r["backflow_pct"])
    # steady at the very end: nothing left to average
    br2 = np.array([50, 30, 20, 20.2, 20.1])
    r = pic.steady_from_series(br2, np.ones(5), 1.0, 0.01)
    assert r["steady_block"] == 4 and r["blocks_averaged"] == 0
