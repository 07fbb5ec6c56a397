"""Learned warm start: dataset generation, training and the warm-vs-cold
evaluation, driving the library's kernels through the C ABI.

Host orchestration only: the particle runs are pic_step graphs, the steady
detector is pic_steady_state, the profiles come from the device's time
averages, the surrogate's forward, backward and Adam steps are sur_* calls,
and the warm load is pic_init_from_profiles.  What runs here is batching,
bookkeeping and the conversion of node fields into training targets.

Steady state (the paper's late-time windows of "Benchmark cases", read as in
pic_steady_state): blocks of `block_steps`; a diode is steady at the end of
the first block whose backflow ratio is within tol_pp of the two blocks
before it and whose live count is within tol_rel of the block before.  The
profiles and the steady backflow ratio are then averaged over the next
`avg_blocks` blocks.

    python -m paper_2605_07083_amd.warmstart generate --n 512 --seed train --out data/train.npz
    python -m paper_2605_07083_amd.warmstart train --data data/train.npz --out data/weights.npz
    python -m paper_2605_07083_amd.warmstart evaluate --data data/heldout.npz --weights data/weights.npz
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import pic, presets

DENSITY_FLOOR = 1e-4      # targets use ln(max(n, floor n0) / n0)
BATCH_DIODES = 32


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def params_of(cfg):
    return [cfg["gamma_emit"], cfg["T_K"], cfg["V"], cfg["ng"]]


def targets_from_fields(cfg, f):
    """Node fields (N + 1) -> cell-centre targets [3][N]: phi / V,
    ln(n_e / n0), ln(n_i / n0) (cell value = mean of its two nodes)."""
    c = lambda a: 0.5 * (a[:-1] + a[1:])
    n0 = cfg["n0"]
    fl = DENSITY_FLOOR * n0
    return np.stack([c(f["phi"]) / cfg["V"], np.log(np.maximum(c(f["n_e"]), fl) / n0),
                     np.log(np.maximum(c(f["n_i"]), fl) / n0)])


def run_to_steady(cfgs, densities=None, block_steps=5000, tol_pp=1.0, tol_rel=5e-4, avg_blocks=4,
                  max_steps=300000, label=""):
    """Run a batch of diodes until each is steady and averaged.  Returns one
    dict per diode: steady_step (-1 if never), backflow_pct over the averaging
    window, targets [3][N] (None if never steady), steps (run length)."""
    import torch
    nd = len(cfgs)
    tp = cfgs[0]["tally_period"]
    if block_steps % tp or any(c["tally_period"] != tp for c in cfgs):
        raise ValueError("block_steps must be a multiple of one common tally period")
    bt = block_steps // tp
    t0 = time.time()
    h = pic.Handle(cfgs, densities=densities)
    phase = ["relax"] * nd
    res = [{"steady_step": -1, "backflow_pct": float("nan"), "targets": None, "steps": 0} for _ in range(nd)]
    avg_start = [0] * nd
    step = 0
    while step < max_steps and any(p != "done" for p in phase):
        h.step(block_steps)
        step += block_steps
        for d in range(nd):
            if phase[d] == "relax":
                s = h.steady_state(d, block_tallies=bt, tol_pp=tol_pp, tol_rel=tol_rel)
                if s["steady"]:
                    res[d]["steady_step"] = int(s["steady_step"])
                    phase[d] = "avg"
                    avg_start[d] = step
                    h.avg_control(d, True)
            elif phase[d] == "avg" and step - avg_start[d] >= avg_blocks * block_steps:
                f = h.fields(d, time_avg=True)
                dg = h.diagnostics(d, window_steps=step - avg_start[d])
                res[d]["targets"] = targets_from_fields(cfgs[d], f)
                res[d]["backflow_pct"] = float(dg["backflow_pct"])
                res[d]["steps"] = step
                h.avg_control(d, False)
                phase[d] = "done"
        if step % (10 * block_steps) == 0 or all(p == "done" for p in phase):
            _log("%s step %d: %d steady, %d done (%.0f s)" % (label, step, sum(p != "relax" for p in phase),
                                                           sum(p == "done" for p in phase), time.time() - t0))
    for d in range(nd):
        if phase[d] != "done":
            res[d]["steps"] = step
    h.sync()
    del h
    torch.cuda.synchronize()
    return res


def generate(n, seed, out, **kw):
    cfgs = presets.surrogate_cases(n, seed)
    P, T, S, B, R = [], [], [], [], []
    for b0 in range(0, n, BATCH_DIODES):
        batch = cfgs[b0:b0 + BATCH_DIODES]
        res = run_to_steady(batch, label="generate %d-%d" % (b0, b0 + len(batch) - 1), **kw)
        for c, r in zip(batch, res):
            P.append(params_of(c))
            T.append(r["targets"] if r["targets"] is not None else np.full((3, c["N"]), np.nan))
            S.append(r["steady_step"])
            B.append(r["backflow_pct"])
            R.append(r["steps"])
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    np.savez(out, params=np.array(P), targets=np.array(T, np.float32), steady_step=np.array(S),
             backflow_pct=np.array(B), steps=np.array(R), seed=seed)
    ok = np.array(S) >= 0
    _log("generated %d cases (%d steady), median steps-to-steady %s -> %s" % (
        n, ok.sum(), np.median(np.array(S)[ok]) if ok.any() else "n/a", out))


def train(data, out, epochs=600, batch=32, lr=2e-3, seed=7, heldout=None):
    import torch
    from .surrogate import Surrogate
    z = np.load(data)
    ok = np.isfinite(z["targets"]).all(axis=(1, 2))
    P = torch.tensor(z["params"][ok], dtype=torch.float32, device="cuda:0")
    T = torch.tensor(z["targets"][ok], dtype=torch.float32, device="cuda:0")
    n, X = T.shape[0], T.shape[2]
    net = Surrogate(batch, X, seed=seed)
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.time()
    steps = 0
    for ep in range(epochs):
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))       # cosine decay
        perm = torch.randperm(n, generator=g)
        tot = 0.0
        nb = 0
        for k in range(0, n - batch + 1, batch):
            idx = perm[k:k + batch].to("cuda:0")
            want = k + 2 * batch > n
            l = net.train_step(P[idx], T[idx], max(lr_ep, 1e-5), want_loss=want)
            steps += 1
            if want:
                tot += l
                nb += 1
        if ep % 25 == 0 or ep == epochs - 1:
            hist.append((ep, tot / max(nb, 1)))
            _log("epoch %d loss %.5g (%.1f s, %d steps)" % (ep, tot / max(nb, 1), time.time() - t0, steps))
    torch.cuda.synchronize()
    train_s = time.time() - t0
    W, b = net.weights()
    np.savez(out, **{"W%d" % l: W[l] for l in range(6)}, **{"b%d" % l: b[l] for l in range(6)})
    rep = {"train_seconds": train_s, "steps": steps, "epochs": epochs, "samples": int(n),
           "train_mse": _mse(net, P, T, batch)}
    if heldout:
        zh = np.load(heldout)
        okh = np.isfinite(zh["targets"]).all(axis=(1, 2))
        rep["heldout_mse"] = _mse(net, torch.tensor(zh["params"][okh], dtype=torch.float32, device="cuda:0"),
                                  torch.tensor(zh["targets"][okh], dtype=torch.float32, device="cuda:0"), batch)
    _log("trained: %s" % rep)
    return rep


def _mse(net, P, T, batch):
    tot, cnt = 0.0, 0
    for k in range(0, P.shape[0], batch):
        o = net.forward(P[k:k + batch])
        tot += float(((o - T[k:k + batch]) ** 2).sum())
        cnt += o.numel()
    return tot / max(cnt, 1)


def load_weights(path):
    z = np.load(path)
    return [z["W%d" % l] for l in range(6)], [z["b%d" % l] for l in range(6)]


def evaluate(data, weights=None, out=None, **kw):
    """Warm runs of the held-out cases against their cold runs (stored in
    `data`).  With weights: from the surrogate's profiles.  Without: from the
    cold runs' own late-time profiles (the best any predictor can do)."""
    import torch
    z = np.load(data)
    seed = int(z["seed"])
    n = len(z["params"])
    cfgs = presets.surrogate_cases(n, seed)
    net = None
    if weights:
        from .surrogate import Surrogate
        W, b = load_weights(weights)
        net = Surrogate(BATCH_DIODES, cfgs[0]["N"])
        net.set_weights(W, b)
    rows = []
    for b0 in range(0, n, BATCH_DIODES):
        batch = cfgs[b0:b0 + BATCH_DIODES]
        n0 = torch.tensor([c["n0"] for c in batch], dtype=torch.float64, device="cuda:0")
        if net is not None:
            p = torch.tensor([params_of(c) for c in batch], dtype=torch.float32, device="cuda:0")
            dens = net.densities(p, n0).contiguous()
        else:
            t = np.nan_to_num(z["targets"][b0:b0 + len(batch)].astype(np.float64), nan=0.0)
            dens = (n0[:, None, None] * torch.exp(torch.tensor(t[:, 1:3], device="cuda:0"))).contiguous()
        res = run_to_steady(batch, densities=dens, label="warm %d-%d" % (b0, b0 + len(batch) - 1), **kw)
        for k, r in enumerate(res):
            i = b0 + k
            rows.append({"case": i, "cold_steady_step": int(z["steady_step"][i]),
                         "warm_steady_step": r["steady_step"], "cold_backflow_pct": float(z["backflow_pct"][i]),
                         "warm_backflow_pct": r["backflow_pct"]})
    ok = [r for r in rows if r["cold_steady_step"] > 0 and r["warm_steady_step"] > 0]
    ratio = np.array([r["cold_steady_step"] / r["warm_steady_step"] for r in ok])
    dbr = np.array([abs(r["warm_backflow_pct"] - r["cold_backflow_pct"]) for r in ok])
    summ = {"cases": n, "both_steady": len(ok),
            "median_cold_steps": float(np.median([r["cold_steady_step"] for r in ok])) if ok else None,
            "median_warm_steps": float(np.median([r["warm_steady_step"] for r in ok])) if ok else None,
            "median_speedup": float(np.median(ratio)) if ok else None,
            "frac_speedup_ge_3": float(np.mean(ratio >= 3)) if ok else None,
            "median_abs_dBR_pp": float(np.median(dbr)) if ok else None,
            "frac_dBR_le_1pp": float(np.mean(dbr <= 1.0)) if ok else None,
            "frac_speedup_ge_3_and_dBR_le_1pp": float(np.mean((ratio >= 3) & (dbr <= 1.0))) if ok else None}
    _log("evaluate: %s" % summ)
    if out:
        json.dump({"summary": summ, "rows": rows}, open(out, "w"), indent=1)
    return summ


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2605_07083_amd.warmstart")
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--n", type=int, default=512)
    g.add_argument("--seed", default="train", help="'train', 'heldout' or an integer")
    g.add_argument("--out", required=True)
    g.add_argument("--max-steps", type=int, default=300000)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--heldout")
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=600)
    t.add_argument("--batch", type=int, default=32)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--report")
    e = sub.add_parser("evaluate")
    e.add_argument("--data", required=True)
    e.add_argument("--weights", help="surrogate weights; omitted: the cold runs' own profiles")
    e.add_argument("--out")
    e.add_argument("--max-steps", type=int, default=300000)
    a = ap.parse_args(argv)
    if a.cmd == "generate":
        seed = {"train": presets.SURROGATE_TRAIN_SEED, "heldout": presets.SURROGATE_HELDOUT_SEED}.get(a.seed)
        generate(a.n, int(a.seed, 0) if seed is None else seed, a.out, max_steps=a.max_steps)
    elif a.cmd == "train":
        rep = train(a.data, a.out, epochs=a.epochs, batch=a.batch, lr=a.lr, heldout=a.heldout)
        if a.report:
            json.dump(rep, open(a.report, "w"), indent=1)
    else:
        evaluate(a.data, a.weights, a.out, max_steps=a.max_steps)


if __name__ == "__main__":
    main()
