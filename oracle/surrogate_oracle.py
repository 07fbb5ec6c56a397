"""FP64 reference of the learned warm-start surrogate.  TEST INFRASTRUCTURE
ONLY: used by tests/, the smoke check and the CPU baseline of bench.py, never
by the product path.

The surrogate maps the four scan parameters of the diode (emission flux,
cathode temperature, bias, neutral density; the swept quantities of "Benchmark
cases" and the operating point of "Model") to the late-time profiles the
paper plots (potential, electron and ion densities; "Results") at the X cell
centres.  The paper has no surrogate; its architecture is a reading: a stack
of six 1D convolutions, kernel 5, zero padding 2, channels 16 -> 64 x 5 -> 39,
tanh between layers, mean squared error, Adam.

Quantised mode (what the BF16 matrix-core path computes, written as a
definition): weights and every layer input are rounded to bfloat16 (round to
nearest even); the gradient reaching every pre-activation is rounded to
bfloat16 too; everything else is FP64 here.

Plain PyTorch CPU ops in float64: conv1d, tanh, autograd.  Pins: brute-force
convolution sums, finite-difference gradient checks, the closed form of the
first Adam steps, feature values at known positions.
"""
import numpy as np
import torch

KS = 5
PAD = 2
LAYERS = [(16, 64), (64, 64), (64, 64), (64, 64), (64, 64), (64, 39)]
N_IN = 16
N_OUT = 39
ADAM_B1 = 0.9
ADAM_B2 = 0.999
ADAM_EPS = 1e-8


def features(params, X):
    """Input channels [B][16][X] in FP64.  params [B][4] = (Gamma m^-2 s^-1,
    T_c K, V volts, n_g m^-3).

    Channels 0-3: the parameters mapped to [-1, 1] over the sampled ranges
    (log scale for flux and density: Gamma in [1e19, 1.2e20], T_c in
    [1800, 2200] K, V in [5, 20] V, n_g in [1e21, 1e22]).  Channels 4-15 are
    functions of the cell-centre coordinate u = (x + 1/2) / X: 2u - 1, 1 - 2u,
    sin and cos of pi u, 2 pi u, 4 pi u, exp(-64 u), exp(-64 (1 - u)),
    exp(-16 u), exp(-16 (1 - u))."""
    p = np.asarray(params, dtype=np.float64).reshape(-1, 4)
    B = p.shape[0]
    u = (np.arange(X, dtype=np.float64) + 0.5) / X
    f = np.empty((B, N_IN, X))
    f[:, 0, :] = (2.0 * np.log10(p[:, 0] / 1e19) / np.log10(12.0) - 1.0)[:, None]
    f[:, 1, :] = ((p[:, 1] - 2000.0) / 200.0)[:, None]
    f[:, 2, :] = ((p[:, 2] - 12.5) / 7.5)[:, None]
    f[:, 3, :] = (2.0 * np.log10(p[:, 3] / 1e21) - 1.0)[:, None]
    pos = [2 * u - 1, 1 - 2 * u,
           np.sin(np.pi * u), np.cos(np.pi * u),
           np.sin(2 * np.pi * u), np.cos(2 * np.pi * u),
           np.sin(4 * np.pi * u), np.cos(4 * np.pi * u),
           np.exp(-64 * u), np.exp(-64 * (1 - u)),
           np.exp(-16 * u), np.exp(-16 * (1 - u))]
    for k, v in enumerate(pos):
        f[:, 4 + k, :] = v[None, :]
    return f


def bf16(t):
    """Round to the nearest bfloat16 (ties to even), back in float64."""
    return t.to(torch.bfloat16).to(torch.float64)


class _RoundSTE(torch.autograd.Function):
    """Forward: bfloat16 rounding.  Backward: identity (the rounding is a
    storage format, its derivative is not taken)."""

    @staticmethod
    def forward(ctx, x):
        return bf16(x)

    @staticmethod
    def backward(ctx, g):
        return g


class _GradRound(torch.autograd.Function):
    """Forward: identity.  Backward: the incoming gradient rounded to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return bf16(g)


def conv(a, w, bias):
    """One layer: y[b][co][x] = bias[co] + sum_{ci, t} w[co][ci][t] a[b][ci][x + t - 2],
    with a = 0 outside [0, X) (torch conv1d is this cross-correlation)."""
    return torch.nn.functional.conv1d(a, w, bias, padding=PAD)


def forward(W, b, feat, quantize=True, keep=False):
    """Network output [B][N_OUT][X].  W, b: lists of arrays or tensors; feat
    [B][16][X].  With keep=True also returns the leaf tensors (for grads)."""
    Wt = [torch.as_tensor(np.asarray(w, dtype=np.float64)).requires_grad_(keep) for w in W]
    bt = [torch.as_tensor(np.asarray(v, dtype=np.float64)).requires_grad_(keep) for v in b]
    a = torch.as_tensor(np.asarray(feat, dtype=np.float64))
    n = len(LAYERS)
    for l in range(n):
        w = Wt[l]
        if quantize:
            a = _RoundSTE.apply(a)
            w = _RoundSTE.apply(w)
        z = conv(a, w, bt[l])
        if quantize:
            z = _GradRound.apply(z)
        a = torch.tanh(z) if l < n - 1 else z
    return (a, Wt, bt) if keep else a.detach().numpy()


def loss_and_grads(W, b, feat, target, quantize=True):
    """Mean squared error over (sample, channel, position) and its gradients
    with respect to every W_l and b_l (FP64)."""
    out, Wt, bt = forward(W, b, feat, quantize=quantize, keep=True)
    t = torch.as_tensor(np.asarray(target, dtype=np.float64))
    loss = ((out - t) ** 2).mean()
    loss.backward()
    return (loss.item(), [w.grad.numpy().copy() for w in Wt], [v.grad.numpy().copy() for v in bt])


def adam(w, m, v, g, t, lr, b1=ADAM_B1, b2=ADAM_B2, eps=ADAM_EPS):
    """One Adam update at step t >= 1 (bias-corrected moments).  Returns the
    new (w, m, v) in FP64."""
    w, m, v, g = (np.asarray(x, dtype=np.float64) for x in (w, m, v, g))
    m1 = b1 * m + (1 - b1) * g
    v1 = b2 * v + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** t)
    vh = v1 / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m1, v1


def train_step(W, b, mW, vW, mb, vb, t, feat, target, lr, quantize=True):
    """Forward, loss, backward and one Adam step on every tensor.  Returns
    (loss, grads_W, grads_b, W', b', mW', vW', mb', vb')."""
    loss, gW, gb = loss_and_grads(W, b, feat, target, quantize)
    W2, b2, mW2, vW2, mb2, vb2 = [], [], [], [], [], []
    for l in range(len(LAYERS)):
        w_, m_, v_ = adam(W[l], mW[l], vW[l], gW[l], t, lr)
        W2.append(w_); mW2.append(m_); vW2.append(v_)
        w_, m_, v_ = adam(b[l], mb[l], vb[l], gb[l], t, lr)
        b2.append(w_); mb2.append(m_); vb2.append(v_)
    return loss, gW, gb, W2, b2, mW2, vW2, mb2, vb2
