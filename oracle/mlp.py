"""FP64 reference of the surrogate network (test infrastructure only).

The surrogate is not part of the paper: it maps control-node velocities to a
predicted log-misfit so that candidate particles can be screened before the
finite-difference fitness. Network: x_hat = (x - lo)/(hi - lo), then hidden
layers h = GELU(W h_prev + b) with the exact erf GELU, then a linear scalar
output. Loss: mean squared error. Optimiser: Adam (Kingma and Ba, 2015).
Pinned by: central finite differences of the loss (backward), GELU identities,
and closed forms of Adam: the first step (-lr * sign(g)), every step under a
constant gradient (bias-corrected moments exactly g and g^2, so each step is
-lr g / (|g| + eps)) and under a gradient of alternating sign (the first
moment a geometric sum).
"""
import math

import numpy as np
from scipy.special import erf


def gelu(x):
    return x * 0.5 * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    phi = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * phi


def init_params(sizes, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, FP64, seeded."""
    rng = np.random.default_rng(seed)
    params = []
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        s = 1.0 / math.sqrt(fin)
        params.append((rng.uniform(-s, s, (fout, fin)), rng.uniform(-s, s, fout)))
    return params


def forward(params, X, lo, hi):
    """Returns (y[n], cache). X[n][D] raw node velocities."""
    h = (np.asarray(X, np.float64) - lo) / (hi - lo)
    cache = [h]
    L = len(params)
    for k, (W, b) in enumerate(params):
        z = h @ W.T + b
        if k < L - 1:
            cache.append(z)
            h = gelu(z)
            cache.append(h)
        else:
            h = z
    return h[:, 0], cache


def loss_and_grads(params, X, t, lo, hi):
    """MSE loss mean((y - t)^2) and its gradient for every W, b."""
    y, cache = forward(params, X, lo, hi)
    n = y.shape[0]
    loss = float(np.mean((y - t) ** 2))
    dy = (2.0 / n) * (y - t)[:, None]
    grads = [None] * len(params)
    L = len(params)
    g = dy
    for k in range(L - 1, -1, -1):
        W, b = params[k]
        hin = cache[0] if k == 0 else cache[2 * k]
        grads[k] = (g.T @ hin, g.sum(axis=0))
        if k > 0:
            z = cache[2 * k - 1]
            g = (g @ W) * gelu_grad(z)
    return loss, grads


def adam_step(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected). step counts from 1. Returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        res = []
        for P_, G_, M_, V_ in ((W, gW, mW, vW), (b, gb, mb, vb)):
            M2 = b1 * M_ + (1 - b1) * G_
            V2 = b2 * V_ + (1 - b2) * G_ * G_
            mh = M2 / (1 - b1 ** step)
            vh = V2 / (1 - b2 ** step)
            res.append((P_ - lr * mh / (np.sqrt(vh) + eps), M2, V2))
        out_p.append((res[0][0], res[1][0]))
        out_m.append((res[0][1], res[1][1]))
        out_v.append((res[0][2], res[1][2]))
    return out_p, out_m, out_v


def zeros_like(params):
    return [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
