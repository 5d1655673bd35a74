"""Multilayer perceptron for the learned constitutive surrogate (oracle, FP64).

The paper notes that a surrogate stress-strain model can replace the designed
material function, with its Jacobian obtained the same way (Sec. III-B).  The
network: dense layers 13 -> 128 -> 128 -> 128 -> 6, SiLU (z * sigmoid(z)) after
each hidden layer, linear output.  Weights are W_l (out, in) and b_l (out,).
  forward:   h_0 = x, z_l = W_l h_{l-1} + b_l, h_l = silu(z_l) (hidden), y = z_L
  Jacobian:  forward-mode tangents t_0 = e_j, t_l = silu'(z_l) * (W_l t_{l-1}), dy/dx_j = W_L t_{L-1}
  backward:  reverse-mode for the mean-squared error (Rumelhart et al. 1986)
  Adam:      Kingma & Ba 2015, bias-corrected first and second moments.
"""
from __future__ import annotations

import numpy as np

LAYERS = (13, 128, 128, 128, 6)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_prime(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params, x):
    """params: list of (W, b).  x (m, 13) -> (y (m, 6), cache of pre-activations)."""
    h = x
    zs = []
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        zs.append(z)
        h = z if li == len(params) - 1 else silu(z)
    return h, dict(x=x, zs=zs)


def jacobian(params, x, cols=range(6)):
    """dy/dx[:, cols] by forward-mode tangents: (m, 6, len(cols))."""
    _, cache = forward(params, x)
    m = x.shape[0]
    cols = list(cols)
    t = np.zeros((m, x.shape[1], len(cols)))
    for k, j in enumerate(cols):
        t[:, j, k] = 1.0
    for li, (W, _) in enumerate(params):
        t = np.einsum("oi,mik->mok", W, t)
        if li < len(params) - 1:
            t = silu_prime(cache["zs"][li])[:, :, None] * t
    return t


def mse_loss(y, target):
    return float(np.mean(np.sum((y - target) ** 2, axis=1)))


def backward(params, cache, y, target):
    """Gradients of mse_loss (mean over rows of the squared error sum) w.r.t. (W, b) per layer."""
    m = y.shape[0]
    g = 2.0 * (y - target) / m                     # dL/dy
    grads = [None] * len(params)
    zs = cache["zs"]
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h_prev = cache["x"] if li == 0 else silu(zs[li - 1])
        grads[li] = (g.T @ h_prev, g.sum(axis=0))
        if li > 0:
            g = (g @ W) * silu_prime(zs[li - 1])
    return grads


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  m, v: moment lists shaped like params. Returns new lists."""
    new_p, new_m, new_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out_p, out_m, out_v = [], [], []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = beta1 * mm + (1 - beta1) * g
            vv = beta2 * vv + (1 - beta2) * g * g
            mhat = mm / (1 - beta1 ** t)
            vhat = vv / (1 - beta2 ** t)
            out_p.append(p - lr * mhat / (np.sqrt(vhat) + eps))
            out_m.append(mm)
            out_v.append(vv)
        new_p.append(tuple(out_p))
        new_m.append(tuple(out_m))
        new_v.append(tuple(out_v))
    return new_p, new_m, new_v
