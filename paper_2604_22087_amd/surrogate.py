"""Learned constitutive surrogate: sample generation and training driver.

Composition of library calls only: samples come from the library's own
return-map residual evaluations (fe_set_capture) along Newton load ramps of the
plastic RVE, and the network is trained by the library's forward, backward and
Adam kernels.  Shuffling and batching are index bookkeeping in torch.

Readings (training details are not in the paper): MSE on the normalised
stress, Adam (beta1 0.9, beta2 0.999, eps 1e-8) with a cosine-decayed learning
rate from 1e-3, Glorot-uniform initial weights from seed 5, batch 8192, 90/10
train/validation split.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import fe, inputs

J2_MATRIX = (3.5, 0.35, 0.05, 0.1)
FIBER = (230.0, 0.2)
INCLUSION = (70.0, 0.22)


def to_lib_layout(params) -> np.ndarray:
    """[(W (out,in), b), ...] -> flat float32 parameters (input-major weights, then bias, per layer)."""
    return np.concatenate([np.concatenate([W.T.ravel(), b]) for W, b in params]).astype(np.float32)


def fiber_problem(n, seed=2, prec="f64"):
    phase = inputs.fiber_phase(n, n_fibers=64, radius=0.05, seed=seed)
    P = fe.Problem(n, prec)
    P.set_materials(torch.tensor(phase, device="cuda"), [fe.J2, fe.LINEAR], [J2_MATRIX, FIBER + (0.0, 0.0)])
    P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
    return P


def sphere_problem(n, prec="f64"):
    """Config-5 geometry: centred sphere r = 0.3 (linear inclusion) in the J2 matrix."""
    phase = inputs.sphere_phase(n)
    P = fe.Problem(n, prec)
    P.set_materials(torch.tensor(phase, device="cuda"), [fe.J2, fe.LINEAR], [J2_MATRIX, INCLUSION + (0.0, 0.0)])
    P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
    return P


def ramp(strain, steps, shear=False):
    out = []
    for k in range(1, steps + 1):
        e = np.zeros((3, 3))
        if shear:
            e[0, 1] = e[1, 0] = 0.5 * strain * k / steps
        else:
            e[0, 0] = strain * k / steps
        out.append(e)
    return out


def capture_samples(problems_and_paths, capacity, stride=1):
    """Run return-map Newton ramps with sample capture on.  Returns (x [m,13], y [m,6]) float32 tensors."""
    x = torch.empty(capacity, 13, dtype=torch.float32, device="cuda")
    y = torch.empty(capacity, 6, dtype=torch.float32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    for P, path, st in problems_and_paths:
        P.set_capture(x, y, count, stride=st if st else stride)
        P.newton(path, state=P.state(), op=fe.OP_MATFREE, newton_rtol=1e-8, pcg_rtol=1e-10, max_newton=30)
        P.set_capture(None)
    m = min(int(count.item()), capacity)
    return x[:m].contiguous(), y[:m].contiguous()


def train(x, y, epochs=20, batch=8192, lr=1e-3, seed=5, val_frac=0.1, log=None):
    """Train the 13-128-128-128-6 network on (x, y).  Returns (W, history)."""
    m = x.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(m, generator=g).to(x.device)
    n_val = int(val_frac * m)
    val_idx, tr_idx = perm[:n_val], perm[n_val:]
    xv, yv = x[val_idx].contiguous(), y[val_idx].contiguous()
    W = torch.tensor(to_lib_layout(inputs.glorot_uniform_params(seed=seed)), device=x.device)
    mom = torch.zeros_like(W)
    vel = torch.zeros_like(W)
    steps_per_epoch = max(1, len(tr_idx) // batch)
    total = epochs * steps_per_epoch
    t = 0
    hist = []
    for ep in range(epochs):
        order = tr_idx[torch.randperm(len(tr_idx), generator=g).to(x.device)]
        tr_loss = 0.0
        for b in range(steps_per_epoch):
            idx = order[b * batch:(b + 1) * batch]
            xb, yb = x[idx].contiguous(), y[idx].contiguous()
            out, _, cache = fe.mlp_forward(W, xb, cache=True)
            dW, loss = fe.mlp_backward(W, xb, cache, out, yb)
            t += 1
            lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * (t - 1) / total))
            fe.adam_step(W, dW, mom, vel, t, lr=lr_t)
            tr_loss += float(loss) if b == steps_per_epoch - 1 else 0.0
        yvp, _, _ = fe.mlp_forward(W, xv)
        val = float(torch.mean(torch.sum((yvp - yv) ** 2, dim=1)))
        hist.append(dict(epoch=ep, train_loss=tr_loss, val_loss=val))
        if log:
            log(f"epoch {ep}: train {tr_loss:.3e} val {val:.3e}")
    return W, hist


def relative_stress_error(W, x, y):
    """Per-sample |sigma_hat - sigma| / max(|sigma|, 1) in the normalised units (stress / sigma_y)."""
    yp, _, _ = fe.mlp_forward(W, x)
    err = torch.linalg.norm(yp - y, dim=1) / torch.clamp(torch.linalg.norm(y, dim=1), min=1.0)
    return err
