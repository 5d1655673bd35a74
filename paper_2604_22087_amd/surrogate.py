"""Learned constitutive surrogate: sample generation and training driver.

Composition of library calls only: samples come from the library's own
return-map residual evaluations (fe_set_capture) along Newton load ramps of the
plastic RVE, and the network is trained by the library's forward, backward and
Adam kernels.  Shuffling and batching are index bookkeeping in torch.

Readings (training details are not in the paper): MSE on the normalised
stress, Adam (beta1 0.9, beta2 0.999, eps 1e-8) with a cosine-decayed learning
rate (2e-3 at the start, 300 epochs, batch 4096 for the shipped parameters),
Glorot-uniform initial weights from seed 5, 90/10 train/validation split.

`python -m paper_2604_22087_amd.surrogate` retrains on the GPU and writes
data/surrogate_j2.npy (+ .json summary).
"""
from __future__ import annotations

import math
import os

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
    capture_samples.last_count = int(count.item())  # points offered, including those past capacity
    m = min(capture_samples.last_count, capacity)
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


DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "surrogate_j2.npy")


def training_set(capacity=10_000_000):
    """Return-map samples of the fiber-RVE matrix material from the plastic-trial points of every
    Newton iterate of four ramps (32^3 uniaxial and shear to 0.03, 64^3 uniaxial and shear to
    0.02), thinned by one common hashed stride so that every ramp contributes in proportion:
    a counting pass gives the number of points offered, the stride is chosen for ~95 % of
    `capacity`, and the second pass captures."""
    p32, p64 = fiber_problem(32), fiber_problem(64)
    ramps = [(p32, ramp(0.03, 10)), (p32, ramp(0.03, 10, shear=True)), (p64, ramp(0.02, 10)),
             (p64, ramp(0.02, 10, shear=True))]
    capture_samples([(P, path, 1) for P, path in ramps], 1)
    offered = capture_samples.last_count
    stride = max(1, math.ceil(offered / (0.95 * capacity)))
    x, y = capture_samples([(P, path, stride) for P, path in ramps], capacity)
    training_set.offered, training_set.stride = offered, stride
    return x, y


def load_weights(path=DEFAULT_WEIGHTS):
    """Trained parameters as a float32 device tensor (None if the file is absent)."""
    if not os.path.exists(path):
        return None
    return torch.tensor(np.load(path).astype(np.float32), device="cuda")


def main(argv=None):
    """Train the surrogate on the GPU and write its parameters (.npy) and a summary (.json)."""
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--samples", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--batch", type=int, default=4096)
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    x, y = training_set(args.samples)
    t1 = time.perf_counter()
    W, hist = train(x, y, epochs=args.epochs, batch=args.batch, lr=args.lr,
                    log=lambda m: print(m, flush=True))
    t2 = time.perf_counter()
    err = relative_stress_error(W, x[:200000], y[:200000]).cpu().numpy()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, W.cpu().numpy())
    meta = dict(samples=int(x.shape[0]), samples_offered=training_set.offered, stride=training_set.stride,
                captured=capture_samples.last_count, epochs=args.epochs, lr=args.lr, batch=args.batch, seed=5,
                capture_seconds=t1 - t0, train_seconds=t2 - t1, final_train_loss=hist[-1]["train_loss"],
                final_val_loss=hist[-1]["val_loss"], rel_stress_err_median=float(np.median(err)),
                rel_stress_err_p99=float(np.percentile(err, 99)))
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
