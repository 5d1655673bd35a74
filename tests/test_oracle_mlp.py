"""Pins of the oracle MLP: SiLU values, the zero-weight closed form, finite
differences of the input Jacobian and of the weight gradients, and the closed
form of Adam's first step (|step| = lr for every weight with non-zero gradient)."""
import numpy as np
import pytest

from oracle import mlp
from paper_2604_22087_amd import inputs

RNG = np.random.default_rng(8)


def _params(scale=1.0, seed=5):
    p = inputs.glorot_uniform_params(seed=seed)
    rng = np.random.default_rng(seed + 1)
    return [(W * scale, rng.normal(scale=0.1, size=b.shape)) for W, b in p]


def test_silu_values():
    assert mlp.silu(np.array([0.0]))[0] == 0.0
    assert mlp.silu_prime(np.array([0.0]))[0] == 0.5
    z = np.array([1.0, -2.0])
    assert np.allclose(mlp.silu(z), z / (1 + np.exp(-z)), rtol=1e-15)
    h = 1e-6
    assert np.allclose((mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), mlp.silu_prime(z), rtol=1e-8)


def test_zero_weights_give_constant_output():
    p = _params()
    p = [(np.zeros_like(W), b) for W, b in p[:3]] + [p[3]]
    x = RNG.normal(size=(4, 13))
    y, _ = mlp.forward(p, x)
    b3 = p[2][1]
    expect = p[3][0] @ (b3 / (1 + np.exp(-b3))) + p[3][1]
    assert np.abs(y - expect[None]).max() < 1e-15


def test_glorot_bounds():
    p = inputs.glorot_uniform_params(seed=5)
    assert [W.shape for W, _ in p] == [(128, 13), (128, 128), (128, 128), (6, 128)]
    for W, b in p:
        a = np.sqrt(6.0 / sum(W.shape))
        assert np.abs(W).max() <= a and np.abs(W).max() > 0.9 * a and not b.any()


def test_jacobian_matches_finite_differences():
    p = _params()
    x = RNG.normal(size=(5, 13))
    Jac = mlp.jacobian(p, x)
    h = 1e-6
    for j in range(6):
        d = np.zeros(13)
        d[j] = h
        fd = (mlp.forward(p, x + d)[0] - mlp.forward(p, x - d)[0]) / (2 * h)
        assert np.abs(fd - Jac[:, :, j]).max() < 1e-8


def test_weight_gradients_match_finite_differences():
    p = _params()
    x = RNG.normal(size=(7, 13))
    t = RNG.normal(size=(7, 6))
    y, cache = mlp.forward(p, x)
    grads = mlp.backward(p, cache, y, t)
    h = 1e-6
    for li, which, idx in ((0, 0, (3, 5)), (1, 0, (10, 20)), (2, 1, (7,)), (3, 0, (2, 100)), (3, 1, (4,))):
        def loss_with(delta):
            q = [list(pp) for pp in p]
            arr = q[li][which].copy()
            arr[idx] += delta
            q[li][which] = arr
            return mlp.mse_loss(mlp.forward([tuple(pp) for pp in q], x)[0], t)
        fd = (loss_with(h) - loss_with(-h)) / (2 * h)
        assert fd == pytest.approx(grads[li][which][idx], rel=1e-6, abs=1e-10)


def test_adam_first_step_closed_form():
    p = _params()
    g = [(RNG.normal(size=W.shape), RNG.normal(size=b.shape)) for W, b in p]
    z = [(np.zeros_like(W), np.zeros_like(b)) for W, b in p]
    lr = 1e-3
    new, m, v = mlp.adam_step(p, g, z, z, 1, lr)
    for (W, b), (W2, b2), (gW, gb) in zip(p, new, g):
        # first step: m_hat = g, v_hat = g^2 -> delta = -lr g / (|g| + eps)
        assert np.allclose(W2 - W, -lr * gW / (np.abs(gW) + 1e-8), rtol=1e-12, atol=1e-18)
        assert np.allclose(b2 - b, -lr * gb / (np.abs(gb) + 1e-8), rtol=1e-12, atol=1e-18)
