"""GPU surrogate-network kernels against the FP64 oracle MLP on identical weights:
forward values and forward-mode Jacobian (FP32 matrix cores), weight gradients of
the mean squared error, one Adam step.  Bars: FP32 rounding of a 35,590-weight
network -- forward and Jacobian <= 1e-5 normwise, gradients <= 1e-4, Adam <= 1e-6."""
import numpy as np
import pytest

from helpers import rel_err
from oracle import mlp
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu


def to_lib(params):
    """Oracle (W (out,in), b) per layer -> flat float32 [Wt (in,out), b] per layer."""
    return np.concatenate([np.concatenate([W.T.ravel(), b]) for W, b in params]).astype(np.float32)


def from_lib(flat):
    out, off = [], 0
    for fi, fo in zip(mlp.LAYERS[:-1], mlp.LAYERS[1:]):
        Wt = flat[off:off + fi * fo].reshape(fi, fo)
        off += fi * fo
        b = flat[off:off + fo]
        off += fo
        out.append((Wt.T.astype(np.float64), b.astype(np.float64)))
    return out


def _params():
    p = inputs.glorot_uniform_params(seed=5)
    rng = np.random.default_rng(6)
    p = [(W, rng.normal(scale=0.1, size=b.shape)) for W, b in p]
    return from_lib(to_lib(p))  # exactly representable in float32


@pytest.mark.parametrize("n", [1, 37, 1000])
def test_forward_and_jacobian(n):
    import torch
    from paper_2604_22087_amd import fe
    p = _params()
    x = np.random.default_rng(n).normal(size=(n, 13)).astype(np.float32).astype(np.float64)
    W = torch.tensor(to_lib(p), device="cuda")
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    y, jac, cache = fe.mlp_forward(W, xt, jacobian=True, cache=True)
    y_ref, c_ref = mlp.forward(p, x)
    assert rel_err(y.double().cpu().numpy(), y_ref) <= 1e-5
    assert rel_err(jac.double().cpu().numpy(), mlp.jacobian(p, x)) <= 1e-5
    z = cache.double().cpu().numpy()
    for layer in range(3):
        assert rel_err(z[:, layer], c_ref["zs"][layer]) <= 1e-5
    y2, _, _ = fe.mlp_forward(W, xt)
    assert rel_err(y2.double().cpu().numpy(), y_ref) <= 1e-5


def test_backward_and_adam():
    import torch
    from paper_2604_22087_amd import fe
    p = _params()
    n = 500
    rng = np.random.default_rng(3)
    x = rng.normal(size=(n, 13)).astype(np.float32).astype(np.float64)
    t = rng.normal(size=(n, 6)).astype(np.float32).astype(np.float64)
    W = torch.tensor(to_lib(p), device="cuda")
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    y, _, cache = fe.mlp_forward(W, xt, cache=True)
    dW, loss = fe.mlp_backward(W, xt, cache, y, tt)
    y_ref, c_ref = mlp.forward(p, x)
    grads = mlp.backward(p, c_ref, y_ref, t)
    g_ref = to_lib([(gW, gb) for gW, gb in grads]).astype(np.float64)
    g_ref = np.concatenate([np.concatenate([gW.T.ravel(), gb]) for gW, gb in grads])
    assert rel_err(dW.double().cpu().numpy(), g_ref) <= 1e-4
    assert float(loss) == pytest.approx(mlp.mse_loss(y_ref, t), rel=1e-5)
    m = torch.zeros_like(W)
    v = torch.zeros_like(W)
    W0 = W.clone()
    fe.adam_step(W, dW, m, v, 1, lr=1e-3)
    gl = from_lib(dW.double().cpu().numpy())
    zero = [(np.zeros_like(a), np.zeros_like(b)) for a, b in p]
    new, _, _ = mlp.adam_step(from_lib(W0.double().cpu().numpy()), gl, zero, zero, 1, 1e-3)
    assert rel_err(W.double().cpu().numpy() - W0.double().cpu().numpy(), to_lib(new) - W0.double().cpu().numpy()) <= 1e-5
