"""The allocation-free network backward (fe_mlp_backward_static, library-owned workspace)
against fe_mlp_backward with a caller workspace, through the C ABI: two calls in a row, the
second with fewer samples, plus the size limit."""
import numpy as np
import pytest
import torch

from paper_2604_22087_amd import fe

pytestmark = pytest.mark.gpu


def _batch(n, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(n, fe.MLP_IN, generator=g, device="cuda", dtype=torch.float32)
    t = torch.randn(n, fe.MLP_OUT, generator=g, device="cuda", dtype=torch.float32)
    return x, t


def _weights(seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    return 0.1 * torch.randn(fe.MLP_PARAMS, generator=g, device="cuda", dtype=torch.float32)


def test_static_backward_matches_workspace_backward():
    W = _weights(11)
    # a large batch first, then a smaller one: the second call must not see the first's rows
    for n, seed in ((fe.MLP_STATIC_MAX, 1), (777, 2)):
        x, t = _batch(n, seed)
        y, _, cache = fe.mlp_forward(W, x, cache=True)
        dW_ref, loss_ref = fe.mlp_backward(W, x, cache, y, t)
        dW, loss = fe.mlp_backward_static(W, x, cache, y, t)
        torch.cuda.synchronize()
        print(f"[no-alloc] n={n} seed={seed}", flush=True)
        a, b = dW.double().cpu().numpy(), dW_ref.double().cpu().numpy()
        # identical products; only the order of the FP32 atomic sums over batch chunks differs
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)
        assert float(loss) == pytest.approx(float(loss_ref), rel=1e-12)


def test_static_backward_rejects_oversized_batch():
    W = _weights(3)
    n = fe.MLP_STATIC_MAX + 1
    x, t = _batch(n, 4)
    y, _, cache = fe.mlp_forward(W, x, cache=True)
    with pytest.raises(fe.FeError) as exc:
        fe.mlp_backward_static(W, x, cache, y, t)
    assert exc.value.status == 1
