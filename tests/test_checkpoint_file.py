"""Load-step snapshot files (paper_2604_22087_amd.checkpoint) on the host: a snapshot written
and read back returns the same tensors, step, path and logs; a snapshot of another problem size
or precision, or a file of another kind, is rejected."""
import types

import numpy as np
import pytest
import torch

from paper_2604_22087_amd import checkpoint


def _fake(n_dof, n_el, dtype=torch.float64):
    return types.SimpleNamespace(n_dof=n_dof, n_el=n_el, dtype=dtype, device=torch.device("cpu"))


def test_snapshot_round_trip(tmp_path):
    P = _fake(81, 8)
    g = torch.Generator().manual_seed(0)
    u = torch.randn(81, dtype=torch.float64, generator=g)
    st = torch.randn(56 * 8, dtype=torch.float64, generator=g)
    up = torch.randn(81, dtype=torch.float64, generator=g)
    path = [np.diag([0.001 * k, 0, 0]) for k in range(1, 4)]
    f = str(tmp_path / "s.safetensors")
    checkpoint.save_snapshot(f, P, 1, path, u, st, up, [[1.0] * 6, [2.0] * 6], [(3, 0, 40), (2, 1, 30)],
                             {"predictor": 1})
    snap = checkpoint.load_snapshot(f, P)
    assert torch.equal(snap["u"], u) and torch.equal(snap["state"], st) and torch.equal(snap["u_prev"], up)
    assert snap["step"] == 1 and snap["sigma_bar"] == [[1.0] * 6, [2.0] * 6]
    assert snap["step_log"] == [[3, 0, 40], [2, 1, 30]] and snap["options"] == {"predictor": 1}
    assert np.array_equal(np.asarray(snap["load_path"]), np.asarray(path).reshape(-1, 9))
    # without state and u_prev
    checkpoint.save_snapshot(f, P, 0, path, u)
    snap = checkpoint.load_snapshot(f, P)
    assert snap["state"] is None and snap["u_prev"] is None and snap["step"] == 0


def test_snapshot_of_another_problem_is_rejected(tmp_path):
    f = str(tmp_path / "s.safetensors")
    checkpoint.save_snapshot(f, _fake(81, 8), 0, [np.eye(3)], torch.zeros(81, dtype=torch.float64))
    with pytest.raises(ValueError):
        checkpoint.load_snapshot(f, _fake(375, 64))
    with pytest.raises(ValueError):
        checkpoint.load_snapshot(f, _fake(81, 8, torch.float32))
    from safetensors.torch import save_file
    other = str(tmp_path / "o.safetensors")
    save_file({"u": torch.zeros(3)}, other, metadata={"snapshot": '{"format": "something else"}'})
    with pytest.raises(ValueError):
        checkpoint.load_snapshot(other, _fake(3, 1))


def test_resume_rejects_a_different_path(tmp_path):
    f = str(tmp_path / "s.safetensors")
    P = _fake(81, 8)
    path = [np.diag([0.001 * k, 0, 0]) for k in range(1, 4)]
    checkpoint.save_snapshot(f, P, 1, path, torch.zeros(81, dtype=torch.float64))
    other = [np.diag([0.002 * k, 0, 0]) for k in range(1, 4)]
    with pytest.raises(ValueError):
        checkpoint.newton_checkpointed(P, other, f, u=torch.zeros(81, dtype=torch.float64))
    with pytest.raises(ValueError):  # the path ends before the snapshot's step
        checkpoint.newton_checkpointed(P, path[:1], f, u=torch.zeros(81, dtype=torch.float64))
