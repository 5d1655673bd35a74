"""Node-structured CSR mat-vec against the general CSR mat-vec and the oracle."""
import numpy as np
import pytest

from helpers import PHASES_CONFIG1, lib_materials, oracle_phases, rel_err
from oracle import assembly
from oracle.rve import RVE
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [5, 17])
def test_nodal_spmv(n, prec):
    import torch
    from paper_2604_22087_amd import fe
    phase = inputs.sphere_phase(n)
    rve = RVE(n, phase, oracle_phases(PHASES_CONFIG1))
    u = inputs.random_displacement(n, seed=1)
    _, k_e, _ = rve.element_residual_tangent(u)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    x = np.random.default_rng(2).normal(size=rve.n_dof)
    y_ref = assembly.csr_matvec(rp, ci, v, x)
    P = fe.Problem(n, prec)
    models, params = lib_materials(PHASES_CONFIG1)
    P.set_materials(torch.tensor(phase, device="cuda"), models, params)
    rpg, cig = P.csr_indices()
    vals = P.tangent_csr(torch.tensor(u, dtype=P.dtype, device="cuda"))
    xg = torch.tensor(x, dtype=P.dtype, device="cuda")
    y1 = P.apply_csr(rpg, cig, vals, xg).double().cpu().numpy()
    y2 = P.apply_csr_nodal(rpg, cig, vals, xg).double().cpu().numpy()
    tol = 1e-13 if prec == "f64" else 1e-5
    assert rel_err(y2, y_ref) <= tol
    assert rel_err(y2, y1) <= tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_general_spmv_arbitrary_rows(prec):
    """fe_apply_csr on a matrix that is not a mesh pattern: random row lengths 0..100 (empty rows,
    single entries, lengths on both sides of the kernel's two-step batches), random columns,
    against the oracle's CSR mat-vec."""
    import torch
    from paper_2604_22087_amd import fe
    print(f"[general spmv arbitrary rows] {prec}", flush=True)
    P = fe.Problem(5, prec)
    rng = np.random.default_rng(7)
    lens = rng.integers(0, 101, size=P.n_dof)
    lens[:40] = np.arange(40)  # every short length, 0 .. 39, at least once
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = rng.integers(0, P.n_dof, size=int(rp[-1])).astype(np.int32)
    v = rng.normal(size=int(rp[-1]))
    x = rng.normal(size=P.n_dof)
    y_ref = assembly.csr_matvec(rp, ci, v, x)
    y = P.apply_csr(torch.tensor(rp, device="cuda"), torch.tensor(ci, device="cuda"),
                    torch.tensor(v, dtype=P.dtype, device="cuda"), torch.tensor(x, dtype=P.dtype, device="cuda"))
    y = y.double().cpu().numpy()
    assert np.all(y[lens == 0] == 0)
    assert rel_err(y, y_ref) <= (1e-13 if prec == "f64" else 1e-5)
