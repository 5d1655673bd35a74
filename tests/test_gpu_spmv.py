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
