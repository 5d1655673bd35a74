"""FP32 problems with FP32 nodal sums (`fe_set_fp32_accumulation`) against the FP64 oracle,
beside the default FP32 problems whose element forces are summed at the nodes in FP64.

Both must meet the FP32 bar of the other parity tests (1e-5 normwise on the residual, the
matrix-free operator and the diagonal; a node sums at most 8 element contributions, so FP32
accumulation adds at most ~8 units of 6e-8 relative to the largest of them); the errors of the
two variants are printed side by side.  The CSR tangent is not affected by the switch (its
blocks are summed per lane in the problem's precision either way)."""
import numpy as np
import pytest

from helpers import PHASES_J2_FIBER, lib_materials, oracle_phases, rel_err, state_from_lib, state_to_lib
from oracle import assembly, solver
from oracle.rve import RVE
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu


def _setup(n):
    import torch
    from paper_2604_22087_amd import fe
    phase = inputs.fiber_phase(n, n_fibers=4, radius=0.18, seed=2)
    rve = RVE(n, phase, oracle_phases(PHASES_J2_FIBER))
    amp = 0.012 / n
    u = rve.affine_lift(np.diag([0.03, -0.01, 0.0])) + inputs.random_displacement(n, -amp, amp, seed=7)
    rng = np.random.default_rng(11)
    st = rve.zero_state()
    ep = rng.normal(scale=2e-3, size=st["eps_p"].shape)
    ep[..., 2] = -ep[..., 0] - ep[..., 1]
    st["eps_p"] = ep * (rve.phase == 0)[:, None, None]
    st["alpha"] = rng.uniform(0, 2e-3, st["alpha"].shape) * (rve.phase == 0)[:, None]
    P = fe.Problem(n, "f32")
    models, params = lib_materials(PHASES_J2_FIBER)
    P.set_materials(torch.tensor(phase, dtype=torch.uint8, device="cuda"), models, params)
    return rve, u, st, P


@pytest.mark.parametrize("n", [6, 17])
def test_fp32_accumulation_matches_oracle(n):
    import torch
    print(f"[fp32 accumulation] n={n}", flush=True)
    rve, u, st, P = _setup(n)
    r_e, k_e, trial = rve.element_residual_tangent(u, st)
    R = assembly.assemble_vector(rve.conn, r_e, rve.n_dof)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    x = np.random.default_rng(3).normal(size=rve.n_dof)
    mask = inputs.boundary_dof_mask(n)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda")
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    s_in = torch.tensor(state_to_lib(st["eps_p"], st["alpha"]), dtype=torch.float32, device="cuda")
    errs = {}
    for acc32 in (False, True):
        P.set_dirichlet(None)
        P.set_fp32_accumulation(acc32)
        r_g = P.residual(ut, s_in, P.state(), store_tangent=True)
        e = {"residual": rel_err(r_g.double().cpu().numpy(), R),
             "K*x": rel_err(P.apply_matfree(xt).double().cpu().numpy(), assembly.csr_matvec(rp, ci, v, x)),
             "diag": rel_err(P.diagonal().double().cpu().numpy(), solver.matfree_diagonal(rve.conn, k_e, rve.n_dof))}
        P.set_dirichlet(torch.tensor(mask, device="cuda"))
        e["K*x bc"] = rel_err(P.apply_matfree(xt, apply_bc=True).double().cpu().numpy(),
                              solver.matfree_apply(rve.conn, k_e, x, mask))
        errs["fp32 sums" if acc32 else "fp64 sums"] = e
        for k, val in e.items():
            assert val <= 1e-5, (acc32, k, val)
    for k in errs["fp64 sums"]:
        print(f"  {k:10s} fp64 sums {errs['fp64 sums'][k]:.2e}   fp32 sums {errs['fp32 sums'][k]:.2e}", flush=True)


def test_fp32_accumulation_rejected_on_fp64():
    from paper_2604_22087_amd import fe
    P = fe.Problem(4, "f64")
    with pytest.raises(fe.FeError):
        P.set_fp32_accumulation(True)
