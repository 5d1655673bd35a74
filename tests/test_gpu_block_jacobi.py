"""Node-block Jacobi PCG on the GPU against the oracle's block-Jacobi PCG.

Config-1 problem (8^3 two-phase sphere, linear) and a plastic J2 linearisation
(6^3 fiber RVE): iterates of CG are a deterministic function of the operator
and the preconditioner, so the GPU iteration count matches the oracle's
(within a few iterations of rounding drift) and the solutions agree to the
solve tolerance.  A wrong block (entry, symmetry or Dirichlet elimination)
changes the CG path and fails the iteration-count check.
"""
import numpy as np
import pytest

from helpers import PHASES_CONFIG1, PHASES_J2_FIBER, lib_materials, oracle_phases, rel_err, state_to_lib
from oracle import assembly, solver
from oracle.rve import RVE
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.parametrize("op", ["matfree", "csr"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_block_jacobi_config1(op, prec):
    import torch
    from paper_2604_22087_amd import fe
    n = 8
    print(f"[block jacobi config1] op={op} prec={prec}", flush=True)
    phase = inputs.sphere_phase(n)
    rve = RVE(n, phase, oracle_phases(PHASES_CONFIG1))
    eb = np.diag([0.01, 0.0, 0.0])
    u0 = rve.affine_lift(eb)
    r_e, k_e, _ = rve.element_residual_tangent(u0)
    rhs = -assembly.assemble_vector(rve.conn, r_e, rve.n_dof) * rve.free
    pre = solver.block_jacobi(solver.matfree_node_blocks(rve.conn, k_e, rve.n_dof, rve.mask))
    rtol = 1e-12 if prec == "f64" else 1e-5
    w_ref, it_ref, st_ref, _ = solver.pcg(lambda x: solver.matfree_apply(rve.conn, k_e, x, rve.mask), None, rhs,
                                          rtol, 5000, precond=pre)
    assert st_ref == solver.OK
    _, it_pj, _, _ = solver.pcg(lambda x: solver.matfree_apply(rve.conn, k_e, x, rve.mask),
                                solver.matfree_diagonal(rve.conn, k_e, rve.n_dof, rve.mask), rhs, rtol, 5000)

    P = fe.Problem(n, prec)
    models, params = lib_materials(PHASES_CONFIG1)
    P.set_materials(torch.tensor(phase, device="cuda"), models, params)
    P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
    P.set_preconditioner(fe.PC_BLOCK_JACOBI)
    u = P.vector()
    P.lift(eb, u, zero_free=True)
    b = P.residual(u, apply_bc=True, store_tangent=True)
    b.neg_()
    if op == "matfree":
        w, res = P.pcg(b, op=fe.OP_MATFREE, rtol=rtol, max_it=5000)
    else:
        rp, ci = P.csr_indices()
        vb = P.tangent_csr(u, apply_bc=True)
        w, res = P.pcg(b, op=fe.OP_CSR, csr=(rp, ci, vb), rtol=rtol, max_it=5000)
    assert res.status == 0
    assert abs(res.iterations - it_ref) <= (2 if prec == "f64" else 6)
    print(f"  iterations: block {res.iterations} (oracle {it_ref}), point Jacobi oracle {it_pj}", flush=True)
    tol = 1e-9 if prec == "f64" else 3e-4
    assert rel_err(_np(w), w_ref) <= tol
    assert P.read_flags() == 0
    # switching back gives point-Jacobi CG again
    P.set_preconditioner(fe.PC_JACOBI)
    _, res2 = P.pcg(b, op=fe.OP_MATFREE, rtol=rtol, max_it=5000)
    assert abs(res2.iterations - it_pj) <= (2 if prec == "f64" else 6)


def test_block_jacobi_j2_newton():
    """Plastic fiber RVE: a Newton ramp with block-Jacobi inner solves reaches the same
    converged fields as with point Jacobi (the preconditioner changes only the path of CG)."""
    import torch
    from paper_2604_22087_amd import fe
    n = 12
    phase = inputs.fiber_phase(n, n_fibers=4, radius=0.18, seed=2)
    path = [np.diag([0.004 * k, 0.0, 0.0]) for k in range(1, 4)]
    out = {}
    for kind in (fe.PC_JACOBI, fe.PC_BLOCK_JACOBI):
        P = fe.Problem(n, "f64")
        models, params = lib_materials(PHASES_J2_FIBER)
        P.set_materials(torch.tensor(phase, device="cuda"), models, params)
        P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
        P.set_preconditioner(kind)
        u, st, sig, info = P.newton(path, state=P.state(), op=fe.OP_MATFREE, newton_rtol=1e-10, pcg_rtol=1e-12)
        assert info["steps_done"] == 3
        out[kind] = (_np(u), np.array(sig), info)
    (u0, s0, i0), (u1, s1, i1) = out[fe.PC_JACOBI], out[fe.PC_BLOCK_JACOBI]
    print(f"  pcg iterations: point {i0['pcg_iterations']}, block {i1['pcg_iterations']}", flush=True)
    assert rel_err(u1, u0) <= 1e-8
    assert np.abs(s1 - s0).max() <= 1e-8 * np.abs(s0).max()
