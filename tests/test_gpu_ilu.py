"""Device preconditioners against the oracle: z = M^-1 r for point Jacobi, node-block
Jacobi and the 8-colour node-block ILU(0) (FP64 and FP32) on the config-1 CSR matrix;
GMRES, CG and BiCGStab with ILU(0) against the oracle's solvers with the oracle's ILU(0); Newton
ramps with GMRES + ILU(0) and CG + ILU(0) inner solves; the 64^3 plastic fiber RVE; and
the rejected combinations."""
import numpy as np
import pytest

from helpers import PHASES_CONFIG1, lib_materials, oracle_phases, rel_err
from oracle import assembly, ilu, solver
from oracle.rve import RVE
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu


def _config1(prec="f64"):
    import torch
    from paper_2604_22087_amd import fe
    n = 8
    phase = inputs.sphere_phase(n)
    rve = RVE(n, phase, oracle_phases(PHASES_CONFIG1))
    P = fe.Problem(n, prec)
    models, params = lib_materials(PHASES_CONFIG1)
    P.set_materials(torch.tensor(phase, device="cuda"), models, params)
    P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
    eb = np.diag([0.01, 0.0, 0.0])
    u0 = rve.affine_lift(eb)
    r_e, k_e, _ = rve.element_residual_tangent(u0)
    rhs = -assembly.assemble_vector(rve.conn, r_e, rve.n_dof) * rve.free
    u = P.vector()
    P.lift(eb, u, zero_free=True)
    b = P.residual(u, apply_bc=True, store_tangent=True)
    b.neg_()
    rp, ci = P.csr_indices()
    csr = (rp, ci, P.tangent_csr(u, apply_bc=True))
    return n, rve, k_e, rhs, P, b, csr


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_preconditioner_application_matches_oracle(prec):
    import torch
    from paper_2604_22087_amd import fe
    print(f"[pc apply] prec={prec}", flush=True)
    n, rve, k_e, rhs, P, b, csr = _config1(prec)
    rp, ci, v = rve.bc_csr(k_e)
    r = np.random.default_rng(3).normal(size=rve.n_dof)
    rt = torch.tensor(r, dtype=P.dtype, device="cuda")
    tol = 1e-12 if prec == "f64" else 2e-5
    want = {fe.PC_JACOBI: r / assembly.csr_diagonal(rp, ci, v),
            fe.PC_BLOCK_JACOBI: solver.block_jacobi(solver.matfree_node_blocks(rve.conn, k_e, rve.n_dof,
                                                                               rve.mask))(r),
            fe.PC_ILU0: ilu.bilu0_preconditioner(n, rp, ci, v)(r)}
    for kind, z_ref in want.items():
        P.set_preconditioner(kind)
        z = P.apply_preconditioner(rt, csr=csr).double().cpu().numpy()
        err = rel_err(z, z_ref)
        print(f"  kind {kind}: rel err {err:.2e}", flush=True)
        assert err <= tol
    assert P.read_flags() == 0


def test_gmres_ilu_matches_oracle():
    from paper_2604_22087_amd import fe
    n, rve, k_e, rhs, P, b, csr = _config1()
    rp, ci, v = rve.bc_csr(k_e)
    pre = ilu.bilu0_preconditioner(n, rp, ci, v)
    x_ref, it_ref, st, _ = solver.gmres(lambda x: assembly.csr_matvec(rp, ci, v, x), rhs, 1e-11, 2000, restart=30,
                                        precond=pre)
    assert st == solver.OK
    P.set_preconditioner(fe.PC_ILU0)
    x, res = P.pcg(b, op=fe.OP_CSR, csr=csr, rtol=1e-11, max_it=2000, solver=fe.SOLVER_GMRES, restart=30)
    P.set_preconditioner(fe.PC_JACOBI)
    _, res_j = P.pcg(b, op=fe.OP_CSR, csr=csr, rtol=1e-11, max_it=2000, solver=fe.SOLVER_GMRES, restart=30)
    print(f"  GMRES + ILU(0): iterations {res.iterations} (oracle {it_ref}; Jacobi {res_j.iterations})", flush=True)
    assert res.status == 0 and abs(res.iterations - it_ref) <= 2
    assert res.iterations < res_j.iterations
    assert rel_err(x.cpu().numpy(), x_ref) <= 1e-8
    # a longer restart reallocates the GMRES basis only; the ILU factors and the CG
    # workspaces stay valid for the solves that follow
    P.set_preconditioner(fe.PC_ILU0)
    for kw in (dict(solver=fe.SOLVER_GMRES, restart=50), dict(solver=fe.SOLVER_CG), dict(solver=fe.SOLVER_GMRES,
                                                                                           restart=64)):
        x2, r2 = P.pcg(b, op=fe.OP_CSR, csr=csr, rtol=1e-11, max_it=2000, **kw)
        assert r2.status == 0 and rel_err(x2.cpu().numpy(), x_ref) <= 1e-8


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cg_ilu_matches_oracle(prec):
    """CG with ILU(0) (symmetric operator, so M = L D L^T is symmetric) against the oracle's
    CG with the oracle's ILU(0): iteration count and solution."""
    from paper_2604_22087_amd import fe
    n, rve, k_e, rhs, P, b, csr = _config1(prec)
    rp, ci, v = rve.bc_csr(k_e)
    rtol = 1e-11 if prec == "f64" else 1e-5
    x_ref, it_ref, st, _ = solver.pcg(lambda x: assembly.csr_matvec(rp, ci, v, x), None, rhs, rtol, 2000,
                                      precond=ilu.bilu0_preconditioner(n, rp, ci, v))
    assert st == solver.OK
    P.set_preconditioner(fe.PC_ILU0)
    x, res = P.pcg(b, op=fe.OP_CSR, csr=csr, rtol=rtol, max_it=2000)
    print(f"  CG + ILU(0) {prec}: iterations {res.iterations} (oracle {it_ref})", flush=True)
    assert res.status == 0 and abs(res.iterations - it_ref) <= (1 if prec == "f64" else 3)
    assert rel_err(x.double().cpu().numpy(), x_ref) <= (1e-9 if prec == "f64" else 1e-4)


def test_bicgstab_ilu_nonsymmetric_matches_oracle():
    """BiCGStab with ILU(0) of a nonsymmetric matrix (the config-1 pattern with perturbed
    off-diagonal values) against the oracle's BiCGStab with the oracle's ILU(0), and fewer
    iterations than with Jacobi (Fig. 7's observation for BiCGStab)."""
    import torch
    from paper_2604_22087_amd import fe
    n, rve, k_e, rhs, P, b, csr = _config1()
    rp, ci, v = rve.bc_csr(k_e)
    rows = assembly.csr_rows(rp)
    rng = np.random.default_rng(12)
    free = (rve.mask[rows] == 0) & (rve.mask[ci] == 0) & (rows != ci)
    v = v.copy()
    v[free] += 0.05 * np.abs(v[free]) * rng.uniform(-1, 1, free.sum())
    bb = rng.normal(size=rve.n_dof) * rve.free
    matvec = lambda x: assembly.csr_matvec(rp, ci, v, x)
    x_ref, it_ref, st, _ = solver.bicgstab(matvec, bb, 1e-12, 2000, precond=ilu.bilu0_preconditioner(n, rp, ci, v))
    assert st == solver.OK
    csr_n = (torch.tensor(rp, dtype=torch.int32, device="cuda"), torch.tensor(ci, dtype=torch.int32, device="cuda"),
             torch.tensor(v, device="cuda"))
    bt = torch.tensor(bb, device="cuda")
    P.set_preconditioner(fe.PC_ILU0)
    x, res = P.pcg(bt, op=fe.OP_CSR, csr=csr_n, rtol=1e-12, max_it=2000, solver=fe.SOLVER_BICGSTAB)
    P.set_preconditioner(fe.PC_JACOBI)
    _, res_j = P.pcg(bt, op=fe.OP_CSR, csr=csr_n, rtol=1e-12, max_it=2000, solver=fe.SOLVER_BICGSTAB)
    print(f"  BiCGStab + ILU(0): iterations {res.iterations} (oracle {it_ref}; Jacobi {res_j.iterations})", flush=True)
    assert res.status == 0 and abs(res.iterations - it_ref) <= 2
    assert res.iterations < res_j.iterations
    assert rel_err(x.cpu().numpy(), x_ref) <= 1e-8


def test_ilu_singular_pivot_is_reported():
    """A zero diagonal block at an interior node makes its ILU(0) pivot singular: bit 2 of the
    flags is raised and GMRES ends with FE_ERR_NONFINITE instead of returning garbage."""
    import torch
    from paper_2604_22087_amd import fe
    n, rve, k_e, rhs, P, b, csr = _config1()
    rp, ci, v = (t.cpu().numpy() for t in csr)
    node = 4 + 9 * (4 + 9 * 4)  # the centre node of the 8^3 mesh (interior)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    blk = (rows // 3 == node) & (ci // 3 == node)
    v = v.copy()
    v[blk] = 0.0
    csr0 = (csr[0], csr[1], torch.tensor(v, device="cuda"))
    P.set_preconditioner(fe.PC_ILU0)
    assert P.read_flags() == 0
    _, res = P.pcg(b, op=fe.OP_CSR, csr=csr0, rtol=1e-10, max_it=100, check=False, solver=fe.SOLVER_GMRES)
    assert res.status == 6  # FE_ERR_NONFINITE
    assert P.read_flags() & 4


def test_ilu_rejected_combinations():
    import torch
    from paper_2604_22087_amd import fe
    n, rve, k_e, rhs, P, b, csr = _config1()
    P.set_preconditioner(fe.PC_ILU0)
    with pytest.raises(fe.FeError):
        P.pcg(b, op=fe.OP_MATFREE, solver=fe.SOLVER_BICGSTAB)  # no CSR values to factor
    with pytest.raises(fe.FeError):
        P.pcg(b, op=fe.OP_MATFREE)
    with pytest.raises(fe.FeError):
        P.pcg(b, op=fe.OP_MATFREE, solver=fe.SOLVER_GMRES)    # no CSR values to factor
    with pytest.raises(fe.FeError):
        P.apply_preconditioner(b)
    with pytest.raises(fe.FeError):
        P.set_preconditioner(3)


def test_newton_gmres_ilu_matches_cg():
    """J2 ramp: matrix-free operator, CSR tangent assembled each iteration for ILU(0),
    GMRES inner solves; same homogenised stress as the Jacobi-CG ramp."""
    import torch
    from paper_2604_22087_amd import fe
    n = 8
    phase = inputs.sphere_phase(n)
    models, params = lib_materials([("j2", 3.5, 0.35, 0.05, 0.1), ("linear", 70.0, 0.22)])
    out = {}
    for name, pc, solv in (("cg", fe.PC_JACOBI, fe.SOLVER_CG), ("gmres-ilu", fe.PC_ILU0, fe.SOLVER_GMRES),
                           ("cg-ilu", fe.PC_ILU0, fe.SOLVER_CG)):
        P = fe.Problem(n, "f64")
        P.set_materials(torch.tensor(phase, device="cuda"), models, params)
        P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
        P.set_preconditioner(pc)
        path = [np.diag([0.004 * k, 0.0, 0.0]) for k in range(1, 5)]
        _, _, sig, info = P.newton(path, state=P.state(), op=fe.OP_MATFREE, assemble_csr=True, newton_rtol=1e-10,
                                   pcg_rtol=1e-12, solver=solv, restart=30)
        out[name] = (np.array(sig), info)
        print(f"  {name}: {info}", flush=True)
        assert info["steps_done"] == len(path)
    for name in ("gmres-ilu", "cg-ilu"):
        assert out[name][1]["pcg_iterations"] < out["cg"][1]["pcg_iterations"]
        assert np.max(np.abs(out[name][0] - out["cg"][0])) <= 1e-9 * np.max(np.abs(out["cg"][0]))


def test_gmres_ilu_fiber64():
    """64^3 fiber RVE at a plastic linearisation, CSR operator: GMRES(30) with ILU(0)
    against Jacobi (iterations, time) and the true residual."""
    import time
    import torch
    from paper_2604_22087_amd import fe
    n = 64
    phase = inputs.fiber_phase(n, n_fibers=64, radius=0.05, seed=2)
    P = fe.Problem(n, "f64")
    P.set_materials(torch.tensor(phase, device="cuda"), [fe.J2, fe.LINEAR],
                    [(3.5, 0.35, 0.05, 0.1), (230.0, 0.2, 0.0, 0.0)])
    P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
    u = P.vector()
    P.lift(np.diag([0.004, 0.0, 0.0]), u, zero_free=False)
    b = P.residual(u, P.state(), P.state(), apply_bc=True, store_tangent=True)
    b.neg_()
    rp, ci = P.csr_indices()
    csr = (rp, ci, P.tangent_csr(u, P.state(), apply_bc=True))
    res = {}
    for name, pc in (("jacobi", fe.PC_JACOBI), ("block", fe.PC_BLOCK_JACOBI), ("ilu", fe.PC_ILU0)):
        P.set_preconditioner(pc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, r = P.pcg(b, op=fe.OP_CSR, csr=csr, rtol=1e-8, max_it=20000, solver=fe.SOLVER_GMRES, restart=30)
        torch.cuda.synchronize()
        res[name] = (r.iterations, time.perf_counter() - t0, x)
        true = float(torch.linalg.norm(b - P.apply_csr(*csr, x)) / torch.linalg.norm(b))
        print(f"  64^3 GMRES(30) {name}: {r.iterations} iterations, {res[name][1]:.3f} s, true residual {true:.2e}",
              flush=True)
        assert r.status == 0 and true <= 2e-8
    assert res["ilu"][0] < res["jacobi"][0]
    assert float(torch.linalg.norm(res["ilu"][2] - res["jacobi"][2]) / torch.linalg.norm(res["jacobi"][2])) <= 1e-5
    # CG: ILU(0) (unfused) against the fused matrix-free Jacobi-CG
    for name, pc, op in (("jacobi (fused, matrix-free)", fe.PC_JACOBI, fe.OP_MATFREE), ("ilu", fe.PC_ILU0, fe.OP_CSR)):
        P.set_preconditioner(pc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, r = P.pcg(b, op=op, csr=csr if op == fe.OP_CSR else None, rtol=1e-8, max_it=20000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        true = float(torch.linalg.norm(b - P.apply_csr(*csr, x)) / torch.linalg.norm(b))
        print(f"  64^3 CG {name}: {r.iterations} iterations, {dt:.3f} s, true residual {true:.2e}", flush=True)
        assert r.status == 0 and true <= 2e-8
