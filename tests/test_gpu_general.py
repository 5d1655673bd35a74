"""GPU parity of the general-mesh path (fe_problem_create_hex8) with the FP64 oracle on
distorted, renumbered hex8 meshes of the unit cube whose elements carry randomly rotated
local node orders (inputs.distorted_cube_mesh), through the C ABI.

Bars (as for the structured path): CSR indices bit-exact against the oracle's sorted COO
assembly; residual, trial state, CSR values, K*u (matrix-free and CSR), diagonal and VJP
<= 1e-12 normwise relative in FP64 and <= 1e-5 in FP32; solves <= 1e-8 relative when both
sides solve to 1e-13.  Also: the general path on the structured mesh reproduces the
structured kernels, the CSR values are bit-identical from run to run (sorted gather, no
atomics), and malformed meshes are rejected before any solve.
"""
import numpy as np
import pytest

from helpers import PHASES_CONFIG1, PHASES_J2_FIBER, lib_materials, oracle_phases, rel_err, state_from_lib, state_to_lib
from oracle import assembly, solver
from oracle.mesh import structured_hex8
from oracle.rve import RVE, phase_params
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _mesh(n, seed=7):
    return inputs.distorted_cube_mesh(n, amplitude=0.25, seed=seed, permute=True)


def _problem(mesh, prec, phase, spec, scale=None):
    import torch
    from paper_2604_22087_amd import fe
    P = fe.Problem(precision=prec, mesh=mesh)
    models, params = lib_materials(spec)
    sc = None if scale is None else torch.tensor(scale, dtype=P.dtype, device="cuda")
    P.set_materials(torch.tensor(phase, dtype=torch.uint8, device="cuda"), models, params, sc)
    return P


def _t(P, a):
    import torch
    return torch.tensor(np.asarray(a), dtype=P.dtype, device="cuda")


def _np(t):
    return t.detach().double().cpu().numpy()


def _plastic_state(rve, seed):
    rng = np.random.default_rng(seed)
    st = rve.zero_state()
    ep = rng.normal(scale=2e-3, size=st["eps_p"].shape)
    ep[..., 2] = -ep[..., 0] - ep[..., 1]
    st["eps_p"] = ep * (rve.phase == 0)[:, None, None]
    st["alpha"] = rng.uniform(0, 2e-3, st["alpha"].shape) * (rve.phase == 0)[:, None]
    return st


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [5, 17])
def test_general_linear_operators(n, prec):
    import torch
    print(f"[general linear] n={n} prec={prec}", flush=True)
    coords, conn = _mesh(n)
    phase = inputs.sphere_phase_mesh(coords, conn)
    u = inputs.random_field_mesh(len(coords), seed=1)
    rve = RVE(None, phase, oracle_phases(PHASES_CONFIG1), mesh=(coords, conn))
    r_e, k_e, _ = rve.element_residual_tangent(u)
    R = assembly.assemble_vector(rve.conn, r_e, rve.n_dof)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)

    P = _problem((coords, conn), prec, phase, PHASES_CONFIG1)
    assert P.nnz == len(ci)
    tol = TOL[prec]
    ut = _t(P, u)
    assert rel_err(_np(P.residual(ut)), R) <= tol
    rp_g, ci_g = P.csr_indices()
    assert np.array_equal(rp_g.cpu().numpy().astype(np.int64), rp)
    assert np.array_equal(ci_g.cpu().numpy().astype(np.int64), ci)
    v_g = P.tangent_csr(ut)
    assert rel_err(_np(v_g), v) <= tol
    ku = assembly.csr_matvec(rp, ci, v, u)
    assert rel_err(_np(P.apply_matfree(ut)), ku) <= tol
    assert rel_err(_np(P.apply_csr(rp_g, ci_g, v_g, ut)), ku) <= tol
    assert rel_err(_np(P.apply_csr_nodal(rp_g, ci_g, v_g, ut)), ku) <= tol
    assert rel_err(_np(P.diagonal()), solver.matfree_diagonal(rve.conn, k_e, rve.n_dof)) <= tol

    mask = inputs.boundary_dof_mask_mesh(coords)
    assert np.array_equal(mask, rve.mask)
    P.set_dirichlet(torch.tensor(mask, device="cuda"))
    x = np.random.default_rng(5).normal(size=rve.n_dof)
    xt = _t(P, x)
    y_ref = solver.matfree_apply(rve.conn, k_e, x, mask)
    assert rel_err(_np(P.apply_matfree(xt, apply_bc=True)), y_ref) <= tol
    vb = assembly.dirichlet_csr(rp, ci, v, mask)
    vb_g = P.tangent_csr(ut, apply_bc=True)
    assert rel_err(_np(vb_g), vb) <= tol
    assert rel_err(_np(P.apply_csr(rp_g, ci_g, vb_g, xt)), y_ref) <= tol
    assert rel_err(_np(P.diagonal(apply_bc=True)), solver.matfree_diagonal(rve.conn, k_e, rve.n_dof, mask)) <= tol
    assert rel_err(_np(P.residual(ut, apply_bc=True)), R * (1 - mask)) <= tol
    # affine lift from the stored coordinates
    eb = np.array([[0.01, 0.002, 0.0], [0.002, -0.003, 0.001], [0.0, 0.001, 0.004]])
    ul = P.vector()
    P.lift(eb, ul)
    assert rel_err(_np(ul), rve.affine_lift(eb)) <= (1e-15 if prec == "f64" else 1e-7)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_general_j2_residual_state_tangent(prec):
    import torch
    n = 9
    print(f"[general j2] n={n} prec={prec}", flush=True)
    coords, conn = _mesh(n, seed=3)
    phase = inputs.sphere_phase_mesh(coords, conn)   # phase 0: J2 matrix, phase 1: linear
    rve = RVE(None, phase, oracle_phases(PHASES_J2_FIBER), mesh=(coords, conn))
    amp = 0.012 / n
    u = (coords @ np.diag([0.01, -0.01 / 3, 0.0]).T).ravel() + inputs.random_field_mesh(len(coords), -amp, amp, seed=7)
    st = _plastic_state(rve, 11)
    r_e, k_e, trial = rve.element_residual_tangent(u, st)
    frac = trial["plastic"][rve.phase == 0].mean()
    assert 0.2 < frac < 0.95
    R = assembly.assemble_vector(rve.conn, r_e, rve.n_dof)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)

    P = _problem((coords, conn), prec, phase, PHASES_J2_FIBER)
    tol = TOL[prec]
    ut = _t(P, u)
    s_in = _t(P, state_to_lib(st["eps_p"], st["alpha"]))
    s_out = P.state()
    r_g = P.residual(ut, s_in, s_out, store_tangent=True)
    assert rel_err(_np(r_g), R) <= tol
    ep_g, al_g = state_from_lib(_np(s_out), len(conn))
    assert rel_err(ep_g, trial["eps_p"]) <= (1e-11 if prec == "f64" else 1e-4)
    assert rel_err(al_g, trial["alpha"]) <= (1e-11 if prec == "f64" else 1e-4)
    if prec == "f64":
        assert int(np.sum((al_g > st["alpha"]) != trial["plastic"])) == 0
    x = np.random.default_rng(3).normal(size=rve.n_dof)
    xt = _t(P, x)
    assert rel_err(_np(P.apply_matfree(xt)), assembly.csr_matvec(rp, ci, v, x)) <= tol
    assert rel_err(_np(P.diagonal()), solver.matfree_diagonal(rve.conn, k_e, rve.n_dof)) <= tol
    v_g = P.tangent_csr(ut, s_in)
    assert rel_err(_np(v_g), v) <= tol
    # committing the trial state copies it bit for bit
    committed = P.state()
    P.commit_state(s_out, committed)
    assert torch.equal(committed, s_out)
    # mean stress: sum_q w detJ sigma / mesh volume
    sig = P.mean_stress(ut, s_in)
    assert rel_err(sig, rve.mean_stress(trial["sigma_all"])) <= (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_general_neohooke(prec):
    import torch
    n = 6
    print(f"[general neo-hookean] prec={prec}", flush=True)
    coords, conn = _mesh(n, seed=5)
    spec = [("neohooke", 2.6, 0.3), ("linear", 8.0, 0.25)]
    phase = inputs.sphere_phase_mesh(coords, conn)
    scale = inputs.uniform_field(len(conn), 0.5, 2.0, seed=9)
    rve = RVE(None, phase, oracle_phases(spec), scale=scale, mesh=(coords, conn))
    F = np.array([[0.08, 0.02, 0.0], [0.01, -0.03, 0.02], [0.0, 0.015, 0.05]])
    u = (coords @ F.T).ravel() + inputs.random_field_mesh(len(coords), -0.01 / n, 0.01 / n, seed=4)
    r_e, k_e, _ = rve.element_residual_tangent(u)
    R = assembly.assemble_vector(rve.conn, r_e, rve.n_dof)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    P = _problem((coords, conn), prec, phase, spec, scale)
    tol = TOL[prec]
    ut = _t(P, u)
    assert rel_err(_np(P.residual(ut, store_tangent=True)), R) <= tol
    x = np.random.default_rng(8).normal(size=rve.n_dof)
    assert rel_err(_np(P.apply_matfree(_t(P, x))), assembly.csr_matvec(rp, ci, v, x)) <= tol
    assert rel_err(_np(P.tangent_csr(ut)), v) <= tol
    assert rel_err(_np(P.diagonal()), solver.matfree_diagonal(rve.conn, k_e, rve.n_dof)) <= tol
    assert P.read_flags() == 0
    del torch


def test_general_vjp_matches_oracle():
    n = 7
    print("[general vjp]", flush=True)
    coords, conn = _mesh(n, seed=13)
    spec = [("linear", 1.0, 0.3)]
    E = inputs.uniform_field(len(conn), 1.0, 10.0, seed=4)
    phase = np.zeros(len(conn), dtype=np.uint8)
    rve1 = RVE(None, phase, oracle_phases(spec), mesh=(coords, conn))   # unit modulus: K_hat
    u = inputs.random_field_mesh(len(coords), seed=2)
    lam = inputs.random_field_mesh(len(coords), seed=3)
    _, k_hat, _ = rve1.element_residual_tangent(u)
    dofs = 3 * rve1.conn[:, :, None] + np.arange(3)[None, None, :]
    ue, le = u[dofs.reshape(len(conn), 24)], lam[dofs.reshape(len(conn), 24)]
    ref = np.einsum("ei,eij,ej->e", le, k_hat, ue)
    P = _problem((coords, conn), "f64", phase, spec, E)
    g = P.vjp(_t(P, u), _t(P, lam))
    assert rel_err(_np(g), ref) <= 1e-12


@pytest.mark.parametrize("op", ["matfree", "csr"])
def test_general_linear_solve(op):
    import torch
    from paper_2604_22087_amd import fe
    n = 17
    print(f"[general solve] op={op}", flush=True)
    coords, conn = _mesh(n, seed=21)
    phase = inputs.sphere_phase_mesh(coords, conn)
    rve = RVE(None, phase, oracle_phases(PHASES_CONFIG1), mesh=(coords, conn))
    eb = np.diag([0.01, 0.0, 0.0])
    u_ref, info = rve.solve_linear(eb, rtol=1e-13)
    assert info["status"] == solver.OK
    P = _problem((coords, conn), "f64", phase, PHASES_CONFIG1)
    P.set_dirichlet(torch.tensor(rve.mask, device="cuda"))
    u, _, sig, ninfo = P.newton([eb], op=fe.OP_MATFREE if op == "matfree" else fe.OP_CSR, pcg_rtol=1e-13)
    assert ninfo["status"] == 0
    assert rel_err(_np(u), u_ref) <= 1e-8
    print(f"  pcg iterations {ninfo['pcg_iterations']} (oracle {info['iterations']})", flush=True)
    assert abs(ninfo["pcg_iterations"] - info["iterations"]) <= max(3, info["iterations"] // 50)
    _, _, trial = rve.element_residual_tangent(u_ref)
    assert rel_err(sig[0], rve.mean_stress(trial["sigma_all"])) <= 1e-8


@pytest.mark.parametrize("solver_kind", ["bicgstab", "gmres"])
def test_general_other_krylov(solver_kind):
    import torch
    from paper_2604_22087_amd import fe
    n = 8
    print(f"[general {solver_kind}]", flush=True)
    coords, conn = _mesh(n, seed=17)
    phase = inputs.sphere_phase_mesh(coords, conn)
    rve = RVE(None, phase, oracle_phases(PHASES_CONFIG1), mesh=(coords, conn))
    eb = np.diag([0.01, 0.0, 0.0])
    u_ref, _ = rve.solve_linear(eb, rtol=1e-13)
    P = _problem((coords, conn), "f64", phase, PHASES_CONFIG1)
    P.set_dirichlet(torch.tensor(rve.mask, device="cuda"))
    kind = fe.SOLVER_BICGSTAB if solver_kind == "bicgstab" else fe.SOLVER_GMRES
    for pc in (fe.PC_JACOBI, fe.PC_BLOCK_JACOBI):
        P.set_preconditioner(pc)
        u, _, _, ninfo = P.newton([eb], op=fe.OP_MATFREE, pcg_rtol=1e-13, solver=kind, restart=40)
        assert ninfo["status"] == 0
        assert rel_err(_np(u), u_ref) <= 1e-8


def test_general_j2_newton_ramp():
    import torch
    from paper_2604_22087_amd import fe
    n = 5
    print("[general j2 newton]", flush=True)
    coords, conn = _mesh(n, seed=23)
    phase = inputs.sphere_phase_mesh(coords, conn)
    rve = RVE(None, phase, oracle_phases(PHASES_J2_FIBER), mesh=(coords, conn))
    path = [np.diag([0.006 * k, 0.0, 0.0]) for k in range(1, 5)]
    u_ref, st_ref, hist = rve.newton(path, newton_rtol=1e-11, pcg_rtol=1e-13)
    assert hist[-1]["plastic_fraction"] > 0.2
    P = _problem((coords, conn), "f64", phase, PHASES_J2_FIBER)
    P.set_dirichlet(torch.tensor(rve.mask, device="cuda"))
    for op in (fe.OP_MATFREE, fe.OP_CSR):
        state = P.state()
        u, state, sig, info = P.newton(path, state=state, op=op, newton_rtol=1e-11, pcg_rtol=1e-13,
                                       assemble_csr=True)
        assert info["steps_done"] == len(path)
        assert rel_err(_np(u), u_ref) <= 1e-8
        _, al_g = state_from_lib(_np(state), len(conn))
        assert rel_err(al_g, st_ref["alpha"]) <= 1e-7
        for k, h in enumerate(hist):
            assert rel_err(sig[k], h["sigma_bar"]) <= 1e-9


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_general_path_on_structured_mesh_equals_structured_kernels(prec):
    """The general kernels fed the structured mesh give the structured kernels' results."""
    import torch
    n = 12
    print(f"[general vs structured] prec={prec}", flush=True)
    coords, conn = structured_hex8(n)
    phase = inputs.fiber_phase(n, n_fibers=8, radius=0.1, seed=2)
    rng = np.random.default_rng(9)
    u = inputs.random_displacement(n, -2e-3, 2e-3, seed=6) + (coords @ np.diag([0.02, 0.0, 0.0]).T).ravel()
    Pg = _problem((coords, conn), prec, phase, PHASES_J2_FIBER)
    from paper_2604_22087_amd import fe
    Ps = fe.Problem(n, prec)
    models, params = lib_materials(PHASES_J2_FIBER)
    Ps.set_materials(torch.tensor(phase, dtype=torch.uint8, device="cuda"), models, params)
    tol = TOL[prec]
    outs = []
    for P in (Pg, Ps):
        ut = _t(P, u)
        s_out = P.state()
        r = P.residual(ut, None, s_out, store_tangent=True)
        x = _t(P, rng.normal(size=P.n_dof)) if not outs else outs[0][3]
        outs.append((_np(r), _np(s_out), _np(P.tangent_csr(ut)), x, _np(P.apply_matfree(x))))
    (rg, sg, vg, _, kg), (rs, ss, vs, _, ks) = outs
    assert rel_err(rg, rs) <= tol
    assert rel_err(sg, ss) <= tol
    assert rel_err(vg, vs) <= tol
    assert rel_err(kg, ks) <= tol
    rpg, cig = Pg.csr_indices()
    rps, cis = Ps.csr_indices()
    assert torch.equal(rpg, rps) and torch.equal(cig, cis)


def test_general_tangent_is_bit_reproducible():
    n = 10
    print("[general reproducible]", flush=True)
    coords, conn = _mesh(n, seed=29)
    phase = inputs.sphere_phase_mesh(coords, conn)
    P = _problem((coords, conn), "f64", phase, PHASES_J2_FIBER)
    u = _t(P, (coords @ np.diag([0.03, -0.01, 0.0]).T).ravel())
    import torch
    a = P.tangent_csr(u).clone()
    b = P.tangent_csr(u).clone()
    assert torch.equal(a, b)


def test_general_mesh_errors():
    import torch
    from paper_2604_22087_amd import fe
    print("[general errors]", flush=True)
    coords, conn = _mesh(3, seed=1)
    bad = conn.copy()
    bad[4, 2] = len(coords)  # node id out of range
    with pytest.raises(fe.FeError) as exc:
        fe.Problem(precision="f64", mesh=(coords, bad))
    assert exc.value.status == 1
    inv = conn.copy()
    inv[7] = inv[7][[4, 5, 6, 7, 0, 1, 2, 3]]  # top and bottom faces swapped: left-handed element
    with pytest.raises(fe.FeError) as exc:
        fe.Problem(precision="f64", mesh=(coords, inv))
    assert exc.value.status == 1
    P = fe.Problem(precision="f64", mesh=(coords, conn))
    with pytest.raises(fe.FeError):
        P.set_preconditioner(fe.PC_ILU0)
    W = torch.zeros(fe.MLP_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(fe.FeError):
        P.set_surrogate(W, 1e-3)
