"""GPU parity of the compressible Neo-Hookean path (config: log-normal shear
modulus field, finite strain) with the FP64 oracle: residual, CSR tangent,
matrix-free operator at the stored linearisation, diagonal, Newton stretch,
inverted-element detection, VJP with respect to the modulus scale."""
import numpy as np
import pytest

from helpers import lib_materials, oracle_phases, rel_err
from oracle import assembly, solver
from oracle.mesh import element_dofs
from oracle.rve import RVE
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu
TOL = {"f64": 1e-12, "f32": 1e-5}
SPEC = [("neohooke", 2.6, 0.3)]  # mu = 1, lam = 1.5 before the per-element scale


def _problem(n, prec, scale):
    import torch
    from paper_2604_22087_amd import fe
    P = fe.Problem(n, prec)
    models, params = lib_materials(SPEC)
    P.set_materials(torch.zeros(n ** 3, dtype=torch.uint8, device="cuda"), models, params,
                    torch.tensor(scale, dtype=P.dtype, device="cuda"))
    return P


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [6, 17])
def test_nh_residual_tangent_operator(n, prec):
    import torch
    print(f"[nh parity] n={n} prec={prec}", flush=True)
    scale = inputs.lognormal_field(n, seed=3)
    rve = RVE(n, np.zeros(n ** 3, dtype=int), oracle_phases(SPEC), scale=scale)
    amp = 0.3 / n
    u = (rve.coords @ np.array([[0.08, 0.02, 0.0], [0.0, -0.03, 0.01], [0.01, 0.0, 0.05]]).T).ravel() \
        + inputs.random_displacement(n, -amp, amp, seed=9)
    r_e, k_e, _ = rve.element_residual_tangent(u)
    R = assembly.assemble_vector(rve.conn, r_e, rve.n_dof)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    P = _problem(n, prec, scale)
    tol = TOL[prec]
    ut = torch.tensor(u, dtype=P.dtype, device="cuda")
    assert rel_err(_np(P.residual(ut, store_tangent=True)), R) <= tol
    assert P.read_flags() == 0
    x = np.random.default_rng(1).normal(size=rve.n_dof)
    xt = torch.tensor(x, dtype=P.dtype, device="cuda")
    assert rel_err(_np(P.apply_matfree(xt)), assembly.csr_matvec(rp, ci, v, x)) <= tol
    assert rel_err(_np(P.diagonal()), solver.matfree_diagonal(rve.conn, k_e, rve.n_dof)) <= tol
    assert rel_err(_np(P.tangent_csr(ut)), v) <= tol
    # VJP with respect to the modulus scale: lambda_e . r_e(u; s = 1)
    lam_v = np.random.default_rng(2).normal(size=rve.n_dof)
    r_hat, _, _ = RVE(n, np.zeros(n ** 3, dtype=int), oracle_phases(SPEC)).element_residual_tangent(u, want_tangent=False)
    vjp_ref = np.einsum("ei,ei->e", lam_v[element_dofs(rve.conn)], r_hat)
    got = _np(P.vjp(ut, torch.tensor(lam_v, dtype=P.dtype, device="cuda")))
    assert rel_err(got, vjp_ref) <= tol


def test_nh_newton_matches_oracle():
    import torch
    from paper_2604_22087_amd import fe
    n = 6
    scale = inputs.lognormal_field(n, seed=3)
    rve = RVE(n, np.zeros(n ** 3, dtype=int), oracle_phases(SPEC), scale=scale)
    path = [np.diag([0.02 * k, 0.0, 0.0]) for k in range(1, 6)]  # F_xx -> 1.1 in 5 steps
    u_ref, _, hist = rve.newton(path, newton_rtol=1e-11, pcg_rtol=1e-13)
    P = _problem(n, "f64", scale)
    P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
    u, _, sig, info = P.newton(path, op=fe.OP_MATFREE, newton_rtol=1e-11, pcg_rtol=1e-13)
    assert info["steps_done"] == 5
    assert rel_err(_np(u), u_ref) <= 1e-8
    for k, h in enumerate(hist):
        assert rel_err(sig[k], h["sigma_bar"]) <= 1e-8


def test_nh_inverted_element_flag():
    import torch
    n = 4
    P = _problem(n, "f64", np.ones(n ** 3))
    P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
    u = P.vector()
    P.lift(np.diag([-1.5, 0.0, 0.0]), u, zero_free=False)  # F_xx = -0.5 on boundary elements
    P.residual(u)
    assert P.read_flags() & 1
    assert P.read_flags() == 0  # reading clears


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_nh_with_linear_phase(prec):
    """A linear sphere inside a Neo-Hookean matrix (n = 9: node rows split into ragged tiles):
    residual, CSR tangent (plain and with the constrained dofs eliminated), matrix-free operator
    and diagonal against the oracle -- the tangent kernel's Neo-Hookean sets and its linear sets,
    the latter summed in closed form, in one assembly."""
    import torch
    from paper_2604_22087_amd import fe
    print(f"[nh + linear phase] prec={prec}", flush=True)
    n = 9
    spec = [("neohooke", 2.6, 0.3), ("linear", 70.0, 0.22)]
    phase = inputs.sphere_phase(n)
    rve = RVE(n, phase, oracle_phases(spec))
    amp = 0.3 / n
    u = (rve.coords @ np.array([[0.06, 0.01, 0.0], [0.0, -0.02, 0.01], [0.01, 0.0, 0.04]]).T).ravel() \
        + inputs.random_displacement(n, -amp, amp, seed=4)
    r_e, k_e, _ = rve.element_residual_tangent(u)
    R = assembly.assemble_vector(rve.conn, r_e, rve.n_dof)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    mask = inputs.boundary_dof_mask(n)
    P = fe.Problem(n, prec)
    models, params = lib_materials(spec)
    P.set_materials(torch.tensor(phase, dtype=torch.uint8, device="cuda"), models, params)
    P.set_dirichlet(torch.tensor(mask, device="cuda"))
    tol = TOL[prec]
    ut = torch.tensor(u, dtype=P.dtype, device="cuda")
    assert rel_err(_np(P.residual(ut, store_tangent=True)), R) <= tol
    assert rel_err(_np(P.tangent_csr(ut)), v) <= tol
    # eliminated: rows and columns of constrained dofs zero, unit diagonal there
    rows = assembly.csr_rows(rp)
    fixed = (mask[rows] != 0) | (mask[ci] != 0)
    v_bc = np.where(fixed, np.where(rows == ci, 1.0, 0.0), v)
    assert rel_err(_np(P.tangent_csr(ut, apply_bc=True)), v_bc) <= tol
    x = np.random.default_rng(5).normal(size=rve.n_dof)
    xt = torch.tensor(x, dtype=P.dtype, device="cuda")
    assert rel_err(_np(P.apply_matfree(xt)), assembly.csr_matvec(rp, ci, v, x)) <= tol
    assert rel_err(_np(P.diagonal()), solver.matfree_diagonal(rve.conn, k_e, rve.n_dof)) <= tol
