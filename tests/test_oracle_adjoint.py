"""Pins of the oracle's adjoint gradient (per-element modulus field, compliance).

Expected values: the adjoint solution equals the forward interior displacement
(closed form for the reaction-work objective), the gradient equals
u_e^T K_hat_e u_e, Euler's theorem for the degree-1 homogeneous objective
(sum_e E_e dJ/dE_e = J), positivity, and central finite differences of the
objective re-solved to 1e-13."""
import numpy as np
import pytest

from oracle import adjoint, assembly
from oracle.rve import RVE, phase_params
from paper_2604_22087_amd import inputs


def _rve(n, E):
    return RVE(n, np.zeros(n ** 3, dtype=int), [phase_params("linear", 1.0, 0.3)], scale=E)


def _solve(rve, exx=0.01):
    u, info = rve.solve_linear(np.diag([exx, 0, 0]), rtol=1e-14)
    assert info["status"] == "ok"
    return u


def test_adjoint_equals_forward_and_euler_identity():
    n = 4
    E = inputs.uniform_field(n ** 3, 1.0, 10.0, seed=4)
    rve = _rve(n, E)
    u = _solve(rve)
    g, lam = adjoint.gradient(rve, u)
    assert np.linalg.norm(lam - u * rve.free) <= 1e-10 * np.linalg.norm(u * rve.free)
    J = adjoint.reaction_objective(rve, u)
    # energy form u.K u equals the reaction work at equilibrium
    r_e, k_e, _ = rve.element_residual_tangent(u)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    assert u @ assembly.csr_matvec(rp, ci, v, u) == pytest.approx(J, rel=1e-12)
    assert np.dot(E, g) == pytest.approx(J, rel=1e-11)
    assert np.all(g > 0)
    g_direct = adjoint.vjp_scale(rve, u, u)
    assert np.linalg.norm(g - g_direct) <= 1e-10 * np.linalg.norm(g)


def test_gradient_matches_central_differences():
    n = 3
    E = inputs.uniform_field(n ** 3, 1.0, 10.0, seed=4)
    rve = _rve(n, E)
    g, _ = adjoint.gradient(rve, _solve(rve))
    h = 1e-4
    for k in (0, 5, 13, 26):
        Jp, Jm = [], []
        for sgn, out in ((1, Jp), (-1, Jm)):
            Ek = E.copy()
            Ek[k] += sgn * h
            r2 = _rve(n, Ek)
            u2 = _solve(r2)
            out.append(adjoint.reaction_objective(r2, u2))
        fd = (Jp[0] - Jm[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-7)
