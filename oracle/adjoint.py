"""Adjoint sensitivities of a compliance objective to a per-element modulus field (oracle).

Differentiability through the solve is the paper's motivation (Sec. I); the
discrete adjoint here follows the Lagrangian L = J(u, E) + lambda_f^T R_f(u, E):
  adjoint equation   K_ff lambda_f = -dJ/du_f
  gradient           dJ/dE_e = dJ/dE_e|_u + lambda_f^T dR_f/dE_e.
With every element's moduli scaled by E_e (linear elasticity, fixed nu), the
element residual is r_e = E_e K_hat_e u_e, so dR/dE_e = A_e^T K_hat_e u_e and the
vector-Jacobian product is lambda_e^T K_hat_e u_e.

Objective under prescribed boundary displacements (macro strain): the work of
the reactions J = u_b^T R_b(u, E) = u^T K(E) u at equilibrium.  Then
dJ/du_f = K_fb u_b and the adjoint solution equals the forward one, lambda_f = u_f;
both routes give dJ/dE_e = u_e^T K_hat_e u_e.
"""
from __future__ import annotations

import numpy as np

from . import assembly
from .mesh import element_dofs


def unit_scale_residuals(rve, u):
    """Element residuals with every modulus scale set to 1: r_hat_e = K_hat_e u_e (linear)."""
    saved = rve.scale
    rve.scale = np.ones_like(saved)
    try:
        r_hat, _, _ = rve.element_residual_tangent(u, want_tangent=False)
    finally:
        rve.scale = saved
    return r_hat


def vjp_scale(rve, u, lam):
    """lambda_e^T dr_e/dE_e for every element."""
    return np.einsum("ei,ei->e", lam[element_dofs(rve.conn)], unit_scale_residuals(rve, u))


def reaction_objective(rve, u):
    """J = u_b . R_b(u)."""
    R, _ = rve.residual(u)
    return float(np.dot(u * rve.mask, R))


def adjoint_rhs(rve, u):
    """-dJ/du_f for J = u_b . R_b(u, E): -(K_fb u_b), zero on constrained dofs."""
    _, k_e, _ = rve.element_residual_tangent(u)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    return -assembly.csr_matvec(rp, ci, v, u * rve.mask) * rve.free


def gradient(rve, u, rtol=1e-13):
    """dJ/dE_e through the adjoint solve.  Returns (gradient, lambda_f)."""
    _, k_e, _ = rve.element_residual_tangent(u)
    lam, it, status, _ = rve.solve_update(k_e, adjoint_rhs(rve, u), rtol, 100000)
    if status != "ok":
        raise RuntimeError(f"adjoint solve failed: {status}")
    partial = vjp_scale(rve, u, u * rve.mask)        # dJ/dE_e at fixed u (boundary rows)
    return partial + vjp_scale(rve, u, lam), lam
