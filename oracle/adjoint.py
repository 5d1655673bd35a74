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


# ---- path-dependent (J2) load paths ---------------------------------------------------
# For an incremental plastic load path the objective is the work of the boundary
# reactions at the last step, J = u_b . R_b(u_N; h_{N-1}, s), where h_{N-1} is the
# plastic history committed after step N-1 and s the per-element modulus scale
# (the elastic moduli of every phase are multiplied by s_e; sigma_y and H are not).
# Its gradient is taken here by the complex step: every quantity of the path is
# analytic in s away from yield-state switches, so with s_e -> s_e + i h,
# dJ/ds_e = Im J / h exactly up to rounding (Squire & Trapp 1998; Martins, Sturdza
# & Alonso 2003), with no subtraction and no derivative code of its own.


def dense_operator(rve, k_e):
    """A = P_f K P_f + P_b as a dense matrix (small meshes only)."""
    dofs = element_dofs(rve.conn)
    a = np.zeros((rve.n_dof, rve.n_dof), dtype=k_e.dtype)
    np.add.at(a, (dofs[:, :, None], dofs[:, None, :]), k_e)
    f = rve.free
    a = a * f[:, None] * f[None, :]
    a[np.arange(rve.n_dof), np.arange(rve.n_dof)] += rve.mask
    return a


def path_reaction_work(rve, path, newton_rtol=1e-13, max_newton=40, extra=2):
    """J = u_b . R(u_N; h_{N-1}) along the load path (full Newton steps, dense solves).

    Works for real or complex scale fields.  After the real parts have converged,
    `extra` further Newton steps settle the complex-step part.  Returns (J, u_N)."""
    cplx = np.iscomplexobj(rve.scale)
    u = np.zeros(rve.n_dof, dtype=complex if cplx else float)
    state = rve.zero_state()
    for eps_bar in path:
        u = u * rve.free + rve.affine_lift(eps_bar)
        r0, left = None, None
        for it in range(max_newton + 1):
            r_e, k_e, trial = rve.element_residual_tangent(u, state)
            rf = assembly.assemble_vector(rve.conn, r_e, rve.n_dof) * rve.free
            rn = np.linalg.norm(np.real(rf))
            r0 = rn if r0 is None else r0
            if left is None and (rn <= newton_rtol * r0 or rn == 0.0):
                left = extra if cplx else 0
            if left is not None:
                if left == 0:
                    break
                left -= 1
            if it == max_newton:
                raise RuntimeError("Newton did not converge")
            u = u + np.linalg.solve(dense_operator(rve, k_e), -rf)
        state = dict(eps_p=trial["eps_p"], alpha=trial["alpha"])
    R = assembly.assemble_vector(rve.conn, r_e, rve.n_dof)
    return np.dot(u * rve.mask, R), u


def path_gradient_complex_step(rve, path, elements=None, h=1e-30, **kw):
    """dJ/ds_e for the listed elements (default all) by the complex step."""
    elements = np.arange(len(rve.conn)) if elements is None else np.asarray(elements)
    s0 = np.asarray(rve.scale, dtype=np.float64)
    g = np.zeros(len(elements))
    try:
        for k, e in enumerate(elements):
            sc = s0.astype(complex)
            sc[e] += 1j * h
            rve.scale = sc
            g[k] = np.imag(path_reaction_work(rve, path, **kw)[0]) / h
    finally:
        rve.scale = s0
    return g
