"""Differentiable compliance of a linear RVE with respect to a per-element modulus field.

torch.autograd.Function around the library: the forward pass solves the
displacement-driven RVE (fe_newton, one linear load step), the backward pass
solves the adjoint system with the same Jacobi-PCG (fe_pcg) and contracts it
with the residual's modulus derivative (fe_vjp).  Objective: the work of the
boundary reactions J = u_b . R_b(u, E) (= u^T K u at equilibrium), whose
adjoint right-hand side is -P_f K u_b.  Only marshalling and sign/mask glue run
in torch; every finite-element operation runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import fe


class Compliance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, problem, phase, mask, eps_bar, rtol):
        P = problem
        P.set_materials(phase, [fe.LINEAR], [(1.0, 0.3)], E.detach().contiguous())
        P.set_dirichlet(mask)
        u, _, _, info = P.newton([np.asarray(eps_bar)], op=fe.OP_MATFREE, pcg_rtol=rtol, newton_rtol=1e-12)
        ub = u * mask.to(u.dtype)
        R = P.residual(u)                       # R(u): reactions on constrained dofs, ~0 elsewhere
        J = torch.dot(ub, R)
        ctx.save_for_backward(u, ub)
        ctx.problem, ctx.rtol = P, rtol
        ctx.info = info
        return J

    @staticmethod
    def backward(ctx, gJ):
        u, ub = ctx.saved_tensors
        P = ctx.problem
        rhs = P.residual(ub, apply_bc=True)     # P_f K u_b (linear: R(u_b) = K u_b)
        rhs.neg_()
        lam, res = P.pcg(rhs, op=fe.OP_MATFREE, rtol=ctx.rtol, max_it=200000)
        ctx.adjoint_iterations = res.iterations
        g = P.vjp(u, ub + lam)                  # dJ/dE_e|_u + lambda_f . dR_f/dE_e
        return g * gJ, None, None, None, None, None


def compliance(E, problem, phase, mask, eps_bar=np.diag([0.01, 0.0, 0.0]), rtol=1e-13):
    return Compliance.apply(E, problem, phase, mask, eps_bar, rtol)
