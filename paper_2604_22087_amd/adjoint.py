"""Differentiable objectives with respect to a per-element modulus field.

`Compliance` (linear RVE, one load step) and `ReactionWorkPath` (plastic load
path with the history checkpointed per step, below).

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


class ReactionWorkPath(torch.autograd.Function):
    """Work of the boundary reactions after an incremental load path with J2 (and
    linear) phases, J = u_b . R(u_N; h_{N-1}, s), differentiable in the per-element
    modulus scale s (FP64 problems).

    Forward: one Newton solve per load step (fe_newton), keeping a checkpoint of the
    plastic history h_{n-1} before each step and of the converged u_n after it.
    Backward, from the last step to the first (discrete adjoint through the return map):
      K_n lambda_n = P_f (K_N u_b  at n = N;  d(mu_n . h_n)/du  otherwise)     (fe_pcg)
      c_n = [u_b at n = N] - lambda_n
      mu_{n-1} = d(c_n . R_n + mu_n . h_n)/d h_{n-1},  dJ/ds += d(same)/ds    (fe_vjp_path)
    with mu_N = 0.  K_n is the consistent tangent at the checkpoint (u_n, h_{n-1}).
    """

    @staticmethod
    def forward(ctx, s, problem, phase, models, params, mask, path, newton_rtol, pcg_rtol):
        P = problem
        if P.prec != fe.F64:
            raise ValueError("the path adjoint needs an FP64 problem")
        P.set_materials(phase, models, params, s.detach().contiguous())
        P.set_dirichlet(mask)
        u, state = P.vector(), P.state()
        us, hs, infos = [], [], []
        for eb in path:
            hs.append(state.clone())
            _, _, _, info = P.newton([np.asarray(eb)], u=u, state=state, op=fe.OP_MATFREE, newton_rtol=newton_rtol,
                                     pcg_rtol=pcg_rtol, max_newton=40)
            us.append(u.clone())
            infos.append(info)
        ub = u * mask.to(u.dtype)
        J = torch.dot(ub, P.residual(u, hs[-1]))
        ctx.problem, ctx.pcg_rtol, ctx.mask = P, pcg_rtol, mask
        ctx.us, ctx.hs, ctx.ub, ctx.infos = us, hs, ub, infos
        return J

    @staticmethod
    def backward(ctx, gJ):
        P, us, hs, ub = ctx.problem, ctx.us, ctx.hs, ctx.ub
        free = 1.0 - ctx.mask.to(ub.dtype)
        grad = torch.zeros(P.n_el, dtype=ub.dtype, device=ub.device)
        mu = None
        ctx.adjoint_iterations = []
        for n in reversed(range(len(us))):
            un, hn = us[n], hs[n]
            P.residual(un, hn, P.state(), apply_bc=True, store_tangent=True)   # K_n at the checkpoint
            if n == len(us) - 1:
                rhs = P.apply_matfree(ub, apply_bc=False)                      # K_N u_b
            else:
                rhs = P.vector()
                P.vjp_path(un, hn, mu_in=mu, u_bar=rhs)                        # d(mu_n . h_n)/du
            rhs *= free
            lam, res = P.pcg(rhs, op=fe.OP_MATFREE, rtol=ctx.pcg_rtol, max_it=200000)
            ctx.adjoint_iterations.append(res.iterations)
            c = (ub - lam) if n == len(us) - 1 else -lam
            mu = P.vjp_path(un, hn, c=c, mu_in=mu, s_bar=grad)
        return grad * gJ, None, None, None, None, None, None, None, None


def reaction_work_path(s, problem, phase, models, params, mask, path, newton_rtol=1e-12, pcg_rtol=1e-13):
    return ReactionWorkPath.apply(s, problem, phase, models, params, mask, path, newton_rtol, pcg_rtol)
