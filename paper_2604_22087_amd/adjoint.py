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

import functools

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
        # the Problem may be given other materials or constraints before backward runs
        # (e.g. a sum of objectives over several fields): keep the forward's own
        ctx.field = (E.detach().clone(), phase, mask)
        ctx.info = info
        return J

    @staticmethod
    def backward(ctx, gJ):
        u, ub = ctx.saved_tensors
        P = ctx.problem
        E, phase, mask = ctx.field
        P.set_materials(phase, [fe.LINEAR], [(1.0, 0.3)], E)
        P.set_dirichlet(mask)
        rhs = P.residual(ub, apply_bc=True)     # P_f K u_b (linear: R(u_b) = K u_b)
        rhs.neg_()
        lam, res = P.pcg(rhs, op=fe.OP_MATFREE, rtol=ctx.rtol, max_it=200000)
        ctx.adjoint_iterations = res.iterations
        g = P.vjp(u, ub + lam)                  # dJ/dE_e|_u + lambda_f . dR_f/dE_e
        return g * gJ, None, None, None, None, None


def compliance(E, problem, phase, mask, eps_bar=np.diag([0.01, 0.0, 0.0]), rtol=1e-13):
    return Compliance.apply(E, problem, phase, mask, eps_bar, rtol)


@functools.lru_cache(maxsize=None)
def _revolve(steps, slots):
    """(forward load-step solves, first split) of the cheapest recursive reversal of `steps`
    steps when the state before the first is held and at most `slots` more states may be
    held at once (binomial checkpointing, Griewank & Walther, ACM TOMS 26, 2000).
    Reversing one step from the state before it costs one solve (the step is re-run to
    recover u_n); with no free slot the steps are reversed by re-running from the start;
    otherwise advance k steps, keep that state, reverse the last steps - k with one slot
    fewer, then the first k with the same slots."""
    if steps == 1:
        return 1, 0
    if slots == 0:
        return steps * (steps + 1) // 2, 0
    return min((k + _revolve(steps - k, slots - 1)[0] + _revolve(k, slots)[0], k) for k in range(1, steps))


def revolve_cost(steps, slots):
    """Forward load-step solves spent by the backward sweep with `slots` checkpoints."""
    return _revolve(int(steps), int(slots))[0]


class ReactionWorkPath(torch.autograd.Function):
    """Work of the boundary reactions after an incremental load path with J2 (and
    linear) phases, J = u_b . R(u_N; h_{N-1}, s), differentiable in the per-element
    modulus scale s (FP64 problems).

    Forward: one Newton solve per load step (fe_newton).  With checkpoints=None every
    step keeps the plastic history h_{n-1} before it and the converged u_n after it;
    with checkpoints=c only the initial state is kept and the backward sweep re-runs
    steps from at most c + 1 held states at a time (binomial schedule, see _revolve).
    Backward, from the last step to the first (discrete adjoint through the return map):
      K_n lambda_n = P_f (K_N u_b  at n = N;  d(mu_n . h_n)/du  otherwise)     (fe_pcg)
      c_n = [u_b at n = N] - lambda_n
      mu_{n-1} = d(c_n . R_n + mu_n . h_n)/d h_{n-1},  dJ/ds += d(same)/ds    (fe_vjp_path)
    with mu_N = 0.  K_n is the consistent tangent at (u_n, h_{n-1}).
    """

    @staticmethod
    def forward(ctx, s, problem, phase, models, params, mask, path, newton_rtol, pcg_rtol, checkpoints=None):
        P = problem
        if P.prec != fe.F64:
            raise ValueError("the path adjoint needs an FP64 problem")
        if checkpoints is not None and int(checkpoints) < 0:
            raise ValueError("checkpoints must be >= 0 or None")
        P.set_materials(phase, models, params, s.detach().contiguous())
        P.set_dirichlet(mask)
        ctx.problem, ctx.pcg_rtol, ctx.mask, ctx.path = P, pcg_rtol, mask, [np.asarray(e) for e in path]
        ctx.field = (phase, list(models), list(params), s.detach().clone())
        ctx.newton_rtol, ctx.checkpoints = newton_rtol, checkpoints
        u, state = P.vector(), P.state()
        ctx.start = (u.clone(), state.clone())
        us, hs, infos = [], [], []
        h_last = None
        for eb in ctx.path:
            h_last = state.clone()
            _, _, _, info = P.newton([eb], u=u, state=state, op=fe.OP_MATFREE, newton_rtol=newton_rtol,
                                     pcg_rtol=pcg_rtol, max_newton=40)
            if checkpoints is None:
                hs.append(h_last)
                us.append(u.clone())
            infos.append(info)
        ub = u * mask.to(u.dtype)
        J = torch.dot(ub, P.residual(u, h_last))
        ctx.us, ctx.hs, ctx.ub, ctx.infos = us, hs, ub, infos
        return J

    @staticmethod
    def _advance(ctx, held, first, last):
        """State (u, h) after step `last` from the state after step `first` (steps are 1-based)."""
        u, h = held[0].clone(), held[1].clone()
        for n in range(first + 1, last + 1):
            ctx.problem.newton([ctx.path[n - 1]], u=u, state=h, op=fe.OP_MATFREE, newton_rtol=ctx.newton_rtol,
                               pcg_rtol=ctx.pcg_rtol, max_newton=40)
            ctx.recompute_solves += 1
        return u, h

    @staticmethod
    def _adjoint_step(ctx, n, un, hn, mu, grad):
        """One backward step at load step n (1-based) with u_n and h_{n-1}; returns mu_{n-1}."""
        P, ub = ctx.problem, ctx.ub
        last = n == len(ctx.path)
        P.residual(un, hn, P.state(), apply_bc=True, store_tangent=True)   # K_n at (u_n, h_{n-1})
        if last:
            rhs = P.apply_matfree(ub, apply_bc=False)                      # K_N u_b
        else:
            rhs = P.vector()
            P.vjp_path(un, hn, mu_in=mu, u_bar=rhs)                        # d(mu_n . h_n)/du
        rhs *= 1.0 - ctx.mask.to(ub.dtype)
        lam, res = P.pcg(rhs, op=fe.OP_MATFREE, rtol=ctx.pcg_rtol, max_it=200000)
        ctx.adjoint_iterations.append(res.iterations)
        c = (ub - lam) if last else -lam
        return P.vjp_path(un, hn, c=c, mu_in=mu, s_bar=grad)

    @staticmethod
    def _reverse(ctx, held, first, last, slots, mu, grad):
        """Backward steps last, last-1, ..., first+1 from the held state after step `first`."""
        R = ReactionWorkPath
        if last - first == 1:
            un, _ = R._advance(ctx, held, first, last)
            return R._adjoint_step(ctx, last, un, held[1], mu, grad)
        if slots == 0:
            for t in range(last, first, -1):
                before = R._advance(ctx, held, first, t - 1)
                mu = R._reverse(ctx, before, t - 1, t, 0, mu, grad)
            return mu
        k = _revolve(last - first, slots)[1]
        mid = R._advance(ctx, held, first, first + k)
        mu = R._reverse(ctx, mid, first + k, last, slots - 1, mu, grad)
        del mid
        return R._reverse(ctx, held, first, first + k, slots, mu, grad)

    @staticmethod
    def backward(ctx, gJ):
        P, ub = ctx.problem, ctx.ub
        phase, models, params, s = ctx.field   # re-instate the forward's materials and constraints
        P.set_materials(phase, models, params, s)
        P.set_dirichlet(ctx.mask)
        grad = torch.zeros(P.n_el, dtype=ub.dtype, device=ub.device)
        ctx.adjoint_iterations, ctx.recompute_solves = [], 0
        if ctx.checkpoints is None:
            mu = None
            for n in range(len(ctx.path), 0, -1):
                mu = ReactionWorkPath._adjoint_step(ctx, n, ctx.us[n - 1], ctx.hs[n - 1], mu, grad)
        else:
            ReactionWorkPath._reverse(ctx, ctx.start, 0, len(ctx.path), int(ctx.checkpoints), None, grad)
        return grad * gJ, None, None, None, None, None, None, None, None, None


def reaction_work_path(s, problem, phase, models, params, mask, path, newton_rtol=1e-12, pcg_rtol=1e-13,
                       checkpoints=None):
    return ReactionWorkPath.apply(s, problem, phase, models, params, mask, path, newton_rtol, pcg_rtol, checkpoints)


def fit_phase_scales(problem, phase, models, params, mask, paths, targets, theta0, max_iter=12, tol=1e-9,
                     newton_rtol=1e-12, pcg_rtol=1e-13, checkpoints=None, log=None):
    """Material-parameter inverse problem: one modulus scale per phase, s_e = theta[phase_e],
    fitted so that the reaction work of every load path matches its target.  Gauss-Newton on
    r_i = J_i(theta) / J_i* - 1 with dr_i/dtheta_p = (sum over phase-p elements of dJ_i/ds_e) / J_i*,
    the gradients from the path adjoint (ReactionWorkPath).  Returns (theta, history)."""
    phase_idx = phase.long()
    n_par = len(models)
    theta = torch.tensor(np.asarray(theta0, dtype=np.float64), device=phase.device)
    hist = []
    for it in range(max_iter):
        r = torch.empty(len(paths), dtype=torch.float64)
        jac = torch.empty(len(paths), n_par, dtype=torch.float64)
        for i, (path, jt) in enumerate(zip(paths, targets)):
            s = theta[phase_idx].clone().requires_grad_(True)
            J = reaction_work_path(s, problem, phase, models, params, mask, path, newton_rtol, pcg_rtol, checkpoints)
            J.backward()
            r[i] = float(J.detach()) / jt - 1.0
            g = torch.zeros(n_par, dtype=torch.float64, device=phase.device).index_add_(0, phase_idx, s.grad)
            jac[i] = (g / jt).cpu()
        hist.append({"theta": theta.cpu().tolist(), "residual": r.tolist()})
        if log:
            log(f"Gauss-Newton {it}: theta {hist[-1]['theta']} residual {hist[-1]['residual']}")
        if float(torch.linalg.norm(r)) <= tol:
            break
        step = torch.linalg.lstsq(jac, -r.unsqueeze(1)).solution.squeeze(1)
        theta = theta + step.to(theta.device)
    return theta.cpu().numpy(), hist
