"""Two-phase RVE problem: residual, Jacobian, Dirichlet lift, Newton (oracle).

The paper solves R(u) = 0 by Newton's method with K = dR/du (Sec. II-A); each
phase contributes its own element residuals and Jacobians, assembled into one
sparse Jacobian per Newton iteration and solved by a Krylov method (Sec. V-A).

Readings where the paper is silent:
  * boundary: affine Dirichlet u = eps_bar . x on every node of the cube faces
    (all three dofs), x measured from the corner (0,0,0);
  * update solve: A w = -P_f R(u), A = P_f K P_f + P_b (symmetric elimination);
  * Newton per load step: predictor moves only the boundary values; stop when
    ||P_f R|| <= newton_rtol * ||P_f R||_first (or it is exactly 0), at most
    max_newton iterations; the plastic state is committed on convergence and
    every evaluation starts from the last committed state;
  * globalisation: the step u + s w starts at s = 1 and is halved while
    ||P_f R(u + s w)|| >= ||P_f R(u)||, at most max_halvings times (the last
    trial is taken).  Full steps cycle when many ligament points switch between
    elastic and plastic; the halving line search is the textbook remedy.
"""
from __future__ import annotations

import numpy as np

from . import assembly, element, j2, neohooke, solver
from .elasticity import lame
from .hex8 import gauss_points, physical_gradients
from .mesh import boundary_nodes, structured_hex8


def phase_params(model, E, nu, sigma_y=0.0, H=0.0):
    return dict(model=model, E=float(E), nu=float(nu), sigma_y=float(sigma_y), H=float(H))


class RVE:
    """Unit-cube RVE with per-element phase and modulus scale: the structured n^3 hex8
    mesh, or any hex8 mesh given as mesh=(coords (n_nodes,3), conn (n_el,8))."""

    def __init__(self, n, phase, phases, scale=None, elements=None, mesh=None):
        self.n = n
        if mesh is None:
            self.coords, conn = structured_hex8(n)
        else:
            self.coords = np.asarray(mesh[0], dtype=np.float64)
            conn = np.asarray(mesh[1], dtype=np.int64)
        n_el = len(conn)
        self.phase_all = np.asarray(phase, dtype=np.int64)
        self.scale_all = np.ones(n_el) if scale is None else np.asarray(scale, dtype=np.float64)
        # optional subset of elements (used to evaluate element quantities one by one)
        self.elements = np.arange(n_el) if elements is None else np.asarray(elements)
        self.conn = conn[self.elements]
        self.phase = self.phase_all[self.elements]
        self.scale = self.scale_all[self.elements]
        self.phases = phases
        self.n_dof = 3 * len(self.coords)
        self.mask = np.repeat(boundary_nodes(self.coords), 3).astype(np.uint8)
        self.free = 1.0 - self.mask

    # ---- constitutive evaluation ------------------------------------------------
    def zero_state(self):
        ne = len(self.conn)
        return dict(eps_p=np.zeros((ne, 8, 6)), alpha=np.zeros((ne, 8)))

    def _material(self, state_n, trial):
        ne = len(self.conn)
        lam_e = np.zeros(ne, dtype=np.result_type(self.scale, np.float64))
        mu_e = np.zeros_like(lam_e)
        for pid, p in enumerate(self.phases):
            lam, mu = lame(p["E"], p["nu"])
            sel = self.phase == pid
            lam_e[sel], mu_e[sel] = lam * self.scale[sel], mu * self.scale[sel]
        lin = element.linear_material(lam_e, mu_e)
        j2_ids = [pid for pid, p in enumerate(self.phases) if p["model"] == "j2"]

        def material(q, eps):
            sig, d = lin(q, eps)
            sig, d = sig.copy(), d.copy()
            for pid in j2_ids:
                sel = self.phase == pid
                if not np.any(sel):
                    continue
                p = self.phases[pid]
                rm = j2.return_map(eps[sel], state_n["eps_p"][sel, q], state_n["alpha"][sel, q],
                                   p["E"] * self.scale[sel], p["nu"], p["sigma_y"], p["H"])
                sig[sel], d[sel] = rm["sigma"], rm["D"]
                trial["eps_p"][sel, q] = rm["eps_p"]
                trial["alpha"][sel, q] = rm["alpha"]
                trial["plastic"][sel, q] = rm["plastic"]
                trial["sigma"][sel, q] = rm["sigma"]
            trial["sigma_all"][:, q] = sig
            return sig, d

        return material

    def element_residual_tangent(self, u, state_n=None, want_tangent=True):
        """Element residuals (n_el,24), tangents (n_el,24,24) and the trial state."""
        if state_n is None:
            state_n = self.zero_state()
        ne = len(self.conn)
        dt = np.result_type(u, self.scale, state_n["eps_p"], np.float64)
        trial = dict(eps_p=state_n["eps_p"].astype(dt), alpha=state_n["alpha"].astype(dt),
                     plastic=np.zeros((ne, 8), dtype=bool), sigma=np.zeros((ne, 8, 6), dtype=dt),
                     sigma_all=np.zeros((ne, 8, 6), dtype=dt))
        r_e, k_e = element.residual_and_tangent(self.coords, self.conn, u,
                                                self._material(state_n, trial), want_tangent)
        nh_ids = [pid for pid, p in enumerate(self.phases) if p["model"] == "neohooke"]
        if nh_ids:  # finite-strain phases replace their small-strain evaluation
            sel = np.isin(self.phase, nh_ids)
            mu_e, lam_e = np.zeros(ne), np.zeros(ne)
            for pid in nh_ids:
                lam, mu = lame(self.phases[pid]["E"], self.phases[pid]["nu"])
                s = self.phase == pid
                lam_e[s], mu_e[s] = lam * self.scale[s], mu * self.scale[s]
            r_n, k_n, p_qp = neohooke.residual_tangent(self.coords, self.conn[sel], u, mu_e[sel], lam_e[sel],
                                                       want_tangent)
            r_e[sel] = r_n
            if want_tangent:
                k_e[sel] = k_n
            trial["sigma_all"][sel] = np.stack([p_qp[..., 0, 0], p_qp[..., 1, 1], p_qp[..., 2, 2],
                                                p_qp[..., 1, 2], p_qp[..., 0, 2], p_qp[..., 0, 1]], axis=-1)
        return r_e, k_e, trial

    def residual(self, u, state_n=None):
        r_e, _, trial = self.element_residual_tangent(u, state_n, want_tangent=False)
        return assembly.assemble_vector(self.conn, r_e, self.n_dof), trial

    # ---- boundary conditions ----------------------------------------------------
    def affine_lift(self, eps_bar):
        """Boundary displacements eps_bar . x (zero on free dofs)."""
        ub = (self.coords @ np.asarray(eps_bar, dtype=np.float64).T).ravel()
        return ub * self.mask

    # ---- operators ----------------------------------------------------------------
    def bc_csr(self, k_e):
        rp, ci, v = assembly.assemble_csr(self.conn, k_e, self.n_dof)
        return rp, ci, assembly.dirichlet_csr(rp, ci, v, self.mask)

    def solve_update(self, k_e, rhs, rtol, max_it, op="csr"):
        """PCG on A w = rhs with A = P_f K P_f + P_b (rhs must vanish on constrained dofs)."""
        if op == "csr":
            rp, ci, v = self.bc_csr(k_e)
            diag = assembly.csr_diagonal(rp, ci, v)
            return solver.pcg(lambda x: assembly.csr_matvec(rp, ci, v, x), diag, rhs, rtol, max_it)
        diag = solver.matfree_diagonal(self.conn, k_e, self.n_dof, self.mask)
        return solver.pcg(lambda x: solver.matfree_apply(self.conn, k_e, x, self.mask),
                          diag, rhs, rtol, max_it)

    # ---- solves -----------------------------------------------------------------
    def solve_linear(self, eps_bar, rtol=1e-10, max_it=20000, op="csr"):
        """One Newton update from the affine lift (exact for linear phases)."""
        u = self.affine_lift(eps_bar)
        r_e, k_e, _ = self.element_residual_tangent(u)
        rhs = -assembly.assemble_vector(self.conn, r_e, self.n_dof) * self.free
        w, it, status, rel = self.solve_update(k_e, rhs, rtol, max_it, op)
        return u + w, dict(iterations=it, status=status, true_relres=rel)

    def newton(self, load_path, newton_rtol=1e-8, max_newton=20, pcg_rtol=1e-10,
               pcg_max_it=20000, op="csr", max_halvings=5):
        """Load stepping: for each macro strain in load_path, Newton to tolerance."""
        u = np.zeros(self.n_dof)
        state = self.zero_state()
        history = []

        def evaluate(v):
            r_e, k_e, trial = self.element_residual_tangent(v, state)
            rf = assembly.assemble_vector(self.conn, r_e, self.n_dof) * self.free
            return rf, np.linalg.norm(rf), k_e, trial

        for eps_bar in load_path:
            u = u * self.free + self.affine_lift(eps_bar)
            rec = dict(eps_bar=np.asarray(eps_bar), residuals=[], pcg_iterations=[], steps=[])
            rf, rn, k_e, trial = evaluate(u)
            r0 = rn
            for it in range(max_newton + 1):
                rec["residuals"].append(rn)
                if rn <= newton_rtol * r0 or rn == 0.0:
                    break
                if it == max_newton:
                    raise RuntimeError("Newton did not converge")
                w, pit, status, _ = self.solve_update(k_e, -rf, pcg_rtol, pcg_max_it, op)
                if status != solver.OK:
                    raise RuntimeError(f"PCG failed: {status}")
                rec["pcg_iterations"].append(pit)
                s = 1.0
                for halving in range(max_halvings + 1):
                    trial_eval = evaluate(u + s * w)
                    if trial_eval[1] < rn or halving == max_halvings:
                        break
                    s *= 0.5
                rec["steps"].append(s)
                u = u + s * w
                rf, rn, k_e, trial = trial_eval
            state = dict(eps_p=trial["eps_p"], alpha=trial["alpha"])
            rec["sigma_bar"] = self.mean_stress(trial["sigma_all"])
            rec["plastic_fraction"] = float(np.mean(trial["plastic"]))
            history.append(rec)
        return u, state, history

    # ---- homogenised output ---------------------------------------------------------
    def qp_volumes(self):
        """(n_el, 8) w_q detJ_q."""
        xe = self.coords[self.conn]
        pts, w = gauss_points()
        return np.stack([w[q] * physical_gradients(xe, pts[q])[1] for q in range(8)], axis=1)

    def mean_stress(self, sigma_qp):
        """Volume average of (n_el, 8, 6) stresses: sum_q w detJ sigma_q / sum_q w detJ."""
        v = self.qp_volumes()
        return np.einsum("eq,eqi->i", v, sigma_qp) / v.sum()
