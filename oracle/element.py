"""Element residuals and element Jacobians, small strain (oracle).

Residual form of the paper's problem (Sec. II-A): the element internal force is
r_e = sum_q w_q detJ_q B_q^T sigma_q with sigma_q the constitutive response to
eps_q = B_q u_e, and the element Jacobian is its derivative
K_e = dr_e/du_e = sum_q w_q detJ_q B_q^T D_q B_q with D_q = dsigma/deps at q
(the dense local Jacobians that Sec. III-B obtains by forward-mode AD).
Loops over the 8 quadrature points; each step is batched over the elements given.
"""
from __future__ import annotations

import numpy as np

from .hex8 import bmatrix, gauss_points, physical_gradients
from .mesh import element_dofs


def qp_strains(coords, conn, u):
    """List over q of (n_el, 6) small strains eps_q = B_q u_e (engineering shear)."""
    xe = coords[conn]
    ue = u[element_dofs(conn)]
    pts, _ = gauss_points()
    out = []
    for q in range(8):
        dndx, _ = physical_gradients(xe, pts[q])
        out.append(np.einsum("eij,ej->ei", bmatrix(dndx), ue))
    return out


def residual_and_tangent(coords, conn, u, material, want_tangent=True):
    """Element residuals (n_el,24) and tangents (n_el,24,24) for a small-strain law.

    material(q, eps) -> (sigma (n_el,6) tensor Voigt, D (n_el,6,6)) evaluates the
    constitutive law at quadrature point q of every element.
    """
    xe = coords[conn]
    ue = u[element_dofs(conn)]
    pts, w = gauss_points()
    ne = len(conn)
    r = k = None
    for q in range(8):
        dndx, det = physical_gradients(xe, pts[q])
        b = bmatrix(dndx)
        eps = np.einsum("eij,ej->ei", b, ue)
        sig, d = material(q, eps)
        if r is None:  # real, or complex when a complex-step perturbation is carried
            dt = np.result_type(sig, d, ue, np.float64)
            r = np.zeros((ne, 24), dtype=dt)
            k = np.zeros((ne, 24, 24), dtype=dt) if want_tangent else None
        wdet = w[q] * det
        r += np.einsum("eji,ej->ei", b, sig) * wdet[:, None]
        if want_tangent:
            k += np.matmul(b.transpose(0, 2, 1), np.matmul(d, b)) * wdet[:, None, None]
    return r, k


def linear_material(lam_e, mu_e):
    """Hooke's law per element with Lame parameters lam_e, mu_e (arrays over elements)."""
    lam_e = np.asarray(lam_e)
    mu_e = np.asarray(mu_e)
    d = np.zeros((len(lam_e), 6, 6), dtype=np.result_type(lam_e, mu_e, np.float64))
    d[:, :3, :3] = lam_e[:, None, None]
    for i in range(3):
        d[:, i, i] += 2.0 * mu_e
        d[:, 3 + i, 3 + i] += mu_e

    def material(q, eps):
        return np.matmul(d, eps[:, :, None])[:, :, 0], d

    return material


def linear_residual_tangent(coords, conn, u, lam_e, mu_e, want_tangent=True):
    """Linear-elastic element residuals and tangents (r_e = K_e u_e)."""
    return residual_and_tangent(coords, conn, u, linear_material(lam_e, mu_e), want_tangent)
