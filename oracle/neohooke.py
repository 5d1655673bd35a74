"""Compressible Neo-Hookean solid in total-Lagrangian form (oracle).

One of the phase laws the paper's heterogeneous RVE admits (Sec. V-A leaves the
laws open); the variant used is the common compressible one
(e.g. Bonet & Wood, Nonlinear Continuum Mechanics for FE Analysis, 2008, Sec. 6.4.3):
  W(F) = mu/2 (tr(F^T F) - 3 - 2 ln J) + lam/2 (ln J)^2,   J = det F,  F = I + grad_X u
  P = dW/dF = mu (F - F^-T) + lam ln J F^-T
  A_iJkL = dP_iJ/dF_kL = mu d_ik d_JL + (mu - lam ln J) Finv_Jk Finv_Li + lam Finv_Ji Finv_Lk
Element residual r_e[a,i] = sum_q w_q detJ_q P_iJ dN_a/dX_J and Jacobian
K_e[(a,i),(b,k)] = sum_q w_q detJ_q dN_a/dX_J A_iJkL dN_b/dX_L (Sec. II-A: K = dR/du).
"""
from __future__ import annotations

import numpy as np

from .hex8 import gauss_points, physical_gradients
from .mesh import element_dofs


class InvertedElement(RuntimeError):
    pass


def energy(F, mu, lam):
    """Strain energy density W(F) for (m,3,3) deformation gradients."""
    J = np.linalg.det(F)
    lnJ = np.log(J)
    i1 = np.einsum("mij,mij->m", F, F)
    return 0.5 * mu * (i1 - 3.0 - 2.0 * lnJ) + 0.5 * lam * lnJ ** 2


def stress_tangent(H, mu, lam):
    """P (m,3,3) and A (m,3,3,3,3) from displacement gradients H = grad_X u (m,3,3)."""
    m = H.shape[0]
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (m,))
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (m,))
    F = np.eye(3)[None] + H
    J = np.linalg.det(F)
    if np.any(J <= 0.0):
        raise InvertedElement("det F <= 0")
    Finv = np.linalg.inv(F)
    FiT = Finv.transpose(0, 2, 1)
    lnJ = np.log(J)
    P = mu[:, None, None] * (F - FiT) + (lam * lnJ)[:, None, None] * FiT
    eye = np.eye(3)
    A = (mu[:, None, None, None, None] * np.einsum("ik,JL->iJkL", eye, eye)[None]
         + (mu - lam * lnJ)[:, None, None, None, None] * np.einsum("mJk,mLi->miJkL", Finv, Finv)
         + lam[:, None, None, None, None] * np.einsum("mJi,mLk->miJkL", Finv, Finv))
    return P, A


def residual_tangent(coords, conn, u, mu_e, lam_e, want_tangent=True):
    """Element residuals (n_el,24), Jacobians (n_el,24,24) and first PK stresses (n_el,8,3,3)."""
    xe = coords[conn]
    ue = u[element_dofs(conn)].reshape(len(conn), 8, 3)
    pts, w = gauss_points()
    ne = len(conn)
    r = np.zeros((ne, 8, 3))
    k = np.zeros((ne, 8, 3, 8, 3)) if want_tangent else None
    p_all = np.zeros((ne, 8, 3, 3))
    for q in range(8):
        dndx, det = physical_gradients(xe, pts[q])
        H = np.einsum("eai,eaJ->eiJ", ue, dndx)
        P, A = stress_tangent(H, mu_e, lam_e)
        p_all[:, q] = P
        wdet = w[q] * det
        r += np.einsum("eiJ,eaJ->eai", P, dndx) * wdet[:, None, None]
        if want_tangent:
            k += np.einsum("eaJ,eiJkL,ebL->eaibk", dndx, A, dndx) * wdet[:, None, None, None, None]
    return r.reshape(ne, 24), (k.reshape(ne, 24, 24) if want_tangent else None), p_all
