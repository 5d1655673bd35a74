"""Small-strain J2 plasticity with linear isotropic hardening (oracle).

The paper's nonlinear phase-dependent constitutive response (Sec. I, Sec. V-A)
is not specified; the plastic matrix phase here is von Mises plasticity
integrated by the radial-return map with its consistent tangent (Simo & Hughes,
Computational Inelasticity, 1998, Sec. 3.3 and Box 3.2).  Every evaluation
starts from the last converged state (eps_p_n, alpha_n):

  trial elastic strain  e_tr = eps - eps_p_n              (tensor form)
  p = K tr e_tr,  s_tr = 2G dev e_tr,  q_tr = sqrt(3/2) |s_tr|_F
  f_tr = q_tr - (sigma_y + H alpha_n)
  f_tr <= 0:  sigma = s_tr + p I, state unchanged, D = elastic
  f_tr  > 0:  dgam = f_tr / (3G + H),  N = s_tr / |s_tr|_F
              sigma = (1 - 3G dgam/q_tr) s_tr + p I
              eps_p = eps_p_n + sqrt(3/2) dgam N,  alpha = alpha_n + dgam
              D = K 1x1 + 2G theta I_dev + 6G^2 (dgam/q_tr - 1/(3G+H)) N x N,
              theta = 1 - 3G dgam/q_tr

Voigt conventions: strains [xx,yy,zz,yz,xz,xy] with engineering shears, stress
with tensor components; I_sym -> diag(1,1,1,1/2,1/2,1/2), N x N uses tensor
components of N.

Every branch is decided on real parts, so complex inputs carry complex-step
derivatives through unchanged (used by the path-adjoint oracle).
"""
from __future__ import annotations

import numpy as np

from .elasticity import bulk_shear

ONE = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
I_SYM = np.diag([1.0, 1.0, 1.0, 0.5, 0.5, 0.5])
I_DEV = I_SYM - np.outer(ONE, ONE) / 3.0


def strain_to_tensor(v):
    """(m,6) engineering Voigt strain -> (m,3,3) tensor."""
    t = np.empty(v.shape[:-1] + (3, 3), dtype=np.result_type(v, np.float64))
    t[..., 0, 0], t[..., 1, 1], t[..., 2, 2] = v[..., 0], v[..., 1], v[..., 2]
    t[..., 1, 2] = t[..., 2, 1] = 0.5 * v[..., 3]
    t[..., 0, 2] = t[..., 2, 0] = 0.5 * v[..., 4]
    t[..., 0, 1] = t[..., 1, 0] = 0.5 * v[..., 5]
    return t


def tensor_to_stress(t):
    """(m,3,3) symmetric tensor -> (m,6) tensor-component Voigt vector."""
    return np.stack([t[..., 0, 0], t[..., 1, 1], t[..., 2, 2],
                     t[..., 1, 2], t[..., 0, 2], t[..., 0, 1]], axis=-1)


def return_map(eps, eps_p_n, alpha_n, E, nu, sigma_y, H):
    """Radial return at m points.

    eps, eps_p_n: (m,6) engineering Voigt; alpha_n: (m,).
    Returns dict: sigma (m,6), eps_p (m,6) engineering, alpha (m,), D (m,6,6),
    plastic (m,) bool, f_trial (m,), dgamma (m,), q_trial (m,), N (m,6) tensor comps.
    """
    m = len(eps)
    K, G = bulk_shear(np.broadcast_to(np.asarray(E), (m,)), nu)
    et = strain_to_tensor(eps - eps_p_n)
    tr = np.trace(et, axis1=-2, axis2=-1)
    eye = np.eye(3)
    p = K * tr
    s_tr = 2.0 * G[:, None, None] * (et - tr[:, None, None] / 3.0 * eye)
    s_norm = np.sqrt(np.sum(s_tr * s_tr, axis=(-2, -1)))
    q_tr = np.sqrt(1.5) * s_norm
    f_tr = q_tr - (sigma_y + H * alpha_n)
    plastic = np.real(f_tr) > 0.0  # real parts decide (complex-step derivatives pass through)

    dgam = np.where(plastic, f_tr / (3.0 * G + H), 0.0)
    safe_norm = np.where(np.real(s_norm) > 0.0, s_norm, 1.0)
    n_t = s_tr / safe_norm[:, None, None]
    safe_q = np.where(np.real(q_tr) > 0.0, q_tr, 1.0)
    theta = np.where(plastic, 1.0 - 3.0 * G * dgam / safe_q, 1.0)

    sig_t = theta[:, None, None] * s_tr + p[:, None, None] * eye
    dep_t = np.sqrt(1.5) * dgam[:, None, None] * n_t
    dep_v = tensor_to_stress(dep_t)
    dep_v[:, 3:] *= 2.0  # engineering shear
    n_v = tensor_to_stress(n_t)

    coef = np.where(plastic, 6.0 * G * G * (dgam / safe_q - 1.0 / (3.0 * G + H)), 0.0)
    d = (K[:, None, None] * np.outer(ONE, ONE)[None]
         + 2.0 * (G * theta)[:, None, None] * I_DEV[None]
         + coef[:, None, None] * np.einsum("mi,mj->mij", n_v, n_v))
    return dict(sigma=tensor_to_stress(sig_t), eps_p=eps_p_n + dep_v, alpha=alpha_n + dgam,
                D=d, plastic=plastic, f_trial=f_tr, dgamma=dgam, q_trial=q_tr, N=n_v)
