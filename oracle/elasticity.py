"""Isotropic linear elasticity (oracle).

The paper's phases each carry their own stress-strain law (Sec. III-B, Sec. V-A)
without stating it; the linear phases follow Hooke's law in Lame form,
sigma = lambda tr(eps) I + 2 mu eps, written in Voigt notation with engineering
shear strains: D = lambda 1 1^T + mu diag(2,2,2,1,1,1).
"""
from __future__ import annotations

import numpy as np


def lame(E, nu):
    """(lambda, mu) from Young's modulus and Poisson ratio."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def bulk_shear(E, nu):
    """(K, G) bulk and shear moduli."""
    return E / (3.0 * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def hooke_voigt(lam, mu) -> np.ndarray:
    """6x6 Voigt stiffness (engineering shear strain in, tensor stress out)."""
    d = np.zeros((6, 6))
    d[:3, :3] = lam
    d += np.diag([2.0 * mu, 2.0 * mu, 2.0 * mu, mu, mu, mu])
    return d
