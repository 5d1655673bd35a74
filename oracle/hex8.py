"""Trilinear hexahedron (8 nodes) with 2x2x2 Gauss quadrature (oracle).

Textbook isoparametric element (e.g. Hughes, The Finite Element Method, 2000,
Sec. 3.5): N_a(xi) = 1/8 (1 + xi_a xi)(1 + eta_a eta)(1 + zeta_a zeta) on the
reference cube [-1,1]^3, Jacobian J_ik = dx_i/dxi_k = sum_a x_a,i dN_a/dxi_k,
physical gradients dN/dx = dN/dxi J^-1.  The paper leaves element type and
quadrature to the batch definition (Sec. III-B); this is the reading used.

Quadrature point q = a + 2b + 4c sits at (s_a, s_b, s_c)/sqrt(3), s_0 = -1,
s_1 = +1, weight 1.  Strain vectors use Voigt order [xx, yy, zz, yz, xz, xy]
with engineering shears; the B-matrix column block of node a with gradient
(b1, b2, b3) is [b1 0 0; 0 b2 0; 0 0 b3; 0 b3 b2; b3 0 b1; b2 b1 0].
"""
from __future__ import annotations

import numpy as np

NODE_XI = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                    [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)


def gauss_points():
    """(8,3) reference coordinates and (8,) weights of the 2x2x2 Gauss rule."""
    g = 1.0 / np.sqrt(3.0)
    s = (-1.0, 1.0)
    pts = np.array([[s[a] * g, s[b] * g, s[c] * g]
                    for c in range(2) for b in range(2) for a in range(2)])
    return pts, np.ones(8)


def shape_functions(xi) -> np.ndarray:
    """(8,) values N_a at reference point xi."""
    xi = np.asarray(xi, dtype=np.float64)
    return 0.125 * np.prod(1.0 + NODE_XI * xi[None, :], axis=1)


def shape_gradients_ref(xi) -> np.ndarray:
    """(8,3) dN_a/dxi_k at reference point xi."""
    xi = np.asarray(xi, dtype=np.float64)
    f = 1.0 + NODE_XI * xi[None, :]  # (8,3) one-dimensional factors
    d = np.empty((8, 3))
    d[:, 0] = 0.125 * NODE_XI[:, 0] * f[:, 1] * f[:, 2]
    d[:, 1] = 0.125 * f[:, 0] * NODE_XI[:, 1] * f[:, 2]
    d[:, 2] = 0.125 * f[:, 0] * f[:, 1] * NODE_XI[:, 2]
    return d


def physical_gradients(xe: np.ndarray, xi):
    """Gradients for a batch of elements at one reference point.

    xe: (n_el, 8, 3) nodal coordinates.  Returns (dNdx (n_el,8,3), detJ (n_el,)).
    """
    dn = shape_gradients_ref(xi)                      # (8,3)
    jac = np.einsum("eai,ak->eik", xe, dn)            # J_ik = dx_i/dxi_k
    det = np.linalg.det(jac)
    jinv = np.linalg.inv(jac)                          # (J^-1)_ki = dxi_k/dx_i
    dndx = np.einsum("ak,eki->eai", dn, jinv)
    return dndx, det


def bmatrix(dndx: np.ndarray) -> np.ndarray:
    """(n_el, 6, 24) small-strain B matrices from (n_el, 8, 3) gradients."""
    ne = dndx.shape[0]
    b = np.zeros((ne, 6, 24))
    for a in range(8):
        b1, b2, b3 = dndx[:, a, 0], dndx[:, a, 1], dndx[:, a, 2]
        c = 3 * a
        b[:, 0, c + 0] = b1
        b[:, 1, c + 1] = b2
        b[:, 2, c + 2] = b3
        b[:, 3, c + 1] = b3
        b[:, 3, c + 2] = b2
        b[:, 4, c + 0] = b3
        b[:, 4, c + 2] = b1
        b[:, 5, c + 0] = b2
        b[:, 5, c + 1] = b1
    return b
