"""Structured trilinear hexahedral mesh of the unit cube (oracle).

The paper's element batches are elements of one type with a map from local to
global dofs (Sec. IV, Construction); the element type and numbering are not
given, so the reading here is an n^3 grid of 8-node bricks on [0,1]^3:
  node (i,j,k), 0 <= i,j,k <= n:  id i + (n+1)(j + (n+1)k), x = (i,j,k)/n
  element (a,b,c), 0 <= a,b,c < n:  id a + n(b + nc)
  local node order (offsets):  0 (0,0,0) 1 (1,0,0) 2 (1,1,0) 3 (0,1,0)
                               4 (0,0,1) 5 (1,0,1) 6 (1,1,1) 7 (0,1,1)
  dof = 3*node + component (x, y, z).
"""
from __future__ import annotations

import numpy as np

LOCAL_OFFSETS = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                          [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)


def node_id(n, i, j, k):
    return i + (n + 1) * (j + (n + 1) * k)


def structured_hex8(n: int):
    """Return (coords (n_nodes,3) float64, conn (n_el,8) int64)."""
    h = 1.0 / n
    coords = np.zeros(((n + 1) ** 3, 3))
    for k in range(n + 1):
        for j in range(n + 1):
            for i in range(n + 1):
                coords[node_id(n, i, j, k)] = (i * h, j * h, k * h)
    conn = np.zeros((n ** 3, 8), dtype=np.int64)
    for c in range(n):
        for b in range(n):
            for a in range(n):
                e = a + n * (b + n * c)
                for loc, (di, dj, dk) in enumerate(LOCAL_OFFSETS):
                    conn[e, loc] = node_id(n, a + di, b + dj, c + dk)
    return coords, conn


def element_dofs(conn: np.ndarray) -> np.ndarray:
    """(n_el, 24) global dofs of each element, local dof = 3*local_node + component."""
    return (3 * conn[:, :, None] + np.arange(3)[None, None, :]).reshape(len(conn), 24)


def boundary_nodes(coords: np.ndarray, tol: float = 1e-12) -> np.ndarray:
    """Boolean per node: on a face of the unit cube."""
    return np.any((coords < tol) | (coords > 1.0 - tol), axis=1)
