"""Node-block incomplete LU factorisation, ILU(0), of the assembled operator (oracle).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

Sec. V-B (Fig. 7) compares Jacobi with ILU preconditioning of the assembled
matrix (ILU needs the explicit matrix).  Here ILU(0) acts on 3x3 node blocks (the
three displacement components of a node are one block unknown), keeps no fill
beyond the block pattern of the matrix (node pairs that share an element), and
takes the nodes in an 8-colour order: colour = (i mod 2) + 2 (j mod 2) + 4 (k mod 2)
of the node's grid indices, nodes sorted by (colour, node id).  No two nodes of one
colour share an element, so each colour is one level of the triangular solves.

Factorisation: the IKJ form of Gaussian elimination restricted to the pattern
(Saad, Iterative Methods for Sparse Linear Systems, 2003, Alg. 10.4), on blocks:
for each block row i in order and each k before i in row i's pattern, in order,
    A_ik <- A_ik A_kk^-1,   A_ij <- A_ij - A_ik A_kj  for every j after k that is in
    the pattern of row i (and of row k).
L is the unit block lower part, U the upper part with the diagonal blocks.
M z = r is solved by L y = r (forward) and U z = y (backward).
"""
from __future__ import annotations

import numpy as np

from .mesh import node_id


def node_color(n, node):
    i = node % (n + 1)
    j = (node // (n + 1)) % (n + 1)
    k = node // (n + 1) ** 2
    return (i % 2) + 2 * (j % 2) + 4 * (k % 2)


def color_order(n):
    """perm[position] = node id and pos[node id] = position, nodes sorted by (colour, id)."""
    nodes = np.arange((n + 1) ** 3)
    perm = np.array(sorted(nodes, key=lambda a: (node_color(n, a), a)))
    pos = np.empty_like(perm)
    pos[perm] = np.arange(perm.size)
    return perm, pos


def neighbours(n, node):
    """Nodes sharing an element with `node` (itself included), ascending ids."""
    i = node % (n + 1)
    j = (node // (n + 1)) % (n + 1)
    k = node // (n + 1) ** 2
    out = []
    for c in (k - 1, k, k + 1):
        for b in (j - 1, j, j + 1):
            for a in (i - 1, i, i + 1):
                if 0 <= a <= n and 0 <= b <= n and 0 <= c <= n:
                    out.append(node_id(n, a, b, c))
    return out


def csr_blocks(n, row_ptr, col_idx, vals):
    """{(I, J): 3x3 block} of a CSR matrix on the structured dof numbering dof = 3 node + c,
    for every node pair in the block pattern (absent entries are zero)."""
    blocks = {}
    n_nodes = (n + 1) ** 3
    for a in range(n_nodes):
        for b in neighbours(n, a):
            blocks[(a, b)] = np.zeros((3, 3))
    for r in range(3 * n_nodes):
        for q in range(row_ptr[r], row_ptr[r + 1]):
            c = col_idx[q]
            blocks[(r // 3, c // 3)][r % 3, c % 3] += vals[q]
    return blocks


def bilu0(n, blocks):
    """Block ILU(0) in the colour order.  Returns {(I, J): block}: L_IJ (I after J),
    U_IJ (I before J) and the diagonal U_II."""
    _, pos = color_order(n)
    f = {key: b.copy() for key, b in blocks.items()}
    perm, _ = color_order(n)
    for i in perm:
        row = sorted(neighbours(n, i), key=lambda a: pos[a])
        for k in row:
            if pos[k] >= pos[i]:
                break
            f[(i, k)] = f[(i, k)] @ np.linalg.inv(f[(k, k)])
            for j in row:
                if pos[j] > pos[k] and (k, j) in f:
                    f[(i, j)] = f[(i, j)] - f[(i, k)] @ f[(k, j)]
    return f


def bilu0_solve(n, f, r):
    """z = (L U)^-1 r."""
    perm, pos = color_order(n)
    y = r.reshape(-1, 3).astype(np.result_type(r, 1.0)).copy()
    for i in perm:
        for k in neighbours(n, i):
            if pos[k] < pos[i]:
                y[i] -= f[(i, k)] @ y[k]
    z = y
    for i in perm[::-1]:
        t = z[i].copy()
        for j in neighbours(n, i):
            if pos[j] > pos[i]:
                t -= f[(i, j)] @ z[j]
        z[i] = np.linalg.solve(f[(i, i)], t)
    return z.ravel()


def bilu0_preconditioner(n, row_ptr, col_idx, vals):
    """r -> M^-1 r for the ILU(0) of the CSR matrix."""
    f = bilu0(n, csr_blocks(n, row_ptr, col_idx, vals))
    return lambda r: bilu0_solve(n, f, r)
