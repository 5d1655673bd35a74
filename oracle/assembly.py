"""Global assembly: vectors, COO -> sorted CSR, Dirichlet elimination (oracle).

Sec. III-B builds the global Jacobian by collecting every element's dense local
Jacobian with its global (row, col) indices, sorting the pairs and combining
duplicates into one sparse tuple whose size is known beforehand.  The reading
here: duplicates are summed (K = sum_e A_e^T K_e A_e, Sec. II-A), rows are dofs,
columns are sorted ascending within a row, and every (row, col) pair that some
element touches is kept even when its value is zero (structural pattern).

Dirichlet conditions (Sec. II-B mentions their treatment without a method) are
applied by symmetric elimination: constrained rows and columns are zeroed and
their diagonal set to 1, i.e. A = P_f K P_f + P_b.
"""
from __future__ import annotations

import numpy as np

from .mesh import element_dofs


def assemble_vector(conn, r_e, n_dof):
    """R = sum_e A_e^T r_e."""
    out = np.zeros(n_dof, dtype=np.result_type(r_e, np.float64))
    np.add.at(out, element_dofs(conn).ravel(), r_e.ravel())
    return out


def coo_from_elements(conn, k_e):
    """Unrolled (rows, cols, vals) of all element Jacobians, 576 per element."""
    dofs = element_dofs(conn)
    rows = np.repeat(dofs[:, :, None], 24, axis=2).ravel()
    cols = np.repeat(dofs[:, None, :], 24, axis=1).ravel()
    return rows, cols, k_e.ravel()


def coo_to_csr(rows, cols, vals, n_rows):
    """Sort (row, col) pairs, sum duplicates, return (row_ptr, col_idx, vals) int64/float64."""
    order = np.lexsort((cols, rows))
    r, c, v = rows[order], cols[order], vals[order]
    first = np.ones(len(r), dtype=bool)
    first[1:] = (r[1:] != r[:-1]) | (c[1:] != c[:-1])
    starts = np.flatnonzero(first)
    summed = np.add.reduceat(v, starts) if len(v) else v
    ur, uc = r[starts], c[starts]
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.add.at(row_ptr, ur + 1, 1)
    return np.cumsum(row_ptr), uc, summed


def assemble_csr(conn, k_e, n_dof):
    """Global sparse Jacobian in CSR from element Jacobians."""
    rows, cols, vals = coo_from_elements(conn, k_e)
    return coo_to_csr(rows, cols, vals, n_dof)


def csr_rows(row_ptr):
    """Row index of every stored entry."""
    return np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))


def csr_matvec(row_ptr, col_idx, vals, x):
    """y = K x for a CSR matrix."""
    return np.bincount(csr_rows(row_ptr), weights=vals * x[col_idx], minlength=len(row_ptr) - 1)


def csr_diagonal(row_ptr, col_idx, vals):
    rows = csr_rows(row_ptr)
    d = np.zeros(len(row_ptr) - 1)
    on = rows == col_idx
    d[rows[on]] = vals[on]
    return d


def dirichlet_csr(row_ptr, col_idx, vals, mask):
    """Symmetric elimination: zero constrained rows/cols, unit diagonal. Returns new vals."""
    rows = csr_rows(row_ptr)
    c = mask.astype(bool)
    out = vals.copy()
    out[c[rows] | c[col_idx]] = 0.0
    out[c[rows] & (rows == col_idx)] = 1.0
    return out
