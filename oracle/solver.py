"""Operators and the Jacobi-preconditioned conjugate-gradient solve (oracle).

Sec. III-A contrasts a matrix-free operator (the action y = K x evaluated
element by element, never forming K) with the matrix-explicit one (assembled
sparse K); Fig. 5 reports that both give the same solver behaviour.  Fig. 4 runs
conjugate gradients with a Jacobi preconditioner in double precision to a
relative residual tolerance.  The CG recursion is the textbook one
(Hestenes & Stiefel 1952; Saad, Iterative Methods for Sparse Linear Systems,
2003, Alg. 9.1): x0 = 0, r0 = b, z = M^-1 r, p = z; each iteration q = A p,
alpha = (r.z)/(p.q), x += alpha p, r -= alpha q, stop when ||r||_2 <= rtol ||b||_2,
z = M^-1 r, beta = (r.z)_new/(r.z)_old, p = z + beta p.  M = diag(A).
"""
from __future__ import annotations

import numpy as np

from .mesh import element_dofs

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE = "ok", "not_converged", "breakdown", "nonfinite"


def matfree_apply(conn, k_e, x, mask=None):
    """y = P_f (sum_e A_e^T K_e A_e) P_f x + P_b x, element by element.

    mask: uint8/bool per dof, 1 = constrained (None: no constraints).
    """
    dofs = element_dofs(conn)
    xf = x.copy()
    if mask is not None:
        xf[mask.astype(bool)] = 0.0
    ye = np.einsum("eij,ej->ei", k_e, xf[dofs])
    y = np.zeros_like(x)
    np.add.at(y, dofs.ravel(), ye.ravel())
    if mask is not None:
        c = mask.astype(bool)
        y[c] = x[c]
    return y


def matfree_diagonal(conn, k_e, n_dof, mask=None):
    """diag(A) of the same operator: sum of element diagonals, 1 on constrained dofs."""
    d = np.zeros(n_dof)
    np.add.at(d, element_dofs(conn).ravel(), np.einsum("eii->ei", k_e).ravel())
    if mask is not None:
        d[mask.astype(bool)] = 1.0
    return d


def pcg(apply_a, diag, b, rtol, max_it):
    """Jacobi-PCG. Returns (x, iterations, status, true relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    if not np.all(np.isfinite(b)) or not np.all(np.isfinite(diag)):
        return x, 0, NONFINITE, np.nan
    if bnorm == 0.0:
        return x, 0, OK, 0.0
    z = r / diag
    p = z.copy()
    rz = r @ z
    status, it = NOT_CONVERGED, 0
    while it < max_it:
        q = apply_a(p)
        pq = p @ q
        if not np.isfinite(pq):
            status = NONFINITE
            break
        if pq <= 0.0:
            status = BREAKDOWN
            break
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        if np.linalg.norm(r) <= rtol * bnorm:
            status = OK
            break
        z = r / diag
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    true_rel = np.linalg.norm(b - apply_a(x)) / bnorm
    return x, it, status, true_rel
