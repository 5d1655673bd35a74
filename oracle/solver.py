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

Fig. 4 also runs GMRES and BiCGStab on the same systems; both are kept here for
nonsymmetric operators (right preconditioning, so the stopping test is on the
unpreconditioned residual like CG's).

Sec. V-B (Fig. 7) compares point Jacobi with stronger preconditioning of the
assembled matrix.  The first step beyond point Jacobi kept here is node-block
Jacobi: M = the 3x3 blocks of A that couple the three displacement components
of one node (zero elsewhere).
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


def matfree_node_blocks(conn, k_e, n_dof, mask=None):
    """The 3x3 diagonal blocks of the same operator, one per node: [n_nodes, 3, 3].

    Block of node a = sum over elements containing a of K_e restricted to a's
    three dofs.  Constrained dofs get a zero row and column and a 1 on the
    diagonal, as in A = P_f K P_f + P_b.
    """
    n_nodes = n_dof // 3
    blocks = np.zeros((n_nodes, 3, 3))
    for a in range(8):
        np.add.at(blocks, conn[:, a], k_e[:, 3 * a:3 * a + 3, 3 * a:3 * a + 3])
    if mask is not None:
        c = mask.astype(bool).reshape(n_nodes, 3)
        for i in range(3):
            blocks[c[:, i], i, :] = 0.0
            blocks[c[:, i], :, i] = 0.0
            blocks[c[:, i], i, i] = 1.0
    return blocks


def block_jacobi(blocks):
    """z = M^-1 r for the node-block preconditioner (one 3x3 solve per node)."""
    inv = np.linalg.inv(blocks)

    def apply(r):
        return np.einsum("nij,nj->ni", inv, r.reshape(-1, 3)).ravel()
    return apply


def pcg(apply_a, diag, b, rtol, max_it, precond=None):
    """Preconditioned CG. M^-1 r = r / diag (point Jacobi), or precond(r) when given
    (diag is then only checked for finiteness and may be None).
    Returns (x, iterations, status, true relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    minv = precond if precond is not None else (lambda v: v / diag)
    if not np.all(np.isfinite(b)) or (diag is not None and not np.all(np.isfinite(diag))):
        return x, 0, NONFINITE, np.nan
    if bnorm == 0.0:
        return x, 0, OK, 0.0
    z = minv(r)
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
        z = minv(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    true_rel = np.linalg.norm(b - apply_a(x)) / bnorm
    return x, it, status, true_rel


def bicgstab(apply_a, b, rtol, max_it, precond=None):
    """Right-preconditioned BiCGStab (van der Vorst 1992; Saad, Iterative Methods for
    Sparse Linear Systems, 2003, Alg. 7.7) for nonsymmetric operators, x0 = 0,
    shadow residual r_hat = r0.  Stops when ||r||_2 <= rtol ||b||_2 (checked on the
    half-step residual s as well).  One iteration = two operator applications.
    Returns (x, iterations, status, true relative residual)."""
    minv = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    if not np.all(np.isfinite(b)):
        return x, 0, NONFINITE, np.nan
    if bnorm == 0.0:
        return x, 0, OK, 0.0
    r_hat = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    status, it = NOT_CONVERGED, 0
    while it < max_it:
        rho = r_hat @ r
        if rho == 0.0 or omega == 0.0:
            status = BREAKDOWN
            break
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        p_hat = minv(p)
        v = apply_a(p_hat)
        rv = r_hat @ v
        if rv == 0.0 or not np.isfinite(rv):
            status = BREAKDOWN if np.isfinite(rv) else NONFINITE
            break
        alpha = rho / rv
        s = r - alpha * v
        it += 1
        if np.linalg.norm(s) <= rtol * bnorm:
            x += alpha * p_hat
            status = OK
            break
        s_hat = minv(s)
        t = apply_a(s_hat)
        tt = t @ t
        omega = (t @ s) / tt if tt > 0.0 else 0.0
        x += alpha * p_hat + omega * s_hat
        r = s - omega * t
        rho_old = rho
        if not np.all(np.isfinite(r)):
            status = NONFINITE
            break
        if np.linalg.norm(r) <= rtol * bnorm:
            status = OK
            break
    true_rel = np.linalg.norm(b - apply_a(x)) / bnorm
    return x, it, status, true_rel


def gmres(apply_a, b, rtol, max_it, restart=30, precond=None):
    """Right-preconditioned restarted GMRES(m) (Saad & Schultz 1986; Saad, Iterative
    Methods for Sparse Linear Systems, 2003, Alg. 6.9 with right preconditioning,
    Sec. 9.3.2), x0 = 0.  A cycle builds an orthonormal basis v_0..v_k of the Krylov
    space of A M^-1 from v_0 = r/||r|| by Arnoldi with modified Gram-Schmidt, reduces
    the Hessenberg matrix to triangular form with Givens rotations applied to
    g = ||r|| e_1, and stops when |g_{k}| (the residual norm of the least-squares
    iterate) <= rtol ||b||_2.  After m steps without convergence the iterate
    x += M^-1 V y (y from the triangular system) is formed and the cycle restarts
    from the true residual b - A x.  One iteration = one Arnoldi step (one operator
    application).  Returns (x, iterations, status, true relative residual)."""
    minv = precond if precond is not None else (lambda v: v)
    m = int(restart)
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if not np.all(np.isfinite(b)):
        return x, 0, NONFINITE, np.nan
    if bnorm == 0.0:
        return x, 0, OK, 0.0
    tol = rtol * bnorm
    it, status = 0, NOT_CONVERGED
    r = b.copy()
    while True:
        beta = np.linalg.norm(r)
        if beta <= tol:
            status = OK
            break
        if it >= max_it:
            break
        V = np.zeros((m + 1, b.size))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k, stop = 0, None
        for j in range(m):
            w = apply_a(minv(V[j]))
            for i in range(j + 1):          # modified Gram-Schmidt
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            h_next = np.linalg.norm(w)
            H[j + 1, j] = h_next
            if not np.isfinite(h_next):
                stop = NONFINITE
                break
            for i in range(j):              # earlier rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = np.hypot(H[j, j], H[j + 1, j])
            if rho == 0.0:                  # singular least-squares problem
                stop = BREAKDOWN
                break
            cs[j], sn[j] = H[j, j] / rho, H[j + 1, j] / rho
            H[j, j], H[j + 1, j] = rho, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            if abs(g[j + 1]) <= tol:
                stop = OK
                break
            if it >= max_it:
                stop = NOT_CONVERGED
                break
            V[j + 1] = w / h_next
        if k > 0:
            y = np.zeros(k)                 # back substitution on the triangular block
            for i in range(k - 1, -1, -1):
                y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
            x += minv(V[:k].T @ y)
        if stop is not None:
            status = stop
            break
        r = b - apply_a(x)
    true_rel = np.linalg.norm(b - apply_a(x)) / bnorm
    return x, it, status, true_rel
