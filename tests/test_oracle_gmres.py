"""Pins of the oracle's restarted GMRES against what fixes it independently:
the minimal-residual property over the Krylov space (brute-force least squares on
an explicit Krylov basis), finite termination with few distinct eigenvalues,
GMRES(1) = the minimal-residual iteration (closed-form step length), dense solves,
and the trivial cases."""
import numpy as np

from oracle import assembly, solver
from oracle.mesh import structured_hex8
from paper_2604_22087_amd import inputs

RNG = np.random.default_rng(31)


def _nonsym(n, shift, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, n)) + shift * np.eye(n)


def test_gmres_minimal_residual_over_krylov_space():
    """x_k minimises ||b - A x|| over x in M^-1 K_k(A M^-1, b), for every k (no restart)."""
    n = 30
    a = _nonsym(n, 4.0, 1)
    d = np.abs(np.diag(a)) + 1.0
    b = RNG.normal(size=n)
    am = lambda v: a @ (v / d)
    for k in range(1, 9):
        x, it, status, _ = solver.gmres(lambda v: a @ v, b, 0.0, k, restart=50, precond=lambda v: v / d)
        assert it == k and status == solver.NOT_CONVERGED
        kry = np.empty((n, k))
        kry[:, 0] = b
        for i in range(1, k):
            kry[:, i] = am(kry[:, i - 1])
        q, _ = np.linalg.qr(kry)
        y = np.linalg.lstsq(np.column_stack([am(q[:, i]) for i in range(k)]), b, rcond=None)[0]
        x_bf = (q @ y) / d
        r_bf = np.linalg.norm(b - a @ x_bf)
        assert abs(np.linalg.norm(b - a @ x) - r_bf) <= 1e-10 * np.linalg.norm(b)
        assert np.linalg.norm(x - x_bf) <= 1e-8 * np.linalg.norm(x_bf)


def test_gmres_finite_termination():
    """A diagonalisable matrix with 5 distinct eigenvalues: the minimal polynomial has
    degree 5, so unrestarted GMRES is exact after 5 steps."""
    n = 40
    s = np.eye(n) + 0.3 * RNG.normal(size=(n, n)) / np.sqrt(n)
    lam = np.repeat([1.0, 2.5, -3.0, 7.0, 0.5], n // 5)
    a = s @ np.diag(lam) @ np.linalg.inv(s)
    b = RNG.normal(size=n)
    x, it, status, rel = solver.gmres(lambda v: a @ v, b, 1e-10, 100, restart=n)
    assert status == solver.OK and it == 5 and rel <= 1e-10
    assert np.linalg.norm(x - np.linalg.solve(a, b)) <= 1e-9 * np.linalg.norm(x)


def test_gmres1_is_the_minimal_residual_iteration():
    """GMRES(1): each cycle is one step x += alpha r with alpha = (r, A r) / (A r, A r)."""
    n = 25
    a = _nonsym(n, 8.0, 2)
    b = RNG.normal(size=n)
    x_mr = np.zeros(n)
    for _ in range(6):
        r = b - a @ x_mr
        ar = a @ r
        x_mr = x_mr + (r @ ar) / (ar @ ar) * r
    x, it, status, _ = solver.gmres(lambda v: a @ v, b, 0.0, 6, restart=1)
    assert it == 6 and status == solver.NOT_CONVERGED
    assert np.linalg.norm(x - x_mr) <= 1e-12 * np.linalg.norm(x_mr)


def test_gmres_restarted_against_dense_solves():
    """Restarted GMRES reaches the dense solution: a nonsymmetric diagonally dominant
    matrix (with and without Jacobi), and the Dirichlet-eliminated two-phase FE operator
    with point Jacobi (SPD, where CG reaches the same solution)."""
    m = 60
    a = _nonsym(m, 12.0, 3)
    b = RNG.normal(size=m)
    x_ref = np.linalg.solve(a, b)
    for pre in (None, lambda v: v / np.diag(a)):
        for restart in (5, 30):
            x, it, status, rel = solver.gmres(lambda v: a @ v, b, 1e-13, 2000, restart=restart, precond=pre)
            assert status == solver.OK and rel <= 1e-12
            assert np.linalg.norm(x - x_ref) <= 1e-11 * np.linalg.norm(x_ref)
    n = 3
    coords, conn = structured_hex8(n)
    rng = np.random.default_rng(4)
    ndof = 3 * len(coords)
    k_e = np.empty((len(conn), 24, 24))
    for e in range(len(conn)):
        g = rng.normal(size=(24, 24))
        k_e[e] = g @ g.T / 24 + np.eye(24)
    mask = inputs.boundary_dof_mask(n)
    rp, ci, v = assembly.assemble_csr(conn, k_e, ndof)
    vb = assembly.dirichlet_csr(rp, ci, v, mask)
    dense = np.zeros((ndof, ndof))
    dense[assembly.csr_rows(rp), ci] = vb
    b = RNG.normal(size=ndof) * (1 - mask)
    dg = assembly.csr_diagonal(rp, ci, vb)
    x, it, status, rel = solver.gmres(lambda p: assembly.csr_matvec(rp, ci, vb, p), b, 1e-13, 2000, restart=20,
                                      precond=lambda r: r / dg)
    assert status == solver.OK and rel <= 1e-13
    assert np.linalg.norm(x - np.linalg.solve(dense, b)) <= 1e-11 * np.linalg.norm(x)


def test_gmres_trivial_cases():
    n = 12
    x, it, status, rel = solver.gmres(lambda v: v, np.zeros(n), 1e-10, 10)
    assert it == 0 and status == solver.OK and not x.any()
    b = RNG.normal(size=n)
    x, it, status, rel = solver.gmres(lambda v: v, b, 1e-12, 10)
    assert it == 1 and status == solver.OK and np.allclose(x, b, rtol=1e-14)
    x, it, status, _ = solver.gmres(lambda v: 2 * v, b, 1e-12, 0)
    assert it == 0 and status == solver.NOT_CONVERGED and not x.any()
