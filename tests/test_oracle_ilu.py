"""Pins of the oracle's node-block ILU(0): the colouring is a proper colouring of the
block graph, ILU(0) is exact where the pattern has no fill (one element: all 8 nodes
coupled; a block-diagonal matrix), (L U)_IJ = A_IJ on the pattern (the definition of
ILU(0)), and for a symmetric matrix U_IJ = D_I L_JI^T (symmetric factorisation)."""
import numpy as np

from oracle import assembly, ilu, solver
from oracle.mesh import structured_hex8
from paper_2604_22087_amd import inputs


def _fe_csr(n, seed, mask=True):
    coords, conn = structured_hex8(n)
    rng = np.random.default_rng(seed)
    ndof = 3 * len(coords)
    k_e = np.empty((len(conn), 24, 24))
    for e in range(len(conn)):
        g = rng.normal(size=(24, 24))
        k_e[e] = g @ g.T / 24 + 0.5 * np.eye(24)
    rp, ci, v = assembly.assemble_csr(conn, k_e, ndof)
    if mask:
        v = assembly.dirichlet_csr(rp, ci, v, inputs.boundary_dof_mask(n))
    return rp, ci, v, ndof


def _dense(rp, ci, v, ndof):
    a = np.zeros((ndof, ndof))
    a[assembly.csr_rows(rp), ci] = v
    return a


def test_colouring_is_proper():
    n = 3
    for a in range((n + 1) ** 3):
        for b in ilu.neighbours(n, a):
            if b != a:
                assert ilu.node_color(n, a) != ilu.node_color(n, b)
    perm, pos = ilu.color_order(n)
    assert sorted(perm) == list(range((n + 1) ** 3)) and np.all(perm[pos] == np.arange(perm.size))
    assert all(ilu.node_color(n, perm[p]) <= ilu.node_color(n, perm[p + 1]) for p in range(perm.size - 1))


def test_ilu0_exact_without_fill():
    """One element couples all 8 nodes, so the block pattern is full and ILU(0) is LU;
    a block-diagonal matrix has nothing to fill either."""
    rp, ci, v, ndof = _fe_csr(1, seed=1, mask=False)
    a = _dense(rp, ci, v, ndof)
    r = np.random.default_rng(2).normal(size=ndof)
    z = ilu.bilu0_preconditioner(1, rp, ci, v)(r)
    assert np.linalg.norm(z - np.linalg.solve(a, r)) <= 1e-12 * np.linalg.norm(z)
    n = 2
    rng = np.random.default_rng(3)
    nn = (n + 1) ** 3
    blocks = {}
    for i in range(nn):
        for j in ilu.neighbours(n, i):
            g = rng.normal(size=(3, 3))
            blocks[(i, j)] = g @ g.T + 3 * np.eye(3) if i == j else np.zeros((3, 3))
    f = ilu.bilu0(n, blocks)
    r = rng.normal(size=3 * nn)
    z = ilu.bilu0_solve(n, f, r)
    want = np.concatenate([np.linalg.solve(blocks[(i, i)], r[3 * i:3 * i + 3]) for i in range(nn)])
    assert np.linalg.norm(z - want) <= 1e-13 * np.linalg.norm(want)


def test_ilu0_product_matches_matrix_on_pattern():
    n = 4  # 3^3 free nodes: not all pairs share an element, so ILU(0) drops fill
    rp, ci, v, ndof = _fe_csr(n, seed=4)
    a = _dense(rp, ci, v, ndof)
    f = ilu.bilu0(n, ilu.csr_blocks(n, rp, ci, v))
    _, pos = ilu.color_order(n)
    nn = (n + 1) ** 3
    L = np.eye(ndof)
    U = np.zeros((ndof, ndof))
    for (i, j), b in f.items():
        if pos[i] > pos[j]:
            L[3 * i:3 * i + 3, 3 * j:3 * j + 3] = b
        else:
            U[3 * i:3 * i + 3, 3 * j:3 * j + 3] = b
    lu = L @ U
    for i in range(nn):
        for j in ilu.neighbours(n, i):
            blk = (slice(3 * i, 3 * i + 3), slice(3 * j, 3 * j + 3))
            assert np.abs(lu[blk] - a[blk]).max() <= 1e-12 * np.abs(a).max()
    # the solve inverts L U exactly
    r = np.random.default_rng(5).normal(size=ndof)
    z = ilu.bilu0_solve(n, f, r)
    assert np.linalg.norm(lu @ z - r) <= 1e-12 * np.linalg.norm(r)
    # and L U differs from A (fill was dropped), so this is not an exact factorisation
    assert np.abs(lu - a).max() > 1e-6 * np.abs(a).max()


def test_ilu0_symmetric_factorisation():
    """For symmetric A the IKJ elimination keeps U_IJ = U_II L_JI^T."""
    n = 2
    rp, ci, v, ndof = _fe_csr(n, seed=6)
    f = ilu.bilu0(n, ilu.csr_blocks(n, rp, ci, v))
    _, pos = ilu.color_order(n)
    for (i, j), b in f.items():
        if pos[i] < pos[j]:
            assert np.abs(b - f[(i, i)] @ f[(j, i)].T).max() <= 1e-12 * max(1.0, np.abs(b).max())


def test_ilu0_preconditioned_gmres_solves():
    n = 4
    rp, ci, v, ndof = _fe_csr(n, seed=7)
    a = _dense(rp, ci, v, ndof)
    b = np.random.default_rng(8).normal(size=ndof) * (1 - inputs.boundary_dof_mask(n))
    pre = ilu.bilu0_preconditioner(n, rp, ci, v)
    x, it, st, rel = solver.gmres(lambda p: assembly.csr_matvec(rp, ci, v, p), b, 1e-13, 500, restart=30,
                                  precond=pre)
    d = assembly.csr_diagonal(rp, ci, v)
    _, it_j, _, _ = solver.gmres(lambda p: assembly.csr_matvec(rp, ci, v, p), b, 1e-13, 500, restart=30,
                                 precond=lambda r: r / d)
    assert st == solver.OK and rel <= 1e-13 and it < it_j
    assert np.linalg.norm(x - np.linalg.solve(a, b)) <= 1e-11 * np.linalg.norm(x)
