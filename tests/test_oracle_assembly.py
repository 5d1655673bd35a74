"""Pins of the oracle's global assembly, operators and PCG.

Expected values: the closed-form structural pattern of the brick mesh, dense
assembly by explicit loops (brute force), the rigid-body nullspace, a dense
library solve on small meshes, and the Voigt/Reuss and Hill-Mandel identities
of the homogenisation problem.
"""
import numpy as np
import pytest

from oracle import assembly, element, elasticity, mesh, solver
from oracle.rve import RVE, phase_params
from paper_2604_22087_amd import inputs

RNG = np.random.default_rng(7)


def _lin_phases():
    return [phase_params("linear", 3.5, 0.35), phase_params("linear", 70.0, 0.22)]


def _two_phase_tangents(n, seed=0):
    coords, conn = mesh.structured_hex8(n)
    lam = np.random.default_rng(seed).uniform(1, 5, n ** 3)
    mu = np.random.default_rng(seed + 1).uniform(1, 5, n ** 3)
    _, k = element.linear_residual_tangent(coords, conn, np.zeros(3 * len(coords)), lam, mu)
    return coords, conn, k


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_csr_pattern_closed_form(n):
    coords, conn, k = _two_phase_tangents(n)
    rp, ci, _ = assembly.assemble_csr(conn, k, 3 * len(coords))
    assert len(ci) == 9 * (3 * n + 1) ** 3
    # row length = 3 * prod over axes of (2 on a face, 3 inside)
    idx = np.arange(n + 1)
    c1 = np.where((idx == 0) | (idx == n), 2, 3)
    lens = np.array([3 * c1[i] * c1[j] * c1[kk] for kk in range(n + 1) for j in range(n + 1)
                     for i in range(n + 1)])
    assert np.array_equal(np.diff(rp), np.repeat(lens, 3))
    for r in range(len(rp) - 1):
        cols = ci[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cols) > 0)
    # pattern symmetric
    rows = assembly.csr_rows(rp)
    a = set(zip(rows.tolist(), ci.tolist()))
    assert all((c, r) in a for r, c in a)


@pytest.mark.parametrize("n", [1, 2])
def test_csr_equals_brute_force_dense(n):
    coords, conn, k = _two_phase_tangents(n, seed=3)
    ndof = 3 * len(coords)
    dense = np.zeros((ndof, ndof))
    for e in range(len(conn)):
        for a in range(8):
            for i in range(3):
                for b in range(8):
                    for j in range(3):
                        dense[3 * conn[e, a] + i, 3 * conn[e, b] + j] += k[e, 3 * a + i, 3 * b + j]
    rp, ci, v = assembly.assemble_csr(conn, k, ndof)
    back = np.zeros((ndof, ndof))
    back[assembly.csr_rows(rp), ci] = v
    assert np.abs(back - dense).max() <= 1e-14 * np.abs(dense).max()


def test_global_symmetry_nullspace_and_matfree():
    n = 4
    coords, conn, k = _two_phase_tangents(n, seed=5)
    ndof = 3 * len(coords)
    rp, ci, v = assembly.assemble_csr(conn, k, ndof)
    dense = np.zeros((ndof, ndof))
    dense[assembly.csr_rows(rp), ci] = v
    kmax = np.abs(dense).max()
    assert np.abs(dense - dense.T).max() <= 1e-14 * kmax
    for t in np.eye(3):
        assert np.abs(assembly.csr_matvec(rp, ci, v, np.tile(t, len(coords)))).max() < 1e-12 * kmax
    for w in np.eye(3):
        assert np.abs(assembly.csr_matvec(rp, ci, v, np.cross(w, coords).ravel())).max() < 1e-12 * kmax
    x = RNG.normal(size=ndof)
    y_csr = assembly.csr_matvec(rp, ci, v, x)
    y_mf = solver.matfree_apply(conn, k, x)
    assert np.linalg.norm(y_csr - y_mf) <= 1e-14 * np.linalg.norm(y_csr)
    # masked operator: csr with symmetric elimination == matrix-free with mask
    mask = inputs.boundary_dof_mask(n)
    vb = assembly.dirichlet_csr(rp, ci, v, mask)
    y1 = assembly.csr_matvec(rp, ci, vb, x)
    y2 = solver.matfree_apply(conn, k, x, mask)
    assert np.linalg.norm(y1 - y2) <= 1e-14 * np.linalg.norm(y1)
    assert np.array_equal(assembly.csr_diagonal(rp, ci, vb), solver.matfree_diagonal(conn, k, ndof, mask)) or \
        np.abs(assembly.csr_diagonal(rp, ci, vb) - solver.matfree_diagonal(conn, k, ndof, mask)).max() < 1e-13 * kmax


def test_linear_residual_is_stiffness_times_u():
    n = 3
    ph = inputs.sphere_phase(n, 0.3)
    rve = RVE(n, ph, _lin_phases())
    u = RNG.uniform(-1e-3, 1e-3, rve.n_dof)
    r_e, k_e, _ = rve.element_residual_tangent(u)
    R = assembly.assemble_vector(rve.conn, r_e, rve.n_dof)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    assert np.linalg.norm(R - assembly.csr_matvec(rp, ci, v, u)) <= 1e-14 * np.linalg.norm(R) * 10


@pytest.mark.parametrize("n", [2, 3])
def test_pcg_matches_dense_solve(n):
    coords, conn, k = _two_phase_tangents(n, seed=11)
    ndof = 3 * len(coords)
    mask = inputs.boundary_dof_mask(n)
    rp, ci, v = assembly.assemble_csr(conn, k, ndof)
    vb = assembly.dirichlet_csr(rp, ci, v, mask)
    dense = np.zeros((ndof, ndof))
    dense[assembly.csr_rows(rp), ci] = vb
    b = RNG.normal(size=ndof) * (1 - mask)
    x_ref = np.linalg.solve(dense, b)
    x, it, status, rel = solver.pcg(lambda p: assembly.csr_matvec(rp, ci, vb, p),
                                    assembly.csr_diagonal(rp, ci, vb), b, 1e-14, 1000)
    assert status == solver.OK and rel <= 1e-13
    assert np.linalg.norm(x - x_ref) <= 1e-12 * np.linalg.norm(x_ref)


def test_pcg_error_paths():
    a = np.array([[2.0, 0.0], [0.0, -1.0]])
    b = np.array([0.0, 1.0])
    _, _, status, _ = solver.pcg(lambda p: a @ p, np.array([2.0, 1.0]), b, 1e-12, 10)
    assert status == solver.BREAKDOWN
    _, _, status, _ = solver.pcg(lambda p: a @ p, np.array([2.0, 1.0]), np.array([np.nan, 1.0]), 1e-12, 10)
    assert status == solver.NONFINITE
    spd = np.array([[4.0, 1.0, 0.0], [1.0, 3.0, 1.0], [0.0, 1.0, 2.0]])
    _, it, status, _ = solver.pcg(lambda p: spd @ p, np.diag(spd), np.ones(3), 1e-14, 1)
    assert status == solver.NOT_CONVERGED and it == 1


def test_homogeneous_rve_closed_form():
    """Equal phases: the affine field is the exact solution, C_app = lambda + 2 mu."""
    n = 4
    rve = RVE(n, inputs.sphere_phase(n), [phase_params("linear", 3.5, 0.35)] * 2)
    eb = np.diag([0.01, 0.0, 0.0])
    u_aff = (rve.coords @ eb.T).ravel()
    R, _ = rve.residual(u_aff)
    assert np.abs(R * rve.free).max() < 1e-15
    u, info = rve.solve_linear(eb, rtol=1e-13)
    assert np.abs(u - u_aff).max() < 1e-15
    r_e, k_e, _ = rve.element_residual_tangent(u)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    capp = u @ assembly.csr_matvec(rp, ci, v, u) / 0.01 ** 2
    assert capp == pytest.approx(5.617283950617283, rel=1e-13)


def test_config1_bounds_and_hill_mandel():
    """8^3 sphere RVE: Reuss <= C_app <= Voigt and u.Ku / V = sigma_bar_xx eps_xx."""
    n = 8
    phase = inputs.sphere_phase(n)
    assert phase.sum() == 56
    rve = RVE(n, phase, _lin_phases())
    exx = 0.01
    for op in ("csr", "matfree"):
        u, info = rve.solve_linear(np.diag([exx, 0, 0]), rtol=1e-13, op=op)
        assert info["status"] == "ok" and info["true_relres"] < 1e-12
        r_e, k_e, trial = rve.element_residual_tangent(u)
        rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
        energy = u @ assembly.csr_matvec(rp, ci, v, u)
        capp = energy / exx ** 2
        phi = 56 / 512
        cm = elasticity.hooke_voigt(*elasticity.lame(3.5, 0.35))
        ci_ = elasticity.hooke_voigt(*elasticity.lame(70.0, 0.22))
        voigt = (phi * ci_ + (1 - phi) * cm)[0, 0]
        reuss = np.linalg.inv(phi * np.linalg.inv(ci_) + (1 - phi) * np.linalg.inv(cm))[0, 0]
        assert voigt == pytest.approx(13.743928354584092, rel=1e-14)
        assert reuss < capp < voigt
        sbar = rve.mean_stress(trial["sigma_all"])
        assert energy == pytest.approx(sbar[0] * exx, rel=1e-9)


@pytest.mark.parametrize("n", [2, 3])
def test_node_blocks_equal_dense_blocks(n):
    """Node blocks of the element-by-element operator = 3x3 diagonal blocks read off
    the assembled, Dirichlet-eliminated dense matrix."""
    coords, conn, k = _two_phase_tangents(n, seed=3)
    ndof = 3 * len(coords)
    mask = inputs.boundary_dof_mask(n)
    rp, ci, v = assembly.assemble_csr(conn, k, ndof)
    vb = assembly.dirichlet_csr(rp, ci, v, mask)
    dense = np.zeros((ndof, ndof))
    dense[assembly.csr_rows(rp), ci] = vb
    blocks = solver.matfree_node_blocks(conn, k, ndof, mask)
    for a in range(len(coords)):
        assert np.abs(blocks[a] - dense[3 * a:3 * a + 3, 3 * a:3 * a + 3]).max() <= 1e-14 * np.abs(dense).max()


def test_block_jacobi_pcg_special_cases():
    """(i) a block-diagonal SPD matrix is solved exactly in one iteration;
    (ii) with diagonal blocks the iterates equal point-Jacobi PCG;
    (iii) on the config-1 problem it converges to the dense solution."""
    rng = np.random.default_rng(5)
    nb = 7
    g = rng.normal(size=(nb, 3, 3))
    blocks = np.einsum("nij,nkj->nik", g, g) + 3 * np.eye(3)
    dense = np.zeros((3 * nb, 3 * nb))
    for a in range(nb):
        dense[3 * a:3 * a + 3, 3 * a:3 * a + 3] = blocks[a]
    b = rng.normal(size=3 * nb)
    x, it, status, rel = solver.pcg(lambda p: dense @ p, None, b, 1e-14, 10, precond=solver.block_jacobi(blocks))
    assert status == solver.OK and it == 1 and rel <= 1e-14
    spd = rng.normal(size=(3 * nb, 3 * nb))
    spd = spd @ spd.T + 3 * nb * np.eye(3 * nb)
    dg = np.diag(spd).copy()
    diag_blocks = np.zeros((nb, 3, 3))
    for a in range(nb):
        diag_blocks[a] = np.diag(dg[3 * a:3 * a + 3])
    for max_it in (1, 2, 5):
        x1, _, _, _ = solver.pcg(lambda p: spd @ p, dg, b, 1e-30, max_it)
        x2, _, _, _ = solver.pcg(lambda p: spd @ p, None, b, 1e-30, max_it, precond=solver.block_jacobi(diag_blocks))
        assert np.abs(x1 - x2).max() <= 1e-13 * np.abs(x1).max()
    n = 3
    coords, conn, k = _two_phase_tangents(n, seed=11)
    ndof = 3 * len(coords)
    mask = inputs.boundary_dof_mask(n)
    rp, ci, v = assembly.assemble_csr(conn, k, ndof)
    vb = assembly.dirichlet_csr(rp, ci, v, mask)
    dense = np.zeros((ndof, ndof))
    dense[assembly.csr_rows(rp), ci] = vb
    b = RNG.normal(size=ndof) * (1 - mask)
    x_ref = np.linalg.solve(dense, b)
    pre = solver.block_jacobi(solver.matfree_node_blocks(conn, k, ndof, mask))
    x, it, status, rel = solver.pcg(lambda p: solver.matfree_apply(conn, k, p, mask), None, b, 1e-14, 1000, precond=pre)
    assert status == solver.OK and rel <= 1e-13
    assert np.linalg.norm(x - x_ref) <= 1e-12 * np.linalg.norm(x_ref)


def test_bicgstab_nonsymmetric_and_spd():
    """BiCGStab against a dense library solve: a nonsymmetric diagonally dominant
    matrix (with and without Jacobi preconditioning) and the SPD config-1-type
    operator, where it must reach the same solution as CG."""
    rng = np.random.default_rng(9)
    m = 60
    a = rng.normal(size=(m, m)) + 12.0 * np.eye(m)
    b = rng.normal(size=m)
    x_ref = np.linalg.solve(a, b)
    for pre in (None, lambda v: v / np.diag(a)):
        x, it, status, rel = solver.bicgstab(lambda v: a @ v, b, 1e-13, 500, precond=pre)
        assert status == solver.OK and rel <= 1e-12
        assert np.linalg.norm(x - x_ref) <= 1e-11 * np.linalg.norm(x_ref)
    n = 3
    coords, conn, k = _two_phase_tangents(n, seed=11)
    ndof = 3 * len(coords)
    mask = inputs.boundary_dof_mask(n)
    rp, ci, v = assembly.assemble_csr(conn, k, ndof)
    vb = assembly.dirichlet_csr(rp, ci, v, mask)
    dense = np.zeros((ndof, ndof))
    dense[assembly.csr_rows(rp), ci] = vb
    b = RNG.normal(size=ndof) * (1 - mask)
    d = assembly.csr_diagonal(rp, ci, vb)
    x, it, status, rel = solver.bicgstab(lambda p: assembly.csr_matvec(rp, ci, vb, p), b, 1e-14, 1000,
                                         precond=lambda r: r / d)
    assert status == solver.OK and rel <= 1e-13
    assert np.linalg.norm(x - np.linalg.solve(dense, b)) <= 1e-12 * np.linalg.norm(x)
