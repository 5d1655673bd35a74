"""Pins of the oracle on general (distorted, renumbered) hex8 meshes.

The isoparametric element (oracle/hex8.py) and the sorted COO assembly (oracle/assembly.py)
are the definitions the general-mesh GPU path is checked against; on a distorted mesh with
random node and element numbering and randomly rotated local orders they must still
satisfy what the mathematics fixes:
  * the generated mesh fills the unit cube: sum of w detJ = 1, every detJ > 0;
  * patch test: an affine displacement u = E x gives eps = sym(E) at every Gauss point
    (trilinear elements reproduce linear fields exactly, whatever their shape);
  * an affine lift solves the homogeneous problem: P_f R(eps_bar x) = 0, and the solve
    returns u = eps_bar x (the exact solution lies in the FE space);
  * K is symmetric and annihilates the 3 translations and 3 infinitesimal rotations;
  * renumbering: the K of the renumbered mesh is the renumbered K of the plain one
    (so the sort-based assembly and the rotated local orders carry no hidden order);
  * CSR pattern: one 3x3 block per pair of nodes sharing an element, rows sorted.
"""
import numpy as np

from oracle import assembly, element
from oracle.elasticity import lame
from oracle.hex8 import gauss_points, physical_gradients
from oracle.rve import RVE, phase_params
from paper_2604_22087_amd import inputs


def _mesh(n=4, seed=7, permute=True):
    return inputs.distorted_cube_mesh(n, amplitude=0.25, seed=seed, permute=permute)


def test_mesh_fills_unit_cube():
    c, e = _mesh(5)
    pts, w = gauss_points()
    dets = np.stack([physical_gradients(c[e], pts[q])[1] for q in range(8)], axis=1)
    assert np.all(dets > 0)
    assert abs(dets.sum() - 1.0) < 1e-13
    # every node is used and every element has 8 distinct nodes
    assert set(np.unique(e)) == set(range(len(c)))
    assert all(len(set(row)) == 8 for row in e)


def test_patch_test_distorted():
    c, e = _mesh(4)
    rng = np.random.default_rng(11)
    E = rng.standard_normal((3, 3))
    u = (c @ E.T).ravel()
    eps = element.qp_strains(c, e, u)
    ex = np.array([E[0, 0], E[1, 1], E[2, 2], E[1, 2] + E[2, 1], E[0, 2] + E[2, 0], E[0, 1] + E[1, 0]])
    for q in range(8):
        assert np.max(np.abs(eps[q] - ex)) < 1e-13


def test_homogeneous_solve_exact_on_distorted_mesh():
    c, e = _mesh(4)
    rve = RVE(None, np.zeros(len(e), dtype=int), [phase_params("linear", 3.5, 0.35)], mesh=(c, e))
    eb = np.diag([0.01, -0.003, 0.002]) + 0.004 * (np.eye(3, k=1) + np.eye(3, k=-1))
    ex = (c @ eb.T).ravel()
    R, _ = rve.residual(ex)
    assert np.max(np.abs(R * rve.free)) < 1e-15
    u, info = rve.solve_linear(eb, rtol=1e-13)
    assert np.max(np.abs(u - ex)) < 1e-12
    lam, mu = lame(3.5, 0.35)
    r_e, _, trial = rve.element_residual_tangent(u)
    s = rve.mean_stress(trial["sigma_all"])
    tr = np.trace(eb)
    assert abs(s[0] - (lam * tr + 2 * mu * eb[0, 0])) < 1e-12
    assert abs(s[5] - 2 * mu * eb[0, 1]) < 1e-12


def test_stiffness_symmetry_and_rigid_modes():
    c, e = _mesh(3)
    ph = inputs.sphere_phase_mesh(c, e)
    rve = RVE(None, ph, [phase_params("linear", 3.5, 0.35), phase_params("linear", 70.0, 0.22)], mesh=(c, e))
    _, k_e, _ = rve.element_residual_tangent(np.zeros(rve.n_dof))
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    K = np.zeros((rve.n_dof, rve.n_dof))
    K[assembly.csr_rows(rp), ci] = v
    assert np.max(np.abs(K - K.T)) <= 1e-14 * np.max(np.abs(K))
    modes = []
    for d in range(3):
        t = np.zeros((len(c), 3))
        t[:, d] = 1
        modes.append(t.ravel())
    for w in np.eye(3):
        modes.append(np.cross(w, c).ravel())
    for m in modes:
        assert np.max(np.abs(K @ m)) <= 1e-13 * np.max(np.abs(K)) * np.max(np.abs(m))
    # exactly six zero eigenvalues
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == 6


def test_renumbering_is_a_permutation_of_K():
    """The same distorted mesh numbered two ways gives the same matrix up to renumbering."""
    n = 3
    c0, e0 = _mesh(n, seed=5, permute=False)
    rng = np.random.default_rng(3)
    perm = rng.permutation(len(c0))                  # new id of old node
    c1 = np.empty_like(c0)
    c1[perm] = c0
    e1 = perm[e0][rng.permutation(len(e0))]
    # rotate each element's local order by a cube rotation (node p -> node at R s_p)
    signs = 2 * inputs.LOCAL_CORNERS - 1
    rots = inputs._cube_rotations()
    rot_perm = np.array([[int(np.flatnonzero((signs == v).all(axis=1))[0]) for v in signs @ r.T] for r in rots])
    e1 = np.take_along_axis(e1, rot_perm[rng.integers(0, 24, len(e1))], axis=1)
    mats = []
    for c, e in ((c0, e0), (c1, e1)):
        rve = RVE(None, np.zeros(len(e), dtype=int), [phase_params("linear", 3.5, 0.35)], mesh=(c, e))
        _, k_e, _ = rve.element_residual_tangent(np.zeros(rve.n_dof))
        rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
        K = np.zeros((rve.n_dof, rve.n_dof))
        K[assembly.csr_rows(rp), ci] = v
        mats.append(K)
    dof_perm = (3 * perm[:, None] + np.arange(3)).ravel()   # new dof of old dof
    K0p = np.zeros_like(mats[0])
    K0p[np.ix_(dof_perm, dof_perm)] = mats[0]
    assert np.max(np.abs(K0p - mats[1])) <= 1e-13 * np.max(np.abs(mats[1]))


def test_csr_pattern_is_node_pair_blocks():
    c, e = _mesh(3)
    n_dof = 3 * len(c)
    k_e = np.ones((len(e), 24, 24))
    rp, ci, _ = assembly.assemble_csr(e, k_e, n_dof)
    # brute force: node pairs sharing an element
    pairs = set()
    for row in e:
        for a in row:
            for b in row:
                pairs.add((int(a), int(b)))
    expect = sorted((3 * a + i, 3 * b + k) for (a, b) in pairs for i in range(3) for k in range(3))
    got = list(zip(assembly.csr_rows(rp).tolist(), ci.tolist()))
    assert got == expect
