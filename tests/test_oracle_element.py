"""Pins of the oracle's element layer against closed forms and invariants.

Every expected value here comes from mathematics written independently of the
oracle's code: the partition of unity and Kronecker property of the trilinear
basis, the patch test, the trace of the brick stiffness (derived from 1-D
integrals of the linear basis), the rigid-body nullspace and finite differences.
"""
import numpy as np
import pytest

from oracle import element, elasticity, hex8, mesh

RNG = np.random.default_rng(123)
LAM_M, MU_M = 3.0246913580246906, 1.2962962962962963  # E = 3.5, nu = 0.35


def test_lame_values():
    lam, mu = elasticity.lame(3.5, 0.35)
    # lambda = E nu / ((1+nu)(1-2nu)) = 1.225 / 0.405, mu = 3.5 / 2.7
    assert lam == pytest.approx(1.225 / 0.405, rel=1e-15)
    assert mu == pytest.approx(3.5 / 2.7, rel=1e-15)
    lam_i, mu_i = elasticity.lame(70.0, 0.22)
    assert lam_i == pytest.approx(22.540983606557376, rel=1e-14)
    assert mu_i == pytest.approx(28.688524590163937, rel=1e-14)


def test_partition_of_unity_and_kronecker():
    for _ in range(10):
        xi = RNG.uniform(-1, 1, 3)
        assert hex8.shape_functions(xi).sum() == pytest.approx(1.0, abs=1e-15)
        assert np.abs(hex8.shape_gradients_ref(xi).sum(axis=0)).max() < 1e-15
    # N_a at node b equals delta_ab
    vals = np.array([hex8.shape_functions(x) for x in hex8.NODE_XI])
    assert np.array_equal(vals, np.eye(8))


def test_gradients_match_finite_differences():
    xi = RNG.uniform(-0.9, 0.9, 3)
    g = hex8.shape_gradients_ref(xi)
    h = 1e-6
    for k in range(3):
        d = np.zeros(3)
        d[k] = h
        fd = (hex8.shape_functions(xi + d) - hex8.shape_functions(xi - d)) / (2 * h)
        assert np.abs(fd - g[:, k]).max() < 1e-9


def _distorted_element():
    x = (hex8.NODE_XI + 1.0) / 2.0 * np.array([0.3, 0.2, 0.25])
    return x + RNG.uniform(-0.03, 0.03, x.shape)


@pytest.mark.parametrize("distorted", [False, True])
def test_patch_test_affine_fields(distorted):
    """u = G x reproduces eps = sym(G) exactly at every Gauss point (cube and distorted brick)."""
    xe = _distorted_element() if distorted else (hex8.NODE_XI + 1.0) / 16.0
    coords, conn = xe, np.arange(8)[None, :]
    for _ in range(6):
        G = RNG.normal(size=(3, 3))
        u = (xe @ G.T).ravel()
        eps = np.array([G[0, 0], G[1, 1], G[2, 2], G[1, 2] + G[2, 1], G[0, 2] + G[2, 0],
                        G[0, 1] + G[1, 0]])
        for e_q in element.qp_strains(coords, conn, u):
            assert np.abs(e_q[0] - eps).max() < 1e-12 * np.abs(G).max()


def test_element_volume_from_quadrature():
    xe = _distorted_element()
    pts, w = hex8.gauss_points()
    vol = sum(w[q] * hex8.physical_gradients(xe[None], pts[q])[1][0] for q in range(8))
    # volume of the trilinear brick from the divergence theorem: (1/3) sum over faces of x.n dA
    # -- here checked instead against a fine midpoint rule of detJ over the reference cube
    m = 24
    s = (np.arange(m) + 0.5) / m * 2 - 1
    fine = 0.0
    for a in s:
        for b in s:
            for c in s:
                fine += hex8.physical_gradients(xe[None], np.array([a, b, c]))[1][0]
    fine *= (2.0 / m) ** 3
    assert vol == pytest.approx(fine, rel=1e-3)


def test_cube_stiffness_trace_closed_form():
    """tr K_e = (lambda + 4 mu) * int sum_a |grad N_a|^2 = (8/3) h (lambda + 4 mu) for a cube."""
    for n in (1, 4, 8):
        coords, conn = mesh.structured_hex8(n)
        h = 1.0 / n
        _, k = element.linear_residual_tangent(coords, conn[:1], np.zeros(len(coords) * 3),
                                               [LAM_M], [MU_M])
        assert np.trace(k[0]) == pytest.approx(8.0 / 3.0 * h * (LAM_M + 4 * MU_M), rel=1e-14)
    assert 8.0 / 3.0 / 8 * (LAM_M + 4 * MU_M) == pytest.approx(2.736625514403292, rel=1e-14)


@pytest.mark.parametrize("distorted", [False, True])
def test_element_stiffness_symmetry_and_nullspace(distorted):
    xe = _distorted_element() if distorted else (hex8.NODE_XI + 1.0) / 16.0
    _, k = element.linear_residual_tangent(xe, np.arange(8)[None, :], np.zeros(24), [LAM_M], [MU_M])
    k = k[0]
    assert np.abs(k - k.T).max() <= 1e-14 * np.abs(k).max()
    ev = np.linalg.eigvalsh(k)
    assert np.sum(np.abs(ev) < 1e-12 * ev.max()) == 6
    assert np.sum(ev > 1e-9 * ev.max()) == 18
    # rigid modes: translations and infinitesimal rotations omega x x
    for t in np.eye(3):
        assert np.abs(k @ np.tile(t, 8)).max() < 1e-13 * np.abs(k).max()
    for w in np.eye(3):
        assert np.abs(k @ np.cross(w, xe).ravel()).max() < 1e-13 * np.abs(k).max()


def test_stiffness_linear_in_lame_parameters():
    xe = _distorted_element()
    c = np.arange(8)[None, :]
    z = np.zeros(24)
    k_l = element.linear_residual_tangent(xe, c, z, [1.0], [0.0])[1][0]
    k_m = element.linear_residual_tangent(xe, c, z, [0.0], [1.0])[1][0]
    k = element.linear_residual_tangent(xe, c, z, [LAM_M], [MU_M])[1][0]
    assert np.abs(k - (LAM_M * k_l + MU_M * k_m)).max() < 1e-14 * np.abs(k).max()


def test_residual_equals_stiffness_times_u():
    xe = _distorted_element()
    u = RNG.uniform(-1e-3, 1e-3, 24)
    r, k = element.linear_residual_tangent(xe, np.arange(8)[None, :], u, [LAM_M], [MU_M])
    assert np.abs(r[0] - k[0] @ u).max() < 1e-14 * np.abs(r).max() * 10
