"""Pins of the oracle's Neo-Hookean law and finite-strain element.

Expected values: P = dW/dF by finite differences of the energy written from its
definition, A = dP/dF by finite differences, the uniaxial closed form
P_xx = mu(s - 1/s) + lam ln(s)/s, P_yy = lam ln(s), material frame indifference
P(QF) = Q P(F), reduction to linear elasticity at u = 0, the superposed
rotation identity K(u) (W x) = W R(u) and translation invariance.
"""
import numpy as np
import pytest

from oracle import assembly, element, neohooke
from oracle.elasticity import lame
from oracle.mesh import structured_hex8
from oracle.rve import RVE, phase_params

RNG = np.random.default_rng(21)
MU, LAM = 1.3, 1.95


def _W(F):
    # strain energy density from its definition (independent of the oracle's helper)
    C = F.T @ F
    J = np.linalg.det(F)
    return 0.5 * MU * (np.trace(C) - 3 - 2 * np.log(J)) + 0.5 * LAM * np.log(J) ** 2


def test_energy_helper_matches_definition():
    F = np.eye(3) + RNG.normal(scale=0.1, size=(3, 3))
    assert neohooke.energy(F[None], MU, LAM)[0] == pytest.approx(_W(F), rel=1e-14)


def test_stress_is_energy_gradient():
    H = RNG.normal(scale=0.15, size=(5, 3, 3))
    P, _ = neohooke.stress_tangent(H, MU, LAM)
    h = 1e-6
    for m in range(5):
        F = np.eye(3) + H[m]
        for i in range(3):
            for J in range(3):
                d = np.zeros((3, 3))
                d[i, J] = h
                fd = (_W(F + d) - _W(F - d)) / (2 * h)
                assert fd == pytest.approx(P[m, i, J], abs=1e-8)


def test_tangent_is_stress_gradient():
    H = RNG.normal(scale=0.15, size=(4, 3, 3))
    _, A = neohooke.stress_tangent(H, MU, LAM)
    h = 1e-7
    for k in range(3):
        for L in range(3):
            d = np.zeros((3, 3))
            d[k, L] = h
            fd = (neohooke.stress_tangent(H + d, MU, LAM)[0] - neohooke.stress_tangent(H - d, MU, LAM)[0]) / (2 * h)
            assert np.abs(fd - A[:, :, :, k, L]).max() < 1e-7


def test_uniaxial_closed_form_and_objectivity():
    for s in (0.8, 1.1, 1.5):
        H = np.diag([s - 1.0, 0.0, 0.0])[None]
        P, _ = neohooke.stress_tangent(H, MU, LAM)
        assert P[0, 0, 0] == pytest.approx(MU * (s - 1 / s) + LAM * np.log(s) / s, rel=1e-14)
        assert P[0, 1, 1] == pytest.approx(LAM * np.log(s), rel=1e-14, abs=1e-16)
    F = np.eye(3) + RNG.normal(scale=0.1, size=(3, 3))
    a = RNG.normal(size=3)
    a /= np.linalg.norm(a)
    th = 0.7
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    Q = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    P1, _ = neohooke.stress_tangent((F - np.eye(3))[None], MU, LAM)
    P2, _ = neohooke.stress_tangent((Q @ F - np.eye(3))[None], MU, LAM)
    assert np.abs(P2[0] - Q @ P1[0]).max() < 1e-14


def test_reduces_to_linear_elasticity_at_zero_displacement():
    coords, conn = structured_hex8(2)
    z = np.zeros(3 * len(coords))
    _, k_nh, _ = neohooke.residual_tangent(coords, conn, z, MU, LAM)
    _, k_lin = element.linear_residual_tangent(coords, conn, z, np.full(8, LAM), np.full(8, MU))
    assert np.abs(k_nh - k_lin).max() < 1e-14 * np.abs(k_lin).max()


def _nh_rve(n):
    E, nu = 2.6, 0.3  # mu = 1, lam = 1.5
    scale = np.random.default_rng(4).uniform(0.5, 2.0, n ** 3)
    return RVE(n, np.zeros(n ** 3, dtype=int), [phase_params("neohooke", E, nu)], scale=scale)


def test_global_tangent_fd_rotation_and_translation():
    n = 3
    rve = _nh_rve(n)
    u = (rve.coords @ np.diag([0.1, 0.0, -0.05]).T).ravel() + np.random.default_rng(5).uniform(-0.01, 0.01, rve.n_dof)
    r_e, k_e, _ = rve.element_residual_tangent(u)
    R = assembly.assemble_vector(rve.conn, r_e, rve.n_dof)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    w = RNG.normal(size=rve.n_dof)
    t = 1e-6
    fd = (rve.residual(u + t * w)[0] - rve.residual(u - t * w)[0]) / (2 * t)
    kv = assembly.csr_matvec(rp, ci, v, w)
    assert np.linalg.norm(fd - kv) <= 1e-7 * np.linalg.norm(kv)
    # superposed infinitesimal rotation of the current configuration: K (W x) = W R
    x_cur = rve.coords + u.reshape(-1, 3)
    for axis in np.eye(3):
        W = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
        lhs = assembly.csr_matvec(rp, ci, v, (x_cur @ W.T).ravel())
        rhs = (R.reshape(-1, 3) @ W.T).ravel()
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.abs(v).max() * np.linalg.norm(x_cur)
    for tr in np.eye(3):
        assert np.abs(assembly.csr_matvec(rp, ci, v, np.tile(tr, rve.n_dof // 3))).max() < 1e-12 * np.abs(v).max()


def test_homogeneous_stretch_newton():
    """Affine stretch of a homogeneous NH cube is the exact solution; P_xx from the closed form."""
    n = 2
    E, nu = 2.6, 0.3
    lam, mu = lame(E, nu)
    rve = RVE(n, np.zeros(n ** 3, dtype=int), [phase_params("neohooke", E, nu)])
    path = [np.diag([0.05 * k, 0.0, 0.0]) for k in range(1, 3)]
    u, _, hist = rve.newton(path, newton_rtol=1e-12, pcg_rtol=1e-14)
    s = 1.1
    assert np.abs(u - (rve.coords @ np.diag([0.1, 0, 0]).T).ravel()).max() < 1e-12
    assert hist[-1]["sigma_bar"][0] == pytest.approx(mu * (s - 1 / s) + lam * np.log(s) / s, rel=1e-12)
    assert hist[-1]["sigma_bar"][1] == pytest.approx(lam * np.log(s), rel=1e-12)
