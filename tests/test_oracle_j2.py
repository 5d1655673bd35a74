"""Pins of the oracle's J2 return map and Newton load stepping.

Expected values: the uniaxial-strain closed form of linear-hardening J2
(yield strain sigma_y/2G, plastic multiplier, stresses and the algorithmic
modulus K + 4GH/(3(3G+H))), path independence under proportional loading,
finite differences of the return map and of the global residual.
"""
import numpy as np
import pytest

from oracle import assembly, j2
from oracle.elasticity import bulk_shear
from oracle.rve import RVE, phase_params

E, NU, SY, H = 3.5, 0.35, 0.05, 0.1
K, G = bulk_shear(E, NU)
RNG = np.random.default_rng(99)


def _uni(e):
    return np.array([[e, 0, 0, 0, 0, 0]], dtype=float)


def test_moduli():
    assert K == pytest.approx(3.5 / 0.9, rel=1e-15)
    assert G == pytest.approx(3.5 / 2.7, rel=1e-15)


def test_uniaxial_closed_form_single_point():
    ey = SY / (2 * G)
    assert ey == pytest.approx(0.019285714285714288, rel=1e-14)
    rm = j2.return_map(_uni(0.999 * ey), np.zeros((1, 6)), np.zeros(1), E, NU, SY, H)
    assert not rm["plastic"][0]
    assert rm["sigma"][0, 0] == pytest.approx((K + 4 * G / 3) * 0.999 * ey, rel=1e-14)
    for e in (0.02, 0.05):
        rm = j2.return_map(_uni(e), np.zeros((1, 6)), np.zeros(1), E, NU, SY, H)
        a = (2 * G * e - SY) / (3 * G + H)
        assert rm["plastic"][0]
        assert rm["alpha"][0] == pytest.approx(a, rel=1e-13)
        assert rm["sigma"][0, 0] == pytest.approx(K * e + 2 / 3 * (SY + H * a), rel=1e-13)
        assert rm["sigma"][0, 1] == pytest.approx(K * e - 1 / 3 * (SY + H * a), rel=1e-13)
        assert rm["sigma"][0, 2] == pytest.approx(K * e - 1 / 3 * (SY + H * a), rel=1e-13)
        # algorithmic modulus in the loading direction
        assert rm["D"][0, 0, 0] == pytest.approx(K + 4 * G * H / (3 * (3 * G + H)), rel=1e-12)
    a02 = (2 * G * 0.02 - SY) / (3 * G + H)
    assert a02 == pytest.approx(4.642526e-4, rel=1e-6)
    assert K + 4 * G * H / (3 * (3 * G + H)) == pytest.approx(3.932219127205199, rel=1e-14)


def test_plastic_state_consistency():
    """After return the stress lies on the updated yield surface and eps_p is deviatoric."""
    eps = RNG.normal(scale=0.015, size=(200, 6))
    epn = RNG.normal(scale=0.005, size=(200, 6))
    epn[:, 2] = -epn[:, 0] - epn[:, 1]
    an = RNG.uniform(0, 0.01, 200)
    rm = j2.return_map(eps, epn, an, E, NU, SY, H)
    s = j2.strain_to_tensor(np.concatenate([rm["sigma"][:, :3], 2 * rm["sigma"][:, 3:]], 1))
    dev = s - np.trace(s, axis1=1, axis2=2)[:, None, None] / 3 * np.eye(3)
    q = np.sqrt(1.5 * np.sum(dev * dev, axis=(1, 2)))
    pl = rm["plastic"]
    assert pl.sum() > 50 and (~pl).sum() > 10
    assert np.abs(q[pl] - (SY + H * rm["alpha"][pl])).max() < 1e-13
    assert np.all(q[~pl] <= SY + H * an[~pl] + 1e-15)
    assert np.abs(rm["eps_p"][:, :3].sum(1)).max() < 1e-15


def test_consistent_tangent_matches_finite_differences():
    eps = RNG.normal(scale=0.03, size=(50, 6))
    epn = np.zeros((50, 6))
    an = np.zeros(50)
    rm = j2.return_map(eps, epn, an, E, NU, SY, H)
    h = 1e-7
    for j in range(6):
        d = np.zeros(6)
        d[j] = h
        sp = j2.return_map(eps + d, epn, an, E, NU, SY, H)["sigma"]
        sm = j2.return_map(eps - d, epn, an, E, NU, SY, H)["sigma"]
        fd = (sp - sm) / (2 * h)
        assert np.abs(fd - rm["D"][:, :, j]).max() < 1e-6
    assert np.abs(rm["D"] - rm["D"].transpose(0, 2, 1)).max() < 1e-13


def test_path_independence_homogeneous_rve():
    """Proportional uniaxial loading: 1 step == 10 steps, matches the closed form."""
    n = 2
    rve = RVE(n, np.zeros(n ** 3, dtype=int), [phase_params("j2", E, NU, SY, H)])
    path = [np.diag([e, 0, 0]) for e in np.linspace(0.005, 0.05, 10)]
    _, st10, h10 = rve.newton(path, newton_rtol=1e-13, pcg_rtol=1e-15)
    _, st1, h1 = rve.newton([np.diag([0.05, 0, 0])], newton_rtol=1e-13, pcg_rtol=1e-15)
    a = (2 * G * 0.05 - SY) / (3 * G + H)
    for h, st in ((h10, st10), (h1, st1)):
        assert np.abs(st["alpha"] - a).max() < 1e-12
        assert h[-1]["sigma_bar"][0] == pytest.approx(K * 0.05 + 2 / 3 * (SY + H * a), rel=1e-12)
    assert np.abs(h10[-1]["sigma_bar"] - h1[-1]["sigma_bar"]).max() < 1e-12


def test_global_tangent_matches_residual_finite_difference():
    """K(u) v == (R(u + t v) - R(u - t v)) / 2t in a plastic two-phase state."""
    n = 3
    phase = np.zeros(n ** 3, dtype=int)
    phase[::4] = 1
    rve = RVE(n, phase, [phase_params("j2", E, NU, SY, H), phase_params("linear", 230.0, 0.2)])
    u = rve.affine_lift(np.diag([0.03, 0, 0])) + RNG.uniform(-1e-3, 1e-3, rve.n_dof)
    st = rve.zero_state()
    st["alpha"][:] = RNG.uniform(0, 1e-3, st["alpha"].shape)
    r_e, k_e, trial = rve.element_residual_tangent(u, st)
    assert trial["plastic"].mean() > 0.3
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    w = RNG.normal(size=rve.n_dof)
    t = 1e-7 * np.linalg.norm(u) / np.linalg.norm(w)
    rp_, _ = rve.residual(u + t * w, st)
    rm_, _ = rve.residual(u - t * w, st)
    fd = (rp_ - rm_) / (2 * t)
    kv = assembly.csr_matvec(rp, ci, v, w)
    assert np.linalg.norm(fd - kv) <= 1e-6 * np.linalg.norm(kv)


def test_newton_quadratic_convergence_fiber_rve():
    n = 4
    phase = np.zeros(n ** 3, dtype=int)
    phase[n * n:2 * n * n] = 1
    rve = RVE(n, phase, [phase_params("j2", E, NU, SY, H), phase_params("linear", 230.0, 0.2)])
    path = [np.diag([0.002 * k, 0, 0]) for k in range(1, 11)]
    u, st, hist = rve.newton(path)
    last = hist[-1]
    assert last["plastic_fraction"] > 0.1
    res = last["residuals"]
    assert res[-1] <= 1e-8 * res[0]
    assert len(res) <= 8
    # the unconstrained tangent at the converged state still annihilates translations
    r_e, k_e, _ = rve.element_residual_tangent(u, st)
    rp, ci, v = assembly.assemble_csr(rve.conn, k_e, rve.n_dof)
    for tr in np.eye(3):
        assert np.abs(assembly.csr_matvec(rp, ci, v, np.tile(tr, rve.n_dof // 3))).max() < 1e-12 * np.abs(v).max()
