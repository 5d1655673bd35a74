"""Pins of the path-adjoint oracle (reaction work after a plastic load path).

The oracle's gradient is the complex step of the whole path.  Pinned by:
* the linear special case, where it must equal the closed-form adjoint
  gradient u_e^T K_hat_e u_e;
* central finite differences of the same path objective;
* complex-step derivatives of the return map itself against finite differences
  at plastic points (the branch tests must pass the perturbation through).
"""
import numpy as np

from oracle import adjoint as oadj
from oracle import j2
from oracle.rve import RVE, phase_params
from paper_2604_22087_amd import inputs

J2P = ("j2", 3.5, 0.35, 0.05, 0.1)


def _strain(xx, xy):
    return np.array([[xx, xy, 0.0], [xy, 0.0, 0.0], [0.0, 0.0, 0.0]])


# tension, then added shear, then partial unloading of the tension: the history matters
NONPROPORTIONAL = [_strain(0.012, 0.0), _strain(0.012, 0.008), _strain(0.004, 0.012)]


def _rve(n, phases, seed=4):
    phase = np.zeros(n ** 3, dtype=int)
    phase[n ** 3 // 2] = 1
    return RVE(n, phase, [phase_params(*p) for p in phases], scale=inputs.uniform_field(n ** 3, 0.8, 1.2, seed=seed))


def test_complex_step_equals_closed_form_linear():
    rve = _rve(3, [("linear", 3.5, 0.35), ("linear", 70.0, 0.22)])
    eb = np.diag([0.01, 0.0, 0.0])
    g_cs = oadj.path_gradient_complex_step(rve, [eb])
    u, _ = rve.solve_linear(eb, rtol=1e-14)
    g_ref, _ = oadj.gradient(rve, u, rtol=1e-14)
    assert np.abs(g_cs - g_ref).max() <= 1e-10 * np.abs(g_ref).max()


def test_complex_step_matches_finite_differences_plastic_path():
    rve = _rve(3, [J2P, ("linear", 230.0, 0.2)])
    path = NONPROPORTIONAL
    J, u = oadj.path_reaction_work(rve, path)
    # the path is plastic and its history matters
    _, _, tr = rve.element_residual_tangent(u, None)
    assert tr["plastic"].mean() > 0.2
    J_one_step, _ = oadj.path_reaction_work(rve, path[-1:])
    assert abs(J_one_step - J) > 1e-3 * abs(J)
    picks = [0, 4, 13, 17, 22, 26]
    g = oadj.path_gradient_complex_step(rve, path, elements=picks)
    s0 = rve.scale.copy()
    for k, e in enumerate(picks):
        h = 1e-5 * s0[e]
        rve.scale = s0.copy()
        rve.scale[e] += h
        jp = oadj.path_reaction_work(rve, path)[0]
        rve.scale = s0.copy()
        rve.scale[e] -= h
        jm = oadj.path_reaction_work(rve, path)[0]
        rve.scale = s0
        assert abs((jp - jm) / (2 * h) - g[k]) <= 1e-6 * abs(g[k])


def test_return_map_complex_step_at_plastic_points():
    rng = np.random.default_rng(3)
    m = 50
    eps = rng.normal(scale=0.02, size=(m, 6))
    epn = rng.normal(scale=2e-3, size=(m, 6))
    epn[:, 2] = -epn[:, 0] - epn[:, 1]
    an = rng.uniform(0, 2e-3, m)
    E, nu, sy, H = 3.5, 0.35, 0.05, 0.1
    base = j2.return_map(eps, epn, an, E, nu, sy, H)
    assert base["plastic"].mean() > 0.5
    for j in range(6):
        d = np.zeros(6)
        d[j] = 1.0
        cs = j2.return_map(eps + 1e-30j * d, epn, an, E, nu, sy, H)
        fp = j2.return_map(eps + 1e-7 * d, epn, an, E, nu, sy, H)
        fm = j2.return_map(eps - 1e-7 * d, epn, an, E, nu, sy, H)
        for key in ("sigma", "eps_p"):
            dcs = np.imag(cs[key]) / 1e-30
            dfd = (fp[key] - fm[key]) / 2e-7
            assert np.abs(dcs - dfd).max() <= 1e-6 * (np.abs(dfd).max() + 1e-12)
        # the consistent tangent is the derivative of the stress
        assert np.abs(np.imag(cs["sigma"]) / 1e-30 - base["D"][:, :, j]).max() <= 1e-10 * np.abs(base["D"]).max()
