"""Pins of the surrogate constitutive logic: with the exact return map standing in
for the network (same normalised Mandel interface), the surrogate update must
reproduce the return map's stress, consistent tangent, plastic strain and
hardening variable, with a zero local residual; a network that is 1% off must
be rejected by the fallback test."""
import numpy as np
import pytest

from oracle import j2, surrogate

E, NU, SY, H = 3.5, 0.35, 0.05, 0.1
S_IN, S_OUT = SY / E, SY
RNG = np.random.default_rng(12)


def exact_net(x):
    eps_tr = x[:, :6] * S_IN * surrogate.SHEAR          # Mandel -> engineering Voigt
    epn = x[:, 6:12] * S_IN * surrogate.SHEAR
    an = x[:, 12] * S_IN
    rm = j2.return_map(eps_tr + epn, epn, an, E, NU, SY, H)
    y = surrogate.stress_voigt_to_mandel(rm["sigma"]) / S_OUT
    jac = (S_IN / S_OUT) * rm["D"] * surrogate.SHEAR[None, :, None] * surrogate.SHEAR[None, None, :]
    return y, jac


def _points(m=300):
    eps = RNG.normal(scale=0.02, size=(m, 6))
    epn = RNG.normal(scale=0.004, size=(m, 6))
    epn[:, 2] = -epn[:, 0] - epn[:, 1]
    an = RNG.uniform(0, 0.01, m)
    return eps, epn, an


def test_mandel_work_conjugacy():
    e = RNG.normal(size=(5, 6))
    s = RNG.normal(size=(5, 6))
    assert np.allclose(np.sum(e * s, 1),
                       np.sum(surrogate.strain_voigt_to_mandel(e) * surrogate.stress_voigt_to_mandel(s), 1))
    assert np.allclose(surrogate.stress_mandel_to_voigt(surrogate.stress_voigt_to_mandel(s)), s, rtol=1e-15)


def test_exact_network_reproduces_return_map():
    eps, epn, an = _points()
    rm = j2.return_map(eps, epn, an, E, NU, SY, H)
    out = surrogate.update(eps, epn, an, E, NU, SY, H, exact_net, S_IN, S_OUT, tol=1e-3)
    assert rm["plastic"].sum() > 100
    assert np.array_equal(out["used"], rm["plastic"])
    assert np.abs(out["r_loc"][rm["plastic"]]).max() < 1e-10
    for k in ("sigma", "D", "eps_p", "alpha"):
        assert np.abs(out[k] - rm[k]).max() <= 1e-12 * max(1.0, np.abs(rm[k]).max()), k


def test_inaccurate_network_falls_back():
    eps, epn, an = _points()

    def off_net(x):
        y, jac = exact_net(x)
        return 1.01 * y, jac

    rm = j2.return_map(eps, epn, an, E, NU, SY, H)
    out = surrogate.update(eps, epn, an, E, NU, SY, H, off_net, S_IN, S_OUT, tol=1e-3)
    assert not out["used"].any()
    assert np.abs(out["r_loc"][rm["plastic"]] - 0.01).max() < 2e-3
    assert np.array_equal(out["sigma"], rm["sigma"])
