"""Pins of the seeded input generators that the oracle and the HIP path both read.

The generators hold no finite-element arithmetic, but a wrong recipe (a lost
variance factor of the correlated field, a wrong correlation coefficient, a fiber
overlap) would pass every parity test, because both sides read the same arrays.
These tests check the recipes against what their definitions fix:

* log-normal field (separable exponential correlation, length 0.1, mean 1,
  CoV 0.5): ln mu = m + s g with s^2 = ln(1 + CoV^2), m = -s^2/2 and g a unit
  Gaussian field with Corr(g_i, g_j) = exp(-(|dx|+|dy|+|dz|)/0.1).  Checked over an
  ensemble of seeds: the mean and variance of ln mu, E[mu] = 1, the correlation at
  lags (1,0,0), (0,1,0), (0,0,1), (2,0,0) and (1,1,0) against rho, rho^2, rho^2
  (rho = exp(-h/0.1)), which pins the exponential form and the separability;
  and, at the 128^3 workload itself, the lag-h correlation of seed 3.
* periodic RSA fibers: count, centers in [0,1)^2, pairwise minimum-image distance
  >= 2r (brute force over all pairs), element phase by centroid within r
  (recomputed by explicit loops), discrete volume fraction near pi r^2 N.
* sphere inclusion at 8^3: 56 elements (fraction 0.109375), with no centroid on
  the sphere.
* Dirichlet mask: exactly the nodes with an index in {0, n}.
"""
import math

import numpy as np
import pytest

from paper_2604_22087_amd import inputs

S2 = math.log1p(0.25)          # s^2 of CoV 0.5
M = -0.5 * S2


def _lag_corr(g, shift):
    """Sample correlation of g with itself shifted by `shift` (a, b, c) = (x, y, z) lags.

    g is laid out [c][b][a] (x fastest in element order)."""
    a, b, c = shift
    n = g.shape[0]
    x = g[: n - c, : n - b, : n - a]
    y = g[c:, b:, a:]
    x = x - g.mean()
    y = y - g.mean()
    return float(np.sum(x * y) / math.sqrt(np.sum(x * x) * np.sum(y * y)))


@pytest.fixture(scope="module")
def ensemble():
    n, seeds = 32, range(100, 228)
    fields = [inputs.lognormal_field(n, seed=s).reshape(n, n, n) for s in seeds]
    return n, fields


def test_lognormal_marginal(ensemble):
    n, fields = ensemble
    logs = np.stack([np.log(f) for f in fields])
    # the ensemble mean of ln mu has std ~ s * 0.011 here; of mu ~ 0.006
    assert abs(logs.mean() - M) < 0.02
    assert abs(logs.var() / S2 - 1.0) < 0.05
    mus = np.stack(fields)
    assert abs(mus.mean() - 1.0) < 0.03
    assert abs(mus.std() / mus.mean() - 0.5) < 0.04


def test_lognormal_correlation(ensemble):
    n, fields = ensemble
    rho = math.exp(-(1.0 / n) / 0.1)
    gs = [(np.log(f) - M) / math.sqrt(S2) for f in fields]
    for shift, expect in [((1, 0, 0), rho), ((0, 1, 0), rho), ((0, 0, 1), rho),
                          ((2, 0, 0), rho ** 2), ((1, 1, 0), rho ** 2), ((1, 1, 1), rho ** 3)]:
        est = float(np.mean([_lag_corr(g, shift) for g in gs]))
        # per-field estimates are biased low by the sample-mean subtraction (~ -0.005 here)
        assert abs(est - expect) < 0.015, (shift, est, expect)


def test_lognormal_workload_field():
    n = 128
    mu = inputs.lognormal_field(n, seed=3)
    assert mu.shape == (n ** 3,) and np.all(mu > 0) and np.all(np.isfinite(mu))
    g = ((np.log(mu) - M) / math.sqrt(S2)).reshape(n, n, n)
    rho = math.exp(-(1.0 / n) / 0.1)  # 0.9248488...
    assert rho == pytest.approx(0.9248488132162048, rel=1e-15)
    for shift in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        assert abs(_lag_corr(g, shift) - rho) < 0.02
    # one realisation with correlation length 0.1 of the cube: loose bounds only
    assert abs(mu.mean() - 1.0) < 0.25
    assert 0.3 < mu.std() / mu.mean() < 0.7


def test_rsa_fibers_non_overlapping():
    r = 0.05
    c = inputs.rsa_fiber_centers(64, r, seed=2)
    assert c.shape == (64, 2)
    assert np.all(c >= 0.0) and np.all(c < 1.0)
    dmin = np.inf
    for i in range(64):
        for j in range(i + 1, 64):
            d = c[i] - c[j]
            d = d - np.round(d)
            dmin = min(dmin, math.hypot(d[0], d[1]))
    assert dmin >= 2 * r
    # deterministic for its seed
    assert np.array_equal(c, inputs.rsa_fiber_centers(64, r, seed=2))


def test_fiber_phase_by_centroid_brute_force():
    n, r = 16, 0.05
    c = inputs.rsa_fiber_centers(64, r, seed=2)
    phase = inputs.fiber_phase(n, 64, r, seed=2)
    h = 1.0 / n
    ref = np.zeros(n ** 3, dtype=np.uint8)
    for cc in range(n):
        for b in range(n):
            for a in range(n):
                x, y = (a + 0.5) * h, (b + 0.5) * h
                inside = False
                for f in c:
                    dx = x - f[0] - round(x - f[0])
                    dy = y - f[1] - round(y - f[1])
                    inside |= dx * dx + dy * dy < r * r
                ref[a + n * (b + n * cc)] = inside
    assert np.array_equal(phase, ref)


def test_fiber_volume_fraction_at_workload():
    phi_nominal = 64 * math.pi * 0.05 ** 2  # 0.50265...
    phase = inputs.fiber_phase(64, 64, 0.05, seed=2)
    phi = float(phase.mean())
    # z-aligned fibers: every z layer has the same phase pattern
    lay = phase.reshape(64, 64 * 64)
    assert np.all(lay == lay[0])
    assert abs(phi - phi_nominal) < 0.02, phi


def test_sphere_phase_config1():
    phase = inputs.sphere_phase(8)
    assert int(phase.sum()) == 56 and phase.mean() == 0.109375
    d = inputs.element_centroids(8) - 0.5
    assert np.min(np.abs(np.einsum("ij,ij->i", d, d) - 0.09)) > 0.01


def test_boundary_mask():
    n = 5
    m = inputs.boundary_dof_mask(n).reshape(-1, 3)
    assert np.all(m == m[:, :1])
    for k in range(n + 1):
        for j in range(n + 1):
            for i in range(n + 1):
                on = i in (0, n) or j in (0, n) or k in (0, n)
                assert m[i + (n + 1) * (j + (n + 1) * k), 0] == on
