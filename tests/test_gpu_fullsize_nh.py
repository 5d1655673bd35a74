"""Parity at the full 128^3 size of the finite-strain workload: compressible
Neo-Hookean RVE with a log-normal shear-modulus field (lambda_e = 1.5 mu_e),
in FP32 (the precision that workload runs in) and FP64.

The oracle evaluates the elements around a seeded sample of nodes and sums them
into those rows: residual, matrix-free tangent product at the stored
linearisation and the operator diagonal.  A stretched state with a random
perturbation exercises the nonlinear terms everywhere.
"""
import numpy as np
import pytest

from helpers import lib_materials, oracle_phases
from oracle.mesh import element_dofs
from oracle.rve import RVE
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu
N = 128
SPEC = [("neohooke", 2.6, 0.3)]  # mu = 1, lam = 1.5 before the per-element scale


def _sample(n, count, seed):
    rng = np.random.default_rng(seed)
    ijk = rng.integers(0, n + 1, size=(count, 3))
    ijk[:4] = [[0, 0, 0], [n, n, n], [1, n // 2, n], [n // 2, n // 2, n // 2]]
    els = set()
    for i, j, k in ijk:
        for a in (i - 1, i):
            for b in (j - 1, j):
                for c in (k - 1, k):
                    if 0 <= a < n and 0 <= b < n and 0 <= c < n:
                        els.add(a + n * (b + n * c))
    nodes = ijk[:, 0] + (n + 1) * (ijk[:, 1] + (n + 1) * ijk[:, 2])
    return np.array(sorted(els)), (3 * nodes[:, None] + np.arange(3)).ravel()


@pytest.fixture(scope="module")
def setup128():
    mu = inputs.lognormal_field(N, seed=3)
    els, rows = _sample(N, 40, seed=23)
    rve = RVE(N, np.zeros(N ** 3, dtype=int), oracle_phases(SPEC), scale=mu, elements=els)
    amp = 0.3 / N
    grad = np.array([[0.1, 0.02, 0.0], [0.0, -0.03, 0.01], [0.01, 0.0, 0.04]])
    u = (rve.coords @ grad.T).ravel() + inputs.random_displacement(N, -amp, amp, seed=9)
    r_e, k_e, _ = rve.element_residual_tangent(u)
    x = np.random.default_rng(3).normal(size=rve.n_dof)
    dofs = element_dofs(rve.conn)

    def gather(vec_e):
        out = np.zeros(rve.n_dof)
        np.add.at(out, dofs.ravel(), vec_e.ravel())
        return out[rows]

    diag_e = np.einsum("eii->ei", k_e)
    return dict(mu=mu, u=u, x=x, rows=rows, r=gather(r_e), kx=gather(np.einsum("eij,ej->ei", k_e, x[dofs])),
                d=gather(diag_e))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fullsize_neohooke(setup128, prec):
    import torch
    from paper_2604_22087_amd import fe
    print(f"[fullsize nh 128^3] prec={prec}", flush=True)
    s = setup128
    tol = 1e-12 if prec == "f64" else 1e-5
    P = fe.Problem(N, prec)
    models, params = lib_materials(SPEC)
    P.set_materials(torch.zeros(N ** 3, dtype=torch.uint8, device="cuda"), models, params,
                    torch.tensor(s["mu"], dtype=P.dtype, device="cuda"))
    ut = torch.tensor(s["u"], dtype=P.dtype, device="cuda")
    rows = s["rows"]
    r = P.residual(ut, store_tangent=True)[rows].double().cpu().numpy()
    assert P.read_flags() == 0
    assert np.linalg.norm(r - s["r"]) <= tol * np.linalg.norm(s["r"])
    y = P.apply_matfree(torch.tensor(s["x"], dtype=P.dtype, device="cuda"))[rows].double().cpu().numpy()
    assert np.linalg.norm(y - s["kx"]) <= tol * np.linalg.norm(s["kx"])
    d = P.diagonal()[rows].double().cpu().numpy()
    assert np.linalg.norm(d - s["d"]) <= tol * np.linalg.norm(s["d"])
