"""GPU adjoint gradient (config: linear RVE with E_e ~ U(1,10), compliance under
macro strain 0.01) against the FP64 oracle and central finite differences.

Bars: objective and gradient <= 1e-10 normwise against the oracle's own solve
(small mesh); at 64^3 the per-element gradient at the GPU solution matches the
oracle element by element (<= 1e-12), Euler's identity sum E_e dJ/dE_e = J holds
(<= 1e-10), and central differences with h = 1e-6 on 64 seeded elements agree
(<= 1e-4 relative; the objective is summed exactly from non-negative element
energies so rounding stays far below the 2e-12 relative change the step makes).
"""
import math

import numpy as np
import pytest

from helpers import rel_err
from oracle import adjoint as oadj
from oracle.rve import RVE, phase_params
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu
EB = np.diag([0.01, 0.0, 0.0])


def _torch_setup(n, E):
    import torch
    from paper_2604_22087_amd import fe
    P = fe.Problem(n, "f64")
    phase = torch.zeros(n ** 3, dtype=torch.uint8, device="cuda")
    mask = torch.tensor(inputs.boundary_dof_mask(n), device="cuda")
    Et = torch.tensor(E, device="cuda", requires_grad=True)
    return P, phase, mask, Et


def test_adjoint_gradient_matches_oracle_small():
    from paper_2604_22087_amd.adjoint import compliance
    n = 6
    E = inputs.uniform_field(n ** 3, 1.0, 10.0, seed=4)
    rve = RVE(n, np.zeros(n ** 3, dtype=int), [phase_params("linear", 1.0, 0.3)], scale=E)
    u_ref, _ = rve.solve_linear(EB, rtol=1e-14)
    g_ref, lam_ref = oadj.gradient(rve, u_ref)
    J_ref = oadj.reaction_objective(rve, u_ref)
    P, phase, mask, Et = _torch_setup(n, E)
    J = compliance(Et, P, phase, mask, EB, rtol=1e-13)
    J.backward()
    assert float(J) == pytest.approx(J_ref, rel=1e-10)
    assert rel_err(Et.grad.cpu().numpy(), g_ref) <= 1e-10


def test_adjoint_fullsize_fd_and_euler():
    import torch
    from paper_2604_22087_amd.adjoint import compliance
    n = 64
    E = inputs.uniform_field(n ** 3, 1.0, 10.0, seed=4)
    P, phase, mask, Et = _torch_setup(n, E)
    J = compliance(Et, P, phase, mask, EB, rtol=1e-13)
    J.backward()
    g = Et.grad.double().cpu().numpy()
    print(f"[adjoint 64^3] J={float(J):.10e}", flush=True)
    assert np.all(g > 0)
    assert float(np.dot(E, g)) == pytest.approx(float(J), rel=1e-10)
    # element-level parity of dJ/dE_e at the GPU solution (oracle evaluates sampled elements)
    from paper_2604_22087_amd import fe
    u = P.newton([EB], op=fe.OP_MATFREE, pcg_rtol=1e-13, newton_rtol=1e-12)[0]
    picks = inputs.fd_element_picks(n ** 3, 64, seed=40)
    sub = RVE(n, np.zeros(n ** 3, dtype=int), [phase_params("linear", 1.0, 0.3)], scale=E, elements=picks)
    un = u.double().cpu().numpy()
    assert rel_err(g[picks], oadj.vjp_scale(sub, un, un)) <= 1e-12

    def energy(Evec, rtol=1e-13):
        P.set_materials(phase, [fe.LINEAR], [(1.0, 0.3)], torch.tensor(Evec, device="cuda"))
        uu = P.newton([EB], op=fe.OP_MATFREE, pcg_rtol=rtol, newton_rtol=1e-12)[0]
        e_el = (torch.tensor(Evec, device="cuda") * P.vjp(uu, uu)).double().cpu().numpy()
        return math.fsum(e_el.tolist())

    # Noise floor of one energy evaluation: the same E solved along two CG paths.  A
    # central difference with step h carries about 2 eps_J / (2 h) of that noise; at
    # h = 1e-6 the difference J(E+h) - J(E-h) is ~1e-12 of J, near FP64 resolution.
    eps_j = max(abs(energy(E, 1e-13) - energy(E, 1e-12)), abs(float(J)) * 2.0 ** -52)

    def fd_errors(h, picks_h):
        errs, bounds = [], []
        for k in picks_h:
            Ep, Em = E.copy(), E.copy()
            Ep[k] += h
            Em[k] -= h
            fd = (energy(Ep) - energy(Em)) / (2 * h)
            errs.append(abs(fd - g[k]) / abs(g[k]))
            bounds.append(2 * eps_j / (2 * h) / abs(g[k]))
        return np.array(errs), np.array(bounds)

    errs, noise = fd_errors(1e-6, picks)
    print(f"  FD (h=1e-6) vs adjoint on 64 elements: median {np.median(errs):.2e} max {errs.max():.2e}; "
          f"noise bound median {np.median(noise):.2e} (eps_J {eps_j:.2e})", flush=True)
    assert np.median(errs) <= 1e-4
    assert np.all(errs <= 1e-5 + 4 * noise)
    # a larger step on 16 of the picks: noise 100x lower, truncation ~(h/E)^2
    errs4, noise4 = fd_errors(1e-4, picks[:16])
    print(f"  FD (h=1e-4) on 16 elements: max {errs4.max():.2e}", flush=True)
    assert np.all(errs4 <= 1e-6 + 4 * noise4)


def test_adjoint_two_objectives_share_one_problem():
    """Two compliance objectives over different modulus fields on one Problem, summed and
    differentiated together: each gradient must be the one of its own field (the backward
    pass re-instates the materials its forward pass used)."""
    import torch
    from paper_2604_22087_amd.adjoint import compliance
    n = 6
    E1 = inputs.uniform_field(n ** 3, 1.0, 10.0, seed=4)
    E2 = inputs.uniform_field(n ** 3, 1.0, 10.0, seed=5)
    P, phase, mask, E1t = _torch_setup(n, E1)
    E2t = torch.tensor(E2, device="cuda", requires_grad=True)
    J = compliance(E1t, P, phase, mask, EB, rtol=1e-13) + compliance(E2t, P, phase, mask, EB, rtol=1e-13)
    J.backward()
    for E, Et in ((E1, E1t), (E2, E2t)):
        rve = RVE(n, np.zeros(n ** 3, dtype=int), [phase_params("linear", 1.0, 0.3)], scale=E)
        u_ref, _ = rve.solve_linear(EB, rtol=1e-14)
        g_ref, _ = oadj.gradient(rve, u_ref)
        assert rel_err(Et.grad.cpu().numpy(), g_ref) <= 1e-10
