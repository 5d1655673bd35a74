"""GPU discrete adjoint through a plastic load path (history checkpointed per step)
against the oracle's complex-step gradient of the same path objective, plus
finite differences at a larger size and the linear special case."""
import numpy as np
import pytest

from helpers import rel_err
from oracle import adjoint as oadj
from oracle.rve import RVE, phase_params
from paper_2604_22087_amd import inputs

pytestmark = pytest.mark.gpu
J2P = (3.5, 0.35, 0.05, 0.1)


def _strain(xx, xy):
    return np.array([[xx, xy, 0.0], [xy, 0.0, 0.0], [0.0, 0.0, 0.0]])


PATH = [_strain(0.012, 0.0), _strain(0.012, 0.008), _strain(0.004, 0.012)]


def _gpu(n, phase, s, models, params, path, **kw):
    import torch
    from paper_2604_22087_amd import fe
    from paper_2604_22087_amd.adjoint import reaction_work_path
    P = fe.Problem(n, "f64")
    st = torch.tensor(s, device="cuda", requires_grad=True)
    J = reaction_work_path(st, P, torch.tensor(phase, dtype=torch.uint8, device="cuda"), models, params,
                           torch.tensor(inputs.boundary_dof_mask(n), device="cuda"), path, **kw)
    J.backward()
    return float(J), st.grad.cpu().numpy(), P


def test_path_gradient_matches_complex_step_oracle():
    from paper_2604_22087_amd import fe
    n = 3
    print("[adjoint path] n=3 vs complex step", flush=True)
    phase = np.zeros(n ** 3, dtype=int)
    phase[n ** 3 // 2] = 1
    s = inputs.uniform_field(n ** 3, 0.8, 1.2, seed=4)
    rve = RVE(n, phase, [phase_params("j2", *J2P), phase_params("linear", 230.0, 0.2)], scale=s)
    J_ref, _ = oadj.path_reaction_work(rve, PATH)
    g_ref = oadj.path_gradient_complex_step(rve, PATH)
    J, g, _ = _gpu(n, phase, s, [fe.J2, fe.LINEAR], [J2P, (230.0, 0.2, 0.0, 0.0)], PATH)
    assert J == pytest.approx(float(np.real(J_ref)), rel=1e-10)
    assert np.abs(g - g_ref).max() <= 1e-8 * np.abs(g_ref).max()


def test_path_gradient_linear_special_case():
    import torch
    from paper_2604_22087_amd import fe
    from paper_2604_22087_amd.adjoint import compliance
    n = 6
    phase = inputs.sphere_phase(n)
    s = inputs.uniform_field(n ** 3, 1.0, 3.0, seed=8)
    eb = np.diag([0.01, 0.0, 0.0])
    J, g, _ = _gpu(n, np.zeros(n ** 3, dtype=int), s, [fe.LINEAR], [(1.0, 0.3, 0.0, 0.0)], [eb])
    P = fe.Problem(n, "f64")
    st = torch.tensor(s, device="cuda", requires_grad=True)
    J2 = compliance(st, P, torch.zeros(n ** 3, dtype=torch.uint8, device="cuda"),
                    torch.tensor(inputs.boundary_dof_mask(n), device="cuda"), eb)
    J2.backward()
    assert J == pytest.approx(float(J2), rel=1e-10)
    assert rel_err(g, st.grad.cpu().numpy()) <= 1e-9
    del phase


def test_path_gradient_finite_differences_fiber():
    from paper_2604_22087_amd import fe
    n = 10
    print("[adjoint path] n=10 fiber FD", flush=True)
    phase = inputs.fiber_phase(n, n_fibers=4, radius=0.18, seed=2)
    s = inputs.uniform_field(n ** 3, 0.8, 1.2, seed=5)
    models, params = [fe.J2, fe.LINEAR], [J2P, (230.0, 0.2, 0.0, 0.0)]
    J, g, P = _gpu(n, phase, s, models, params, PATH)
    picks = inputs.fd_element_picks(n ** 3, 6, seed=40)
    errs = []
    for e in picks:
        # truncation is ~(h/s)^2; the quotient divides J's solve error by 2h, so the two
        # evaluations solve to a Newton relative residual of 1e-14 instead of 1e-12 (at
        # 1e-12, J's error over 2h reaches ~1e-6 of the gradient of a weak element)
        h = 1e-4 * s[e]
        sp, sm = s.copy(), s.copy()
        sp[e] += h
        sm[e] -= h
        jp, _, _ = _gpu(n, phase, sp, models, params, PATH, newton_rtol=1e-14)
        jm, _, _ = _gpu(n, phase, sm, models, params, PATH, newton_rtol=1e-14)
        errs.append(abs((jp - jm) / (2 * h) - g[e]) / abs(g[e]))
    print(f"  FD vs adjoint: {np.array(errs)}", flush=True)
    assert max(errs) <= 1e-6


PATH5 = [_strain(0.006, 0.0), _strain(0.012, 0.0), _strain(0.012, 0.006), _strain(0.008, 0.010),
         _strain(0.004, 0.012)]


def test_path_gradient_binomial_checkpoints_match_store_all():
    """Keeping only c + 1 states and re-running steps (binomial schedule) gives the gradient
    of the store-all sweep, with the predicted number of re-run load steps."""
    from paper_2604_22087_amd import fe
    from paper_2604_22087_amd.adjoint import revolve_cost
    n = 8
    print("[adjoint path] n=8 binomial checkpoints", flush=True)
    phase = inputs.fiber_phase(n, n_fibers=4, radius=0.18, seed=2)
    s = inputs.uniform_field(n ** 3, 0.8, 1.2, seed=6)
    models, params = [fe.J2, fe.LINEAR], [J2P, (230.0, 0.2, 0.0, 0.0)]
    J0, g0, _ = _gpu(n, phase, s, models, params, PATH5)
    for c in (0, 1, 2):
        import torch
        from paper_2604_22087_amd.adjoint import reaction_work_path
        P = fe.Problem(n, "f64")
        st = torch.tensor(s, device="cuda", requires_grad=True)
        J = reaction_work_path(st, P, torch.tensor(phase, dtype=torch.uint8, device="cuda"), models, params,
                               torch.tensor(inputs.boundary_dof_mask(n), device="cuda"), PATH5, checkpoints=c)
        J.backward()
        solves = J.grad_fn.recompute_solves
        print(f"  checkpoints {c}: {solves} re-run load steps", flush=True)
        assert solves == revolve_cost(len(PATH5), c)
        assert float(J) == pytest.approx(J0, rel=1e-12)
        assert rel_err(st.grad.cpu().numpy(), g0) <= 1e-9


def test_inverse_fit_recovers_phase_scales():
    """Gauss-Newton on the reaction work of a tension and a shear path recovers the two
    phase modulus scales that produced the targets."""
    import torch
    from paper_2604_22087_amd import fe
    from paper_2604_22087_amd.adjoint import fit_phase_scales, reaction_work_path
    n = 8
    print("[adjoint path] n=8 inverse fit", flush=True)
    phase = torch.tensor(inputs.fiber_phase(n, n_fibers=4, radius=0.18, seed=2), dtype=torch.uint8, device="cuda")
    mask = torch.tensor(inputs.boundary_dof_mask(n), device="cuda")
    models, params = [fe.J2, fe.LINEAR], [J2P, (230.0, 0.2, 0.0, 0.0)]
    paths = [[_strain(0.006, 0.0), _strain(0.012, 0.0)], [_strain(0.0, 0.006), _strain(0.0, 0.012)]]
    true = np.array([1.3, 0.7])
    P = fe.Problem(n, "f64")
    targets = []
    for path in paths:
        s = torch.tensor(true, device="cuda")[phase.long()]
        targets.append(float(reaction_work_path(s, P, phase, models, params, mask, path)))
    theta, hist = fit_phase_scales(P, phase, models, params, mask, paths, targets, [1.0, 1.0], checkpoints=1,
                                   log=lambda m: print("  " + m, flush=True))
    assert np.abs(theta - true).max() <= 1e-6
    assert len(hist) <= 8
