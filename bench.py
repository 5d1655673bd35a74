"""Benchmark of the element-level FE hot path on one MI355X.

Workload (one "step"): the 64^3 two-phase fiber RVE -- 64 periodic RSA
z-fibers (r = 0.05, linear, E = 230, nu = 0.2) in a J2 matrix (E = 3.5,
nu = 0.35, sigma_y = 0.05, H = 0.1), 823,875 dofs, 2,097,152 Gauss points --
driven by affine Dirichlet conditions to eps_xx = 0.002 k, k = 1..10.  Each load
step runs Newton to ||R_f|| <= 1e-8 ||R_f^0||; every Newton iteration evaluates
the residual with the radial-return map at all Gauss points, assembles the CSR
tangent (matrix-explicit Jacobian) and solves the update with matrix-free
Jacobi-PCG (diagonal from the CSR) to 1e-10.  Inputs are resident on the GPU
before the timed region; each step restarts the ramp from zero.

value = whole-step K*u throughput: dofs x operator applications / step time.
The dominant kernel (the single-reduction CG launch: vector updates, M^-1,
matrix-free K*u and three dot products, one launch per iteration) is timed live
with HIP events recorded by the library on the stream it runs on (every 16th
launch of each solve); its algorithmic bytes per launch are the compulsory
traffic at the linearisation in force (r, w, s, p, x, M^-1 read; r, s, p, x, w and
the cleared next w written; phase ids; stored tangent values read).

Further legs (outside the timed region, each recorded in its own entry): K*u
rates of both operators, the FP32 ramp, the 96^3 surrogate against the return
map, the assembled operator at 96^3 and 128^3, the plastic-path adjoint and the
phase-modulus inverse problem at 64^3, the 128^3 Neo-Hookean leg (FP32 element kernels
with FP64 reductions against the FP64 run, with its own roofline), the general-mesh path at
64^3 beside the structured kernels, and
the FP64 CPU oracle on a sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "K*u GDOF/s + quad-pt constitutive evals/s; surrogate vs return-map @ stated err"
HBM_PEAK_GBS = 8000.0
FIBER = (230.0, 0.2)
MATRIX = (3.5, 0.35, 0.05, 0.1)


# inside the timed region only every k-th CG operator launch carries an event pair (each
# pair costs several microseconds of issue time, about 10% of a 64^3 iteration)
CG_TIMING_STRIDE = 16

# MI355X vector peaks (TFLOP/s): 256 CUs x 2.4 GHz; FP32 counts packed FMA, FP64 one FMA per lane
VALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}

# Algorithmic flops of one matrix-free Neo-Hookean K*x per element, for the kernel's own
# algorithm: the sum-factorised gradient of x (per component and direction 4 nodal differences and
# a 2x2 -> 2x2 interpolation, 9 x 36 flops, plus 72 scalings by 1/h), at each of 8 Gauss points the
# linearised stress from the stored F^-T and ln J (F^-1 dH, its product with F^-1, the trace and
# the combination: 160 flops), and the sum-factorised push-back (the transposed interpolation, 396).
NH_APPLY_FLOPS_PER_ELEMENT = 396 + 8 * 160 + 396


def measured_traffic(name="cg_operator_fiber64_f64_traffic.json"):
    """HBM bytes per launch of a fused CG operator from the committed rocprofv3 counter runs
    (FETCH_SIZE / WRITE_SIZE, scaled by a 1 GiB copy), or None when the kernel source has
    changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2604_22087_amd", "csrc")
    h = hashlib.sha256()
    for f in ("fe_kernels.hip", "fe_internal.hpp", "fe_device.hpp"):
        h.update(open(os.path.join(src, f), "rb").read())
    return rec if h.hexdigest() == rec["source_sha256"] else None


def load_path(steps=10, d=0.002):
    return [np.diag([d * k, 0.0, 0.0]) for k in range(1, steps + 1)]


def setup(n, prec):
    import torch
    from paper_2604_22087_amd import fe, inputs
    phase = inputs.fiber_phase(n, n_fibers=64, radius=0.05, seed=2)
    P = fe.Problem(n, prec)
    P.set_materials(torch.tensor(phase, device="cuda"), [fe.J2, fe.LINEAR],
                    [MATRIX, FIBER + (0.0, 0.0)])
    P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
    return P, phase


def run_ramp(P, u, state, path, predictor=0):
    """Newton tolerances: 1e-8 / 1e-10 in FP64; FP32 residuals carry rounding noise near 1e-7
    relative, so the FP32 run stops at 1e-5 / 1e-6 and its error against FP64 is reported."""
    from paper_2604_22087_amd import fe
    u.zero_()
    state.zero_()
    f64 = P.prec == fe.F64
    return P.newton(path, u=u, state=state, op=fe.OP_MATFREE, assemble_csr=True,
                    newton_rtol=1e-8 if f64 else 1e-5, pcg_rtol=1e-10 if f64 else 1e-6, max_newton=30,
                    predictor=predictor)


def predictor_leg(P, path, sig_ref):
    """The same FP64 ramp with the extrapolating Newton predictor (previous converged increment,
    scaled to the load increment) against the boundary-only predictor of the timed steps."""
    import torch
    from paper_2604_22087_amd import fe
    u, state = P.vector(), P.state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, sig, info = run_ramp(P, u, state, path, predictor=fe.PREDICT_EXTRAPOLATE)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s_new = np.array([x[0] for x in sig])
    s_ref = np.array([x[0] for x in sig_ref])
    return {"seconds": dt, "newton_iterations": info["newton_iterations"],
            "line_search_halvings": info["line_search_halvings"], "pcg_iterations": info["pcg_iterations"],
            "per_step": info["steps"], "sigma_bar_xx_max_rel_diff": float(np.max(np.abs(s_new - s_ref) / np.abs(s_ref)))}


def operator_rates(P, u, state, reps=50):
    """K*u rates at the current linearisation: matrix-free and assembled CSR, each hot (back to back,
    as inside PCG) and cold (a 1 GiB read before every launch evicts the 256 MB last-level cache
    without leaving dirty lines behind).
    Times are the library's own HIP events around each launch; bytes are algorithmic."""
    import torch
    from paper_2604_22087_amd import fe
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(P.n_dof, dtype=P.dtype, device="cuda", generator=g)
    y = P.vector()
    flush = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    sink = torch.empty(1, dtype=torch.float64, device="cuda")
    rp, ci = P.csr_indices()
    vals = P.tangent_csr(u, state, apply_bc=True)
    P.residual(u, state, P.state(), apply_bc=True, store_tangent=True)  # matrix-free linearisation = CSR's
    out = {}
    calls = (("matfree", "matfree_apply", lambda: P.apply_matfree(x, y, apply_bc=True)),
             ("csr", "csr_spmv", lambda: P.apply_csr(rp, ci, vals, x, y)),
             ("csr_nodal", "csr_spmv_nodal", lambda: P.apply_csr_nodal(rp, ci, vals, x, y)))
    for name, key, call in calls:
        for mode in ("hot", "cold"):
            for _ in range(5):
                call()
            torch.cuda.synchronize()
            P.profile(True)
            for k in range(reps):
                if mode == "cold":
                    torch.sum(flush, dim=0, keepdim=True, out=sink)
                call()
            c, ms, by = P.profile_read()[key]
            P.profile(False)
            t = ms / c * 1e-3
            out[f"{name}_{mode}"] = {"us": 1e6 * t, "gdofs": P.n_dof / t / 1e9, "GBs": by / c / t / 1e9,
                                     "frac": by / c / t / 1e9 / HBM_PEAK_GBS, "bytes": by / c}
    del vals, flush
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(20):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    out["copy_GBs"] = 20 * 2 * a.numel() * 8 / (s.elapsed_time(e) * 1e-3) / 1e9
    return out


def neohooke_leg(n):
    """Finite-strain leg: n^3 compressible Neo-Hookean RVE with a log-normal shear-modulus field
    (mean 1, CoV 0.5, correlation length 0.1, seed 3; lambda_e = 1.5 mu_e), F_xx -> 1.1 in 5 load
    steps, matrix-free Jacobi-PCG.  Run in FP32 (element kernels and K*u in FP32, PCG scalars and
    Newton norms in FP64) and in FP64; reports times, K*u rates and the FP32 error against FP64."""
    import torch
    from paper_2604_22087_amd import fe, inputs
    mu = inputs.lognormal_field(n, seed=3)
    path = [np.diag([0.02 * k, 0.0, 0.0]) for k in range(1, 6)]
    res, sol = {}, {}
    for prec in ("f32", "f64"):
        P = fe.Problem(n, prec)
        P.set_materials(torch.zeros(n ** 3, dtype=torch.uint8, device="cuda"), [fe.NEOHOOKE],
                        [(2.6, 0.3, 0.0, 0.0)], torch.tensor(mu, dtype=P.dtype, device="cuda"))
        P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask(n), device="cuda"))
        u, state = P.vector(), P.state()
        f64 = prec == "f64"
        torch.cuda.synchronize()
        P.profile(CG_TIMING_STRIDE)
        t0 = time.perf_counter()
        _, _, sig, info = P.newton(path, u=u, state=state, op=fe.OP_MATFREE, newton_rtol=1e-8 if f64 else 1e-5,
                                   pcg_rtol=1e-10 if f64 else 1e-6, max_newton=30)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        c, ms, by = P.profile_read()["matfree_apply"]
        P.profile(False)
        t = ms / max(c, 1) * 1e-3
        flops = NH_APPLY_FLOPS_PER_ELEMENT * P.n_el
        peak = VALU_PEAK_TFLOPS[prec]
        tr = measured_traffic("neohooke128_cg_operator_f64_traffic.json") if (n, prec) == (128, "f64") else None
        res[prec] = {"seconds": dt, "newton_iterations": info["newton_iterations"],
                     "pcg_iterations": info["pcg_iterations"], "ku_applies": info["operator_applies"],
                     "line_search_halvings": info["line_search_halvings"],
                     "ku_us": 1e6 * t, "ku_gdofs": P.n_dof / t / 1e9, "ku_GBs": by / max(c, 1) / t / 1e9,
                     "ku_frac_hbm": by / max(c, 1) / t / 1e9 / HBM_PEAK_GBS,
                     "whole_ramp_gdofs": P.n_dof * info["operator_applies"] / dt / 1e9,
                     "roofline": {"bound": "hbm", "achieved": by / max(c, 1) / t / 1e9, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": by / max(c, 1) / t / 1e9 / HBM_PEAK_GBS,
                                  "traffic": tr["traffic_bytes_per_launch"] if tr else None,
                                  "kernel": f"elem_kernel<{'float' if prec == 'f32' else 'double'}, OP_CG_APPLY, "
                                            f"MS_NH> (fused CG launch; F^-T and ln J of the linearisation read "
                                            f"per Gauss point as stored by the residual)",
                                  "bytes_per_launch": by / max(c, 1), "avg_launch_us": 1e6 * t, "launches": c,
                                  "flops_per_launch": flops, "tflops": flops / t / 1e12,
                                  "frac_valu": flops / t / 1e12 / peak}}
        sol[prec] = (u.double(), np.array(sig))
        del P
    (u32, s32), (u64, s64) = sol["f32"], sol["f64"]
    res["f32_vs_f64"] = {"u_rel_err": float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64)),
                         "stress_bar_max_rel_err": float(np.max(np.abs(s32 - s64)) / np.max(np.abs(s64)))}
    res["workload"] = (f"{n}^3 compressible Neo-Hookean, log-normal mu (mean 1, CoV 0.5, l = 0.1), "
                       f"lambda = 1.5 mu, F_xx -> 1.1 in 5 steps, matrix-free Jacobi-PCG")
    return res


def surrogate_leg(n):
    """Learned-surrogate leg: n^3 sphere RVE (r = 0.3 linear inclusion E = 70, nu = 0.22, J2 matrix of the
    fiber workload), eps_xx ramp to 0.02 in 10 steps, matrix-free Jacobi-PCG, Newton 1e-6 / PCG 1e-8 for
    both constitutive paths; the surrogate runs at plastic-trial points with a 1e-3 local check and
    return-map fallback.  Reports wall times, solver work and the homogenised-stress error."""
    import torch
    from paper_2604_22087_amd import fe
    from paper_2604_22087_amd import surrogate as S
    W = S.load_weights()
    if W is None:
        return {"skipped": "no trained parameters (python -m paper_2604_22087_amd.surrogate writes them)"}
    out = {}
    for mode in ("return_map", "surrogate"):
        P = S.sphere_problem(n)
        if mode == "surrogate":
            P.set_surrogate(W, fallback_tol=1e-3)
        u, st = P.vector(), P.state()
        torch.cuda.synchronize()
        P.profile(CG_TIMING_STRIDE)
        t0 = time.perf_counter()
        _, _, sig, info = P.newton(S.ramp(0.02, 10), u=u, state=st, op=fe.OP_MATFREE, newton_rtol=1e-6,
                                   pcg_rtol=1e-8, max_newton=30, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pr = P.profile_read()
        P.profile(False)
        rc, rms, _ = pr["residual"]
        kc, kms, _ = pr["matfree_apply"]
        out[mode] = {"seconds": dt, "status": info["status"], "newton_iterations": info["newton_iterations"],
                     "pcg_iterations": info["pcg_iterations"], "residual_avg_us": 1e3 * rms / max(rc, 1),
                     "ku_avg_us": 1e3 * kms / max(kc, 1), "sigma_bar_xx": [s_[0] for s_ in sig]}
        if mode == "surrogate":
            out[mode]["points"] = P.surrogate_stats()
        del P
    s_rm = np.array(out["return_map"]["sigma_bar_xx"])
    s_su = np.array(out["surrogate"]["sigma_bar_xx"])
    out["max_rel_sigma_bar_err"] = float(np.max(np.abs(s_su - s_rm) / np.abs(s_rm)))
    out["time_ratio_surrogate_over_return_map"] = out["surrogate"]["seconds"] / out["return_map"]["seconds"]
    out["workload"] = (f"{n}^3 sphere RVE, J2 matrix, eps_xx -> 0.02 in 10 steps, Newton 1e-6, PCG 1e-8; "
                       f"MLP 13-128-128-128-6 with 1e-3 local check and return-map fallback")
    return out


def adjoint_path_leg(n):
    """Adjoint through a plastic load path: n^3 fiber RVE (J2 matrix, per-element modulus scale
    U(0.8, 1.2), seed 5), non-proportional path (tension 0.012, then shear 0.008 added, then tension
    relaxed to 0.004 with shear 0.012), reaction work after the last step and its gradient with
    respect to every element's modulus scale (history checkpointed per step)."""
    import torch
    from paper_2604_22087_amd import fe, inputs
    from paper_2604_22087_amd.adjoint import ReactionWorkPath

    def strain(xx, xy):
        return np.array([[xx, xy, 0.0], [xy, 0.0, 0.0], [0.0, 0.0, 0.0]])
    path = [strain(0.012, 0.0), strain(0.012, 0.008), strain(0.004, 0.012)]
    phase = inputs.fiber_phase(n, n_fibers=64, radius=0.05, seed=2)
    s = torch.tensor(inputs.uniform_field(n ** 3, 0.8, 1.2, seed=5), device="cuda", requires_grad=True)
    P = fe.Problem(n, "f64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = ReactionWorkPath.apply(s, P, torch.tensor(phase, device="cuda"), [fe.J2, fe.LINEAR],
                               [MATRIX, FIBER + (0.0, 0.0)], torch.tensor(inputs.boundary_dof_mask(n), device="cuda"),
                               path, 1e-10, 1e-12)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = s.grad.double()
    out = {"workload": f"{n}^3 fiber RVE, 3-step non-proportional path, dJ/ds for {n ** 3} elements",
           "J": float(J.detach()), "forward_seconds": t1 - t0, "backward_seconds": t2 - t1,
           "grad_norm": float(torch.linalg.norm(g)), "grad_min": float(g.min()), "grad_max": float(g.max()),
           "checkpoint_bytes": 3 * (56 * P.n_el + P.n_dof) * 8}
    # the same gradient keeping one state besides the initial one (binomial schedule)
    s1 = s.detach().clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J1 = ReactionWorkPath.apply(s1, P, torch.tensor(phase, device="cuda"), [fe.J2, fe.LINEAR],
                                [MATRIX, FIBER + (0.0, 0.0)], torch.tensor(inputs.boundary_dof_mask(n), device="cuda"),
                                path, 1e-10, 1e-12, 1)
    J1.backward()
    torch.cuda.synchronize()
    out["one_checkpoint"] = {"seconds": time.perf_counter() - t0, "rerun_load_steps": J1.grad_fn.recompute_solves,
                             "checkpoint_bytes": 2 * (56 * P.n_el + P.n_dof) * 8,
                             "max_rel_grad_diff": float((s1.grad.double() - g).abs().max() / g.abs().max())}
    return out


def inverse_leg(n):
    """Material-parameter inverse problem on the n^3 fiber RVE: the modulus scales of the J2
    matrix and the fibers (1.3, 0.7) behind the reaction work of a 3-step tension path and a
    3-step shear path are recovered from (1, 1) by Gauss-Newton with path-adjoint gradients
    (one checkpoint besides the initial state)."""
    import torch
    from paper_2604_22087_amd import fe, inputs
    from paper_2604_22087_amd.adjoint import fit_phase_scales, reaction_work_path

    def strain(xx, xy):
        return np.array([[xx, xy, 0.0], [xy, 0.0, 0.0], [0.0, 0.0, 0.0]])
    paths = [[strain(0.004 * k, 0.0) for k in (1, 2, 3)], [strain(0.0, 0.004 * k) for k in (1, 2, 3)]]
    phase = torch.tensor(inputs.fiber_phase(n, n_fibers=64, radius=0.05, seed=2), device="cuda")
    mask = torch.tensor(inputs.boundary_dof_mask(n), device="cuda")
    models, params = [fe.J2, fe.LINEAR], [MATRIX, FIBER + (0.0, 0.0)]
    true = np.array([1.3, 0.7])
    P = fe.Problem(n, "f64")
    targets = [float(reaction_work_path(torch.tensor(true, device="cuda")[phase.long()], P, phase, models, params,
                                        mask, path, 1e-10, 1e-12)) for path in paths]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, hist = fit_phase_scales(P, phase, models, params, mask, paths, targets, [1.0, 1.0], newton_rtol=1e-10,
                                   pcg_rtol=1e-12, checkpoints=1,
                                   log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    return {"workload": f"{n}^3 fiber RVE, phase modulus scales from the reaction work of a tension and a shear "
                        f"path (3 steps each)", "true": true.tolist(), "fitted": theta.tolist(),
            "max_abs_error": float(np.abs(theta - true).max()), "gauss_newton_iterations": len(hist),
            "seconds": time.perf_counter() - t0, "history": hist}


def csr_scaling_leg(sizes):
    """Assembled-operator K*u at larger meshes: the fiber RVE's CSR tangent at an affine strain
    eps_xx = 0.004 (elastic linearisation), node-structured and general CSR mat-vec, FP64 and FP32,
    hot and cold (1 GiB read between launches)."""
    import torch
    out = {}
    for n in sizes:
        for prec in ("f64", "f32"):
            P, _ = setup(n, prec)
            u = P.vector()
            P.lift(np.diag([0.004, 0.0, 0.0]), u)
            r = operator_rates(P, u, P.state(), reps=20)
            out[f"{n}^3_{prec}"] = {k: {"us": v["us"], "gdofs": v["gdofs"], "frac": v["frac"]}
                                    for k, v in r.items() if k.startswith("csr")}
            del P, u, r
            torch.cuda.empty_cache()
    return out


def general_leg(n, reps=20):
    """General-mesh path (fe_problem_create_hex8) at n^3 beside the structured kernels: the fiber RVE
    (J2 matrix) on the plain grid fed through the general path, and on a distorted, renumbered mesh
    of the same size, linearised at an affine strain eps_xx = 0.01.  Reports per-kernel times from the
    library's own events (residual, matrix-free K*u, CSR mat-vec), the whole fe_tangent_csr call
    (matrix-core element Jacobians plus the sorted gather) from stream events, one CG iteration, and
    the one-time symbolic set-up."""
    import torch
    from paper_2604_22087_amd import fe, inputs
    out = {}
    eb = np.diag([0.01, 0.0, 0.0])
    for name, amp, perm in (("structured", None, False), ("grid_general", 0.0, False), ("distorted_general", 0.25, True)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        coords, conn = inputs.distorted_cube_mesh(n, amplitude=amp or 0.0, seed=7, permute=perm)
        if amp is None:  # the plain grid numbers nodes and elements as the structured problem does
            P, _ = setup(n, "f64")
        else:
            P = fe.Problem(precision="f64", mesh=(coords, conn))
            P.set_materials(torch.tensor(inputs.fiber_phase_mesh(coords, conn), device="cuda"), [fe.J2, fe.LINEAR],
                            [MATRIX, FIBER + (0.0, 0.0)])
            P.set_dirichlet(torch.tensor(inputs.boundary_dof_mask_mesh(coords), device="cuda"))
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        u = torch.tensor((coords @ eb.T).ravel(), device="cuda")  # the affine field at every node
        st = P.state()
        x = torch.randn(P.n_dof, dtype=torch.float64, device="cuda", generator=torch.Generator(device="cuda").manual_seed(0))
        y = P.vector()
        rp, ci = P.csr_indices()
        vals = P.tangent_csr(u, st, apply_bc=True)
        P.residual(u, st, P.state(), apply_bc=True, store_tangent=True)
        for _ in range(3):
            P.apply_matfree(x, y, apply_bc=True)
            P.tangent_csr(u, st, vals=vals, apply_bc=True)
        torch.cuda.synchronize()
        P.profile(True)
        r = P.vector()
        for _ in range(reps):
            P.residual(u, st, None, r=r, apply_bc=True)
            P.apply_matfree(x, y, apply_bc=True)
            P.apply_csr_nodal(rp, ci, vals, x, y)
        pr = P.profile_read()
        P.profile(False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.tangent_csr(u, st, vals=vals, apply_bc=True)
        e1.record()
        torch.cuda.synchronize()
        t_tan = e0.elapsed_time(e1) / reps * 1e-3
        b = P.residual(u, st, apply_bc=True, store_tangent=True).neg_()
        torch.cuda.synchronize()
        e0.record()
        _, res = P.pcg(b, op=fe.OP_MATFREE, rtol=1e-30, max_it=200, check=False)
        e1.record()
        torch.cuda.synchronize()
        t_cg = e0.elapsed_time(e1) * 1e-3 / max(res.iterations, 1)
        kc, kms, kby = pr["matfree_apply"]
        rc, rms, _ = pr["residual"]
        sc, sms, sby = pr["csr_spmv_nodal"]
        ku = kms / kc * 1e-3
        sp = sms / sc * 1e-3
        out[name] = {"setup_seconds": t_setup, "nnz": P.nnz,
                     "residual_us": 1e3 * rms / rc, "matfree_ku_us": 1e6 * ku, "matfree_gdofs": P.n_dof / ku / 1e9,
                     "matfree_frac_hbm": kby / kc / ku / 1e9 / HBM_PEAK_GBS,
                     "csr_nodal_us": 1e6 * sp, "csr_nodal_frac_hbm": sby / sc / sp / 1e9 / HBM_PEAK_GBS,
                     "tangent_csr_us": 1e6 * t_tan, "cg_iteration_us": 1e6 * t_cg}
        del P, u, st, x, y, vals, r, b, rp, ci, coords, conn
        torch.cuda.empty_cache()
    out["workload"] = (f"{n}^3 fiber RVE (J2 matrix), linearised at eps_xx = 0.01: structured kernels; the same grid "
                       f"through the general-mesh path; a distorted, renumbered {n}^3 mesh (amplitude 0.25 h)")
    return out


def cpu_baseline(n, phase, gpu_info, path):
    """The FP64 oracle on a bounded sample of the same workload, on one host core with the BLAS
    pool limited to one thread, extrapolated to one step.  One evaluation is repeated with the
    BLAS pool at its default size: only BLAS calls inside the oracle are threaded, its einsum and
    scatter loops run on one core either way."""
    from oracle import solver
    from oracle.rve import RVE, phase_params
    from threadpoolctl import threadpool_info, threadpool_limits
    pool = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    rve = RVE(n, phase, [phase_params("j2", *MATRIX), phase_params("linear", *FIBER)])
    samples = [0, len(path) // 2]  # the affine states of the first and a middle load step
    x = np.random.default_rng(0).normal(size=rve.n_dof)
    reps = 5

    def sample(states):
        t0 = time.perf_counter()
        for k in states:
            _, k_e, _ = rve.element_residual_tangent(rve.affine_lift(path[k]), rve.zero_state())
        return (time.perf_counter() - t0) / len(states), k_e

    # the step's work: one residual + tangent per Newton iteration and per load step (the
    # predictor), one residual per line-search halving, one K*u per CG iteration
    applies = gpu_info["operator_applies"]
    n_rt = gpu_info["newton_iterations"] + len(path)
    n_r = gpu_info["line_search_halvings"]
    with threadpool_limits(limits=1):
        t_rt, k_e = sample(samples)
        t0 = time.perf_counter()
        rve.element_residual_tangent(rve.affine_lift(path[samples[-1]]), rve.zero_state(), want_tangent=False)
        t_r = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(reps):
            solver.matfree_apply(rve.conn, k_e, x, rve.mask)
        t_ku = (time.perf_counter() - t0) / reps
    t_rt_pool, _ = sample(samples[:1])  # the same evaluation with the BLAS pool at its default size
    step = t_rt * n_rt + t_r * n_r + t_ku * applies
    return {"value": rve.n_dof * applies / step / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "extrapolated": True,
            "sample": (f"{len(samples)} residual+tangent ({t_rt:.1f} s each), 1 residual-only ({t_r:.1f} s) and "
                       f"{reps} matrix-free K*u ({t_ku:.2f} s each) evaluations of the {n}^3 workload at the affine "
                       f"states of load steps {', '.join(str(k + 1) for k in samples)}, one thread, extrapolated "
                       f"to the step's {n_rt} residual+tangent, {n_r} residual-only and {applies} K*u evaluations"),
            "qp_evals_per_s": 8 * rve.conn.shape[0] / t_r, "step_seconds_est": step,
            "blas_pool_check": {"blas_threads": int(pool), "residual_tangent_seconds": t_rt_pool,
                                "note": "one residual+tangent evaluation with the BLAS pool at its default size: "
                                        "the oracle's einsum and scatter loops run on one core either way"}}


def _leg(fn, *args):
    """An optional leg: a failure there is recorded in its own entry and does not cost the
    benchmark line."""
    try:
        return fn(*args)
    except Exception as exc:  # noqa: BLE001 - reported in the JSON line
        print(f"[bench] {fn.__name__} failed: {exc!r}", file=sys.stderr, flush=True)
        return {"error": repr(exc)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--load-steps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 ramp")
    ap.add_argument("--nh", type=int, default=128, help="n of the finite-strain Neo-Hookean leg (0: skip)")
    ap.add_argument("--surrogate", type=int, default=96, help="n of the surrogate-vs-return-map leg (0: skip)")
    ap.add_argument("--adjoint-path", type=int, default=64, help="n of the plastic-path adjoint leg (0: skip)")
    ap.add_argument("--inverse", type=int, default=64, help="n of the inverse-problem leg (0: skip)")
    ap.add_argument("--csr-sizes", default="96,128", help="mesh sizes of the assembled-operator leg ('' to skip)")
    ap.add_argument("--general", type=int, default=64, help="n of the general-mesh leg (0: skip)")
    ap.add_argument("--copy-calib", action="store_true", help="run only a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the library runs on a single GPU; how the path would shard across GPUs is a design note)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calib:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 8}))
        return

    n = args.n
    path = load_path(args.load_steps)
    P, phase = setup(n, "f64")
    u, state = P.vector(), P.state()
    print(f"[bench] {n}^3 f64 ramp: warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        run_ramp(P, u, state, path)
    torch.cuda.synchronize()
    P.profile(CG_TIMING_STRIDE)
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, _, sig, info = run_ramp(P, u, state, path)
        infos.append(info)
        print(f"[bench] step {k}: {info}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = P.profile_read()
    P.profile(False)
    ms_step = 1e3 * elapsed / args.steps
    applies = sum(i["operator_applies"] for i in infos) / args.steps
    value = P.n_dof * applies / (elapsed / args.steps) / 1e9

    cnt, ms, byts = prof["matfree_apply"]
    ku_avg_ms = ms / max(cnt, 1)
    achieved = byts / max(cnt, 1) / (ku_avg_ms * 1e-3) / 1e9
    traffic = measured_traffic() if n == 64 else None
    rcnt, rms, _ = prof["residual"]
    tcnt, tms, _ = prof["tangent_csr"]
    out = {
        "metric": METRIC, "value": value, "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{n}^3 hex8 two-phase fiber RVE (64 RSA fibers r=0.05 E=230; J2 matrix "
                               f"E=3.5 nu=0.35 sy=0.05 H=0.1), eps_xx ramp to {0.002 * args.load_steps:.3f} in "
                               f"{args.load_steps} load steps, Newton 1e-8 with CSR tangent + matrix-free "
                               f"Jacobi-PCG 1e-10",
                   "n": n, "n_dof": P.n_dof, "n_qp": P.n_qp, "nnz": P.nnz, "load_steps": args.load_steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["traffic_bytes_per_launch"] if traffic else None,
                     "traffic_note": (f"rocprofv3 FETCH_SIZE x {traffic['fetch_scale']:.3f} + WRITE_SIZE x "
                                      f"{traffic['write_scale']:.3f} (1 GiB copy calibration), mean per launch over "
                                      f"{traffic['workload']}, where the algorithmic bytes are "
                                      f"{traffic['algorithmic_bytes_per_launch']:.4g}") if traffic else None,
                     "kernel": "elem_kernel<double, OP_CG_APPLY, MS_J2> (single-reduction CG launch: vector "
                               "updates, M^-1, matrix-free K*u and three dot products)",
                     "avg_launch_us": 1e3 * ku_avg_ms, "launches": cnt,
                     "sampling": f"HIP event pairs on operator launches 0, {CG_TIMING_STRIDE}, "
                                 f"{2 * CG_TIMING_STRIDE}, ... of every CG solve in the timed region",
                     "bytes_per_launch": byts / max(cnt, 1)},
        "ku_kernel_gdofs": P.n_dof / (ku_avg_ms * 1e-3) / 1e9,
        "qp_evals_per_s": P.n_qp / (rms / max(rcnt, 1) * 1e-3),
        "residual_avg_us": 1e3 * rms / max(rcnt, 1),
        "tangent_csr_avg_us": 1e3 * tms / max(tcnt, 1),
        "newton_iterations": infos[-1]["newton_iterations"], "pcg_iterations": infos[-1]["pcg_iterations"],
        "ku_applies": infos[-1]["operator_applies"],
        "line_search_halvings": infos[-1]["line_search_halvings"],
        "per_step": {"fields": ["newton_iterations", "line_search_halvings", "cg_iterations"],
                     "last_timed_step": infos[-1]["steps"],
                     "newton_iterations_over_timed_steps": [i["newton_iterations"] for i in infos]},
        "sigma_bar_xx_last": sig[-1][0],
    }
    out["operators_f64"] = operator_rates(P, u, state)
    print("[bench] predictor leg", file=sys.stderr, flush=True)
    out["extrapolating_predictor"] = _leg(predictor_leg, P, path, sig)
    if not args.no_fp32:
        P32, _ = setup(n, "f32")
        u32, s32 = P32.vector(), P32.state()
        run_ramp(P32, u32, s32, path)  # warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, sig32, info32 = run_ramp(P32, u32, s32, path)
        torch.cuda.synchronize()
        t32 = time.perf_counter() - t1
        s64 = np.array([s[0] for s in sig])
        s32a = np.array([s[0] for s in sig32])
        out["fp32"] = {"value": P32.n_dof * info32["operator_applies"] / t32 / 1e9, "ms_per_step": 1e3 * t32,
                       "sigma_bar_xx_max_rel_err_vs_f64": float(np.max(np.abs(s32a - s64) / np.abs(s64))),
                       "u_rel_err_vs_f64": float(torch.linalg.norm(u32.double() - u) / torch.linalg.norm(u)),
                       "pcg_iterations": info32["pcg_iterations"],
                       "operators": operator_rates(P32, u32, s32)}
        del P32
        # the same ramp with the nodal sums in FP32 as well (default: FP64 sums in FP32 problems)
        P32, _ = setup(n, "f32")
        P32.set_fp32_accumulation(True)
        u32, s32 = P32.vector(), P32.state()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, sig32, info32 = run_ramp(P32, u32, s32, path)
        torch.cuda.synchronize()
        t32 = time.perf_counter() - t1
        s32a = np.array([s[0] for s in sig32])
        out["fp32"]["fp32_nodal_sums"] = {
            "value": P32.n_dof * info32["operator_applies"] / t32 / 1e9, "ms_per_step": 1e3 * t32,
            "sigma_bar_xx_max_rel_err_vs_f64": float(np.max(np.abs(s32a - s64) / np.abs(s64))),
            "u_rel_err_vs_f64": float(torch.linalg.norm(u32.double() - u) / torch.linalg.norm(u)),
            "pcg_iterations": info32["pcg_iterations"]}
        del P32
    if args.surrogate:
        print(f"[bench] surrogate leg {args.surrogate}^3", file=sys.stderr, flush=True)
        out["surrogate"] = _leg(surrogate_leg, args.surrogate)
    if args.csr_sizes:
        sizes = [int(v) for v in args.csr_sizes.split(",") if v]
        print(f"[bench] assembled-operator leg {sizes}", file=sys.stderr, flush=True)
        out["csr_scaling"] = _leg(csr_scaling_leg, sizes)
    if args.adjoint_path:
        print(f"[bench] adjoint path leg {args.adjoint_path}^3", file=sys.stderr, flush=True)
        out["adjoint_path"] = _leg(adjoint_path_leg, args.adjoint_path)
    if args.inverse:
        print(f"[bench] inverse-problem leg {args.inverse}^3", file=sys.stderr, flush=True)
        out["inverse"] = _leg(inverse_leg, args.inverse)
    if args.nh:
        print(f"[bench] neo-hookean leg {args.nh}^3", file=sys.stderr, flush=True)
        out["neohooke"] = _leg(neohooke_leg, args.nh)
    if args.general:
        print(f"[bench] general-mesh leg {args.general}^3", file=sys.stderr, flush=True)
        out["general_mesh"] = _leg(general_leg, args.general)
    if not args.no_cpu:
        print("[bench] cpu oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(n, phase, infos[-1], path)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
