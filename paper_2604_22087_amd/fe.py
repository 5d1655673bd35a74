"""Thin Python binding of libfe (include/fe.h): argument marshalling only.

Every computation runs in the HIP library; this module converts torch device
tensors to raw pointers, passes the current torch stream as the hipStream_t and
turns non-zero statuses into FeError.  There is no CPU fallback: if libfe.so is
missing or no GPU is visible, calls fail.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfe.so")

F64, F32 = 0, 1
LINEAR, J2, NEOHOOKE = 0, 1, 2
OP_CSR, OP_MATFREE = 0, 1
PC_JACOBI, PC_BLOCK_JACOBI, PC_ILU0 = 0, 1, 2
SOLVER_CG, SOLVER_BICGSTAB, SOLVER_GMRES = 0, 1, 2
APPLY_BC, STORE_TANGENT = 1, 2

STATUS = {0: "ok", 1: "invalid argument", 2: "HIP runtime error", 3: "out of device memory",
          4: "iteration limit reached", 5: "CG breakdown", 6: "non-finite value",
          7: "inverted element", 8: "required state missing"}

_vp, _i32, _i64, _dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double


class PcgInfo(ctypes.Structure):
    _fields_ = [("iterations", _i32), ("status", _i32), ("relres", _dbl), ("bnorm", _dbl)]


class NewtonOpts(ctypes.Structure):
    _fields_ = [("op", _i32), ("assemble_csr", _i32), ("max_newton", _i32), ("newton_rtol", _dbl), ("pcg_rtol", _dbl),
                ("pcg_max_it", _i32), ("solver", _i32), ("restart", _i32), ("predictor", _i32),
                ("step_log_host", ctypes.POINTER(_i32))]


PREDICT_BOUNDARY, PREDICT_EXTRAPOLATE = 0, 1


class NewtonInfo(ctypes.Structure):
    _fields_ = [("newton_iterations", _i32), ("pcg_iterations", _i32), ("operator_applies", _i32),
                ("steps_done", _i32), ("line_search_halvings", _i32), ("status", _i32), ("last_residual", _dbl)]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("fe_problem_create", _i32, [ctypes.POINTER(_vp), _i32, _i32]),
    ("fe_problem_create_hex8", _i32, [ctypes.POINTER(_vp), _i64, _i64, _vp, _vp, _i32, _vp]),
    ("fe_commit_state", _i32, [_vp, _vp, _vp, _vp]),
    ("fe_set_deterministic", _i32, [_vp, _i32]),
    ("fe_set_fp32_accumulation", _i32, [_vp, _i32]),
    ("fe_problem_destroy", None, [_vp]),
    ("fe_problem_sizes", _i32, [_vp, ctypes.POINTER(_i64)]),
    ("fe_set_materials", _i32, [_vp, _vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_dbl), _vp, _vp]),
    ("fe_set_dirichlet", _i32, [_vp, _vp, _vp]),
    ("fe_lift", _i32, [_vp, ctypes.POINTER(_dbl), _vp, _i32, _vp]),
    ("fe_residual", _i32, [_vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    ("fe_csr_nnz", _i32, [_vp, ctypes.POINTER(_i64)]),
    ("fe_csr_indices", _i32, [_vp, _vp, _vp, _vp]),
    ("fe_tangent_csr", _i32, [_vp, _vp, _vp, _vp, _i32, _vp]),
    ("fe_apply_matfree", _i32, [_vp, _vp, _vp, _i32, _vp]),
    ("fe_apply_csr", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("fe_diagonal", _i32, [_vp, _vp, _i32, _vp]),
    ("fe_set_preconditioner", _i32, [_vp, _i32]),
    ("fe_apply_csr_nodal", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("fe_set_surrogate_tangent", _i32, [_vp, _i32]),
    ("fe_vjp_path", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("fe_pcg", _i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _dbl, _i32, ctypes.POINTER(PcgInfo), _vp]),
    ("fe_bicgstab", _i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _dbl, _i32, ctypes.POINTER(PcgInfo), _vp]),
    ("fe_apply_preconditioner", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("fe_gmres", _i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _dbl, _i32, _i32, ctypes.POINTER(PcgInfo), _vp]),
    ("fe_vjp", _i32, [_vp, _vp, _vp, _vp, _vp]),
    ("fe_newton", _i32, [_vp, ctypes.POINTER(_dbl), _i32, ctypes.POINTER(NewtonOpts), _vp, _vp,
                         ctypes.POINTER(_dbl), ctypes.POINTER(NewtonInfo), _vp]),
    ("fe_newton_resume", _i32, [_vp, ctypes.POINTER(_dbl), _i32, _i32, ctypes.POINTER(NewtonOpts), _vp, _vp,
                                _vp, ctypes.POINTER(_dbl), ctypes.POINTER(NewtonInfo), _vp]),
    ("fe_mean_stress", _i32, [_vp, _vp, _vp, ctypes.POINTER(_dbl), _vp]),
    ("fe_read_flags", _i32, [_vp, ctypes.POINTER(_i32), _vp]),
    ("fe_profile", _i32, [_vp, _i32]),
    ("fe_profile_read", _i32, [_vp, ctypes.POINTER(_dbl)]),
    ("fe_linearization_stats", _i32, [_vp, ctypes.POINTER(_i64), _vp]),
    ("fe_mlp_forward", _i32, [_vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    ("fe_mlp_backward", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    ("fe_mlp_backward_static", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    ("fe_set_surrogate", _i32, [_vp, _vp, _dbl]),
    ("fe_surrogate_stats", _i32, [_vp, ctypes.POINTER(_i64), _vp]),
    ("fe_set_capture", _i32, [_vp, _vp, _vp, _i64, _vp, _i32]),
    ("fe_adam_step", _i32, [_vp, _vp, _vp, _vp, _i64, _dbl, _dbl, _dbl, _dbl, _i32, _vp]),
    ("fe_status_string", ctypes.c_char_p, [_i32]),
    ("fe_last_error", ctypes.c_char_p, []),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} not found: build it with paper_2604_22087_amd/csrc/build.py")
        lib = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class FeError(RuntimeError):
    def __init__(self, status, where):
        lib = load_library()
        msg = lib.fe_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg})")
        self.status = status


def _check(status, where):
    if status != 0:
        raise FeError(status, where)


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return _vp(0) if t is None else _vp(t.data_ptr())


@dataclass
class PcgResult:
    iterations: int
    status: int
    relres: float
    bnorm: float


class Problem:
    """Hex8 RVE problem on the current GPU (precision 'f64' or 'f32'): the structured n^3 mesh
    of the unit cube, or a general mesh given as mesh=(coords (n_nodes, 3), conn (n_el, 8))
    (numpy or torch; node ids of each element in the local order of include/fe.h)."""

    def __init__(self, n: int | None = None, precision: str = "f64", device=None, mesh=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the finite-element library runs on the GPU only")
        self.lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.prec = F64 if precision == "f64" else F32
        self.dtype = torch.float64 if self.prec == F64 else torch.float32
        h = _vp()
        with torch.cuda.device(self.device):
            if mesh is None:
                _check(self.lib.fe_problem_create(ctypes.byref(h), int(n), self.prec), "fe_problem_create")
            else:
                coords = torch.as_tensor(mesh[0], dtype=torch.float64)
                conn = torch.as_tensor(mesh[1])
                if coords.ndim != 2 or coords.shape[1] != 3 or conn.ndim != 2 or conn.shape[1] != 8:
                    raise ValueError("mesh must be (coords (n_nodes, 3), conn (n_el, 8))")
                c_soa = coords.t().contiguous().to(self.device)              # [3][n_nodes]
                e_soa = conn.to(torch.int32).t().contiguous().to(self.device)  # [8][n_el]
                _check(self.lib.fe_problem_create_hex8(ctypes.byref(h), coords.shape[0], conn.shape[0], _ptr(c_soa),
                                                       _ptr(e_soa), self.prec, _stream()), "fe_problem_create_hex8")
        self.handle = h
        sz = (_i64 * 6)()
        _check(self.lib.fe_problem_sizes(h, sz), "fe_problem_sizes")
        self.n, self.n_el, self.n_nodes, self.n_dof, self.n_qp, self.nnz = (int(v) for v in sz)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fe_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -------------------------------------------------------------------
    def _real(self, t, size, name):
        if t is None:
            return None
        if t.device != self.device or t.dtype != self.dtype or not t.is_contiguous() or t.numel() != size:
            raise ValueError(f"{name}: expected contiguous {self.dtype} tensor of {size} elements on {self.device}")
        return t

    def vector(self):
        return torch.zeros(self.n_dof, dtype=self.dtype, device=self.device)

    def state(self):
        return torch.zeros(7 * 8 * self.n_el, dtype=self.dtype, device=self.device)

    def set_deterministic(self, on=True):
        """Fixed summation orders (no floating-point atomics) in residual, K*x and diagonal."""
        _check(self.lib.fe_set_deterministic(self.handle, int(bool(on))), "fe_set_deterministic")

    def set_fp32_accumulation(self, on=True):
        """FP32 problems: sum the element forces at the nodes in FP32 too (default: FP64 sums)."""
        _check(self.lib.fe_set_fp32_accumulation(self.handle, int(bool(on))), "fe_set_fp32_accumulation")

    def commit_state(self, trial, state):
        """state <- trial (the plastic history of a converged step)."""
        self._real(trial, 7 * 8 * self.n_el, "trial")
        self._real(state, 7 * 8 * self.n_el, "state")
        _check(self.lib.fe_commit_state(self.handle, _ptr(trial), _ptr(state), _stream()), "fe_commit_state")

    # -- setup ---------------------------------------------------------------------
    def set_materials(self, phase, models, params, scale=None):
        """phase: uint8 [n_el] (device); models: list of LINEAR/J2/NEOHOOKE;
        params: list of (E, nu, sigma_y, H); scale: real [n_el] or None."""
        if phase.dtype != torch.uint8 or phase.numel() != self.n_el or phase.device != self.device:
            raise ValueError("phase must be a uint8 device tensor with one entry per element")
        phase = phase.contiguous()
        k = len(models)
        m = (_i32 * k)(*models)
        flat = [float(v) for row in params for v in (list(row) + [0.0] * (4 - len(row)))]
        pr = (_dbl * (4 * k))(*flat)
        self._real(scale, self.n_el, "scale")
        _check(self.lib.fe_set_materials(self.handle, _ptr(phase), k, m, pr, _ptr(scale), _stream()),
               "fe_set_materials")

    def set_dirichlet(self, mask):
        if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != self.n_dof):
            raise ValueError("mask must be uint8 with one entry per dof")
        _check(self.lib.fe_set_dirichlet(self.handle, _ptr(mask), _stream()), "fe_set_dirichlet")

    def lift(self, eps_bar, u, zero_free=False):
        e = (_dbl * 9)(*[float(v) for v in torch.as_tensor(eps_bar, dtype=torch.float64).reshape(-1)])
        self._real(u, self.n_dof, "u")
        _check(self.lib.fe_lift(self.handle, e, _ptr(u), int(zero_free), _stream()), "fe_lift")
        return u

    # -- element operations ------------------------------------------------------------
    def residual(self, u, state_in=None, state_out=None, r=None, apply_bc=False, store_tangent=False):
        self._real(u, self.n_dof, "u")
        self._real(state_in, 56 * self.n_el, "state_in")
        self._real(state_out, 56 * self.n_el, "state_out")
        r = self.vector() if r is None else self._real(r, self.n_dof, "r")
        flags = (APPLY_BC if apply_bc else 0) | (STORE_TANGENT if store_tangent else 0)
        _check(self.lib.fe_residual(self.handle, _ptr(u), _ptr(state_in), _ptr(state_out), _ptr(r), flags,
                                    _stream()), "fe_residual")
        return r

    def csr_indices(self):
        rp = torch.empty(self.n_dof + 1, dtype=torch.int32, device=self.device)
        ci = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        _check(self.lib.fe_csr_indices(self.handle, _ptr(rp), _ptr(ci), _stream()), "fe_csr_indices")
        return rp, ci

    def tangent_csr(self, u, state_in=None, vals=None, apply_bc=False):
        self._real(u, self.n_dof, "u")
        self._real(state_in, 56 * self.n_el, "state_in")
        vals = torch.empty(self.nnz, dtype=self.dtype, device=self.device) if vals is None else \
            self._real(vals, self.nnz, "vals")
        _check(self.lib.fe_tangent_csr(self.handle, _ptr(u), _ptr(state_in), _ptr(vals), int(apply_bc),
                                       _stream()), "fe_tangent_csr")
        return vals

    def apply_matfree(self, x, y=None, apply_bc=False):
        self._real(x, self.n_dof, "x")
        y = self.vector() if y is None else self._real(y, self.n_dof, "y")
        _check(self.lib.fe_apply_matfree(self.handle, _ptr(x), _ptr(y), int(apply_bc), _stream()),
               "fe_apply_matfree")
        return y

    def apply_csr(self, row_ptr, col_idx, vals, x, y=None):
        self._real(x, self.n_dof, "x")
        y = self.vector() if y is None else self._real(y, self.n_dof, "y")
        _check(self.lib.fe_apply_csr(self.handle, _ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(x), _ptr(y),
                                     _stream()), "fe_apply_csr")
        return y

    def apply_csr_nodal(self, row_ptr, col_idx, vals, x, y=None):
        """y = A x for a matrix in the node-structured pattern of csr_indices()."""
        self._real(x, self.n_dof, "x")
        y = self.vector() if y is None else self._real(y, self.n_dof, "y")
        _check(self.lib.fe_apply_csr_nodal(self.handle, _ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(x), _ptr(y),
                                           _stream()), "fe_apply_csr_nodal")
        return y

    def diagonal(self, apply_bc=False, d=None):
        d = self.vector() if d is None else self._real(d, self.n_dof, "d")
        _check(self.lib.fe_diagonal(self.handle, _ptr(d), int(apply_bc), _stream()), "fe_diagonal")
        return d

    def set_preconditioner(self, kind):
        """PC_JACOBI (point) or PC_BLOCK_JACOBI (3x3 node blocks) for pcg and newton."""
        _check(self.lib.fe_set_preconditioner(self.handle, int(kind)), "fe_set_preconditioner")

    def pcg(self, b, x=None, op=OP_MATFREE, csr=None, rtol=1e-10, max_it=100000, check=True, solver=SOLVER_CG,
            restart=30):
        """Preconditioned CG (BiCGStab with solver=SOLVER_BICGSTAB, GMRES(restart) with
        solver=SOLVER_GMRES) on the masked operator."""
        self._real(b, self.n_dof, "b")
        x = self.vector() if x is None else self._real(x, self.n_dof, "x")
        rp, ci, v = csr if csr is not None else (None, None, None)
        info = PcgInfo()
        args = (self.handle, int(op), _ptr(rp), _ptr(ci), _ptr(v), _ptr(b), _ptr(x), float(rtol), int(max_it))
        if solver == SOLVER_GMRES:
            name = "fe_gmres"
            st = self.lib.fe_gmres(*args, int(restart), ctypes.byref(info), _stream())
        else:
            fn, name = (self.lib.fe_bicgstab, "fe_bicgstab") if solver == SOLVER_BICGSTAB else \
                (self.lib.fe_pcg, "fe_pcg")
            st = fn(*args, ctypes.byref(info), _stream())
        if check:
            _check(st, name)
        return x, PcgResult(info.iterations, info.status, info.relres, info.bnorm)

    def apply_preconditioner(self, r, csr=None, z=None):
        """z = M^-1 r for the current preconditioner (from the CSR matrix when given)."""
        self._real(r, self.n_dof, "r")
        z = self.vector() if z is None else self._real(z, self.n_dof, "z")
        rp, ci, v = csr if csr is not None else (None, None, None)
        _check(self.lib.fe_apply_preconditioner(self.handle, _ptr(rp), _ptr(ci), _ptr(v), _ptr(r), _ptr(z),
                                                _stream()), "fe_apply_preconditioner")
        return z

    def vjp(self, u, lam, out=None):
        self._real(u, self.n_dof, "u")
        self._real(lam, self.n_dof, "lambda")
        out = torch.empty(self.n_el, dtype=self.dtype, device=self.device) if out is None else \
            self._real(out, self.n_el, "out")
        _check(self.lib.fe_vjp(self.handle, _ptr(u), _ptr(lam), _ptr(out), _stream()), "fe_vjp")
        return out

    def vjp_path(self, u, state_in, c=None, mu_in=None, mu_out=None, u_bar=None, s_bar=None):
        """One backward step through the return map (FP64): writes mu_out = d(c.R + mu_in.h)/d h_in,
        accumulates u_bar += d(mu_in.h)/du and s_bar += d(c.R + mu_in.h)/ds.  Returns mu_out."""
        self._real(u, self.n_dof, "u")
        mu_out = self.state() if mu_out is None else self._real(mu_out, 56 * self.n_el, "mu_out")
        for t, size, name in ((state_in, 56 * self.n_el, "state_in"), (c, self.n_dof, "c"),
                              (mu_in, 56 * self.n_el, "mu_in"), (u_bar, self.n_dof, "u_bar"),
                              (s_bar, self.n_el, "s_bar")):
            if t is not None:
                self._real(t, size, name)
        _check(self.lib.fe_vjp_path(self.handle, _ptr(u), _ptr(state_in), _ptr(c), _ptr(mu_in), _ptr(mu_out),
                                    _ptr(u_bar), _ptr(s_bar), _stream()), "fe_vjp_path")
        return mu_out

    def newton(self, load_path, u=None, state=None, op=OP_MATFREE, max_newton=20, newton_rtol=1e-8,
               pcg_rtol=1e-10, pcg_max_it=100000, assemble_csr=False, check=True, solver=SOLVER_CG, restart=0,
               predictor=PREDICT_BOUNDARY, first_step=0, u_prev=None):
        """Load stepping; load_path: sequence of 3x3 macro strains. Returns (u, state, sigma_bar, info);
        info["steps"] lists (Newton iterations, line-search halvings, Krylov iterations) per load step.
        first_step > 0 resumes the same path at that step (fe_newton_resume): u and state are then
        the converged field and committed state of step first_step - 1, u_prev the field of step
        first_step - 2 (extrapolating predictor only); sigma_bar and info["steps"] cover the
        resumed steps."""
        path = torch.as_tensor(np.asarray(load_path, dtype=np.float64)).reshape(-1, 9)
        k = path.shape[0]
        pa = (_dbl * (9 * k))(*path.reshape(-1).tolist())
        u = self.vector() if u is None else self._real(u, self.n_dof, "u")
        self._real(state, 56 * self.n_el, "state")
        self._real(u_prev, self.n_dof, "u_prev")
        log = (_i32 * (3 * max(k, 1)))()
        opts = NewtonOpts(int(op), int(bool(assemble_csr)), int(max_newton), float(newton_rtol), float(pcg_rtol),
                          int(pcg_max_it), int(solver), int(restart), int(predictor),
                          ctypes.cast(log, ctypes.POINTER(_i32)))
        sig = (_dbl * (6 * max(k, 1)))()
        info = NewtonInfo()
        if first_step:
            st = self.lib.fe_newton_resume(self.handle, pa, k, int(first_step), ctypes.byref(opts), _ptr(u),
                                           _ptr(u_prev), _ptr(state), sig, ctypes.byref(info), _stream())
        else:
            st = self.lib.fe_newton(self.handle, pa, k, ctypes.byref(opts), _ptr(u), _ptr(state), sig,
                                    ctypes.byref(info), _stream())
        if check:
            _check(st, "fe_newton_resume" if first_step else "fe_newton")
        f0 = int(first_step)
        sb = [list(sig[6 * i:6 * i + 6]) for i in range(f0, k)]
        out = {f: getattr(info, f) for f, _ in NewtonInfo._fields_}
        out["steps"] = [tuple(log[3 * i:3 * i + 3]) for i in range(f0, f0 + info.steps_done)]
        return u, state, sb, out

    def mean_stress(self, u, state_in=None):
        self._real(u, self.n_dof, "u")
        out = (_dbl * 6)()
        _check(self.lib.fe_mean_stress(self.handle, _ptr(u), _ptr(state_in), out, _stream()), "fe_mean_stress")
        return list(out)

    def read_flags(self):
        f = _i32()
        _check(self.lib.fe_read_flags(self.handle, ctypes.byref(f), _stream()), "fe_read_flags")
        return f.value

    # -- measurement -------------------------------------------------------------------
    KERNEL_CLASSES = ("matfree_apply", "csr_spmv", "residual", "tangent_csr", "csr_spmv_nodal")

    def profile(self, enable=True):
        _check(self.lib.fe_profile(self.handle, int(enable)), "fe_profile")

    def profile_read(self):
        """{class: (launches, total_ms, algorithmic_bytes)} since profiling was enabled (synchronises)."""
        out = (_dbl * 15)()
        _check(self.lib.fe_profile_read(self.handle, out), "fe_profile_read")
        return {k: (int(out[3 * i]), float(out[3 * i + 1]), float(out[3 * i + 2]))
                for i, k in enumerate(self.KERNEL_CLASSES)}

    def set_surrogate(self, W, fallback_tol=1e-3):
        """Use the network (float32 [35590] device tensor, kept alive by the caller) at plastic-trial J2 points."""
        if W is not None:
            _f32(W, MLP_PARAMS, "W")
        self._sur_W = W
        _check(self.lib.fe_set_surrogate(self.handle, _ptr(W), float(fallback_tol)), "fe_set_surrogate")

    def set_surrogate_tangent(self, full):
        """True: the network Jacobian itself as tangent (nonsymmetric; use solver=SOLVER_BICGSTAB)."""
        _check(self.lib.fe_set_surrogate_tangent(self.handle, int(bool(full))), "fe_set_surrogate_tangent")

    def surrogate_stats(self):
        out = (_i64 * 3)()
        _check(self.lib.fe_surrogate_stats(self.handle, out, _stream()), "fe_surrogate_stats")
        return dict(listed=int(out[0]), accepted=int(out[1]), fallback=int(out[2]))

    def set_capture(self, x=None, y=None, count=None, stride=1):
        """Append (normalised input, exact stress) samples at plastic-trial J2 points on every residual."""
        cap = 0 if x is None else x.shape[0]
        self._capture = (x, y, count)
        _check(self.lib.fe_set_capture(self.handle, _ptr(x), _ptr(y), cap, _ptr(count), int(stride)),
               "fe_set_capture")

    def linearization_stats(self):
        out = (_i64 * 2)()
        _check(self.lib.fe_linearization_stats(self.handle, out, _stream()), "fe_linearization_stats")
        return int(out[0]), int(out[1])


# ---- surrogate network (float32 device tensors) ---------------------------------------
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 13, 128, 6, 35590


def _f32(t, size, name):
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != size:
        raise ValueError(f"{name}: expected a contiguous float32 CUDA tensor of {size} elements")
    return t


def mlp_forward(W, x, jacobian=False, cache=False):
    """y [n,6] (+ jac [n,6,6] = dy/dx[:, :6], + pre-activation cache [n,3,128])."""
    lib = load_library()
    n = x.shape[0]
    _f32(W, MLP_PARAMS, "W")
    _f32(x, n * MLP_IN, "x")
    y = torch.empty(n, MLP_OUT, dtype=torch.float32, device=x.device)
    jac = torch.empty(n, MLP_OUT, MLP_OUT, dtype=torch.float32, device=x.device) if jacobian else None
    c = torch.empty(n, 3, MLP_HIDDEN, dtype=torch.float32, device=x.device) if cache else None
    _check(lib.fe_mlp_forward(_ptr(W), _ptr(x), _ptr(y), _ptr(jac), _ptr(c), n, _stream()), "fe_mlp_forward")
    return y, jac, c


def mlp_backward(W, x, cache, y, target):
    """(dW [35590], loss (device double scalar)) of the mean squared error of one batch."""
    lib = load_library()
    n = x.shape[0]
    dW = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float64, device=x.device)
    work = torch.empty(n, 3 * MLP_HIDDEN + MLP_OUT, dtype=torch.float32, device=x.device)
    _check(lib.fe_mlp_backward(_ptr(W), _ptr(x), _ptr(cache), _ptr(y), _ptr(target), _ptr(dW), _ptr(loss),
                               _ptr(work), n, _stream()), "fe_mlp_backward")
    return dW, loss


MLP_STATIC_MAX = 8192


def mlp_backward_static(W, x, cache, y, target, dW=None, loss=None):
    """mlp_backward through the entry point that allocates nothing (library-owned workspace,
    n <= MLP_STATIC_MAX); dW and loss may be given to keep the call allocation-free here too."""
    lib = load_library()
    n = x.shape[0]
    if dW is None:
        dW = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(lib.fe_mlp_backward_static(_ptr(W), _ptr(x), _ptr(cache), _ptr(y), _ptr(target), _ptr(dW), _ptr(loss),
                                      n, _stream()), "fe_mlp_backward_static")
    return dW, loss


def adam_step(W, dW, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    lib = load_library()
    _check(lib.fe_adam_step(_ptr(W), _ptr(dW), _ptr(m), _ptr(v), W.numel(), float(lr), float(beta1), float(beta2),
                            float(eps), int(t), _stream()), "fe_adam_step")
