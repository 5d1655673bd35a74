"""Load-step snapshots of a Newton ramp and a load-stepping driver that resumes from them.

A snapshot holds what the next load step of the ramp depends on (Sec. II-A: each step solves
R(u) = 0 from the converged field of the previous one; Sec. V-A: the plastic history of the J2
phases is committed at the end of every step): the converged displacement u, the committed
state (plastic strain and equivalent plastic strain per Gauss point, [7][8][n_el]), and for the
extrapolating predictor the converged field one step earlier, together with the load path, the
index of the last converged step, the homogenised stresses and the per-step solver log.  The
file is safetensors (tensors on the host, metadata as JSON text), written to a temporary name
and renamed, so an interrupted write leaves the previous snapshot in place.

Resuming calls fe_newton_resume, which runs exactly the arithmetic of an uninterrupted
fe_newton call over the same path: in deterministic mode a resumed ramp is bit-identical to
one that was never stopped.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

FORMAT = "fe-load-step-snapshot/1"


def save_snapshot(file, P, step, load_path, u, state=None, u_prev=None, sigma_bar=(), step_log=(), options=None):
    """Write the snapshot taken after load step `step` (0-based) of `load_path` to `file`."""
    from safetensors.torch import save_file
    tensors = {"u": u.detach().contiguous().cpu()}
    if state is not None:
        tensors["state"] = state.detach().contiguous().cpu()
    if u_prev is not None:
        tensors["u_prev"] = u_prev.detach().contiguous().cpu()
    path = np.asarray(load_path, dtype=np.float64).reshape(-1, 9)
    meta = {"format": FORMAT, "n_dof": P.n_dof, "n_el": P.n_el, "dtype": str(P.dtype).replace("torch.", ""),
            "step": int(step), "load_path": path.tolist(), "sigma_bar": [list(map(float, s)) for s in sigma_bar],
            "step_log": [list(map(int, t)) for t in step_log], "options": options or {}}
    tmp = f"{file}.tmp"
    save_file(tensors, tmp, metadata={"snapshot": json.dumps(meta)})
    os.replace(tmp, file)


def load_snapshot(file, P):
    """Read a snapshot for problem P: a dict with u, state, u_prev (tensors on P's device, or
    None) and the metadata fields.  Raises ValueError when the file belongs to another problem
    size or precision."""
    from safetensors import safe_open
    with safe_open(file, framework="pt", device="cpu") as f:
        meta = json.loads(f.metadata()["snapshot"])
        if meta.get("format") != FORMAT:
            raise ValueError(f"{file}: not a load-step snapshot")
        if meta["n_dof"] != P.n_dof or meta["n_el"] != P.n_el:
            raise ValueError(f"{file}: snapshot of a problem with {meta['n_dof']} dofs / {meta['n_el']} elements")
        if meta["dtype"] != str(P.dtype).replace("torch.", ""):
            raise ValueError(f"{file}: snapshot in {meta['dtype']}, problem in {P.dtype}")
        keys = set(f.keys())
        out = dict(meta)
        for k in ("u", "state", "u_prev"):
            out[k] = f.get_tensor(k).to(P.device) if k in keys else None
    return out


def newton_checkpointed(P, load_path, file, u=None, state=None, every=1, resume=True, stop_after=None,
                        **newton_kwargs):
    """Newton load stepping over `load_path` with a snapshot in `file` after every `every`-th
    converged step (and after the last).  With resume=True and `file` present, the ramp
    continues after the snapshot's step (the path must agree with the stored one).
    stop_after: return once that many steps (counted over the whole path) have converged.
    Other keywords go to Problem.newton.  Returns (u, state, sigma_bar, info) over the whole
    path: sigma_bar and info["steps"] include the steps taken before a resume."""
    path = np.asarray(load_path, dtype=np.float64).reshape(-1, 9)
    K = path.shape[0]
    u = P.vector() if u is None else u
    u_prev = None
    k0, sig, log = 0, [], []
    extrapolate = newton_kwargs.get("predictor", 0) != 0
    if resume and os.path.exists(file):
        snap = load_snapshot(file, P)
        stored = np.asarray(snap["load_path"], dtype=np.float64).reshape(-1, 9)
        done = snap["step"] + 1
        if done > K or not np.array_equal(stored[:done], path[:done]):
            raise ValueError(f"{file}: snapshot of a different load path")
        u.copy_(snap["u"])
        if state is not None:
            if snap["state"] is None:
                raise ValueError(f"{file}: snapshot holds no state")
            state.copy_(snap["state"])
        u_prev = snap["u_prev"]
        k0 = snap["step"] + 1
        sig, log = list(snap["sigma_bar"]), [tuple(t) for t in snap["step_log"]]
    totals = {"newton_iterations": 0, "pcg_iterations": 0, "operator_applies": 0, "line_search_halvings": 0}
    info = {"status": 0}
    last = K if stop_after is None else min(K, int(stop_after))
    for k in range(k0, last):
        before = u.clone() if extrapolate else None
        # one step per call: path[:k + 1] resumed at step k runs the uninterrupted ramp's step k
        _, _, sb, info = P.newton(path[:k + 1], u=u, state=state, first_step=k,
                                  u_prev=u_prev if (extrapolate and k >= 2) else None, **newton_kwargs)
        if info["steps_done"] != 1:
            break
        sig += sb
        log += info["steps"]
        for f in totals:
            totals[f] += info[f]
        u_prev = before
        if (k + 1 - k0) % every == 0 or k + 1 == last:
            save_snapshot(file, P, k, path, u, state, u_prev if extrapolate else None, sig, log,
                          {key: (v if isinstance(v, (int, float, bool)) else str(v)) for key, v in newton_kwargs.items()})
    out = dict(info)
    out.update(totals)
    out["steps"] = log
    out["steps_done"] = len(log)
    return u, state, sig, out
