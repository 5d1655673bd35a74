"""Learned constitutive surrogate in place of the J2 return map (oracle).

The paper remarks that a surrogate model can replace the designed stress-strain
function with its Jacobian extracted the same way (Sec. III-B).  Readings used:
  * the network sees x = [eps_trial (6), eps_p_n (6), alpha_n] / s_in with
    eps_trial = eps_{n+1} - eps_p_n, strains in Mandel form (shear components
    times sqrt(2) of the tensor ones), and returns sigma_Mandel / s_out;
    s_in = sigma_y / E, s_out = sigma_y of the plastic phase;
  * the tangent is d sigma / d eps_{n+1} = (s_out / s_in) dy/dx[:, :6]; in the
    Voigt form used by the B-operator (tensor stress, engineering shear strain)
    shear rows and shear columns are each divided by sqrt(2);
  * history from the predicted stress: eps_p_{n+1} = eps_{n+1} - C^-1 sigma_hat,
    alpha_{n+1} = alpha_n + sqrt(2/3) |eps_p_{n+1} - eps_p_n|_F (tensor norm);
  * it runs only at plastic-phase points whose elastic trial is plastic
    (f_trial > 0); elsewhere the exact law is used;
  * local check r_loc = max(|q(sigma_hat) - sigma_y - H alpha_{n+1}| / sigma_y,
    |dev sigma_hat / |dev sigma_hat| - N_trial|_F); above `tol` the exact return
    map is used instead (fallback).
"""
from __future__ import annotations

import numpy as np

from . import j2
from .elasticity import hooke_voigt, lame

SQ2 = np.sqrt(2.0)
SHEAR = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])


def strain_voigt_to_mandel(e):
    """engineering-shear Voigt strain -> Mandel (shear = sqrt(2) * tensor = gamma / sqrt(2))."""
    return e * np.array([1.0, 1.0, 1.0, 1 / SQ2, 1 / SQ2, 1 / SQ2])


def stress_voigt_to_mandel(s):
    return s * SHEAR


def stress_mandel_to_voigt(m):
    return m / SHEAR


def network_inputs(eps, eps_p_n, alpha_n, s_in):
    """(m, 13) normalised network inputs."""
    x = np.concatenate([strain_voigt_to_mandel(eps - eps_p_n), strain_voigt_to_mandel(eps_p_n),
                        alpha_n[:, None]], axis=1)
    return x / s_in


def update(eps, eps_p_n, alpha_n, E, nu, sigma_y, H, net, s_in, s_out, tol):
    """Surrogate constitutive update at m points.

    net(x) -> (y (m,6), dy/dx[:, :, :6] (m,6,6)) on normalised inputs.
    Returns dict(sigma, D, eps_p, alpha, used (surrogate accepted), plastic_trial, r_loc).
    """
    exact = j2.return_map(eps, eps_p_n, alpha_n, E, nu, sigma_y, H)
    trial = exact["plastic"]
    out = dict(sigma=exact["sigma"].copy(), D=exact["D"].copy(), eps_p=exact["eps_p"].copy(),
               alpha=exact["alpha"].copy(), used=np.zeros(len(eps), dtype=bool), plastic_trial=trial,
               r_loc=np.zeros(len(eps)))
    idx = np.flatnonzero(trial)
    if len(idx) == 0:
        return out
    x = network_inputs(eps[idx], eps_p_n[idx], alpha_n[idx], s_in)
    y, jac = net(x)
    sig = stress_mandel_to_voigt(s_out * y)
    d_m = (s_out / s_in) * jac
    c = 1.0 / SHEAR
    D = d_m * c[None, :, None] * c[None, None, :]
    lam, mu = lame(E, nu)
    comp = np.linalg.inv(hooke_voigt(lam, mu))
    ep = eps[idx] - sig @ comp.T
    dep = j2.strain_to_tensor(ep - eps_p_n[idx])
    al = alpha_n[idx] + np.sqrt(2.0 / 3.0) * np.sqrt(np.sum(dep * dep, axis=(1, 2)))
    # local residual of the prediction
    st = j2.strain_to_tensor(np.concatenate([sig[:, :3], 2 * sig[:, 3:]], axis=1))
    dev = st - np.trace(st, axis1=1, axis2=2)[:, None, None] / 3 * np.eye(3)
    dn = np.sqrt(np.sum(dev * dev, axis=(1, 2)))
    q = np.sqrt(1.5) * dn
    n_tr = j2.strain_to_tensor(np.concatenate([exact["N"][idx][:, :3], 2 * exact["N"][idx][:, 3:]], axis=1))
    dir_err = np.sqrt(np.sum((dev / np.where(dn > 0, dn, 1)[:, None, None] - n_tr) ** 2, axis=(1, 2)))
    r_loc = np.maximum(np.abs(q - sigma_y - H * al) / sigma_y, dir_err)
    ok = r_loc <= tol
    acc = idx[ok]
    out["sigma"][acc] = sig[ok]
    out["D"][acc] = D[ok]
    out["eps_p"][acc] = ep[ok]
    out["alpha"][acc] = al[ok]
    out["used"][acc] = True
    out["r_loc"][idx] = r_loc
    return out
