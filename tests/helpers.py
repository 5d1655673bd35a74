"""Shared test utilities: layout conversion between the oracle and the library, error norms."""
import numpy as np

PHASES_CONFIG1 = [("linear", 3.5, 0.35), ("linear", 70.0, 0.22)]
PHASES_J2_FIBER = [("j2", 3.5, 0.35, 0.05, 0.1), ("linear", 230.0, 0.2)]


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def state_to_lib(eps_p, alpha):
    """Oracle state (n_el,8,6), (n_el,8) -> library layout [7][8][n_el] (flat)."""
    return np.concatenate([eps_p.transpose(2, 1, 0), alpha.T[None]], axis=0).reshape(-1).copy()


def state_from_lib(flat, n_el):
    a = np.asarray(flat, dtype=np.float64).reshape(7, 8, n_el)
    return a[:6].transpose(2, 1, 0).copy(), a[6].T.copy()


def oracle_phases(spec):
    from oracle.rve import phase_params
    return [phase_params(*s) for s in spec]


def lib_materials(spec):
    from paper_2604_22087_amd import fe
    kinds = {"linear": fe.LINEAR, "j2": fe.J2, "neohooke": fe.NEOHOOKE}
    models = [kinds[s[0]] for s in spec]
    params = [tuple(s[1:]) + (0.0,) * (5 - len(s)) for s in spec]
    return models, params
