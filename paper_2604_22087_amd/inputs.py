"""Seeded synthetic inputs for the heterogeneous micromechanics RVE.

The paper's benchmark (Sec. V-A) is a two-phase composite RVE whose meshes,
microstructures and fields are not published; these generators stand in for
them.  Every array is a pure function of its arguments and seed.  This module
holds geometry and random-number recipes only: no finite-element arithmetic
(no shape functions, stresses, assembly or solves), so the CPU oracle and the
HIP path can both be fed from it without sharing any of the method.

Conventions of the structured cube mesh on [0,1]^3 with n elements per side:
  element (a,b,c) has id a + n*(b + n*c) and centroid ((a+.5)h, (b+.5)h, (c+.5)h)
  node (i,j,k) has id i + (n+1)*(j + (n+1)*k); dof = 3*node + component.
Phase ids: 0 = matrix, 1 = inclusion / fiber.
"""
from __future__ import annotations

import numpy as np

MATRIX, INCLUSION = 0, 1


def element_centroids(n: int) -> np.ndarray:
    """(n^3, 3) centroids of the elements of the n^3 unit-cube mesh, element order."""
    h = 1.0 / n
    c1 = (np.arange(n) + 0.5) * h
    cz, cy, cx = np.meshgrid(c1, c1, c1, indexing="ij")  # a (x) varies fastest
    return np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)


def sphere_phase(n: int, radius: float = 0.3, center=(0.5, 0.5, 0.5)) -> np.ndarray:
    """Centered spherical inclusion: phase 1 where |centroid - center| < radius (strict)."""
    d = element_centroids(n) - np.asarray(center, dtype=np.float64)
    return (np.einsum("ij,ij->i", d, d) < radius * radius).astype(np.uint8)


def rsa_fiber_centers(n_fibers: int = 64, radius: float = 0.05, seed: int = 2,
                      max_attempts: int = 10_000_000) -> np.ndarray:
    """Periodic random sequential addition of non-overlapping disks in [0,1)^2.

    Candidates are successive uniform pairs from numpy's default_rng(seed)
    (PCG64); a candidate is kept when its minimum-image distance to every kept
    center is at least 2*radius.  Raises if max_attempts candidates run out.
    """
    rng = np.random.default_rng(seed)
    centers = np.empty((0, 2))
    attempts, block = 0, 4096
    min_d2 = (2.0 * radius) ** 2
    while len(centers) < n_fibers:
        cand = rng.random((block, 2))
        for p in cand:
            attempts += 1
            if attempts > max_attempts:
                raise RuntimeError("RSA did not place all fibers")
            if len(centers):
                d = centers - p
                d -= np.round(d)  # minimum image on the unit torus
                if np.min(np.einsum("ij,ij->i", d, d)) < min_d2:
                    continue
            centers = np.vstack([centers, p])
            if len(centers) == n_fibers:
                break
    return centers


def fiber_phase(n: int, n_fibers: int = 64, radius: float = 0.05, seed: int = 2) -> np.ndarray:
    """z-aligned cylindrical fibers: phase 1 where the centroid's (x,y) lies strictly
    within radius of a fiber center (minimum image)."""
    centers = rsa_fiber_centers(n_fibers, radius, seed)
    xy = element_centroids(n)[:, :2]
    phase = np.zeros(len(xy), dtype=np.uint8)
    for c in centers:
        d = xy - c
        d -= np.round(d)
        phase |= (np.einsum("ij,ij->i", d, d) < radius * radius).astype(np.uint8)
    return phase


def lognormal_field(n: int, mean: float = 1.0, cov: float = 0.5, corr_len: float = 0.1,
                    seed: int = 3) -> np.ndarray:
    """Per-element log-normal field with separable exponential correlation.

    g is a unit Gaussian field with covariance exp(-(|dx|+|dy|+|dz|)/corr_len) on
    the element centroids, sampled exactly by a stationary AR(1) recursion along
    each axis (g_0 = xi_0, g_k = rho g_{k-1} + sqrt(1-rho^2) xi_k, rho = exp(-h/corr_len)).
    The field is mean * exp(m + s g) with s^2 = ln(1 + cov^2), m = -s^2/2.
    """
    h = 1.0 / n
    rho = np.exp(-h / corr_len)
    c = np.sqrt(1.0 - rho * rho)
    g = np.random.default_rng(seed).standard_normal((n, n, n))  # [c][b][a]
    for axis in (2, 1, 0):
        g = np.moveaxis(g, axis, 0).copy()
        for k in range(1, n):
            g[k] = rho * g[k - 1] + c * g[k]
        g = np.moveaxis(g, 0, axis)
    s2 = np.log1p(cov * cov)
    return mean * np.exp(-0.5 * s2 + np.sqrt(s2) * g.reshape(-1))


def uniform_field(n_items: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """i.i.d. U(lo, hi) per item from default_rng(seed)."""
    return np.random.default_rng(seed).uniform(lo, hi, n_items)


def random_displacement(n: int, lo: float = -1e-3, hi: float = 1e-3, seed: int = 1) -> np.ndarray:
    """U(lo, hi) on every dof of the n^3 mesh (interleaved dof = 3*node + c)."""
    return np.random.default_rng(seed).uniform(lo, hi, 3 * (n + 1) ** 3)


def boundary_dof_mask(n: int) -> np.ndarray:
    """uint8 per dof: 1 for all three dofs of every node with an index in {0, n}."""
    idx = np.arange(n + 1)
    on = (idx == 0) | (idx == n)
    kk, jj, ii = np.meshgrid(on, on, on, indexing="ij")
    node = (ii | jj | kk).ravel().astype(np.uint8)
    return np.repeat(node, 3)


def glorot_uniform_params(layers=(13, 128, 128, 128, 6), seed: int = 5):
    """Initial MLP weights: W_l (out, in) ~ U(-a, a), a = sqrt(6 / (in + out)), b_l = 0,
    drawn layer by layer from default_rng(seed).  Returns a list of (W, b) float64 arrays."""
    rng = np.random.default_rng(seed)
    params = []
    for fan_in, fan_out in zip(layers[:-1], layers[1:]):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        params.append((rng.uniform(-a, a, (fan_out, fan_in)), np.zeros(fan_out)))
    return params


def fd_element_picks(n_el: int, count: int = 64, seed: int = 40) -> np.ndarray:
    """Element ids for the finite-difference gradient check."""
    return np.sort(np.random.default_rng(seed).choice(n_el, count, replace=False))


# ---- general (unstructured-numbered, distorted) hexahedral meshes of the unit cube ------------

def _cube_rotations():
    """The 24 proper rotations of the cube as 3x3 integer matrices."""
    gens = [np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]]), np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]])]
    found = [np.eye(3, dtype=np.int64)]
    frontier = list(found)
    while frontier:
        nxt = []
        for r in frontier:
            for g in gens:
                m = g @ r
                if not any(np.array_equal(m, f) for f in found):
                    found.append(m)
                    nxt.append(m)
        frontier = nxt
    return found


# corner offsets of the local node order (0,0,0) (1,0,0) (1,1,0) (0,1,0) (0,0,1) (1,0,1) (1,1,1) (0,1,1)
LOCAL_CORNERS = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                          [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)


def distorted_cube_mesh(n: int, amplitude: float = 0.25, seed: int = 7, permute: bool = True):
    """Hex8 mesh of [0,1]^3 with n elements per side, distorted and renumbered.

    Starts from the n^3 grid; interior nodes move by U(-a h, a h) per component, face
    nodes (not on an edge) within their face, edge nodes along their edge, corners stay
    (a = amplitude), so the mesh still fills the unit cube exactly.  With permute: the
    nodes and the elements are renumbered by random permutations, and each element's
    local node order is one of the 24 proper rotations of the reference cube, drawn per
    element (every local order stays right-handed).  All draws come from
    default_rng(seed).  Returns (coords (n_nodes, 3) float64, conn (n_el, 8) int64 with
    conn[e, p] = node of local node p).
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    idx = np.arange(n + 1)
    kk, jj, ii = np.meshgrid(idx, idx, idx, indexing="ij")
    grid = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)        # node (i,j,k), i fastest
    coords = grid * h
    on = (grid == 0) | (grid == n)                                        # per component: on a boundary plane
    move = ~on                                                            # a component moves unless pinned
    coords = coords + move * rng.uniform(-amplitude * h, amplitude * h, coords.shape)
    a, b, c = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([c.ravel(), b.ravel(), a.ravel()], axis=1)            # element (a,b,c), a fastest
    corner = base[:, None, :] + LOCAL_CORNERS[None, :, :]                 # (n_el, 8, 3)
    conn = corner[..., 0] + (n + 1) * (corner[..., 1] + (n + 1) * corner[..., 2])
    if permute:
        rots = _cube_rotations()
        # local node p of the rotated element sits at corner R (s_p) of the original one
        signs = 2 * LOCAL_CORNERS - 1
        perms = []
        for r in rots:
            img = signs @ r.T
            perms.append([int(np.flatnonzero((signs == v).all(axis=1))[0]) for v in img])
        perms = np.array(perms)
        pick = rng.integers(0, len(rots), len(conn))
        conn = np.take_along_axis(conn, perms[pick], axis=1)
        node_perm = rng.permutation(len(coords))                          # new id of old node
        new_coords = np.empty_like(coords)
        new_coords[node_perm] = coords
        coords = new_coords
        conn = node_perm[conn]
        conn = conn[rng.permutation(len(conn))]
    return coords, conn


def mesh_centroids(coords, conn) -> np.ndarray:
    """(n_el, 3) mean of each element's 8 node positions."""
    return np.asarray(coords)[np.asarray(conn)].mean(axis=1)


def sphere_phase_mesh(coords, conn, radius: float = 0.3, center=(0.5, 0.5, 0.5)) -> np.ndarray:
    """Phase 1 where the element's node-mean centroid lies strictly within radius of center."""
    d = mesh_centroids(coords, conn) - np.asarray(center, dtype=np.float64)
    return (np.einsum("ij,ij->i", d, d) < radius * radius).astype(np.uint8)


def fiber_phase_mesh(coords, conn, n_fibers: int = 64, radius: float = 0.05, seed: int = 2) -> np.ndarray:
    """fiber_phase on a general mesh: phase 1 where the element's node-mean centroid (x,y)
    lies strictly within radius of a fiber center (minimum image)."""
    centers = rsa_fiber_centers(n_fibers, radius, seed)
    xy = mesh_centroids(coords, conn)[:, :2]
    phase = np.zeros(len(xy), dtype=np.uint8)
    for c in centers:
        d = xy - c
        d -= np.round(d)
        phase |= (np.einsum("ij,ij->i", d, d) < radius * radius).astype(np.uint8)
    return phase


def boundary_dof_mask_mesh(coords, tol: float = 1e-12) -> np.ndarray:
    """uint8 per dof: 1 for all three dofs of every node on a face of the unit cube."""
    c = np.asarray(coords)
    node = np.any((c < tol) | (c > 1.0 - tol), axis=1).astype(np.uint8)
    return np.repeat(node, 3)


def random_field_mesh(n_nodes: int, lo: float = -1e-3, hi: float = 1e-3, seed: int = 1) -> np.ndarray:
    """U(lo, hi) on every dof of a mesh with n_nodes nodes."""
    return np.random.default_rng(seed).uniform(lo, hi, 3 * n_nodes)
