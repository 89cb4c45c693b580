"""Seeded synthetic inputs for the hex-mesh mass/diffusion workloads.

This module only draws random numbers and evaluates the problem data (the
manufactured solution, its right-hand side and the variable coefficient).  It
holds none of the finite element arithmetic (no basis, quadrature, geometric
factors or assembly), so both the GPU library's callers and the CPU oracle may
import it.

Workload recipe (the synthetic stand-in for the CEED bake-off problems BP1,
BP3 and BPS3 named in the paper's section on exascale performance):

* unit cube [0,1]^3 split into nx*ny*nz hexahedra on a lattice; the interior
  vertices are moved independently in each coordinate by U[-0.1 h, 0.1 h]
  (h = 1/n in that direction), boundary vertices stay put, so the domain stays
  the unit cube and every element stays valid;
* vertex array layout [(nx+1)*(ny+1)*(nz+1)][3], x index fastest;
* operator input vectors are U[-1, 1];
* Poisson data: u = sin(pi x) sin(pi y) sin(pi z), f = 3 pi^2 u;
* variable coefficient k(x) = 1 + 0.5 sin(2 pi x).
"""
from __future__ import annotations

import math

import numpy as np

PERTURB_FRACTION = 0.1


def mesh_seed(p: int, n: int) -> int:
    """Seed of the vertex perturbation for an n^3 mesh used at order p."""
    return 2402 + 1000 * p + n


def vector_seed(p: int, n: int) -> int:
    """Seed of the operator input vector for an n^3 mesh at order p."""
    return mesh_seed(p, n) + 1


def lattice_vertices(nx: int, ny: int, nz: int) -> np.ndarray:
    """Unperturbed lattice vertices of [0,1]^3, shape [(nx+1)(ny+1)(nz+1), 3], x fastest."""
    xs = np.arange(nx + 1, dtype=np.float64) / nx
    ys = np.arange(ny + 1, dtype=np.float64) / ny
    zs = np.arange(nz + 1, dtype=np.float64) / nz
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def perturbed_vertices(nx: int, ny: int, nz: int, seed: int | None,
                       fraction: float = PERTURB_FRACTION) -> np.ndarray:
    """Lattice vertices with interior vertices jittered by U[-fraction*h, fraction*h].

    ``seed=None`` returns the unperturbed (affine) lattice.
    """
    v = lattice_vertices(nx, ny, nz)
    if seed is None or fraction == 0.0:
        return v
    rng = np.random.default_rng(seed)
    h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    d = rng.uniform(-1.0, 1.0, size=v.shape) * (fraction * h)
    i = np.arange(nx + 1)
    j = np.arange(ny + 1)
    k = np.arange(nz + 1)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    boundary = ((I == 0) | (I == nx) | (J == 0) | (J == ny) | (K == 0) | (K == nz)).ravel()
    d[boundary] = 0.0
    return v + d


def random_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Operator input vector, U[-1, 1]."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n).astype(dtype)


def u_exact(x, y, z):
    """Manufactured solution u = sin(pi x) sin(pi y) sin(pi z) (vanishes on the cube's boundary)."""
    return np.sin(math.pi * x) * np.sin(math.pi * y) * np.sin(math.pi * z)


def f_manufactured(x, y, z):
    """-div(grad u) for the manufactured solution: 3 pi^2 u."""
    return 3.0 * math.pi ** 2 * u_exact(x, y, z)


def coef_sin_x(x, y=None, z=None, amp: float = 0.5):
    """Variable diffusion coefficient k = 1 + amp sin(2 pi x)."""
    return 1.0 + amp * np.sin(2.0 * math.pi * x)


def mesh_n_for_dofs(p: int, target_dofs: float) -> int:
    """Elements per direction so that (N p + 1)^3 is closest to target_dofs."""
    return max(1, int(round((target_dofs ** (1.0 / 3.0) - 1.0) / p)))


def poisson_arrivals(n_requests: int, rate_per_s: float, seed: int = 15940,
                     n_range=(8, 64), p_range=(2, 8)):
    """Serving request stream: exponential inter-arrival times, N and p uniform.

    Returns a list of dicts with keys t_arrive (s), N, p, mesh_seed.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.integers(n_range[0], n_range[1] + 1, size=n_requests)
    ps = rng.integers(p_range[0], p_range[1] + 1, size=n_requests)
    out = []
    for i in range(n_requests):
        out.append({"t_arrive": float(t[i]), "N": int(ns[i]), "p": int(ps[i]),
                    "mesh_seed": int(seed * 7 + i)})
    return out
