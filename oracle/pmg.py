"""Plain FP64 CPU oracle of the p-multigrid preconditioned conjugate gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports this module;
only the tests and the benchmark's CPU-baseline leg may call it.  It shares
no code with the HIP path.

What it computes (section "Matrix-free solvers for high-order finite
elements" of the paper): a hierarchy of H1 spaces of decreasing polynomial
degree on the same mesh; because they are nested, the natural injection of a
coarse space into a finer one gives the prolongation P (fine nodal values of
the coarse function) and its transpose the restriction; every level but the
coarsest is smoothed with Chebyshev-accelerated Jacobi (the diagonal is all
that is needed of the operator); the coarsest level is solved approximately.
The paper leaves the details open; the readings fixed here are

* orders p, floor(p/2), floor(p/4), ..., 1 on the same mesh, each level with
  its own q = p_level + 2 Gauss rule and the constrained operator (identity on
  the boundary rows and columns);
* P is assembled node by node: fine node i takes the coarse interpolant at
  its position, i.e. row i holds the coarse basis functions evaluated there
  (a fine node shared by several elements is filled once); the restricted
  residual has its boundary entries set to zero;
* smoother: Chebyshev iteration for D^-1 A (Saad, Iterative Methods for
  Sparse Linear Systems, 2nd ed., section 12.3, Chebyshev acceleration) on
  the interval [lower * lmax, lmax], `degree` steps from x = 0, the same
  polynomial before and after the coarse correction (a symmetric V-cycle);
* coarsest level: exactly `coarse_iters` Jacobi-PCG steps from 0 (fewer only
  if the residual vanishes), a fixed, deterministic number;
* outer solver: flexible CG (Notay 2000) with one V-cycle as preconditioner:
  beta = z_{k+1} . (r_{k+1} - r_k) / (z_k . r_k), which equals the classical
  beta when the preconditioner is linear and symmetric.

Everything here is FP64 sparse linear algebra on matrices from oracle.fem.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem


def order_hierarchy(p: int) -> list[int]:
    """[p, p // 2, ..., 1]: the polynomial degree halves from level to level."""
    out = [p]
    while out[-1] > 1:
        out.append(out[-1] // 2)
    return out


def interpolation_1d(pc: int, pf: int) -> np.ndarray:
    """I[i, j] = l^c_j(x^f_i): coarse GLL Lagrange functions at the fine GLL nodes."""
    return fem.lagrange_values(fem.gll_nodes(pc), fem.gll_nodes(pf))


def prolongation(nx: int, ny: int, nz: int, pc: int, pf: int) -> sp.csr_matrix:
    """P [ndofs(pf), ndofs(pc)]: nodal values of the fine-space copy of a coarse function.

    On element e the coarse function is sum_j u_j phi^c_j with phi^c_j the
    tensor products of the coarse 1D Lagrange functions in the reference
    coordinates; its value at the fine node (a, b, c) of e is therefore the
    row (a, b, c) of kron(I, kron(I, I)) (x the last factor, as for the local
    numbering) applied to the element's coarse values.  Each fine node takes
    the row of the first element (ascending number) that contains it.
    """
    I1 = interpolation_1d(pc, pf)
    Pe = np.kron(I1, np.kron(I1, I1))
    Ef = fem.element_restriction(nx, ny, nz, pf)
    Ec = fem.element_restriction(nx, ny, nz, pc)
    nf = fem.ndofs(nx, ny, nz, pf)
    taken = np.zeros(nf, dtype=bool)
    rows, cols, vals = [], [], []
    for e in range(Ef.shape[0]):
        for l, i in enumerate(Ef[e]):
            if taken[i]:
                continue
            taken[i] = True
            nzc = np.nonzero(Pe[l])[0]
            rows.append(np.full(len(nzc), i))
            cols.append(Ec[e][nzc])
            vals.append(Pe[l][nzc])
    assert taken.all()
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nf, fem.ndofs(nx, ny, nz, pc))).tocsr()


def constrained_matrix(A: sp.csr_matrix, ess: np.ndarray) -> sp.csr_matrix:
    """A with the rows and columns of the essential dofs replaced by the identity."""
    keep = np.ones(A.shape[0])
    keep[ess] = 0.0
    Z = sp.diags(keep)
    E = sp.diags(1.0 - keep)
    return (Z @ A @ Z + E).tocsr()


def chebyshev(A, dinv, b, lmax, degree, lower):
    """`degree` steps of Chebyshev-accelerated Jacobi for A x = b from x = 0.

    Eigenvalues of D^-1 A are assumed in [lower lmax, lmax]; theta and delta
    are the centre and half-width of that interval.  Returns (x, b - A x).
    """
    a = lower * lmax
    theta = 0.5 * (lmax + a)
    delta = 0.5 * (lmax - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = np.zeros_like(b)
    r = b.copy()
    d = (dinv * r) / theta
    for _ in range(degree):
        x = x + d
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = (rho_new * rho) * d + (2.0 * rho_new / delta) * (dinv * r)
        rho = rho_new
    return x, r


def cg_fixed(A, dinv, b, iters):
    """Exactly `iters` Jacobi-PCG steps from x = 0 (fewer only if r . z becomes 0)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    pdir = z.copy()
    rz = r @ z
    for _ in range(iters):
        if rz == 0.0:
            break
        Ap = A @ pdir
        alpha = rz / (pdir @ Ap)
        x = x + alpha * pdir
        r = r - alpha * Ap
        z = dinv * r
        rz_new = r @ z
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
    return x


class Level:
    """One order of the hierarchy: constrained operator, Jacobi diagonal, essential dofs."""

    def __init__(self, verts, nx, ny, nz, p, kind="diffusion", coef=None):
        self.p = p
        q = p + 2
        coef_q = None
        if coef is not None:
            xq = fem.qpoint_coords(verts, nx, ny, nz, q)
            coef_q = coef(xq[:, 0, :], xq[:, 1, :], xq[:, 2, :])
        self.ess = fem.essential_dofs(nx, ny, nz, p)
        self.A = constrained_matrix(fem.assemble(kind, verts, nx, ny, nz, p, q, coef_q), self.ess)
        self.dinv = 1.0 / self.A.diagonal()
        self.lmax = None
        self.P = None  # prolongation from the next coarser level


def build_levels(verts, nx, ny, nz, p, kind="diffusion", coef=None):
    orders = order_hierarchy(p)
    levels = [Level(verts, nx, ny, nz, pk, kind, coef) for pk in orders]
    for k in range(len(levels) - 1):
        levels[k].P = prolongation(nx, ny, nz, orders[k + 1], orders[k])
    return levels


def vcycle(levels, r, degree=2, lower=0.1, coarse_iters=20, k=0):
    """z = V r: pre-smoothing, coarse correction (recursively), post-smoothing."""
    L = levels[k]
    if k == len(levels) - 1:
        return cg_fixed(L.A, L.dinv, r, coarse_iters)
    z, t = chebyshev(L.A, L.dinv, r, L.lmax, degree, lower)
    rc = L.P.T @ t
    rc[levels[k + 1].ess] = 0.0
    zc = vcycle(levels, rc, degree, lower, coarse_iters, k + 1)
    z = z + L.P @ zc
    t = r - L.A @ z
    z2, _ = chebyshev(L.A, L.dinv, t, L.lmax, degree, lower)
    return z + z2


def pmg_fcg(levels, b, rtol=1e-10, maxit=500, degree=2, lower=0.1, coarse_iters=20):
    """Flexible CG on the finest level's constrained operator, one V-cycle per step.

    Returns (x, iterations, recursive relative residual history)."""
    A = levels[0].A
    x = np.zeros_like(b)
    r = b.copy()
    z = vcycle(levels, r, degree, lower, coarse_iters)
    pdir = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while hist[-1] > rtol and it < maxit:
        Ap = A @ pdir
        alpha = rz / (pdir @ Ap)
        x = x + alpha * pdir
        r_new = r - alpha * Ap
        z = vcycle(levels, r_new, degree, lower, coarse_iters)
        beta = (z @ (r_new - r)) / rz
        rz = r_new @ z
        pdir = z + beta * pdir
        r = r_new
        it += 1
        hist.append(np.linalg.norm(r) / nb)
    return x, it, hist
