"""Pins of the p-multigrid oracle (oracle/pmg.py) against what mathematics fixes.

* the 1D interpolation and the assembled prolongation reproduce polynomials of
  the coarse degree exactly (nested spaces), checked with polynomials of the
  lattice coordinates evaluated at the node positions directly;
* on an affine mesh with exact quadrature the coarse operator equals the
  Galerkin product P^T A_fine P (the coarse space is a subspace of the fine);
* the Chebyshev smoother's error after k steps is the scaled Chebyshev
  polynomial T_k((theta - lambda) / delta) / T_k(theta / delta) on each
  eigencomponent (numpy's Chebyshev series as the reference);
* the fixed-step coarse CG reproduces the textbook PCG iterate, and finite
  termination gives the exact solution;
* the V-cycle with an exact coarse solve is a symmetric operator, and the
  preconditioned flexible CG solves the Poisson problem in a small fraction of
  the Jacobi-PCG iterations, to the same solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import chebyshev as npcheb

from oracle import fem, pmg
from paper_2402_15940_amd import inputs


def test_order_hierarchy():
    assert pmg.order_hierarchy(1) == [1]
    assert pmg.order_hierarchy(2) == [2, 1]
    assert pmg.order_hierarchy(6) == [6, 3, 1]
    assert pmg.order_hierarchy(7) == [7, 3, 1]
    assert pmg.order_hierarchy(8) == [8, 4, 2, 1]


@pytest.mark.parametrize("pf", range(2, 9))
def test_interpolation_1d_reproduces_coarse_polynomials(pf):
    pc = pf // 2
    I1 = pmg.interpolation_1d(pc, pf)
    xc, xf = fem.gll_nodes(pc), fem.gll_nodes(pf)
    assert I1.shape == (pf + 1, pc + 1)
    for k in range(pc + 1):
        np.testing.assert_allclose(I1 @ (xc ** k), xf ** k, atol=1e-14)
    # degree pc + 1 is not reproduced (the spaces differ)
    assert np.abs(I1 @ (xc ** (pc + 1)) - xf ** (pc + 1)).max() > 1e-6


def _lattice_coords(n_el, p):
    """Lattice coordinate (element index + reference GLL position) of each node along one axis."""
    g = fem.gll_nodes(p)
    out = np.empty(n_el * p + 1)
    for I in range(n_el * p + 1):
        e = min(I // p, n_el - 1)
        out[I] = e + g[I - e * p]
    return out


@pytest.mark.parametrize("pf", [2, 3, 4, 6, 7])
def test_prolongation_reproduces_coarse_polynomials(pf):
    pc = pf // 2
    nx, ny, nz = 3, 2, 2
    P = pmg.prolongation(nx, ny, nz, pc, pf)
    assert P.shape == (fem.ndofs(nx, ny, nz, pf), fem.ndofs(nx, ny, nz, pc))
    rng = np.random.default_rng(pf)

    def nodal(p):
        X, Y, Z = (_lattice_coords(n, p) for n in (nx, ny, nz))
        return np.meshgrid(Z, Y, X, indexing="ij")  # lattice order: x fastest

    for _ in range(3):
        # a random polynomial of degree <= pc in each lattice coordinate; on each
        # element it is a polynomial of that degree in the reference coordinates
        C = rng.uniform(-1, 1, (pc + 1, pc + 1, pc + 1))

        def g(Z, Y, X):
            v = np.zeros_like(X)
            for i in range(pc + 1):
                for j in range(pc + 1):
                    for k in range(pc + 1):
                        v += C[i, j, k] * X ** i * Y ** j * Z ** k
            return v.ravel()

        uc, uf = g(*nodal(pc)), g(*nodal(pf))
        np.testing.assert_allclose(P @ uc, uf, atol=1e-12 * np.abs(uf).max())
    # each row sums to one (constants are reproduced) and P has no empty row
    np.testing.assert_allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0, atol=1e-14)


@pytest.mark.parametrize("kind", ["mass", "diffusion"])
@pytest.mark.parametrize("pf", [2, 3, 4])
def test_galerkin_coarse_operator_on_affine_mesh(kind, pf):
    """Nested spaces and exact quadrature: P^T A_f P equals the coarse matrix."""
    pc = pf // 2
    n = 2
    v = inputs.perturbed_vertices(n, n, n, seed=None)
    Af = fem.assemble(kind, v, n, n, n, pf)
    Ac = fem.assemble(kind, v, n, n, n, pc)
    P = pmg.prolongation(n, n, n, pc, pf)
    G = (P.T @ Af @ P).toarray()
    np.testing.assert_allclose(G, Ac.toarray(), atol=1e-13 * np.abs(Ac).max())


def test_chebyshev_error_polynomial():
    lam = np.linspace(0.05, 2.0, 40)
    A = sp.diags(lam).tocsr()
    dinv = np.ones_like(lam)
    b = np.random.default_rng(3).uniform(-1, 1, lam.size)
    lmax, lower = 2.1, 0.1
    a = lower * lmax
    theta, delta = 0.5 * (lmax + a), 0.5 * (lmax - a)
    for k in range(1, 6):
        x, r = pmg.chebyshev(A, dinv, b, lmax, k, lower)
        ck = np.zeros(k + 1)
        ck[k] = 1.0
        damp = npcheb.chebval((theta - lam) / delta, ck) / npcheb.chebval(theta / delta, ck)
        np.testing.assert_allclose(x, (1.0 - damp) * b / lam, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(r, b - A @ x, atol=1e-13)
        # the smoothing interval is damped by at most 1 / T_k(theta / delta)
        on = lam >= a
        assert np.all(np.abs(damp[on]) <= 1.0 / npcheb.chebval(theta / delta, ck) + 1e-12)


def test_cg_fixed_matches_textbook_pcg_and_terminates():
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    A = sp.csr_matrix(Q @ np.diag(np.linspace(1, 30, 12)) @ Q.T)
    dinv = 1.0 / A.diagonal()
    b = rng.uniform(-1, 1, 12)
    for k in (1, 3, 6):
        xk = pmg.cg_fixed(A, dinv, b, k)
        xr, it, _ = fem.pcg(A, b, dinv, rtol=0.0, maxit=k)
        assert it == k
        np.testing.assert_allclose(xk, xr, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(pmg.cg_fixed(A, dinv, b, 12), spla.spsolve(A.tocsc(), b),
                               rtol=1e-8)


@pytest.fixture(scope="module")
def small_levels():
    n, p = 3, 4
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    levels = pmg.build_levels(v, n, n, n, p)
    for L in levels[:-1]:
        L.lmax = 1.1 * np.abs(spla.eigs(sp.diags(L.dinv) @ L.A, k=1, which="LM",
                                        return_eigenvectors=False)[0])
    return v, n, p, levels


def test_vcycle_is_symmetric_with_exact_coarse_solve(small_levels):
    _, _, _, levels = small_levels
    nc = levels[-1].A.shape[0]
    rng = np.random.default_rng(7)
    r1, r2 = (rng.uniform(-1, 1, levels[0].A.shape[0]) for _ in range(2))
    for r in (r1, r2):
        r[levels[0].ess] = 0.0
    z1 = pmg.vcycle(levels, r1, degree=3, lower=0.1, coarse_iters=nc)
    z2 = pmg.vcycle(levels, r2, degree=3, lower=0.1, coarse_iters=nc)
    assert abs(z1 @ r2 - r1 @ z2) <= 1e-10 * abs(z1 @ r2)
    assert z1 @ r1 > 0 and z2 @ r2 > 0


def test_pmg_fcg_solves_poisson(small_levels):
    v, n, p, levels = small_levels
    b = fem.rhs(v, n, n, n, p, f=inputs.f_manufactured)
    b[levels[0].ess] = 0.0
    x, it, hist = pmg.pmg_fcg(levels, b, rtol=1e-10, degree=3, lower=0.1, coarse_iters=20)
    assert hist[-1] <= 1e-10
    xd = spla.spsolve(levels[0].A.tocsc(), b)
    np.testing.assert_allclose(x, xd, atol=1e-8 * np.abs(xd).max())
    _, it_j, _ = fem.pcg(levels[0].A, b, levels[0].dinv, rtol=1e-10)
    assert it <= it_j // 3, (it, it_j)
