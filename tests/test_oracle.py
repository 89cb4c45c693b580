"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks the oracle against a closed form, an exact integral, an
invariant of the Galerkin operators, brute force on a tiny case, or a textbook
a-priori estimate.  A plausible slip in the oracle (a dropped term, a wrong
sign or index, a transposed operand, wrong weights) fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import numpy.polynomial.polynomial as P
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem
from paper_2402_15940_amd import inputs

# ----------------------------------------------------------------------------
# 1D nodes, quadrature, Lagrange tables
# ----------------------------------------------------------------------------


def test_gll_closed_forms():
    # Gauss-Lobatto points on [-1,1]: p=2 {0}, p=3 {+-1/sqrt5}, p=4 {0, +-sqrt(3/7)}
    np.testing.assert_allclose(fem.gll_nodes(1), [0.0, 1.0], atol=0)
    np.testing.assert_allclose(fem.gll_nodes(2), [0.0, 0.5, 1.0], atol=1e-16)
    s5 = 1 / math.sqrt(5)
    np.testing.assert_allclose(fem.gll_nodes(3), [0, (1 - s5) / 2, (1 + s5) / 2, 1], atol=2e-16)
    s37 = math.sqrt(3 / 7)
    np.testing.assert_allclose(fem.gll_nodes(4), [0, (1 - s37) / 2, 0.5, (1 + s37) / 2, 1],
                               atol=2e-16)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_symmetric_and_lobatto_exactness(p):
    x = fem.gll_nodes(p)
    np.testing.assert_allclose(x + x[::-1], 1.0, atol=4e-16)
    # Lobatto weights w_i = 2/(p(p+1) P_p(t_i)^2) make a rule exact to degree 2p-1
    t = 2 * x - 1
    Pp = np.polynomial.legendre.legval(t, [0] * p + [1])
    w = 1.0 / (p * (p + 1) * Pp ** 2)  # mapped to [0,1]
    for k in range(2 * p):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14


@pytest.mark.parametrize("q", range(2, 11))
def test_gauss_legendre_exactness(q):
    x, w = fem.gauss_legendre(q)
    assert abs(w.sum() - 1) < 1e-15
    for k in range(2 * q):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 2e-15, k
    # not exact one degree higher (the rule really has q points)
    assert abs(np.sum(w * x ** (2 * q)) - 1.0 / (2 * q + 1)) > 1e-13


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_reproduces_polynomials(p):
    nodes = fem.gll_nodes(p)
    np.testing.assert_allclose(fem.lagrange_values(nodes, nodes), np.eye(p + 1), atol=1e-15)
    x = np.linspace(-0.1, 1.1, 37)
    L = fem.lagrange_values(nodes, x)
    D = fem.lagrange_derivatives(nodes, x)
    for k in range(p + 1):
        np.testing.assert_allclose(L @ nodes ** k, x ** k, atol=1e-12)
        dk = k * x ** (k - 1) if k > 0 else 0 * x
        np.testing.assert_allclose(D @ nodes ** k, dk, atol=1e-10)


# ----------------------------------------------------------------------------
# Integer maps
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("nx,ny,nz,p", [(1, 1, 1, 1), (2, 3, 1, 2), (3, 2, 2, 3), (2, 2, 2, 5)])
def test_restriction_geometry_and_multiplicity(nx, ny, nz, p):
    v = inputs.perturbed_vertices(nx, ny, nz, seed=7)
    E = fem.element_restriction(nx, ny, nz, p)
    n = p + 1
    N = fem.ndofs(nx, ny, nz, p)
    assert E.shape == (nx * ny * nz, n ** 3) and E.dtype == np.int32
    assert E.min() == 0 and E.max() == N - 1
    # shared nodes sit at the same physical point seen from every element
    X = fem.node_coords(v, nx, ny, nz, p)
    xi = fem.tensor_points(fem.gll_nodes(p))
    EV = fem.element_vertices(v, nx, ny, nz)
    for e in range(len(E)):
        Xe, _ = fem.trilinear(EV[e], xi)
        np.testing.assert_allclose(X[E[e]], Xe, atol=1e-14)
    # multiplicity: interior 1, face 2, edge 4, vertex 8
    mult = np.bincount(E.ravel(), minlength=N)
    I = np.arange(N) % (nx * p + 1)
    J = (np.arange(N) // (nx * p + 1)) % (ny * p + 1)
    K = np.arange(N) // ((nx * p + 1) * (ny * p + 1))

    def shared(i, m):
        return ((i % p) == 0) & (i > 0) & (i < m * p)

    expect = 2 ** (shared(I, nx).astype(int) + shared(J, ny) + shared(K, nz))
    np.testing.assert_array_equal(mult, expect)
    # essential dofs: exactly the nodes on the cube's boundary
    ess = fem.essential_dofs(nx, ny, nz, p)
    on_bnd = np.any((np.abs(X) < 1e-14) | (np.abs(X - 1) < 1e-14), axis=1)
    np.testing.assert_array_equal(ess, np.nonzero(on_bnd)[0])
    assert len(ess) == N - (nx * p - 1) * (ny * p - 1) * (nz * p - 1)


def test_restriction_transpose_is_inverse():
    E = fem.element_restriction(2, 2, 3, 3)
    N = fem.ndofs(2, 2, 3, 3)
    off, idx = fem.restriction_transpose(E, N)
    flat = E.ravel()
    for i in range(N):
        pos = idx[off[i]:off[i + 1]]
        assert np.all(flat[pos] == i) and np.all(np.diff(pos) > 0)
    assert off[-1] == flat.size


# ----------------------------------------------------------------------------
# Operators: closed forms and invariants
# ----------------------------------------------------------------------------


def _lagrange_poly(nodes, i):
    others = np.delete(nodes, i)
    c = P.polyfromroots(others)
    return c / P.polyval(nodes[i], c)


def _exact_1d(p, h, m):
    """Assembled 1D mass/stiffness on m uniform elements of size h by exact polynomial integration."""
    nodes = fem.gll_nodes(p)
    polys = [_lagrange_poly(nodes, i) for i in range(p + 1)]
    Me = np.zeros((p + 1, p + 1))
    Ke = np.zeros((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            Me[i, j] = h * P.polyval(1.0, P.polyint(P.polymul(polys[i], polys[j])))
            Ke[i, j] = P.polyval(1.0, P.polyint(P.polymul(P.polyder(polys[i]), P.polyder(polys[j])))) / h
    n = m * p + 1
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    for e in range(m):
        s = slice(e * p, e * p + p + 1)
        M[s, s] += Me
        K[s, s] += Ke
    return M, K, Me, Ke


def test_textbook_1d_element_matrices():
    for h in (1.0, 0.25):
        _, _, Me, Ke = _exact_1d(1, h, 1)
        np.testing.assert_allclose(Me, h / 6 * np.array([[2, 1], [1, 2]]), atol=1e-15)
        np.testing.assert_allclose(Ke, 1 / h * np.array([[1, -1], [-1, 1]]), atol=1e-14)
        _, _, Me, Ke = _exact_1d(2, h, 1)
        np.testing.assert_allclose(Me, h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]),
                                   atol=1e-15)
        np.testing.assert_allclose(Ke, 1 / (3 * h) * np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]),
                                   atol=1e-13)


@pytest.mark.parametrize("nx,ny,nz,p", [(3, 2, 1, 1), (2, 1, 3, 2), (1, 2, 2, 3), (2, 2, 1, 4)])
def test_uniform_mesh_kronecker_form(nx, ny, nz, p):
    """On an axis-aligned uniform mesh M = Mz x My x Mx and K = Kz x My x Mx + ..."""
    v = inputs.perturbed_vertices(nx, ny, nz, seed=None)
    M = fem.assemble("mass", v, nx, ny, nz, p).toarray()
    K = fem.assemble("diffusion", v, nx, ny, nz, p).toarray()
    Mx, Kx, _, _ = _exact_1d(p, 1.0 / nx, nx)
    My, Ky, _, _ = _exact_1d(p, 1.0 / ny, ny)
    Mz, Kz, _, _ = _exact_1d(p, 1.0 / nz, nz)
    Mk = np.kron(Mz, np.kron(My, Mx))
    Kk = np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx))
    np.testing.assert_allclose(M, Mk, atol=1e-15 * np.abs(Mk).max() * 10)
    np.testing.assert_allclose(K, Kk, atol=1e-13 * np.abs(Kk).max())


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_volume_nullspace_symmetry_perturbed(p):
    n = 3
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    M = fem.assemble("mass", v, n, n, n, p)
    K = fem.assemble("diffusion", v, n, n, n, p)
    one = np.ones(M.shape[0])
    assert abs(one @ (M @ one) - 1.0) < 1e-13
    assert np.abs(K @ one).max() < 1e-12 * np.abs(K.diagonal()).max()
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((2, M.shape[0]))
    for A in (M, K):
        assert abs(x @ (A @ y) - y @ (A @ x)) < 1e-13 * abs(x @ (A @ y)) + 1e-13
        # positive (semi)definite on random vectors
        assert x @ (A @ x) > 0


@pytest.mark.parametrize("p", [2, 3])
def test_exact_energies_affine_polynomial(p):
    """u = x^2 y z on the unit cube: int u^2 = 1/45, int |grad u|^2 = 38/135."""
    n = 2
    v = inputs.perturbed_vertices(n, n, n, seed=None)
    X = fem.node_coords(v, n, n, n, p)
    u = X[:, 0] ** 2 * X[:, 1] * X[:, 2]
    M = fem.assemble("mass", v, n, n, n, p)
    K = fem.assemble("diffusion", v, n, n, n, p)
    assert abs(u @ (M @ u) - float(Fraction(1, 45))) < 1e-14
    assert abs(u @ (K @ u) - float(Fraction(38, 135))) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 4])
def test_exact_energies_linear_on_perturbed_mesh(p):
    """u = a.x + c lies in the space on any trilinear mesh; energies are closed forms."""
    n = 3
    v = inputs.perturbed_vertices(n, n, n, seed=11 + p)
    X = fem.node_coords(v, n, n, n, p)
    a = np.array([0.3, -1.2, 0.7])
    c = 0.4
    u = X @ a + c
    M = fem.assemble("mass", v, n, n, n, p)
    K = fem.assemble("diffusion", v, n, n, n, p)
    exact_m = (a @ a) / 3 + (a.sum() ** 2 - a @ a) / 4 + c * a.sum() + c * c
    assert abs(u @ (K @ u) - a @ a) < 1e-13
    assert abs(u @ (M @ u) - exact_m) < 1e-13


def _cube_moment(i, j, k):
    """Exact integral of x^i y^j z^k over the unit cube."""
    return Fraction(1, (i + 1) * (j + 1) * (k + 1))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_variable_coefficient_energies_on_perturbed_mesh(p):
    """rho = k = 1 + x sampled at the quadrature points through qpoint_coords.

    For u = a.x + c (in the space on any trilinear mesh), grad u = a, so
    u^T K u = |a|^2 int (1 + x) = 3/2 |a|^2 and u^T M u = int (1 + x)(a.x + c)^2,
    both exact under q = p+2 (the integrands have degree <= 5 per reference
    direction).  The coefficient must reach the right quadrature points: an
    ordering slip in qpoint_coords (e.g. qz fastest) misses by about 1e-4.
    """
    n = 3
    v = inputs.perturbed_vertices(n, n, n, seed=31 + p)
    q = p + 2
    XQ = fem.qpoint_coords(v, n, n, n, q)        # [ne, 3, q^3]
    kq = 1.0 + XQ[:, 0, :]
    X = fem.node_coords(v, n, n, n, p)
    af = (Fraction(3, 10), Fraction(-6, 5), Fraction(7, 10))
    cf = Fraction(2, 5)
    a = np.array([float(t) for t in af])
    c = float(cf)
    u = X @ a + c
    K = fem.assemble("diffusion", v, n, n, n, p, coef_q=kq)
    M = fem.assemble("mass", v, n, n, n, p, coef_q=kq)
    aa = sum(t * t for t in af)
    assert abs(u @ (K @ u) - float(Fraction(3, 2) * aa)) < 1e-13
    # (1 + x)(a1 x + a2 y + a3 z + c)^2 expanded into monomials x^i y^j z^k
    lin = {(1, 0, 0): af[0], (0, 1, 0): af[1], (0, 0, 1): af[2], (0, 0, 0): cf}
    sq = {}
    for m1, c1 in lin.items():
        for m2, c2 in lin.items():
            key = tuple(s + t for s, t in zip(m1, m2))
            sq[key] = sq.get(key, 0) + c1 * c2
    exact = Fraction(0)
    for (i, j, k), cc in sq.items():
        exact += cc * (_cube_moment(i, j, k) + _cube_moment(i + 1, j, k))
    assert abs(u @ (M @ u) - float(exact)) < 1e-13
    # a constant coefficient through the same path is the plain operator scaled
    K2 = fem.assemble("diffusion", v, n, n, n, p, coef_q=np.full_like(kq, 2.0))
    K1 = fem.assemble("diffusion", v, n, n, n, p)
    assert abs(K2 - 2.0 * K1).max() < 1e-14 * abs(K1).max()


def test_qpoint_coords_affine_closed_form():
    """On the unperturbed lattice, point (qx, qy, qz) of element (ex, ey, ez) sits at
    ((ex + t_qx)/nx, (ey + t_qy)/ny, (ez + t_qz)/nz) with t the Gauss points on [0,1]."""
    nx, ny, nz, q = 3, 2, 4, 5
    v = inputs.perturbed_vertices(nx, ny, nz, seed=None)
    XQ = fem.qpoint_coords(v, nx, ny, nz, q)
    t, _ = np.polynomial.legendre.leggauss(q)
    t = (t + 1) / 2
    e = 0
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                m = 0
                for qz in range(q):
                    for qy in range(q):
                        for qx in range(q):
                            want = ((ex + t[qx]) / nx, (ey + t[qy]) / ny, (ez + t[qz]) / nz)
                            np.testing.assert_allclose(XQ[e, :, m], want, atol=1e-15)
                            m += 1
                e += 1


def _brute_element(v8, p, q, kind):
    """Scalar triple loop over (i, j, point) with its own Lagrange, Jacobian and inverse (adjugate)."""
    nodes = list(fem.gll_nodes(p))
    xs, ws = np.polynomial.legendre.leggauss(q)
    xs = [(t + 1) / 2 for t in xs]
    ws = [w / 2 for w in ws]
    n = p + 1

    def lag(i, x):
        r = 1.0
        for k in range(n):
            if k != i:
                r *= (x - nodes[k]) / (nodes[i] - nodes[k])
        return r

    def dlag(i, x, hstep=None):
        s = 0.0
        for j in range(n):
            if j == i:
                continue
            t = 1.0 / (nodes[i] - nodes[j])
            for k in range(n):
                if k != i and k != j:
                    t *= (x - nodes[k]) / (nodes[i] - nodes[k])
            s += t
        return s

    A = np.zeros((n ** 3, n ** 3))
    for qz in range(q):
        for qy in range(q):
            for qx in range(q):
                s, t, u = xs[qx], xs[qy], xs[qz]
                w = ws[qx] * ws[qy] * ws[qz]
                J = [[0.0] * 3 for _ in range(3)]
                for k in range(2):
                    for j in range(2):
                        for i in range(2):
                            vv = v8[i + 2 * j + 4 * k]
                            fs = (s if i else 1 - s, t if j else 1 - t, u if k else 1 - u)
                            ds = (1 if i else -1, 1 if j else -1, 1 if k else -1)
                            d = (ds[0] * fs[1] * fs[2], fs[0] * ds[1] * fs[2], fs[0] * fs[1] * ds[2])
                            for r in range(3):
                                for cc in range(3):
                                    J[r][cc] += vv[r] * d[cc]
                det = (J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                       - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                       + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]))
                adj = [[J[(cc + 1) % 3][(r + 1) % 3] * J[(cc + 2) % 3][(r + 2) % 3]
                        - J[(cc + 1) % 3][(r + 2) % 3] * J[(cc + 2) % 3][(r + 1) % 3]
                        for cc in range(3)] for r in range(3)]
                inv = [[adj[r][cc] / det for cc in range(3)] for r in range(3)]
                vals = []
                grads = []
                for c in range(n):
                    for b in range(n):
                        for a in range(n):
                            vals.append(lag(a, s) * lag(b, t) * lag(c, u))
                            gr = (dlag(a, s) * lag(b, t) * lag(c, u),
                                  lag(a, s) * dlag(b, t) * lag(c, u),
                                  lag(a, s) * lag(b, t) * dlag(c, u))
                            # physical gradient: J^-T grad_ref
                            grads.append([sum(inv[m][d] * gr[m] for m in range(3)) for d in range(3)])
                for i in range(n ** 3):
                    for j in range(n ** 3):
                        if kind == "mass":
                            A[i, j] += w * det * vals[i] * vals[j]
                        else:
                            A[i, j] += w * det * sum(grads[i][d] * grads[j][d] for d in range(3))
    return A


@pytest.mark.parametrize("p", [1, 2])
def test_single_element_brute_force(p):
    rng = np.random.default_rng(3)
    v8 = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], float)
    v8 = v8 * np.array([1.3, 0.8, 1.1]) + rng.uniform(-0.15, 0.15, size=(8, 3))
    q = p + 2
    for kind, fn in (("mass", fem.element_mass), ("diffusion", fem.element_diffusion)):
        ref = _brute_element(v8, p, q, kind)
        got = fn(v8, p, q)
        np.testing.assert_allclose(got, ref, atol=1e-13 * np.abs(ref).max())
    # mass is integrated exactly by q = p+2 (integrand degree <= 2p+2 per direction)
    np.testing.assert_allclose(fem.element_mass(v8, p, q), fem.element_mass(v8, p, 12),
                               atol=1e-14 * np.abs(fem.element_mass(v8, p, 12)).max())


def test_qdata_reference_agrees_with_adjugate_form():
    rng = np.random.default_rng(5)
    v8 = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], float)
    v8 += rng.uniform(-0.1, 0.1, size=(8, 3))
    q = 4
    detJ, S = fem.element_qdata_reference(v8, q)
    pts, wts = fem.gauss_legendre(q)
    xi = fem.tensor_points(pts)
    w = fem.tensor_weights(wts)
    _, J = fem.trilinear(v8, xi)
    for m in range(len(w)):
        Jm = J[m]
        cof = np.array([[np.linalg.det(np.delete(np.delete(Jm, r, 0), c, 1)) * (-1) ** (r + c)
                         for c in range(3)] for r in range(3)])
        adj = cof.T
        np.testing.assert_allclose(S[m], w[m] * adj @ adj.T / detJ[m], rtol=1e-13, atol=1e-16)


def test_rhs_constant_and_linear_moments():
    n, p = 3, 3
    v = inputs.perturbed_vertices(n, n, n, seed=9)
    b1 = fem.rhs(v, n, n, n, p, f=lambda x, y, z: np.ones_like(x))
    assert abs(b1.sum() - 1.0) < 1e-13           # partition of unity: int 1 = |Omega|
    X = fem.node_coords(v, n, n, n, p)
    assert abs(b1 @ X[:, 1] - 0.5) < 1e-13       # int y dx = 1/2
    bx = fem.rhs(v, n, n, n, p, f=lambda x, y, z: x)
    assert abs(bx @ X[:, 0] - 1.0 / 3.0) < 1e-13  # int x^2 = 1/3 (exact quadrature)


def test_constrained_apply_is_free_submatrix():
    n, p = 2, 2
    v = inputs.perturbed_vertices(n, n, n, seed=1)
    K = fem.assemble("diffusion", v, n, n, n, p)
    ess = fem.essential_dofs(n, n, n, p)
    free = np.setdiff1d(np.arange(K.shape[0]), ess)
    x = np.random.default_rng(2).standard_normal(K.shape[0])
    y = fem.constrained_apply(K, x, ess)
    np.testing.assert_allclose(y[free], K[free][:, free] @ x[free], rtol=1e-14, atol=1e-14)
    np.testing.assert_array_equal(y[ess], x[ess])
    d = fem.constrained_diagonal(K, ess)
    np.testing.assert_array_equal(d[ess], 1.0)
    np.testing.assert_array_equal(d[free], K.diagonal()[free])


# ----------------------------------------------------------------------------
# Solve
# ----------------------------------------------------------------------------


def test_pcg_matches_direct_solve():
    n, p = 3, 2
    v = inputs.perturbed_vertices(n, n, n, seed=21)
    res = fem.solve_poisson(v, n, n, n, p, f=inputs.f_manufactured, rtol=1e-12)
    A, b, free = res["A"], res["b"], res["free"]
    xd = spla.spsolve(A[free][:, free].tocsc(), b[free])
    np.testing.assert_allclose(res["x"][free], xd, rtol=1e-9, atol=1e-12)
    assert res["rel_res"] <= 1e-12 and res["true_rel_res"] < 1e-11


def test_poisson_config_small_affine():
    """4^3 affine mesh, p = 2, q = 4, manufactured sine solution, Jacobi-PCG to 1e-10.

    The expected values come from an independent script that assembled the same
    problem in Kronecker form (1D matrices, no element loop) and ran its own
    Jacobi-PCG: 4 iterations, max nodal error 1.1683e-3 against sin sin sin, and
    discrete energy u_h^T K u_h = 3.699126 (the continuous one is 3 pi^2 / 8 =
    3.701102).  A dropped Jacobi scaling, a wrong right-hand side or a wrong
    stopping rule changes at least one of them.
    """
    n, p = 4, 2
    v = inputs.perturbed_vertices(n, n, n, seed=None)
    res = fem.solve_poisson(v, n, n, n, p, f=inputs.f_manufactured, rtol=1e-10)
    X = fem.node_coords(v, n, n, n, p)
    x = res["x"]
    err = np.abs(x - inputs.u_exact(X[:, 0], X[:, 1], X[:, 2])).max()
    assert res["rel_res"] <= 1e-10 and res["true_rel_res"] <= 1e-10
    assert res["iterations"] == 4
    assert abs(err - 1.1683e-3) <= 1e-7, err
    assert abs(x @ (res["A"] @ x) - 3.699126) <= 1e-6
    assert abs(3 * math.pi ** 2 / 8 - 3.701102) < 1e-6  # the continuous energy quoted above


def test_pcg_iterate_is_krylov_energy_minimizer():
    """The k-th Jacobi-PCG iterate minimizes the A-norm error over x0 + K_k(D^-1 A, D^-1 r0).

    That characterization of preconditioned CG does not use its recurrences: the
    minimizer is computed here from an explicit Krylov basis and a small dense
    solve.  A wrong preconditioner (scaling, transposition) changes the space.
    """
    rng = np.random.default_rng(17)
    m = 12
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    S = Q @ np.diag(np.linspace(1.0, 30.0, m)) @ Q.T
    Dh = np.diag(rng.uniform(0.5, 3.0, m))
    A = sp.csr_matrix(Dh @ S @ Dh)  # SPD with a non-constant diagonal
    b = rng.standard_normal(m)
    dinv = 1.0 / A.diagonal()
    for k in (1, 2, 3, 5):
        xk, it, _ = fem.pcg(A, b, dinv, rtol=1e-300, maxit=k)
        assert it == k
        Ad = A.toarray()
        V = np.empty((m, k))
        v = dinv * b
        for j in range(k):
            V[:, j] = v
            v = dinv * (Ad @ v)
        V, _ = np.linalg.qr(V)
        y = np.linalg.solve(V.T @ Ad @ V, V.T @ b)
        np.testing.assert_allclose(xk, V @ y, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2])
def test_discretization_convergence_rate(p):
    """|| u_h - I_h u ||_M decays at least like h^(p+1) (a-priori estimate)."""
    errs = []
    for n in (4, 8):
        v = inputs.perturbed_vertices(n, n, n, seed=None)
        res = fem.solve_poisson(v, n, n, n, p, f=inputs.f_manufactured, rtol=1e-12)
        X = fem.node_coords(v, n, n, n, p)
        e = res["x"] - inputs.u_exact(X[:, 0], X[:, 1], X[:, 2])
        M = fem.assemble("mass", v, n, n, n, p)
        errs.append(math.sqrt(e @ (M @ e)))
    rate = math.log2(errs[0] / errs[1])
    assert rate > p + 1 - 0.3, (errs, rate)


def test_all_cores_csr_spmv_equals_scipy():
    """The CPU baseline's OpenMP CSR product is the plain definition: equal to scipy's."""
    import ctypes as C
    import os
    import shutil
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from oracle import build_csr
    lib = C.CDLL(build_csr.build())
    n, p = 3, 3
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    A = fem.assemble("diffusion", v, n, n, n, p)
    x = inputs.random_vector(A.shape[0], 4)
    y = np.empty_like(x)
    rp = A.indptr.astype(np.int64)
    ci = A.indices.astype(np.int32)
    lib.csr_spmv(C.c_int64(A.shape[0]), rp.ctypes.data_as(C.c_void_p),
                 ci.ctypes.data_as(C.c_void_p), A.data.ctypes.data_as(C.c_void_p),
                 x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p))
    np.testing.assert_allclose(y, A @ x, rtol=0, atol=1e-13 * np.abs(A @ x).max())
    assert lib.csr_threads() >= 1
