"""Plain FP64 CPU oracle for the H1 mass/diffusion operators on hex meshes.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports this module;
only the tests, the smoke check and the benchmark's CPU-baseline leg may call
it.  It shares no code with the HIP path.

What it computes.  The paper (section on assembly levels) notes that partial
assembly stores only data at quadrature points, while sparse full assembly
stores the global matrix; both define the same Galerkin operator for the same
quadrature rule.  The operator decomposition of the paper (figure on the
finite element operator decomposition, A = P^T G^T B^T D B G P) is therefore
checked here against its plain definition, assembled the traditional way:

    M_ij = sum_e sum_q w_q rho(x_q) detJ_q phi_i(xi_q) phi_j(xi_q)
    K_ij = sum_e sum_q w_q k(x_q)  detJ_q (J_q^-T grad phi_i) . (J_q^-T grad phi_j)

with dense element matrices formed from explicit basis/gradient matrices (no
sum factorization), scattered to a CSR matrix, then CSR SpMV, diag(A) and a
textbook Jacobi-preconditioned conjugate gradient.  Readings where the paper
is silent (node set, quadrature, numbering, Dirichlet treatment, stopping
rule) follow the problem statement of the hot path:

* basis: tensor-product Lagrange on the p+1 Gauss-Lobatto-Legendre points;
* quadrature: q (default p+2) Gauss-Legendre points per direction;
* reference element [0,1]^3, trilinear geometry from the 8 element vertices;
* dof numbering: lattice-lexicographic, x fastest; elements x fastest; local
  element dofs (a, b, c) with a (x) fastest;
* Dirichlet rows: y_ess = x_ess, free rows see x with essential entries zeroed;
* CG: x0 = 0, stop when ||r||_2 <= rtol ||b||_2 on the recursive residual.

Everything here is FP64.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg

# --------------------------------------------------------------------------
# 1D nodes, quadrature and Lagrange tables
# --------------------------------------------------------------------------


def gll_nodes(p: int) -> np.ndarray:
    """p+1 Gauss-Lobatto-Legendre nodes on [0,1]: the endpoints and the roots of P_p'."""
    if p < 1:
        raise ValueError("p >= 1")
    e_p = np.zeros(p + 1)
    e_p[p] = 1.0
    interior = np.sort(npleg.legroots(npleg.legder(e_p))) if p >= 2 else np.array([])
    t = np.concatenate([[-1.0], interior, [1.0]])
    return 0.5 * (t + 1.0)


def gauss_legendre(q: int):
    """q-point Gauss-Legendre rule mapped to [0,1]; weights sum to 1."""
    t, w = npleg.leggauss(q)
    return 0.5 * (t + 1.0), 0.5 * w


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[m, i] = l_i(x_m), the Lagrange polynomial of node i, by the product formula."""
    n = len(nodes)
    L = np.ones((len(x), n))
    for i in range(n):
        for k in range(n):
            if k != i:
                L[:, i] *= (x - nodes[k]) / (nodes[i] - nodes[k])
    return L


def lagrange_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[m, i] = l_i'(x_m), by differentiating the product: a sum over the dropped factor."""
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for j in range(n):
            if j == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[j]))
            for k in range(n):
                if k != i and k != j:
                    term *= (x - nodes[k]) / (nodes[i] - nodes[k])
            D[:, i] += term
    return D


def basis_tables(p: int, q: int):
    """(B, G, qpts, qwts): B[qx, a] = l_a(xi_qx), G[qx, a] = l_a'(xi_qx) on GLL nodes."""
    nodes = gll_nodes(p)
    pts, wts = gauss_legendre(q)
    return lagrange_values(nodes, pts), lagrange_derivatives(nodes, pts), pts, wts


# --------------------------------------------------------------------------
# Mesh topology: element restriction and essential dofs (integer maps)
# --------------------------------------------------------------------------


def ndofs(nx: int, ny: int, nz: int, p: int) -> int:
    return (nx * p + 1) * (ny * p + 1) * (nz * p + 1)


def element_restriction(nx: int, ny: int, nz: int, p: int) -> np.ndarray:
    """E[e, l] = global dof of local dof l of element e (int32, [ne, (p+1)^3]).

    Built by slicing a lattice of dof numbers: element (ex, ey, ez) covers the
    sub-block [ez p : ez p + p + 1, ey p : ..., ex p : ...] of the lattice.
    """
    n = p + 1
    lattice = np.arange(ndofs(nx, ny, nz, p), dtype=np.int64).reshape(
        nz * p + 1, ny * p + 1, nx * p + 1)
    E = np.empty((nx * ny * nz, n ** 3), dtype=np.int32)
    e = 0
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                blk = lattice[ez * p:ez * p + n, ey * p:ey * p + n, ex * p:ex * p + n]
                E[e] = blk.ravel()  # C order of [c][b][a]: a fastest
                e += 1
    return E


def essential_dofs(nx: int, ny: int, nz: int, p: int) -> np.ndarray:
    """Ascending int32 list of dofs on the boundary of the unit cube."""
    lattice = np.arange(ndofs(nx, ny, nz, p)).reshape(nz * p + 1, ny * p + 1, nx * p + 1)
    mask = np.zeros(lattice.shape, dtype=bool)
    mask[0, :, :] = mask[-1, :, :] = True
    mask[:, 0, :] = mask[:, -1, :] = True
    mask[:, :, 0] = mask[:, :, -1] = True
    return np.sort(lattice[mask]).astype(np.int32)


def restriction_transpose(E: np.ndarray, n_dofs: int):
    """CSR form of E^T: for each dof, the E-vector positions e*(n^3)+l that map to it, ascending."""
    flat = E.ravel().astype(np.int64)
    order = np.argsort(flat, kind="stable")
    counts = np.bincount(flat, minlength=n_dofs)
    offsets = np.zeros(n_dofs + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    return offsets.astype(np.int32), order.astype(np.int32)


# --------------------------------------------------------------------------
# Geometry: trilinear map of each hexahedron
# --------------------------------------------------------------------------


def element_vertices(verts: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """[ne, 8, 3] corner coordinates; corner (i, j, k) at index i + 2 j + 4 k."""
    V = verts.reshape(nz + 1, ny + 1, nx + 1, 3)
    out = np.empty((nx * ny * nz, 8, 3))
    e = 0
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                for k in range(2):
                    for j in range(2):
                        for i in range(2):
                            out[e, i + 2 * j + 4 * k] = V[ez + k, ey + j, ex + i]
                e += 1
    return out


def trilinear(v8: np.ndarray, xi: np.ndarray):
    """Positions [m, 3] and Jacobians J[m, i, j] = d x_i / d xi_j of the trilinear map at xi [m, 3]."""
    s, t, u = xi[:, 0], xi[:, 1], xi[:, 2]
    phi = [(1 - s, s), (1 - t, t), (1 - u, u)]
    dphi = (-1.0, 1.0)
    X = np.zeros((len(xi), 3))
    J = np.zeros((len(xi), 3, 3))
    for k in range(2):
        for j in range(2):
            for i in range(2):
                v = v8[i + 2 * j + 4 * k]
                N = phi[0][i] * phi[1][j] * phi[2][k]
                dN = np.stack([dphi[i] * phi[1][j] * phi[2][k],
                               phi[0][i] * dphi[j] * phi[2][k],
                               phi[0][i] * phi[1][j] * dphi[k]], axis=1)
                X += N[:, None] * v[None, :]
                J += v[None, :, None] * dN[:, None, :]
    return X, J


def tensor_points(pts1d: np.ndarray) -> np.ndarray:
    """[m^3, 3] tensor grid of a 1D point set, x fastest."""
    m = len(pts1d)
    c, b, a = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    return np.stack([pts1d[a.ravel()], pts1d[b.ravel()], pts1d[c.ravel()]], axis=1)


def tensor_weights(w1d: np.ndarray) -> np.ndarray:
    m = len(w1d)
    c, b, a = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    return w1d[a.ravel()] * w1d[b.ravel()] * w1d[c.ravel()]


def qpoint_coords(verts, nx, ny, nz, q: int) -> np.ndarray:
    """Physical quadrature points [ne, 3, q^3] (q-point index qx fastest)."""
    pts, _ = gauss_legendre(q)
    xi = tensor_points(pts)
    EV = element_vertices(verts, nx, ny, nz)
    out = np.empty((len(EV), 3, q ** 3))
    for e in range(len(EV)):
        X, _ = trilinear(EV[e], xi)
        out[e] = X.T
    return out


def node_coords(verts, nx, ny, nz, p: int) -> np.ndarray:
    """Physical positions [ndofs, 3] of the GLL nodes (shared nodes agree across elements)."""
    xi = tensor_points(gll_nodes(p))
    EV = element_vertices(verts, nx, ny, nz)
    E = element_restriction(nx, ny, nz, p)
    out = np.empty((ndofs(nx, ny, nz, p), 3))
    for e in range(len(EV)):
        X, _ = trilinear(EV[e], xi)
        out[E[e]] = X
    return out


# --------------------------------------------------------------------------
# Element matrices by direct quadrature (dense, no sum factorization)
# --------------------------------------------------------------------------


def reference_matrices(p: int, q: int):
    """Dense [q^3, n^3] value and reference-gradient matrices of the 3D basis.

    Row (qx, qy, qz) with qx fastest, column (a, b, c) with a fastest.  Formed as
    Kronecker products of the 1D tables, the last factor being the x direction.
    """
    B, G, pts, wts = basis_tables(p, q)
    Phi = np.kron(B, np.kron(B, B))
    Gx = np.kron(B, np.kron(B, G))
    Gy = np.kron(B, np.kron(G, B))
    Gz = np.kron(G, np.kron(B, B))
    return Phi, (Gx, Gy, Gz), tensor_points(pts), tensor_weights(wts)


def element_mass(v8, p, q, rho_q=None, ref=None):
    """M_e = Phi^T diag(w rho detJ) Phi."""
    Phi, _, xi, w = ref if ref is not None else reference_matrices(p, q)
    _, J = trilinear(v8, xi)
    detJ = np.linalg.det(J)
    rho = np.ones(len(w)) if rho_q is None else rho_q
    return Phi.T @ ((w * rho * detJ)[:, None] * Phi)


def element_diffusion(v8, p, q, k_q=None, ref=None):
    """K_e = sum_d (J^-T grad phi)_d^T diag(w k detJ) (J^-T grad phi)_d."""
    _, Gr, xi, w = ref if ref is not None else reference_matrices(p, q)
    _, J = trilinear(v8, xi)
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)  # [m, 3, 3]
    k = np.ones(len(w)) if k_q is None else k_q
    scale = w * k * detJ
    Ke = np.zeros((Gr[0].shape[1], Gr[0].shape[1]))
    for d in range(3):
        # physical derivative d/dx_d = sum_a (J^-1)_{a d} d/dxi_a
        Pd = (Jinv[:, 0, d][:, None] * Gr[0] + Jinv[:, 1, d][:, None] * Gr[1]
              + Jinv[:, 2, d][:, None] * Gr[2])
        Ke += Pd.T @ (scale[:, None] * Pd)
    return Ke


def element_qdata_reference(v8, q, k_q=None):
    """Per-qpoint detJ and the symmetric matrix w k detJ J^-1 J^-T (independent of p).

    Returned as (detJ [q^3], S [q^3, 3, 3]); used to check quadrature data.
    """
    pts, wts = gauss_legendre(q)
    xi = tensor_points(pts)
    w = tensor_weights(wts)
    _, J = trilinear(v8, xi)
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    k = np.ones(len(w)) if k_q is None else k_q
    S = (w * k * detJ)[:, None, None] * np.einsum("mad,mbd->mab", Jinv, Jinv)
    return detJ, S


# --------------------------------------------------------------------------
# Global assembly, apply, diagonal, right-hand side
# --------------------------------------------------------------------------


def assemble(kind: str, verts, nx, ny, nz, p, q=None, coef_q=None) -> sp.csr_matrix:
    """Global CSR matrix of 'mass' or 'diffusion'; coef_q is [ne, q^3] or None (= 1)."""
    q = p + 2 if q is None else q
    ref = reference_matrices(p, q)
    EV = element_vertices(verts, nx, ny, nz)
    E = element_restriction(nx, ny, nz, p)
    nloc = E.shape[1]
    rows = np.repeat(E, nloc, axis=1).ravel()
    cols = np.tile(E, (1, nloc)).ravel()
    vals = np.empty((len(EV), nloc * nloc))
    for e in range(len(EV)):
        c = None if coef_q is None else coef_q[e]
        if kind == "mass":
            Ae = element_mass(EV[e], p, q, c, ref)
        elif kind == "diffusion":
            Ae = element_diffusion(EV[e], p, q, c, ref)
        else:
            raise ValueError(kind)
        vals[e] = Ae.ravel()
    N = ndofs(nx, ny, nz, p)
    return sp.coo_matrix((vals.ravel(), (rows, cols)), shape=(N, N)).tocsr()


def constrained_apply(A: sp.csr_matrix, x: np.ndarray, ess: np.ndarray) -> np.ndarray:
    """y_free = (A x~)_free with x~_ess = 0; y_ess = x_ess."""
    xt = x.copy()
    xt[ess] = 0.0
    y = A @ xt
    y[ess] = x[ess]
    return y


def constrained_diagonal(A: sp.csr_matrix, ess: np.ndarray) -> np.ndarray:
    d = A.diagonal().copy()
    d[ess] = 1.0
    return d


def rhs(verts, nx, ny, nz, p, q=None, f=None) -> np.ndarray:
    """b_i = sum_e sum_q w_q detJ f(x_q) phi_i(x_q), with f a callable f(x, y, z)."""
    q = p + 2 if q is None else q
    Phi, _, xi, w = reference_matrices(p, q)
    EV = element_vertices(verts, nx, ny, nz)
    E = element_restriction(nx, ny, nz, p)
    b = np.zeros(ndofs(nx, ny, nz, p))
    for e in range(len(EV)):
        X, J = trilinear(EV[e], xi)
        fq = f(X[:, 0], X[:, 1], X[:, 2])
        np.add.at(b, E[e], Phi.T @ (w * np.linalg.det(J) * fq))
    return b


# --------------------------------------------------------------------------
# Jacobi-preconditioned conjugate gradient
# --------------------------------------------------------------------------


def pcg(A, b, dinv, rtol=1e-10, maxit=10000, x0=None):
    """Textbook Jacobi-PCG.  Returns (x, iterations, recursive rel. residual history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    z = dinv * r
    pdir = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while hist[-1] > rtol and it < maxit:
        Ap = A @ pdir
        alpha = rz / (pdir @ Ap)
        x += alpha * pdir
        r -= alpha * Ap
        z = dinv * r
        rz_new = r @ z
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
        it += 1
        hist.append(np.linalg.norm(r) / nb)
    return x, it, hist


def solve_poisson(verts, nx, ny, nz, p, q=None, f=None, coef_q=None, rtol=1e-10):
    """Dirichlet Poisson solve on the free-dof submatrix.

    Returns dict with x (full length, zero on the boundary), iterations,
    recursive and true relative residuals, and the assembled A and b.
    """
    A = assemble("diffusion", verts, nx, ny, nz, p, q, coef_q)
    b = rhs(verts, nx, ny, nz, p, q, f)
    ess = essential_dofs(nx, ny, nz, p)
    free = np.setdiff1d(np.arange(A.shape[0]), ess)
    Aff = A[free][:, free].tocsr()
    bf = b[free]
    xf, it, hist = pcg(Aff, bf, 1.0 / Aff.diagonal(), rtol=rtol)
    x = np.zeros(A.shape[0])
    x[free] = xf
    true_res = np.linalg.norm(bf - Aff @ xf) / np.linalg.norm(bf)
    return {"x": x, "iterations": it, "rel_res": hist[-1], "true_rel_res": true_res,
            "A": A, "b": b, "free": free, "ess": ess}
