"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: FP64 apply/diagonal/RHS at relative error <= 1e-12 in the 2-norm
and the max-norm (absolute 1e-12 * ||diag||_inf where the oracle result is
zero, e.g. K 1); FP32 apply at 5e-5 relative (single-precision contractions
of ~(p+2)^3 terms).  Integer maps are bit-exact (tests/test_host_abi.py).
"""
import functools

import numpy as np
import pytest

from oracle import fem
from paper_2402_15940_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MESHES = [(5, 2, 2), (3, 3, 1)]  # 20 and 9 elements: several workgroups, ragged last one


def MODES(pf):
    """Every (E^T scatter, E source) combination the apply kernels implement."""
    return [(s, i) for s in (pf.SCATTER_ATOMIC, pf.SCATTER_DETERMINISTIC)
            for i in (pf.INDEX_LATTICE, pf.INDEX_MAP)]


@pytest.fixture(scope="module")
def pf():
    from paper_2402_15940_amd import pafem
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pafem.lib()
    return pafem


@pytest.fixture(scope="module")
def ctx(pf):
    return pf.Context(0)


@functools.lru_cache(maxsize=None)
def _oracle_matrix(kind, nx, ny, nz, p, seed, coef):
    v = inputs.perturbed_vertices(nx, ny, nz, seed=seed)
    coef_q = None
    if coef == "sinx":
        xq = fem.qpoint_coords(v, nx, ny, nz, p + 2)
        coef_q = inputs.coef_sin_x(xq[:, 0, :])
    return fem.assemble(kind, v, nx, ny, nz, p, coef_q=coef_q)


def _build(pf, ctx, kind, nx, ny, nz, p, seed, coef=None, prec=1):
    v = inputs.perturbed_vertices(nx, ny, nz, seed=seed)
    mesh = pf.Mesh(ctx, nx, ny, nz, v)
    sp = pf.Space(mesh, p)
    op = pf.Operator(sp, pf.DIFFUSION if kind == "diffusion" else pf.MASS)
    if coef == "sinx":
        op.set_coefficient_sinx(0.5)
    op.assemble(prec)
    return v, op


def _relerr(y, yref, scale=None):
    y = np.asarray(y)
    yref = np.asarray(yref)
    d = y - yref
    n2 = np.linalg.norm(yref)
    ninf = np.abs(yref).max()
    if scale is not None and n2 < scale * 1e-8:
        return np.abs(d).max() / scale, np.abs(d).max() / scale
    return np.linalg.norm(d) / n2, np.abs(d).max() / ninf


# ----------------------------------------------------------------------------
# quadrature data and geometry
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("p", [1, 3, 6, 8])
def test_qdata_matches_oracle(pf, ctx, p):
    nx, ny, nz = 3, 2, 2
    q = p + 2
    v, op = _build(pf, ctx, "diffusion", nx, ny, nz, p, seed=100 + p)
    _, opm = _build(pf, ctx, "mass", nx, ny, nz, p, seed=100 + p)
    qd = op.qdata().cpu().numpy()
    qm = opm.qdata().cpu().numpy()
    EV = fem.element_vertices(v, nx, ny, nz)
    pts, wts = fem.gauss_legendre(q)
    w = fem.tensor_weights(wts)
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for e in range(len(EV)):
        detJ, S = fem.element_qdata_reference(EV[e], q)
        np.testing.assert_allclose(qm[e, 0], w * detJ, rtol=1e-13)
        for c, (i, j) in enumerate(iu):
            np.testing.assert_allclose(qd[e, c], S[:, i, j], rtol=1e-12,
                                       atol=1e-13 * np.abs(S).max())
    xq = op.qpoint_coords().cpu().numpy()
    np.testing.assert_allclose(xq, fem.qpoint_coords(v, nx, ny, nz, q), atol=1e-15)


def test_inverted_element_rejected(pf, ctx):
    v = inputs.perturbed_vertices(2, 2, 2, seed=None)
    v[13] = [0.9, 0.9, 0.9]  # drag the centre vertex through a face
    mesh = pf.Mesh(ctx, 2, 2, 2, v)
    op = pf.Operator(pf.Space(mesh, 2), pf.DIFFUSION)
    with pytest.raises(pf.PafemError) as ei:
        op.assemble()
    assert ei.value.name == "INVALID_ARG"
    with pytest.raises(pf.PafemError):
        op.apply(torch.zeros(op.space.ndofs, dtype=torch.float64, device="cuda"))


# ----------------------------------------------------------------------------
# operator apply (FP64), both E^T modes, constrained and plain
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("kind", ["mass", "diffusion"])
def test_apply_fp64_matches_oracle(pf, ctx, kind, p, mesh):
    nx, ny, nz = mesh
    seed = inputs.mesh_seed(p, nx)
    A = _oracle_matrix(kind, nx, ny, nz, p, seed, None)
    v, op = _build(pf, ctx, kind, nx, ny, nz, p, seed)
    n = op.space.ndofs
    x = inputs.random_vector(n, inputs.vector_seed(p, nx))
    xd = torch.from_numpy(x).cuda()
    ess = fem.essential_dofs(nx, ny, nz, p)
    for mode, im in MODES(pf):
        op.set_scatter_mode(mode)
        op.set_restriction_mode(im)
        y = op.apply(xd).cpu().numpy()
        e2, einf = _relerr(y, A @ x)
        assert e2 <= 1e-12 and einf <= 1e-12, (mode, e2, einf)
        yc = op.apply(xd, constrained=True).cpu().numpy()
        e2, einf = _relerr(yc, fem.constrained_apply(A, x, ess))
        assert e2 <= 1e-12 and einf <= 1e-12, (mode, e2, einf)
        np.testing.assert_array_equal(yc[ess], x[ess])


@pytest.mark.parametrize("p", [2, 5])
def test_apply_variable_coefficient(pf, ctx, p):
    nx, ny, nz = 3, 3, 1
    seed = 7
    for kind in ("mass", "diffusion"):
        A = _oracle_matrix(kind, nx, ny, nz, p, seed, "sinx")
        v, op = _build(pf, ctx, kind, nx, ny, nz, p, seed, coef="sinx")
        x = inputs.random_vector(op.space.ndofs, 5)
        y = op.apply(torch.from_numpy(x).cuda()).cpu().numpy()
        e2, einf = _relerr(y, A @ x)
        assert e2 <= 1e-12 and einf <= 1e-12
        # coefficient given at the exported quadrature points gives the same operator
        op2 = pf.Operator(op.space, op.kind)
        xq = op2.qpoint_coords()
        k = (1.0 + 0.5 * torch.sin(2 * np.pi * xq[:, 0, :])).contiguous()
        op2.set_coefficient_qpts(k)
        op2.assemble()
        y2 = op2.apply(torch.from_numpy(x).cuda()).cpu().numpy()
        e2, _ = _relerr(y2, A @ x)
        assert e2 <= 1e-12


@pytest.mark.parametrize("p", [1, 3, 4, 7])
def test_apply_fp32_close_to_oracle(pf, ctx, p):
    nx, ny, nz = 5, 2, 2
    seed = inputs.mesh_seed(p, nx)
    for kind in ("mass", "diffusion"):
        A = _oracle_matrix(kind, nx, ny, nz, p, seed, None)
        v, op = _build(pf, ctx, kind, nx, ny, nz, p, seed, prec=pf.FP64 | pf.FP32)
        x = inputs.random_vector(op.space.ndofs, 9)
        for mode, im in MODES(pf):
            op.set_scatter_mode(mode)
            op.set_restriction_mode(im)
            y = op.apply(torch.from_numpy(x).float().cuda()).double().cpu().numpy()
            e2, _ = _relerr(y, A @ x.astype(np.float32).astype(np.float64))
            assert e2 <= 5e-5, e2


def test_single_element_columns_are_element_matrix(pf, ctx):
    """N = 1: applying to unit vectors reproduces the oracle's element matrix."""
    rng = np.random.default_rng(4)
    v = fem.element_vertices(inputs.lattice_vertices(1, 1, 1), 1, 1, 1)[0]
    v = v + rng.uniform(-0.12, 0.12, size=v.shape)
    verts = v.copy()  # corner order i + 2j + 4k equals the vertex order of a 1x1x1 mesh
    for p in (1, 2, 3):
        mesh = pf.Mesh(ctx, 1, 1, 1, verts)
        sp = pf.Space(mesh, p)
        for kind, fn in (("mass", fem.element_mass), ("diffusion", fem.element_diffusion)):
            op = pf.Operator(sp, pf.MASS if kind == "mass" else pf.DIFFUSION)
            op.assemble()
            n = sp.ndofs
            I = torch.eye(n, dtype=torch.float64, device="cuda")
            cols = torch.stack([op.apply(I[i].contiguous()) for i in range(n)], 1).cpu().numpy()
            Ae = fn(v, p, p + 2)
            np.testing.assert_allclose(cols, Ae, atol=1e-13 * np.abs(Ae).max())


@pytest.mark.parametrize("p,kind", [(4, "diffusion"), (6, "diffusion"), (2, "mass"), (6, "mass")])
def test_deterministic_mode_is_bitwise_reproducible(pf, ctx, p, kind):
    # the lattice-numbered sum takes the tuned cache policies (non-temporal
    # E-vector loads and y stores where measured faster); the stored-map sum
    # takes ordinary ones: the numbers are the same
    nx, ny, nz = 4, 4, 3
    v, op = _build(pf, ctx, kind, nx, ny, nz, p, seed=2, prec=pf.FP64 | pf.FP32)
    op.set_scatter_mode(pf.SCATTER_DETERMINISTIC)
    x = torch.from_numpy(inputs.random_vector(op.space.ndofs, 1)).cuda()
    for xx in (x, x.float()):
        op.set_restriction_mode(pf.INDEX_LATTICE)
        y1 = op.apply(xx).clone()
        y2 = op.apply(xx).clone()
        assert torch.equal(y1, y2)
        c1 = op.apply(xx, constrained=True).clone()
        # the lattice-computed and the stored E^T sum in the same order
        op.set_restriction_mode(pf.INDEX_MAP)
        y3 = op.apply(xx).clone()
        assert torch.equal(y1, y3), (xx.dtype, (y1 - y3).abs().max().item())
        assert torch.equal(c1, op.apply(xx, constrained=True))
    op.set_restriction_mode(pf.INDEX_LATTICE)
    d1 = op.diagonal()
    d2 = op.diagonal()
    assert torch.equal(d1, d2)


# ----------------------------------------------------------------------------
# diagonal, right-hand side, reductions
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("kind", ["mass", "diffusion"])
def test_diagonal_matches_oracle(pf, ctx, kind, p):
    nx, ny, nz = 3, 3, 1
    seed = inputs.mesh_seed(p, nx)
    A = _oracle_matrix(kind, nx, ny, nz, p, seed, None)
    v, op = _build(pf, ctx, kind, nx, ny, nz, p, seed)
    d = op.diagonal().cpu().numpy()
    e2, einf = _relerr(d, A.diagonal())
    assert e2 <= 1e-12 and einf <= 1e-12
    ess = fem.essential_dofs(nx, ny, nz, p)
    dc = op.diagonal(constrained=True).cpu().numpy()
    np.testing.assert_array_equal(dc[ess], 1.0)
    e2, _ = _relerr(dc, fem.constrained_diagonal(A, ess))
    assert e2 <= 1e-12


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_rhs_matches_oracle(pf, ctx, p):
    nx, ny, nz = 3, 2, 2
    v, op = _build(pf, ctx, "diffusion", nx, ny, nz, p, seed=31)
    b = op.rhs().cpu().numpy()
    bo = fem.rhs(v, nx, ny, nz, p, f=inputs.f_manufactured)
    bo[fem.essential_dofs(nx, ny, nz, p)] = 0.0
    e2, einf = _relerr(b, bo)
    assert e2 <= 1e-12 and einf <= 1e-12
    # f supplied at the quadrature points
    xq = op.qpoint_coords()
    fq = (3 * np.pi ** 2 * torch.sin(np.pi * xq[:, 0]) * torch.sin(np.pi * xq[:, 1])
          * torch.sin(np.pi * xq[:, 2])).contiguous()
    b2 = op.rhs(fq).cpu().numpy()
    e2, _ = _relerr(b2, bo)
    assert e2 <= 1e-12


@pytest.mark.parametrize("n", [0, 1, 255, 256, 1000, 123457, 4_000_001])
def test_dot_matches_numpy(pf, ctx, n):
    rng = np.random.default_rng(n)
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    r = ctx.dot(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()).item()
    ref = float(np.dot(x, y))
    assert abs(r - ref) <= 1e-13 * max(1.0, np.abs(x * y).sum())
    r2 = ctx.dot(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()).item()
    assert r == r2


# ----------------------------------------------------------------------------
# solve
# ----------------------------------------------------------------------------


def test_poisson_small_affine_plain_cg(pf, ctx):
    """4^3 affine mesh, p = 2, q = 4, Jacobi-PCG to 1e-10 in FP64."""
    n, p = 4, 2
    v = inputs.perturbed_vertices(n, n, n, seed=None)
    ref = fem.solve_poisson(v, n, n, n, p, f=inputs.f_manufactured, rtol=1e-10)
    mesh = pf.Mesh(ctx, n, n, n, v)
    op = pf.Operator(pf.Space(mesh, p), pf.DIFFUSION)
    op.assemble()
    b = op.rhs()
    x, st = op.solve(b, rtol=1e-10)
    x = x.cpu().numpy()
    assert st["rel_res"] <= 1e-10 and st["true_rel_res"] <= 1e-10
    assert st["iterations"] == ref["iterations"]
    np.testing.assert_allclose(x, ref["x"], atol=1e-12 * np.abs(ref["x"]).max() * 100)


@pytest.mark.parametrize("p", [3, 5, 7])
def test_poisson_perturbed_plain_and_mixed(pf, ctx, p):
    n = 4
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    xq = fem.qpoint_coords(v, n, n, n, p + 2)
    ref = fem.solve_poisson(v, n, n, n, p, f=inputs.f_manufactured,
                            coef_q=inputs.coef_sin_x(xq[:, 0, :]), rtol=1e-12)
    mesh = pf.Mesh(ctx, n, n, n, v)
    op = pf.Operator(pf.Space(mesh, p), pf.DIFFUSION)
    op.set_coefficient_sinx(0.5)
    op.assemble(pf.FP64 | pf.FP32 | pf.BF16)
    b = op.rhs()
    xr = ref["x"]
    its = {}
    for mode, inner in ((pf.SOLVE_PLAIN_FP64, 1e-3), (pf.SOLVE_IR_FP32, 1e-3),
                        (pf.SOLVE_MIXED_FP32, 0.1), (pf.SOLVE_MIXED_BF16, 0.1),
                        (pf.SOLVE_IR_BF16, 1e-3)):
        x, st = op.solve(b, mode=mode, rtol=1e-10, inner_rtol=inner)
        assert st["true_rel_res"] <= 1e-10, (mode, st)
        err = np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr)
        assert err <= 1e-8, (mode, err)
        its[mode] = st["iterations"]
        if mode == pf.SOLVE_IR_FP32:
            assert st["outer_iterations"] >= 2
        if mode == pf.SOLVE_MIXED_FP32:
            # the FP64 residual is confirmed at the end and replaced on the way
            assert st["true_rel_res"] <= 1e-10 and st["outer_iterations"] >= 3
    # one Krylov space: about the plain iteration count (a restarted defect
    # correction needs far more)
    assert its[pf.SOLVE_MIXED_FP32] <= 1.3 * its[pf.SOLVE_PLAIN_FP64] + 5, its


def test_solve_not_converged_reports(pf, ctx):
    n, p = 3, 3
    v = inputs.perturbed_vertices(n, n, n, seed=1)
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p), pf.DIFFUSION)
    op.assemble()
    b = op.rhs()
    x, st = op.solve(b, rtol=1e-14, maxit=3, raise_on_nonconvergence=False)
    assert st["iterations"] == 3 and st["rel_res"] > 1e-14
    with pytest.raises(pf.PafemError) as ei:
        op.solve(b, rtol=1e-14, maxit=3)
    assert ei.value.name == "NOT_CONVERGED"


# ----------------------------------------------------------------------------
# full-size runs: sampled rows against the oracle's element matrices, and
# invariants that hold at any size
# ----------------------------------------------------------------------------


def _corners(verts, nx, ny, nz, e):
    V = verts.reshape(nz + 1, ny + 1, nx + 1, 3)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    return np.array([V[ez + k, ey + j, ex + i] for k in (0, 1) for j in (0, 1) for i in (0, 1)])


def _oracle_rows(kind, verts, nx, ny, nz, p, x, dofs):
    E = fem.element_restriction(nx, ny, nz, p)
    ref = fem.reference_matrices(p, p + 2)
    out = []
    for i in dofs:
        es, ls = np.nonzero(E == i)
        acc = 0.0
        for e, l in zip(es, ls):
            v8 = _corners(verts, nx, ny, nz, e)
            Ae = (fem.element_mass if kind == "mass" else fem.element_diffusion)(v8, p, p + 2,
                                                                               ref=ref)
            acc += Ae[l] @ x[E[e]]
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("p,target", [(2, 1e6), (4, 1e6), (6, 8e6), (8, 1e6)])
def test_full_size_sampled_rows(pf, ctx, p, target):
    N = inputs.mesh_n_for_dofs(p, target)
    seed = inputs.mesh_seed(p, N)
    v = inputs.perturbed_vertices(N, N, N, seed=seed)
    mesh = pf.Mesh(ctx, N, N, N, v)
    sp = pf.Space(mesh, p)
    x = inputs.random_vector(sp.ndofs, inputs.vector_seed(p, N))
    xd = torch.from_numpy(x).cuda()
    rng = np.random.default_rng(p)
    # a vertex, an edge, a face and interior dofs, plus random ones
    L = N * p + 1
    special = [0, L // 2, L * L // 2 + p, (L ** 3) // 2]
    dofs = np.unique(np.concatenate([special, rng.integers(0, sp.ndofs, 12)]))
    for kind in ("diffusion", "mass"):
        op = pf.Operator(sp, pf.DIFFUSION if kind == "diffusion" else pf.MASS)
        op.assemble()
        for mode, im in MODES(pf):
            op.set_scatter_mode(mode)
            op.set_restriction_mode(im)
            y = op.apply(xd)[torch.from_numpy(dofs).cuda()].cpu().numpy()
            yo = _oracle_rows(kind, v, N, N, N, p, x, dofs)
            scale = np.abs(yo).max()
            np.testing.assert_allclose(y, yo, rtol=1e-12, atol=1e-12 * scale)
        del op
        torch.cuda.synchronize()


def _elements_of_node(i, N, p):
    """(element, local index) pairs holding lattice node i of an N^3 mesh of order p."""
    L = N * p + 1
    I, J, K = i % L, (i // L) % L, i // (L * L)

    def cands(c):
        out = []
        for e in (c // p - 1, c // p):
            if 0 <= e < N and 0 <= c - e * p <= p:
                out.append((e, c - e * p))
        return out

    res = []
    for ez, lz in cands(K):
        for ey, ly in cands(J):
            for ex, lx in cands(I):
                res.append((ex + N * (ey + N * ez), lx + (p + 1) * (ly + (p + 1) * lz)))
    return res


@pytest.mark.parametrize("p,N", [(4, 100), (7, 64)])
def test_largest_sizes_sampled_rows(pf, ctx, p, N):
    """The largest stated sizes: p=4 on 64.5M dofs (the apply sweep's top size)
    and p=7 on the 64^3 mesh of 90.5M dofs (the large solve), in the launch
    configuration the benchmark times (deterministic E^T on the lattice
    numbering): sampled rows against the oracle's element matrices."""
    seed = inputs.mesh_seed(p, N)
    v = inputs.perturbed_vertices(N, N, N, seed=seed)
    sp = pf.Space(pf.Mesh(ctx, N, N, N, v), p)
    print(f"largest-size apply p={p} N={N} ndofs={sp.ndofs}", flush=True)
    x = inputs.random_vector(sp.ndofs, inputs.vector_seed(p, N))
    E = fem.element_restriction(N, N, N, p)
    ref = fem.reference_matrices(p, p + 2)
    L = N * p + 1
    rng = np.random.default_rng(100 + p)
    dofs = np.unique(np.concatenate([[0, L - 1, L * L // 2 + p, (L ** 3) // 2, sp.ndofs - 1],
                                     rng.integers(0, sp.ndofs, 10)]))
    op = pf.Operator(sp, pf.DIFFUSION)
    op.assemble()
    y = op.apply(torch.from_numpy(x).cuda())[torch.from_numpy(dofs).cuda()].cpu().numpy()
    yo = []
    for i in dofs:
        acc = 0.0
        for e, l in _elements_of_node(int(i), N, p):
            assert E[e, l] == i
            Ae = fem.element_diffusion(_corners(v, N, N, N, e), p, p + 2, ref=ref)
            acc += Ae[l] @ x[E[e]]
        yo.append(acc)
    yo = np.array(yo)
    np.testing.assert_allclose(y, yo, rtol=1e-12, atol=1e-12 * np.abs(yo).max())
    del op
    torch.cuda.synchronize()


@pytest.mark.parametrize("p,target", [(1, 8e6), (3, 8e6), (6, 8e6), (7, 8e6)])
def test_full_size_invariants(pf, ctx, p, target):
    N = inputs.mesh_n_for_dofs(p, target)
    v = inputs.perturbed_vertices(N, N, N, seed=inputs.mesh_seed(p, N))
    sp = pf.Space(pf.Mesh(ctx, N, N, N, v), p)
    ones = torch.ones(sp.ndofs, dtype=torch.float64, device="cuda")
    M = pf.Operator(sp, pf.MASS)
    M.assemble()
    vol = ctx.dot(ones, M.apply(ones)).item()
    assert abs(vol - 1.0) < 1e-12
    del M
    K = pf.Operator(sp, pf.DIFFUSION)
    K.assemble()
    k1 = K.apply(ones)
    dmax = K.diagonal().abs().max().item()
    assert k1.abs().max().item() <= 1e-12 * dmax
    # linear field: u^T K u = |a|^2 exactly
    X = torch.from_numpy(fem.node_coords(v, N, N, N, p) if N <= 40 else _node_coords_fast(v, N, p))
    a = torch.tensor([0.3, -1.2, 0.7], dtype=torch.float64)
    u = (X @ a + 0.4).cuda()
    e = ctx.dot(u, K.apply(u)).item()
    assert abs(e - float(a @ a)) < 1e-11


def _node_coords_fast(v, N, p):
    """Physical positions of all lattice nodes via the trilinear maps (vectorized)."""
    g = fem.gll_nodes(p)
    L = N * p + 1
    I = np.arange(L)
    el = np.minimum(I // p, N - 1)
    loc = g[I - el * p]
    V = v.reshape(N + 1, N + 1, N + 1, 3)
    out = np.zeros((L, L, L, 3))
    K3, J3, I3 = np.meshgrid(I, I, I, indexing="ij")
    ex, ey, ez = el[I3], el[J3], el[K3]
    s, t, u = loc[I3], loc[J3], loc[K3]
    for k in (0, 1):
        for j in (0, 1):
            for i in (0, 1):
                w = (s if i else 1 - s) * (t if j else 1 - t) * (u if k else 1 - u)
                out += w[..., None] * V[ez + k, ey + j, ex + i]
    return out.reshape(-1, 3)


@pytest.mark.parametrize("kind", ["mass", "diffusion"])
def test_apply_accumulate(pf, ctx, kind):
    nx, ny, nz, p = 3, 2, 2, 3
    seed = 44
    A = _oracle_matrix(kind, nx, ny, nz, p, seed, None)
    v, op = _build(pf, ctx, kind, nx, ny, nz, p, seed)
    n = op.space.ndofs
    x = inputs.random_vector(n, 1)
    y0 = inputs.random_vector(n, 2)
    ess = fem.essential_dofs(nx, ny, nz, p)
    for mode, im in MODES(pf):
        op.set_scatter_mode(mode)
        op.set_restriction_mode(im)
        for constrained in (False, True):
            y = torch.from_numpy(y0.copy()).cuda()
            op.apply(torch.from_numpy(x).cuda(), y, constrained=constrained, accumulate=True)
            Ax = fem.constrained_apply(A, x, ess) if constrained else A @ x
            e2, einf = _relerr(y.cpu().numpy(), y0 + Ax)
            assert e2 <= 1e-12 and einf <= 1e-12, (mode, constrained, e2)


@pytest.mark.parametrize("p", [1, 3, 6, 8])
@pytest.mark.parametrize("kind", ["mass", "diffusion"])
def test_apply_evector_is_element_matrix_action(pf, ctx, kind, p):
    nx, ny, nz = 3, 2, 1
    v, op = _build(pf, ctx, kind, nx, ny, nz, p, seed=60 + p, prec=pf.FP64 | pf.FP32)
    x = inputs.random_vector(op.space.ndofs, 3)
    E = fem.element_restriction(nx, ny, nz, p)
    EV = fem.element_vertices(v, nx, ny, nz)
    fn = fem.element_mass if kind == "mass" else fem.element_diffusion
    ess = np.zeros(op.space.ndofs, bool)
    ess[fem.essential_dofs(nx, ny, nz, p)] = True
    xt = np.where(ess, 0.0, x)
    for im in (pf.INDEX_LATTICE, pf.INDEX_MAP):
        op.set_restriction_mode(im)
        yE = op.apply_evector(torch.from_numpy(x).cuda()).cpu().numpy()
        yEc = op.apply_evector(torch.from_numpy(x).cuda(), constrained=True).cpu().numpy()
        y32 = op.apply_evector(torch.from_numpy(x).float().cuda()).double().cpu().numpy()
        for e in range(len(E)):
            Ae = fn(EV[e], p, p + 2)
            ref = Ae @ x[E[e]]
            np.testing.assert_allclose(yE[e], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
            refc = Ae @ xt[E[e]]
            np.testing.assert_allclose(yEc[e], refc, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
            np.testing.assert_allclose(y32[e], ref, rtol=1e-4, atol=5e-5 * np.abs(ref).max())


@pytest.mark.parametrize("p", [2, 5, 7])
def test_bf16_quadrature_data(pf, ctx, p):
    """BF16 storage of D: every entry is the nearest bfloat16 of the FP32 copy, and the
    FP32-arithmetic apply with it stays within the bfloat16 rounding of the operator."""
    nx, ny, nz = 3, 2, 2
    seed = inputs.mesh_seed(p, nx)
    A = _oracle_matrix("diffusion", nx, ny, nz, p, seed, None)
    v, op = _build(pf, ctx, "diffusion", nx, ny, nz, p, seed, prec=pf.FP64 | pf.FP32 | pf.BF16)
    q32 = op.qdata(pf.FP32).cpu().numpy().ravel()
    q16 = op.qdata(pf.BF16).cpu().numpy().ravel().astype(np.uint16)
    back = (q16.astype(np.uint32) << 16).view(np.float32)
    # nearest bfloat16: error at most half a unit in the 8-bit significand
    assert np.all(np.abs(back - q32) <= np.abs(q32) * 2.0 ** -8 + 1e-45)
    x = inputs.random_vector(op.space.ndofs, 2)
    for mode, im in MODES(pf)[::3]:
        op.set_scatter_mode(mode)
        y = op.apply(torch.from_numpy(x).float().cuda(), bf16=True).double().cpu().numpy()
        e2, _ = _relerr(y, A @ x)
        assert 1e-6 < e2 <= 1e-2, e2


def test_bf16_refined_solve_reaches_fp64_accuracy(pf, ctx):
    n, p = 4, 4
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p), pf.DIFFUSION)
    op.set_coefficient_sinx(0.5)
    op.assemble(pf.FP64 | pf.FP32 | pf.BF16)
    b = op.rhs()
    x64, s64 = op.solve(b, mode=pf.SOLVE_PLAIN_FP64, rtol=1e-12)
    xb, sb = op.solve(b, mode=pf.SOLVE_IR_BF16, rtol=1e-10, inner_rtol=1e-3)
    assert sb["true_rel_res"] <= 1e-10 and sb["outer_iterations"] >= 2
    assert ((xb - x64).norm() / x64.norm()).item() < 1e-8
    xm, sm = op.solve(b, mode=pf.SOLVE_MIXED_BF16, rtol=1e-10, inner_rtol=0.1)
    assert sm["true_rel_res"] <= 1e-10 and sm["outer_iterations"] >= 2
    assert ((xm - x64).norm() / x64.norm()).item() < 1e-8


def test_mixed_solve_limits_and_nonzero_guess(pf, ctx):
    n, p = 3, 3
    v = inputs.perturbed_vertices(n, n, n, seed=2)
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p), pf.DIFFUSION)
    op.assemble(pf.FP64 | pf.FP32)
    b = op.rhs()
    x, st = op.solve(b, mode=pf.SOLVE_MIXED_FP32, rtol=1e-14, inner_rtol=0.1, maxit=3,
                     raise_on_nonconvergence=False)
    assert st["iterations"] == 3 and st["true_rel_res"] > 1e-14
    with pytest.raises(pf.PafemError) as ei:
        op.solve(b, mode=pf.SOLVE_MIXED_FP32, rtol=1e-14, inner_rtol=0.1, maxit=3)
    assert ei.value.name == "NOT_CONVERGED"
    for bad in (0.0, 1.5):
        with pytest.raises(pf.PafemError) as ei:
            op.solve(b, mode=pf.SOLVE_MIXED_FP32, inner_rtol=bad)
        assert ei.value.name == "INVALID_ARG"
    with pytest.raises(pf.PafemError) as ei:
        op.solve(b, mode=7)
    assert ei.value.name == "INVALID_ARG"
    # restart from the last iterate: the first FP64 residual accounts for it
    x2, st2 = op.solve(b, x.clone(), mode=pf.SOLVE_MIXED_FP32, rtol=1e-10, inner_rtol=0.1)
    x64, _ = op.solve(b, mode=pf.SOLVE_PLAIN_FP64, rtol=1e-12)
    assert st2["true_rel_res"] <= 1e-10
    assert ((x2 - x64).norm() / x64.norm()).item() < 1e-8


@pytest.mark.parametrize("p", [2, 3, 6])
def test_fused_cg_step_matches_separate_kernels(pf, ctx, p):
    """On the lattice numbering one CG step runs fused (p . A p formed in the
    element pass, the x and r updates in the ordered E^T sum); on the stored
    map it runs as separate apply, dot and update kernels.  Both are the same
    Jacobi-PCG: same iteration counts (up to one), same solution.  The initial
    guess is nonzero on the boundary, so the essential rows of the direction
    are nonzero and their p_i^2 share of p . A p is exercised."""
    n = 3
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p), pf.DIFFUSION)
    op.set_coefficient_sinx(0.5)
    op.assemble(pf.FP64 | pf.FP32)
    b = op.rhs()
    x0 = torch.from_numpy(inputs.random_vector(op.space.ndofs, 5)).cuda()
    for mode, inner in ((pf.SOLVE_PLAIN_FP64, 1e-3), (pf.SOLVE_IR_FP32, 1e-3),
                        (pf.SOLVE_MIXED_FP32, 0.1)):
        out = {}
        for im in (pf.INDEX_LATTICE, pf.INDEX_MAP):
            op.set_restriction_mode(im)
            x, st = op.solve(b, x0.clone(), mode=mode, rtol=1e-10, inner_rtol=inner)
            assert st["true_rel_res"] <= 1e-10, (mode, im, st)
            out[im] = (x, st["iterations"])
        (xl, il), (xm, im_) = out[pf.INDEX_LATTICE], out[pf.INDEX_MAP]
        assert abs(il - im_) <= 1, (mode, il, im_)
        assert ((xl - xm).norm() / xm.norm()).item() < 1e-9, mode
    op.set_restriction_mode(pf.INDEX_LATTICE)


def test_fused_cg_full_size_matches_separate_kernels(pf, ctx):
    """At the full 7.9M-dof p=6 size, 30 iterations of the fused CG (lattice
    numbering) and of the separate-kernel CG (stored maps) from the same start
    agree: the two differ only in the order of the p.Ap and (r.z, r.r) sums."""
    n, p = 33, 6
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p), pf.DIFFUSION)
    op.set_coefficient_sinx(0.5)
    op.assemble(pf.FP64 | pf.FP32)
    b = op.rhs()
    for mode, tol in ((pf.SOLVE_PLAIN_FP64, 1e-11), (pf.SOLVE_MIXED_FP32, 1e-5)):
        out = {}
        for im in (pf.INDEX_LATTICE, pf.INDEX_MAP):
            op.set_restriction_mode(im)
            x, st = op.solve(b, mode=mode, rtol=1e-30, inner_rtol=0.1, maxit=30, check_every=10,
                             raise_on_nonconvergence=False)
            assert st["iterations"] == 30
            out[im] = (x, st["rel_res"])
            if mode == pf.SOLVE_PLAIN_FP64:
                # the CG invariant: the recursively updated residual is b - A x
                # recomputed through the apply that the sampled-row tests pin
                # to the oracle
                assert abs(st["true_rel_res"] - st["rel_res"]) <= 1e-8 * st["rel_res"], (im, st)
        (xl, rl), (xm, rm) = out[pf.INDEX_LATTICE], out[pf.INDEX_MAP]
        assert ((xl - xm).norm() / xm.norm()).item() < tol, mode
        assert abs(rl - rm) <= tol * rm, (mode, rl, rm)
    op.set_restriction_mode(pf.INDEX_LATTICE)


def test_fused_cg_full_size_solves_to_tolerance(pf, ctx):
    """One fused FP64 Jacobi-PCG solve to 1e-10 at the full 7.9M-dof p=6 size
    (grid-stride branch of the fused E^T step and the wide alpha reduction):
    the residual recomputed in FP64 meets the tolerance, and the solution is
    close to the manufactured one (discretization error, not solver error)."""
    n, p = 33, 6
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    sp_ = pf.Space(pf.Mesh(ctx, n, n, n, v), p)
    op = pf.Operator(sp_, pf.DIFFUSION)
    op.assemble(pf.FP64)
    b = op.rhs()
    x, st = op.solve(b, rtol=1e-10, check_every=50)
    assert st["true_rel_res"] <= 1e-10, st
    assert st["rel_res"] <= 1e-10, st
    # sampled nodal values against u = sin sin sin at the GLL nodes of a few elements
    xn = x.cpu().numpy()
    rng = np.random.default_rng(4)
    for e in rng.integers(0, n ** 3, 6):
        ex, ey, ez = e % n, (e // n) % n, e // (n * n)
        vv = v.reshape(n + 1, n + 1, n + 1, 3)
        v8 = np.array([vv[ez + k, ey + j, ex + i] for k in (0, 1) for j in (0, 1) for i in (0, 1)])
        Xn, _ = fem.trilinear(v8, fem.tensor_points(fem.gll_nodes(p)))
        E = fem.element_restriction(1, 1, 1, p)[0]  # local lattice offsets of one element
        L = n * p + 1
        loc = E % (p + 1) + L * ((E // (p + 1)) % (p + 1)) + L * L * (E // (p + 1) ** 2)
        g = (ex * p) + L * (ey * p) + L * L * (ez * p) + loc
        ue = inputs.u_exact(Xn[:, 0], Xn[:, 1], Xn[:, 2])
        assert np.abs(xn[g] - ue).max() < 1e-6


def test_footprint_counts_qdata_and_workspace(pf, ctx):
    """The operator footprint is the quadrature data plus the E-vector, the
    inverse diagonal, the CG vectors and the partials, and it covers what a
    solve allocates."""
    n, p = 6, 4
    v = inputs.perturbed_vertices(n, n, n, seed=2)
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p), pf.DIFFUSION)
    op.assemble(pf.FP64 | pf.FP32)
    nd, ne = op.space.ndofs, op.space.nelems
    q64 = ne * (p + 2) ** 3 * 6 * 8
    assert op.qdata_bytes(pf.FP64) == q64
    f64 = op.footprint_bytes(pf.FP64)
    f32 = op.footprint_bytes(pf.FP64 | pf.FP32)
    evec = ne * (p + 1) ** 3 * 8
    assert f64 >= q64 + evec + nd * (8 + 4 * 8)
    assert f32 - f64 == q64 // 2 + nd * 4 + nd * 16
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    b = op.rhs()
    op.solve(b, mode=pf.SOLVE_MIXED_FP32, inner_rtol=0.1)
    torch.cuda.synchronize()
    grown = free0 - torch.cuda.mem_get_info()[0]
    assert grown <= f32 - q64 - q64 // 2 + 8 * nd + (4 << 20)
