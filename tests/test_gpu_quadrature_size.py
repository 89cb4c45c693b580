"""GPU parity of operators built with a non-default number of quadrature points
per direction (q1d in p+1 .. 10; the default is p+2) against the CPU oracle,
which integrates with the same Gauss-Legendre rule.

These operators run the run-time-sized element kernel.  Tolerances are those
of the default kernels: FP64 relative error <= 1e-12 (2-norm and max-norm),
FP32 <= 5e-5.
"""
import functools

import numpy as np
import pytest

from oracle import fem
from paper_2402_15940_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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
def _oracle(kind, nx, ny, nz, p, q, seed, coef):
    v = inputs.perturbed_vertices(nx, ny, nz, seed=seed)
    coef_q = None
    if coef == "sinx":
        coef_q = inputs.coef_sin_x(fem.qpoint_coords(v, nx, ny, nz, q)[:, 0, :])
    return fem.assemble(kind, v, nx, ny, nz, p, q=q, coef_q=coef_q)


def _op(pf, ctx, kind, mesh, p, q, seed, coef=None, prec=None):
    v = inputs.perturbed_vertices(*mesh, seed=seed)
    op = pf.Operator(pf.Space(pf.Mesh(ctx, *mesh, v), p),
                     pf.DIFFUSION if kind == "diffusion" else pf.MASS, q1d=q)
    if coef == "sinx":
        op.set_coefficient_sinx(0.5)
    op.assemble(prec if prec is not None else pf.FP64 | pf.FP32)
    return v, op


def _rel(y, yref):
    d = np.asarray(y) - np.asarray(yref)
    return np.linalg.norm(d) / np.linalg.norm(yref), np.abs(d).max() / np.abs(yref).max()


CASES = [(1, 2), (1, 10), (2, 3), (3, 4), (3, 7), (5, 6), (6, 7), (6, 9), (7, 10), (8, 9),
         (8, 10)]


@pytest.mark.parametrize("p,q", CASES)
@pytest.mark.parametrize("kind", ["diffusion", "mass"])
def test_apply_matches_oracle(pf, ctx, kind, p, q):
    mesh = (3, 2, 2)
    seed = inputs.mesh_seed(p, 3) + q
    coef = "sinx" if (p + q) % 2 else None
    _, op = _op(pf, ctx, kind, mesh, p, q, seed, coef)
    assert op.q == q
    A = _oracle(kind, *mesh, p, q, seed, coef)
    x = inputs.random_vector(A.shape[0], inputs.vector_seed(p, q))
    xt = torch.from_numpy(x).cuda()
    ref = A @ x
    ess = fem.essential_dofs(*mesh, p)
    refc = fem.constrained_apply(A, x, ess)
    modes = [(pf.SCATTER_DETERMINISTIC, pf.INDEX_LATTICE), (pf.SCATTER_DETERMINISTIC, pf.INDEX_MAP),
             (pf.SCATTER_ATOMIC, pf.INDEX_LATTICE)]
    for scatter, index in modes:
        op.set_scatter_mode(scatter)
        op.set_restriction_mode(index)
        e2, einf = _rel(op.apply(xt).cpu().numpy(), ref)
        assert e2 <= 1e-12 and einf <= 1e-12, (scatter, index, e2, einf)
        e2, einf = _rel(op.apply(xt, constrained=True).cpu().numpy(), refc)
        assert e2 <= 1e-12 and einf <= 1e-12, (scatter, index, e2, einf)
    y32 = op.apply(xt.float()).double().cpu().numpy()
    assert _rel(y32, ref)[0] <= 5e-5
    # the E-vector is the element matrices' action
    op.set_scatter_mode(pf.SCATTER_DETERMINISTIC)
    op.set_restriction_mode(pf.INDEX_LATTICE)
    yE = op.apply_evector(xt).cpu().numpy().reshape(-1)
    E = fem.element_restriction(*mesh, p)
    EV = fem.element_vertices(inputs.perturbed_vertices(*mesh, seed=seed), *mesh)
    coef_q = None
    if coef == "sinx":
        v = inputs.perturbed_vertices(*mesh, seed=seed)
        coef_q = inputs.coef_sin_x(fem.qpoint_coords(v, *mesh, q)[:, 0, :])
    ref_e = []
    for e in range(len(EV)):
        kq = None if coef_q is None else coef_q[e]
        Ae = (fem.element_diffusion(EV[e], p, q, kq) if kind == "diffusion"
              else fem.element_mass(EV[e], p, q, kq))
        ref_e.append(Ae @ x[E[e]])
    assert _rel(yE, np.concatenate(ref_e))[0] <= 1e-12


@pytest.mark.parametrize("p,q", [(1, 2), (4, 5), (4, 9), (8, 10)])
@pytest.mark.parametrize("kind", ["diffusion", "mass"])
def test_diagonal_matches_oracle(pf, ctx, kind, p, q):
    mesh = (3, 3, 1)
    seed = inputs.mesh_seed(p, 3)
    _, op = _op(pf, ctx, kind, mesh, p, q, seed, prec=pf.FP64)
    A = _oracle(kind, *mesh, p, q, seed, None)
    e2, einf = _rel(op.diagonal().cpu().numpy(), A.diagonal())
    assert e2 <= 1e-12 and einf <= 1e-12
    ess = fem.essential_dofs(*mesh, p)
    assert _rel(op.diagonal(constrained=True).cpu().numpy(),
                fem.constrained_diagonal(A, ess))[0] <= 1e-12


@pytest.mark.parametrize("p,q", [(1, 3), (3, 4), (5, 9), (8, 10)])
def test_rhs_matches_oracle(pf, ctx, p, q):
    mesh = (3, 2, 2)
    v, op = _op(pf, ctx, "diffusion", mesh, p, q, seed=31, prec=pf.FP64)
    bo = fem.rhs(v, *mesh, p, q=q, f=inputs.f_manufactured)
    bo[fem.essential_dofs(*mesh, p)] = 0.0
    e2, einf = _rel(op.rhs().cpu().numpy(), bo)
    assert e2 <= 1e-12 and einf <= 1e-12
    xq = op.qpoint_coords()
    assert tuple(xq.shape) == (12, 3, q ** 3)
    np.testing.assert_allclose(xq.cpu().numpy(), fem.qpoint_coords(v, *mesh, q), rtol=0,
                               atol=1e-14)


@pytest.mark.parametrize("p,q", [(2, 3), (4, 8)])
def test_solves_match_oracle(pf, ctx, p, q):
    n = 4
    seed = inputs.mesh_seed(p, n)
    v, op = _op(pf, ctx, "diffusion", (n, n, n), p, q, seed, "sinx")
    coef_q = inputs.coef_sin_x(fem.qpoint_coords(v, n, n, n, q)[:, 0, :])
    ref = fem.solve_poisson(v, n, n, n, p, q=q, f=inputs.f_manufactured, coef_q=coef_q,
                            rtol=1e-12)
    b = op.rhs()
    xk, sk = op.solve(b, rtol=1e-10)
    assert sk["true_rel_res"] <= 1e-10 and _rel(xk.cpu().numpy(), ref["x"])[0] <= 1e-8
    xg, sg = op.solve(b, rtol=1e-10, launch=pf.LAUNCH_GRAPH)
    assert sg["iterations"] == sk["iterations"] and torch.equal(xg, xk)
    xm, sm = op.solve(b, mode=pf.SOLVE_MIXED_FP32, rtol=1e-10, inner_rtol=0.1)
    assert sm["true_rel_res"] <= 1e-10 and _rel(xm.cpu().numpy(), ref["x"])[0] <= 1e-8
    mg = pf.Multigrid(op)
    xp, st = mg.solve(b, rtol=1e-10)
    assert st["true_rel_res"] <= 1e-10 and _rel(xp.cpu().numpy(), ref["x"])[0] <= 1e-8


def test_unsupported_combinations_are_refused(pf, ctx):
    v = inputs.perturbed_vertices(2, 2, 2, seed=5)
    sp = pf.Space(pf.Mesh(ctx, 2, 2, 2, v), 3)
    for q in (1, 3, 11):
        with pytest.raises(pf.PafemError):
            pf.Operator(sp, pf.DIFFUSION, q1d=q)
    assert pf.Operator(sp, pf.MASS, q1d=0).q == 5
    op = pf.Operator(sp, pf.DIFFUSION, q1d=6)
    with pytest.raises(pf.PafemError):
        op.assemble(pf.FP64 | pf.BF16)
    with pytest.raises(pf.PafemError):
        op.set_assembly_level(pf.ASSEMBLY_MATRIX_FREE)
    op.assemble(pf.FP64)
    with pytest.raises(pf.PafemError):
        op.solve(op.rhs(), launch=pf.LAUNCH_PERSISTENT)
    assert op.qdata_bytes(pf.FP64) == 8 * 6 ** 3 * 6 * 8


def test_allocation_free_apply_with_other_rule(pf, ctx):
    mesh = (3, 2, 2)
    _, op = _op(pf, ctx, "diffusion", mesh, 4, 8, seed=17, prec=pf.FP64)
    x = torch.from_numpy(inputs.random_vector(op.space.ndofs, 3)).cuda()
    y0 = op.apply(x, constrained=True)
    y1 = torch.empty_like(x)
    op.apply_noalloc(x, y1, constrained=True)
    assert torch.equal(y0, y1)
