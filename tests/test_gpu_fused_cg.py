"""The launch forms of the CG iterations (separate kernels, a captured HIP
graph replayed, one persistent cooperative kernel per batch of iterations)
against each other and against the CPU oracle.

Kernels and graph run the same kernels with the same arguments: bitwise equal
solutions and iteration counts, over several solves in a row (the graph is
captured once and replayed with the program's own work in between).  The
persistent kernel sums its reductions in another fixed order: the oracle's
iteration count and solution (within 1e-12 relative on the 4^3 affine
problem), and at full size the CG invariant (recursive residual = FP64
residual) and convergence to 1e-10 on the FP64 residual.
"""
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


def _op(pf, ctx, n, p, kind="diffusion", coef=None, seed=True, prec=None):
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n) if seed else None)
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p),
                     pf.DIFFUSION if kind == "diffusion" else pf.MASS)
    if coef == "sinx":
        op.set_coefficient_sinx(0.5)
    op.assemble(prec if prec is not None else pf.FP64)
    return v, op


@pytest.mark.parametrize("p,check_every,kind", [(2, 1, "diffusion"), (6, 4, "diffusion"),
                                                (3, 3, "mass")])
def test_graph_equals_kernels_over_several_solves(pf, ctx, p, check_every, kind):
    _, op = _op(pf, ctx, 4, p, kind=kind, coef="sinx")
    b0 = op.rhs()
    for k in range(3):
        # a different right-hand side each time; eager work between the replays
        b = b0 * (1.0 + 0.25 * k) + (k * 1e-3) * torch.sin(torch.arange(b0.numel(),
                                                                         device="cuda",
                                                                         dtype=torch.float64))
        ess = torch.from_numpy(np.asarray(op.space.ess_dofs(), dtype=np.int64)).cuda()
        b[ess] = 0.0
        xk, sk = op.solve(b, rtol=1e-10, check_every=check_every, launch=pf.LAUNCH_KERNELS)
        xg, sg = op.solve(b, rtol=1e-10, check_every=check_every, launch=pf.LAUNCH_GRAPH)
        torch.cuda.synchronize()
        assert sk["iterations"] == sg["iterations"] and sk["true_rel_res"] <= 1e-10
        assert torch.equal(xk, xg), (k, (xk - xg).abs().max().item())


def test_graph_ir_inner_solves_equal_kernels(pf, ctx):
    _, op = _op(pf, ctx, 4, 4, coef="sinx", prec=pf.FP64 | pf.FP32)
    b = op.rhs()
    xk, sk = op.solve(b, mode=pf.SOLVE_IR_FP32, rtol=1e-10, inner_rtol=1e-3, check_every=2)
    xg, sg = op.solve(b, mode=pf.SOLVE_IR_FP32, rtol=1e-10, inner_rtol=1e-3, check_every=2,
                      launch=pf.LAUNCH_GRAPH)
    assert sk["iterations"] == sg["iterations"] and sk["outer_iterations"] == sg["outer_iterations"]
    assert torch.equal(xk, xg)


@pytest.mark.parametrize("check_every", [1, 3, 64])
def test_persistent_small_affine_matches_oracle(pf, ctx, check_every):
    n, p = 4, 2
    v = inputs.perturbed_vertices(n, n, n, seed=None)
    ref = fem.solve_poisson(v, n, n, n, p, f=inputs.f_manufactured, rtol=1e-10)
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p), pf.DIFFUSION)
    op.assemble()
    b = op.rhs()
    x, st = op.solve(b, rtol=1e-10, check_every=check_every, launch=pf.LAUNCH_PERSISTENT)
    assert st["iterations"] == ref["iterations"] and st["true_rel_res"] <= 1e-10, st
    x = x.cpu().numpy()
    assert np.linalg.norm(x - ref["x"]) <= 1e-12 * np.linalg.norm(ref["x"])


@pytest.mark.parametrize("p,kind", [(1, "diffusion"), (5, "diffusion"), (8, "diffusion"),
                                    (4, "mass")])
def test_persistent_perturbed_matches_oracle_and_kernels(pf, ctx, p, kind):
    n = 4 if p < 8 else 3
    v, op = _op(pf, ctx, n, p, kind=kind, coef="sinx")
    xq = fem.qpoint_coords(v, n, n, n, p + 2)
    coef_q = inputs.coef_sin_x(xq[:, 0, :])
    A = fem.assemble(kind, v, n, n, n, p, coef_q=coef_q)
    b = op.rhs()
    bo = b.cpu().numpy()
    ess = fem.essential_dofs(n, n, n, p)
    free = np.setdiff1d(np.arange(A.shape[0]), ess)
    Aff = A[free][:, free].tocsr()
    xf, it, _ = fem.pcg(Aff, bo[free], 1.0 / Aff.diagonal(), rtol=1e-12)
    xo = np.zeros_like(bo)
    xo[free] = xf
    xp, sp_ = op.solve(b, rtol=1e-10, check_every=8, launch=pf.LAUNCH_PERSISTENT)
    xk, sk = op.solve(b, rtol=1e-10, check_every=8)
    assert sp_["true_rel_res"] <= 1e-10, sp_
    assert abs(sp_["iterations"] - sk["iterations"]) <= 1, (sp_, sk)
    xp = xp.cpu().numpy()
    assert np.linalg.norm(xp - xo) <= 1e-8 * np.linalg.norm(xo)
    assert np.linalg.norm(xp - xk.cpu().numpy()) <= 1e-9 * np.linalg.norm(xo)


def test_persistent_full_size_invariant_and_solve(pf, ctx):
    """7.9M dofs, p = 6: more element groups than the grid holds, so every
    workgroup walks several; the recursive residual after 30 iterations equals
    the FP64 residual b - A x, and the solve converges on the FP64 residual."""
    n, p = 33, 6
    _, op = _op(pf, ctx, n, p, coef="sinx")
    print(f"persistent CG at n={n} p={p} ndofs={op.space.ndofs}", flush=True)
    b = op.rhs()
    x30, s30 = op.solve(b, rtol=1e-10, maxit=30, check_every=30, launch=pf.LAUNCH_PERSISTENT,
                        raise_on_nonconvergence=False)
    assert s30["iterations"] == 30
    assert abs(s30["rel_res"] - s30["true_rel_res"]) <= 1e-8 * s30["true_rel_res"], s30
    xk30, sk30 = op.solve(b, rtol=1e-10, maxit=30, check_every=30,
                          raise_on_nonconvergence=False)
    assert torch.linalg.norm(x30 - xk30) <= 1e-10 * torch.linalg.norm(xk30)
    x, st = op.solve(b, rtol=1e-10, check_every=100, launch=pf.LAUNCH_PERSISTENT)
    assert st["true_rel_res"] <= 1e-10, st


def test_launch_forms_rejected_where_unavailable(pf, ctx):
    _, op = _op(pf, ctx, 3, 3, prec=None)
    op32 = _op(pf, ctx, 3, 3)[1]
    op32.assemble(pf.FP64 | pf.FP32)
    b = op32.rhs()
    with pytest.raises(pf.PafemError):
        op32.solve(b, mode=pf.SOLVE_MIXED_FP32, inner_rtol=0.1, launch=pf.LAUNCH_GRAPH)
    with pytest.raises(pf.PafemError):
        op32.solve(b, mode=pf.SOLVE_IR_FP32, launch=pf.LAUNCH_PERSISTENT)
    op.set_scatter_mode(pf.SCATTER_ATOMIC)
    with pytest.raises(pf.PafemError):
        op.solve(op.rhs(), launch=pf.LAUNCH_PERSISTENT)
    with pytest.raises(pf.PafemError):
        op.solve(op.rhs(), launch=7)


@pytest.mark.parametrize("n,p", [(1, 3), (2, 2), (2, 5)])
def test_persistent_grid_smaller_than_the_xcd_count(pf, ctx, n, p):
    """Grids of 1..7 workgroups: every workgroup is its own barrier group and
    walks the items with a plain stride; the solve matches the oracle."""
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p), pf.DIFFUSION)
    op.assemble()
    b = op.rhs()
    xk, sk = op.solve(b, rtol=1e-10, check_every=4)
    xp, sp_ = op.solve(b, rtol=1e-10, check_every=4, launch=pf.LAUNCH_PERSISTENT)
    assert sp_["true_rel_res"] <= 1e-10 and abs(sp_["iterations"] - sk["iterations"]) <= 1
    ref = fem.solve_poisson(v, n, n, n, p, f=inputs.f_manufactured, rtol=1e-12)
    xr = ref["x"]
    assert np.linalg.norm(xp.cpu().numpy() - xr) <= 1e-8 * max(np.linalg.norm(xr), 1e-300)
