"""GPU parity of the p-multigrid preconditioner and solve (through the C ABI)
against the CPU oracle (oracle/pmg.py).

Transfers and the smoother are single linear maps: relative error <= 1e-13.
The V-cycle (with the eigenvalue bounds the test sets on both sides) and the
flexible-CG iterates combine a few dozen such steps with a fixed-step coarse
CG: relative error <= 1e-12 for one V-cycle, the same iteration count and a
solution within 1e-9 of the oracle for the solve, whose FP64 residual b - A x
must be <= 1e-10.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem, pmg
from paper_2402_15940_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MESH = (5, 4, 3)  # 60 elements; the order-1 level has 24 free dofs (> coarse steps)


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


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _setup(pf, ctx, p, kind="diffusion", coef=None, mesh=MESH):
    nx, ny, nz = mesh
    v = inputs.perturbed_vertices(nx, ny, nz, seed=inputs.mesh_seed(p, nx))
    op = pf.Operator(pf.Space(pf.Mesh(ctx, nx, ny, nz, v), p),
                     pf.DIFFUSION if kind == "diffusion" else pf.MASS)
    if coef == "sinx":
        op.set_coefficient_sinx(0.5)
    op.assemble(pf.FP64)
    return v, op


def _oracle_levels(v, p, kind="diffusion", coef=None, mesh=MESH):
    nx, ny, nz = mesh
    c = (lambda x, y, z: inputs.coef_sin_x(x)) if coef == "sinx" else None
    levels = pmg.build_levels(v, nx, ny, nz, p, kind, c)
    for L in levels[:-1]:
        lam = spla.eigs(sp.diags(L.dinv) @ L.A, k=1, which="LM", return_eigenvectors=False)[0]
        L.lmax = 1.1 * abs(lam)
    return levels


def _zero_ess(x, ess):
    x = x.copy()
    x[ess] = 0.0
    return x


@pytest.mark.parametrize("pfine", range(2, 9))
def test_transfer_matches_oracle(pf, ctx, pfine):
    nx, ny, nz = 3, 2, 2
    v, op = _setup(pf, ctx, pfine, mesh=(nx, ny, nz))
    mg = pf.Multigrid(op)
    pc = pfine // 2
    assert mg.level_info(1)["p"] == pc
    P = pmg.prolongation(nx, ny, nz, pc, pfine)
    rng = np.random.default_rng(pfine)
    uc = rng.uniform(-1, 1, P.shape[1])
    uf = mg.prolong(0, torch.from_numpy(uc).cuda()).cpu().numpy()
    assert _rel(uf, P @ uc) <= 1e-13
    rf = rng.uniform(-1, 1, P.shape[0])
    rc = mg.restrict(0, torch.from_numpy(rf).cuda()).cpu().numpy()
    ref = _zero_ess(P.T @ rf, fem.essential_dofs(nx, ny, nz, pc))
    assert _rel(rc, ref) <= 1e-13
    # every coarser pair of the hierarchy too
    for k in range(1, mg.num_levels - 1):
        pk, pk1 = mg.level_info(k)["p"], mg.level_info(k + 1)["p"]
        Pk = pmg.prolongation(nx, ny, nz, pk1, pk)
        u = rng.uniform(-1, 1, Pk.shape[1])
        assert _rel(mg.prolong(k, torch.from_numpy(u).cuda()).cpu().numpy(), Pk @ u) <= 1e-13


@pytest.mark.parametrize("p", [2, 5, 8])
def test_smoother_matches_oracle(pf, ctx, p):
    v, op = _setup(pf, ctx, p)
    levels = _oracle_levels(v, p)
    mg = pf.Multigrid(op)
    mg.set_lmax(0, levels[0].lmax)
    b = _zero_ess(np.random.default_rng(p).uniform(-1, 1, levels[0].A.shape[0]), levels[0].ess)
    x = mg.smooth(0, torch.from_numpy(b).cuda()).cpu().numpy()
    xo, _ = pmg.chebyshev(levels[0].A, levels[0].dinv, b, levels[0].lmax,
                          mg.opts.cheb_degree, mg.opts.cheb_lower)
    assert _rel(x, xo) <= 1e-13


def test_eigenvalue_estimate(pf, ctx):
    p = 4
    v, op = _setup(pf, ctx, p)
    levels = _oracle_levels(v, p)
    mg = pf.Multigrid(op, power_iters=30)
    for k in range(mg.num_levels - 1):
        lam = levels[k].lmax / 1.1
        est = mg.level_info(k)["lmax"] / mg.opts.lmax_safety
        # the Rayleigh quotient never exceeds the largest eigenvalue and is close after 30 steps
        assert 0.9 * lam <= est <= lam * (1 + 1e-9), (k, est, lam)


@pytest.mark.parametrize("p,coef", [(2, None), (4, None), (6, "sinx"), (8, None)])
def test_vcycle_matches_oracle(pf, ctx, p, coef):
    v, op = _setup(pf, ctx, p, coef=coef)
    levels = _oracle_levels(v, p, coef=coef)
    mg = pf.Multigrid(op)
    assert mg.num_levels == len(levels)
    for k, L in enumerate(levels[:-1]):
        mg.set_lmax(k, L.lmax)
    r = _zero_ess(np.random.default_rng(10 + p).uniform(-1, 1, levels[0].A.shape[0]),
                  levels[0].ess)
    z = mg.vcycle(torch.from_numpy(r).cuda()).cpu().numpy()
    zo = pmg.vcycle(levels, r, mg.opts.cheb_degree, mg.opts.cheb_lower, mg.opts.coarse_iters)
    assert _rel(z, zo) <= 1e-12


@pytest.mark.parametrize("p,coef", [(3, None), (6, "sinx")])
def test_pmg_solve_matches_oracle(pf, ctx, p, coef):
    nx, ny, nz = MESH
    v, op = _setup(pf, ctx, p, coef=coef)
    levels = _oracle_levels(v, p, coef=coef)
    mg = pf.Multigrid(op)
    for k, L in enumerate(levels[:-1]):
        mg.set_lmax(k, L.lmax)
    b = op.rhs()
    bo = b.cpu().numpy()
    x, st = mg.solve(b, rtol=1e-10)
    assert st["converged"] and st["true_rel_res"] <= 1e-10, st
    xo, it, hist = pmg.pmg_fcg(levels, bo, rtol=1e-10, degree=mg.opts.cheb_degree,
                               lower=mg.opts.cheb_lower, coarse_iters=mg.opts.coarse_iters)
    assert abs(st["iterations"] - it) <= 1, (st, it)
    assert _rel(x.cpu().numpy(), xo) <= 1e-9
    # far fewer iterations than Jacobi-PCG on the same problem, same solution
    xj, stj = op.solve(b, rtol=1e-10)
    assert st["iterations"] * 4 <= stj["iterations"], (st, stj)
    assert _rel(x.cpu().numpy(), xj.cpu().numpy()) <= 1e-8


def test_pmg_solve_at_size(pf, ctx):
    """A 0.9M-dof p=6 problem: the FP64 residual confirms convergence, and the
    solution agrees with plain Jacobi-PCG's."""
    n, p = 16, 6
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p), pf.DIFFUSION)
    op.set_coefficient_sinx(0.5)
    op.assemble(pf.FP64)
    print(f"pmg solve at size: n={n} p={p} ndofs={op.space.ndofs}", flush=True)
    mg = pf.Multigrid(op)
    b = op.rhs()
    x, st = mg.solve(b, rtol=1e-10)
    assert st["converged"] and st["true_rel_res"] <= 1e-10, st
    xj, stj = op.solve(b, rtol=1e-10)
    assert st["iterations"] * 10 <= stj["iterations"], (st, stj)
    assert _rel(x.cpu().numpy(), xj.cpu().numpy()) <= 1e-8


def test_pmg_rejects_bad_input(pf, ctx):
    v, op = _setup(pf, ctx, 2, mesh=(2, 2, 2))
    with pytest.raises(pf.PafemError):
        pf.Multigrid(op, cheb_degree=0)
    with pytest.raises(pf.PafemError):
        pf.Multigrid(op, cheb_lower=1.5)
    mg = pf.Multigrid(op)
    with pytest.raises(pf.PafemError):
        mg.set_lmax(mg.num_levels - 1, 1.0)  # the order-1 level is not smoothed
    op_q = pf.Operator(op.space, pf.DIFFUSION)
    op_q.set_coefficient_qpts(torch.ones(op.space.nelems * 64, dtype=torch.float64,
                                         device="cuda"))
    op_q.assemble(pf.FP64)
    with pytest.raises(pf.PafemError):
        pf.Multigrid(op_q)
