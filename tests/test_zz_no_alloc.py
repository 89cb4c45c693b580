"""The allocation-free apply (pafem_op_apply_noalloc) against pafem_op_apply.

Both run the same element and E^T kernels (deterministic E^T on the lattice
numbering), so the results must agree bitwise; the allocation-free entry point
keeps its E-vector in the library's fixed device array, shared by every call
on the GPU, so two calls in a row (the second on a smaller operator) must each
give the result of the ordinary entry point.
"""
import numpy as np
import pytest

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


def _op(pf, ctx, kind, n, p, prec):
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    sp = pf.Space(pf.Mesh(ctx, n, n, n, v), p)
    op = pf.Operator(sp, kind)
    op.assemble(prec)
    return op


@pytest.mark.parametrize("kind", ["diffusion", "mass"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_apply_matches_apply_twice(pf, kind, dtype):
    ctx = pf.Context(0)
    k = pf.DIFFUSION if kind == "diffusion" else pf.MASS
    td = torch.float64 if dtype == "f64" else torch.float32
    # the second operator is smaller than the first: the shared workspace then
    # holds the first call's values beyond the second's extent
    for n, p, flags in [(9, 5, dict(constrained=True)), (4, 3, dict())]:
        print(f"noalloc apply {kind} {dtype} n={n} p={p} {flags}", flush=True)
        op = _op(pf, ctx, k, n, p, pf.FP64 | pf.FP32)
        x = torch.from_numpy(inputs.random_vector(op.space.ndofs,
                                                  inputs.vector_seed(p, n))).to(td).cuda()
        y_ref = op.apply(x, **flags)
        y = torch.full_like(x, float("nan"))
        op.apply_noalloc(x, y, **flags)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        # accumulate: y += A x
        y0 = torch.from_numpy(inputs.random_vector(op.space.ndofs, 7)).to(td).cuda()
        y_ref2 = y0.clone()
        op.apply(x, y_ref2, accumulate=True, **flags)
        y2 = y0.clone()
        op.apply_noalloc(x, y2, accumulate=True, **flags)
        torch.cuda.synchronize()
        assert torch.equal(y2, y_ref2)


def test_noalloc_apply_rejects_oversize(pf):
    """An operator whose workspace exceeds the fixed array is refused before launch."""
    ctx = pf.Context(0)
    n, p = 24, 6  # 13824 elements * 343 words * 8 B = 37.9 MB > 32 MiB
    op = _op(pf, ctx, pf.DIFFUSION, n, p, pf.FP64)
    x = torch.zeros(op.space.ndofs, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(pf.PafemError) as ei:
        op.apply_noalloc(x, y)
    assert ei.value.name == "INVALID_ARG" and "workspace" in str(ei.value)
    # the FP32 workspace (half the bytes) fits
    op32 = _op(pf, ctx, pf.DIFFUSION, n, p, pf.FP64 | pf.FP32)
    x32 = torch.from_numpy(inputs.random_vector(op32.space.ndofs, 3)).float().cuda()
    y32 = torch.empty_like(x32)
    op32.apply_noalloc(x32, y32)
    torch.cuda.synchronize()
    assert torch.equal(y32, op32.apply(x32))
    assert np.isfinite(y32.cpu().numpy()).all()
