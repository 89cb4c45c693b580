"""The allocation-free apply under HIP graph capture: captured once (through
torch's graph capture on its capture stream), replayed several times with
eager work and synchronizations between the replays; every replay equals the
eager pafem_op_apply bitwise, FP64 and FP32, after the input changed in place.
"""
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


@pytest.fixture(scope="module")
def ctx(pf):
    return pf.Context(0)


@pytest.mark.parametrize("p,kind", [(3, "diffusion"), (6, "diffusion"), (4, "mass")])
def test_captured_noalloc_apply_replays_match_eager(pf, ctx, p, kind):
    n = 5
    v = inputs.perturbed_vertices(n, n, n, seed=inputs.mesh_seed(p, n))
    op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, v), p),
                     pf.DIFFUSION if kind == "diffusion" else pf.MASS)
    op.set_coefficient_sinx(0.5)
    op.assemble(pf.FP64 | pf.FP32)
    nd = op.space.ndofs
    x = torch.from_numpy(inputs.random_vector(nd, inputs.vector_seed(p, n))).cuda()
    x32 = x.float()
    y = torch.zeros_like(x)
    y32 = torch.zeros_like(x32)
    # warm-up on a side stream (as torch's capture recommends), then capture
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        op.apply_noalloc(x, y, constrained=True)
        op.apply_noalloc(x32, y32)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        op.apply_noalloc(x, y, constrained=True)
        op.apply_noalloc(x32, y32)
    for k in range(4):
        # eager work between the replays: new input in place, other applies
        x.mul_(1.0 + 0.125 * k).add_(0.01 * k)
        x32.copy_(x)
        ref = op.apply(x, constrained=True)
        ref32 = op.apply(x32)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (k, (y - ref).abs().max().item())
        assert torch.equal(y32, ref32), k
