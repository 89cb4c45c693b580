"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/pafem.h declares, and its host setup (1D tables, element
restriction, its transpose, essential dofs) matches the oracle -- the
integer maps bit for bit."""
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import fem
from paper_2402_15940_amd import inputs
from paper_2402_15940_amd import pafem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pafem.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pafem_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = pafem.lib()
    declared = _declared()
    assert len(declared) >= 25
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", pafem.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (pafem_\w+)", out))
    assert set(declared) <= exported
    # the binding covers exactly the declared API
    assert set(pafem.exported_symbols()) == set(declared)


@pytest.mark.parametrize("p", range(1, 9))
def test_basis_tables_match_oracle(p):
    q = p + 2
    t = pafem.basis_tables(p, q)
    B, G, pts, wts = fem.basis_tables(p, q)
    np.testing.assert_allclose(t["nodes"], fem.gll_nodes(p), atol=4e-16)
    np.testing.assert_allclose(t["points"], pts, atol=4e-16)
    np.testing.assert_allclose(t["weights"], wts, rtol=1e-14)
    np.testing.assert_allclose(t["B"], B, atol=2e-14)
    np.testing.assert_allclose(t["G"], G, atol=2e-12 * np.abs(G).max())


@pytest.mark.parametrize("nx,ny,nz,p", [(1, 1, 1, 1), (3, 2, 1, 2), (2, 3, 4, 3), (1, 2, 2, 5),
                                        (2, 2, 2, 8), (4, 1, 3, 4)])
def test_integer_maps_bit_exact(nx, ny, nz, p):
    ctx = pafem.Context(-1)
    mesh = pafem.Mesh(ctx, nx, ny, nz, inputs.perturbed_vertices(nx, ny, nz, seed=3))
    sp = pafem.Space(mesh, p)
    N = fem.ndofs(nx, ny, nz, p)
    assert sp.ndofs == N and sp.nelems == nx * ny * nz
    E = fem.element_restriction(nx, ny, nz, p)
    np.testing.assert_array_equal(sp.restriction(), E)
    off, idx = sp.restriction_transpose()
    off_o, idx_o = fem.restriction_transpose(E, N)
    np.testing.assert_array_equal(off, off_o)
    np.testing.assert_array_equal(idx, idx_o)
    np.testing.assert_array_equal(sp.ess_dofs(), fem.essential_dofs(nx, ny, nz, p))


def test_errors_are_reported():
    ctx = pafem.Context(-1)
    v = inputs.perturbed_vertices(2, 2, 2, seed=None)
    mesh = pafem.Mesh(ctx, 2, 2, 2, v)
    with pytest.raises(pafem.PafemError) as ei:
        pafem.Space(mesh, 0)
    assert ei.value.name == "INVALID_ARG" and "p must be" in str(ei.value)
    with pytest.raises(pafem.PafemError):
        pafem.Space(mesh, 9)
    sp = pafem.Space(mesh, 2)
    with pytest.raises(pafem.PafemError) as ei:
        pafem.Operator(sp, pafem.DIFFUSION)
    assert ei.value.name == "UNSUPPORTED"
    with pytest.raises(pafem.PafemError):
        pafem.Mesh(ctx, 0, 1, 1, np.zeros((4, 3)))
    bad = v.copy()
    bad[3, 1] = np.nan
    with pytest.raises(pafem.PafemError):
        pafem.Mesh(ctx, 2, 2, 2, bad)
    with pytest.raises(pafem.PafemError):
        pafem.basis_tables(3, 13)


def test_handles_destroyed_in_any_order():
    from paper_2402_15940_amd.pafem import lib
    ctx = pafem.Context(-1)
    mesh = pafem.Mesh(ctx, 2, 1, 1, inputs.perturbed_vertices(2, 1, 1, seed=None))
    sp = pafem.Space(mesh, 3)
    ctx.close()
    mesh.close()
    # the space still holds its mesh and context
    assert sp.ndofs == 7 * 4 * 4
    np.testing.assert_array_equal(sp.restriction(), fem.element_restriction(2, 1, 1, 3))
    sp.close()


def test_server_needs_gpu_and_footprint_is_consistent():
    ctx = pafem.Context(-1)
    with pytest.raises(pafem.PafemError) as ei:
        pafem.Server(ctx, 1 << 30)
    assert ei.value.name == "UNSUPPORTED"
    # footprint: quadrature data dominates and grows with elements * q^3
    f1 = pafem.request_footprint(8, 8, 8, 4, pafem.SOLVE_PLAIN_FP64)
    f2 = pafem.request_footprint(16, 16, 16, 4, pafem.SOLVE_PLAIN_FP64)
    fir = pafem.request_footprint(8, 8, 8, 4, pafem.SOLVE_IR_FP32)
    qd = 8 ** 3 * 6 ** 3 * 6 * 8
    assert qd < f1 < 2 * qd and 7.5 < f2 / f1 < 8.5
    assert fir - f1 >= 8 ** 3 * 6 ** 3 * 6 * 4       # FP32 copy of the quadrature data


def test_sizes_beyond_32_bit_indexing_are_refused():
    """The kernels index nodes and E-vector words in 32 bits: a space whose
    E-vector or lattice would pass 2^31 - 1 is refused at creation (nothing is
    allocated), the largest that fits is accepted."""
    ctx = pafem.Context(-1)
    n = 162  # p = 8: 162^3 * 9^3 = 3.1e9 E-vector words, 1297^3 = 2.18e9 nodes
    mesh = pafem.Mesh(ctx, n, n, n, inputs.perturbed_vertices(n, n, n, seed=None))
    with pytest.raises(pafem.PafemError) as ei:
        pafem.Space(mesh, 8)
    assert ei.value.name == "INVALID_ARG" and "int32" in str(ei.value)
    # p = 6 on the same mesh: 162^3 * 343 = 1.46e9 words and 973^3 = 9.2e8 nodes fit
    sp = pafem.Space(mesh, 6)
    assert sp.ndofs == 973 ** 3
