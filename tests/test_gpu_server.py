"""GPU tests of the continuous-batching solve server (through the C ABI).

* every served solve (plain FP64, FP64 defect correction around FP32 inner
  solves, and mixed FP32 CG with FP64 residual replacement) reaches its
  residual target and agrees with the single-solve path and with the CPU
  oracle;
* a request's solution is bitwise the same alone and in a mix of other
  requests of different sizes and orders (deterministic E^T, fixed-order
  per-request reductions);
* admission respects the HBM budget (back-pressure, first-in first-out) and a
  request larger than the budget, or one with an inverted element, fails
  without disturbing the others.
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


def _req(n, p, seed, mode, coef=0):
    return dict(nx=n, ny=n, nz=n, p=p, verts=inputs.perturbed_vertices(n, n, n, seed=seed),
                mode=mode, coef_kind=coef, coef_value=0.5 if coef else 1.0)


def _submit(srv, r, **kw):
    from paper_2402_15940_amd import pafem
    if r["mode"] == pafem.SOLVE_MIXED_FP32:
        kw = dict(kw, inner_rtol=0.1)  # the residual-replacement factor
    return srv.submit(r["nx"], r["ny"], r["nz"], r["p"], r["verts"], mode=r["mode"],
                      coef_kind=r["coef_kind"], coef_value=r["coef_value"], **kw)


def test_served_solves_match_single_solves_and_oracle(pf, ctx):
    reqs = [_req(4, 2, 1, pf.SOLVE_PLAIN_FP64), _req(3, 4, 2, pf.SOLVE_IR_FP32),
            _req(5, 3, 3, pf.SOLVE_IR_FP32, coef=pf.COEF_SINX), _req(2, 6, 4, pf.SOLVE_PLAIN_FP64),
            _req(4, 5, 5, pf.SOLVE_MIXED_FP32, coef=pf.COEF_SINX), _req(3, 7, 6, pf.SOLVE_MIXED_FP32)]
    srv = pf.Server(ctx, 8 << 30, max_slots=8, iters_per_round=5)
    tickets = [_submit(srv, r, rtol=1e-10, inner_rtol=1e-3) for r in reqs]
    srv.drain()
    for r, t in zip(reqs, tickets):
        res = srv.poll(t)
        assert res["status"] == pf.REQ_DONE, res
        assert res["rel_res"] <= 1e-10 and res["t_done"] >= res["t_admit"] >= res["t_arrive"]
        if r["mode"] == pf.SOLVE_MIXED_FP32:
            assert res["outer_iterations"] >= 2  # residual replacements
        x = srv.solution(t)
        n = r["nx"]
        op = pf.Operator(pf.Space(pf.Mesh(ctx, n, n, n, r["verts"]), r["p"]), pf.DIFFUSION)
        if r["coef_kind"]:
            op.set_coefficient_sinx(0.5)
        op.assemble(pf.FP64 | pf.FP32)
        xs, st = op.solve(op.rhs(), rtol=1e-12)
        xs = xs.cpu().numpy()
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-8
        coef_q = None
        if r["coef_kind"]:
            coef_q = inputs.coef_sin_x(fem.qpoint_coords(r["verts"], n, n, n, r["p"] + 2)[:, 0, :])
        ref = fem.solve_poisson(r["verts"], n, n, n, r["p"], f=inputs.f_manufactured,
                                coef_q=coef_q, rtol=1e-12)
        assert np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"]) < 1e-8
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["max_active"] >= 2
    srv.close()


@pytest.mark.parametrize("mode", ["plain", "ir", "mixed"])
def test_result_is_bitwise_the_same_alone_and_in_a_mix(pf, ctx, mode):
    m = {"plain": pf.SOLVE_PLAIN_FP64, "ir": pf.SOLVE_IR_FP32, "mixed": pf.SOLVE_MIXED_FP32}[mode]
    target = _req(4, 3, 11, m, coef=pf.COEF_SINX)
    others = [_req(3, 5, 12, pf.SOLVE_IR_FP32), _req(6, 2, 13, pf.SOLVE_PLAIN_FP64),
              _req(2, 8, 14, pf.SOLVE_MIXED_FP32), _req(5, 4, 15, m)]
    srv = pf.Server(ctx, 8 << 30, max_slots=8, iters_per_round=4)
    t = _submit(srv, target, rtol=1e-10, inner_rtol=1e-3)
    srv.drain()
    x_alone = srv.solution(t)
    srv.close()
    srv = pf.Server(ctx, 8 << 30, max_slots=8, iters_per_round=4)
    ts = [_submit(srv, r, rtol=1e-10, inner_rtol=1e-3) for r in others[:2]]
    t = _submit(srv, target, rtol=1e-10, inner_rtol=1e-3)
    ts += [_submit(srv, r, rtol=1e-10, inner_rtol=1e-3) for r in others[2:]]
    srv.drain()
    x_mix = srv.solution(t)
    assert srv.stats()["max_active"] >= 3
    assert all(srv.poll(k)["status"] == pf.REQ_DONE for k in ts)
    srv.close()
    assert np.array_equal(x_alone, x_mix)


def test_admission_respects_the_budget(pf, ctx):
    reqs = [_req(4, 3, 20 + i, pf.SOLVE_IR_FP32) for i in range(4)]
    fp = pf.request_footprint(4, 4, 4, 3, pf.SOLVE_IR_FP32)
    srv = pf.Server(ctx, int(fp * 1.5), max_slots=8, iters_per_round=3)
    ts = [_submit(srv, r, rtol=1e-10, inner_rtol=1e-3) for r in reqs]
    srv.drain()
    res = [srv.poll(t) for t in ts]
    assert all(r["status"] == pf.REQ_DONE for r in res)
    st = srv.stats()
    assert st["max_active"] == 1 and st["peak_bytes"] <= fp * 1.5
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)                  # first in, first out
    for a, b in zip(res[:-1], res[1:]):              # one at a time
        assert b["t_admit"] >= a["t_done"] - 1e-6
    srv.close()


def test_failures_are_isolated(pf, ctx):
    srv = pf.Server(ctx, 1 << 30, max_slots=4, iters_per_round=3)
    good = _req(3, 2, 30, pf.SOLVE_PLAIN_FP64)
    bad = _req(2, 2, None, pf.SOLVE_PLAIN_FP64)
    bad["verts"][13] = [0.9, 0.9, 0.9]               # inverted elements
    huge = _req(64, 8, 31, pf.SOLVE_IR_FP32)         # ~19 GB, over the 1 GiB budget
    t1 = _submit(srv, good, rtol=1e-10)
    t2 = _submit(srv, bad, rtol=1e-10)
    t3 = _submit(srv, huge, rtol=1e-10)
    t4 = _submit(srv, good, rtol=1e-10)
    with pytest.raises(pf.PafemError):
        srv.submit(2, 2, 2, 9, inputs.lattice_vertices(2, 2, 2))
    srv.drain()
    r1, r2, r3, r4 = (srv.poll(t) for t in (t1, t2, t3, t4))
    assert r1["status"] == pf.REQ_DONE and r4["status"] == pf.REQ_DONE
    assert r2["status"] == pf.REQ_FAILED and r2["error"] == -1   # INVALID_ARG
    assert r3["status"] == pf.REQ_FAILED and r3["error"] == -2   # OUT_OF_MEMORY
    assert np.array_equal(srv.solution(t1), srv.solution(t4))
    with pytest.raises(pf.PafemError):
        srv.solution(t2)
    srv.close()
