"""FP32 inner vectors of the refinement sweeps (BF16 blocks): each sweep
solves for a correction e with e, r and q = A p stored in FP32 and adds it
to the FP64 x at its end.  Against the oracle's matrix, with the option on
and off: both meet the tolerance (the FP64 true residual decides), the
sweep and iteration counts stay within 10% of each other, and batched
instances, a warm start, a sweep count above one and graph replay all go
through the correction path; the option does not touch FP32/FP64 blocks."""
import numpy as np
import pytest

from gpu_helpers import random_velocity, require_gpu, sheet, to_dev
from paper_2008_00409_amd import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def B():
    from paper_2008_00409_amd import binding
    return binding


def solve(torch, B, c, v, dtype, inner, precond="block", chunk=0, dv0=None, instances=None, tol=1e-6):
    ctx = B.Context.from_cloth(c)
    try:
        if instances is not None:
            ctx.set_instances(instances)
        ctx.set_option(B.PC_OPT_INNER_FP32, inner)
        ctx.set_option(B.PC_OPT_GRAPH_CHUNK, chunk)
        assert ctx.get_option(B.PC_OPT_INNER_FP32) == inner
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), dtype)
        start = None if dv0 is None else to_dev(torch, dv0)
        dv, info = ctx.cloth_pcg_solve(b, dv=start, tol=tol, precond=precond, warm=dv0 is not None)
        per = ctx.instance_info() if instances is not None else None
        return dv.cpu().numpy(), info, per
    finally:
        ctx.close()


@pytest.mark.parametrize("precond", ["block", "jacobi"])
def test_bf16_inner32_meets_tolerance(torch, B, oracle_mod, precond):
    c = sheet(71, 53, seed=21, flips=0.1)
    v = random_velocity(c, 0.05, seed=2)
    P = oracle_mod.Problem.from_cloth(c)
    A = P.assemble(c.x0, v)
    d1, i1, _ = solve(torch, B, c, v, "bf16", 1, precond)
    d0, i0, _ = solve(torch, B, c, v, "bf16", 0, precond)
    assert i1["sweeps"] > 1
    for d, i in ((d1, i1), (d0, i0)):
        assert i["rel_res_true"] <= 1e-6
        assert P.residual(A, d) <= 1e-6 * (1 + 1e-6)
    assert abs(i1["iters"] - i0["iters"]) <= 0.1 * i0["iters"] + 5, (i1["iters"], i0["iters"])
    assert np.linalg.norm(d1 - d0) <= 1e-4 * np.linalg.norm(d0)


def test_inner32_warm_start_graph_and_instances(torch, B, oracle_mod):
    c = mg.config_batch(seed=93, sizes=[12, 33, 9, 21])
    begins = [r[0] for r in c.sheet_ranges] + [c.nv]
    v = random_velocity(c, 0.05, seed=8)
    P = oracle_mod.Problem.from_cloth(c)
    A = P.assemble(c.x0, v)
    dv_ref, _ = P.pcg(A, tol=1e-10)
    start = dv_ref + 1e-3 * np.random.default_rng(4).normal(size=dv_ref.shape) * np.abs(dv_ref).max()
    start[c.pinned == 1] = 0
    outs = []
    for chunk in (0, 32):
        d, info, per = solve(torch, B, c, v, "bf16", 1, chunk=chunk, dv0=start, instances=begins)
        r = A.b - P.spmv(A, d)
        for k in range(len(begins) - 1):
            sl = slice(begins[k], begins[k + 1])
            assert np.linalg.norm(r[sl]) <= 1e-6 * (1 + 1e-6) * np.linalg.norm(A.b[sl])
        outs.append((d, info["iters"]))
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0].view(np.uint64), outs[1][0].view(np.uint64))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_option_leaves_higher_precision_blocks_alone(torch, B, dtype):
    c = sheet(40, 30, seed=35, flips=0.1)
    v = random_velocity(c, 0.05, seed=9)
    d1, i1, _ = solve(torch, B, c, v, dtype, 1)
    d0, i0, _ = solve(torch, B, c, v, dtype, 0)
    assert i1["iters"] == i0["iters"]
    assert np.array_equal(d1.view(np.uint64), d0.view(np.uint64))


def test_bf16_refinement_falls_back_when_not_contracting(torch, B):
    """The 64-sheet batch with BF16 blocks and the previous-step start: on the
    third step the BF16 sweeps stop contracting for some small sheets (their
    FP64 residual grows); the solver detects a sweep that does not halve its
    starting residual and finishes on the FP64 blocks, so every instance
    still meets the tolerance (before this check, those instances ran 40
    sweeps and ended far above it)."""
    c = mg.config_batch()
    begins = [r[0] for r in c.sheet_ranges] + [c.nv]
    ctx = B.Context.from_cloth(c)
    try:
        ctx.set_instances(begins)
        x = to_dev(torch, c.x0)
        v = to_dev(torch, c.v0)
        dvp = None
        fallbacks = 0
        for step in range(3):
            b = ctx.cloth_assemble(x, v, "bf16")
            dv, info = ctx.cloth_pcg_solve(b, dv=None if dvp is None else dvp.clone(), warm=dvp is not None,
                                           tol=1e-6, precond="block")
            per = ctx.instance_info()
            assert all(d["rel_res_true"] <= 1e-6 for d in per), step
            fallbacks += sum(d["fallback"] for d in per)
            dvp = dv.clone()
            v += dv
            x += c.h * v
    finally:
        ctx.close()
    assert fallbacks > 0


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_sweep_budget_ends_the_first_sweep_at_half_of_maxit(torch, B, dtype):
    """A refinement sweep on the low-precision copy runs at most half of
    maxit iterations if it is the first: with maxit = 40 (far too few for
    the tolerance) the first sweep ends after 20 iterations, the FP64
    residual is checked, and a second sweep (budget 20) uses the rest; the
    solve reports 40 iterations in at least 2 sweeps and PC_ERR_NOT_CONVERGED.
    Without the budget a single sweep would take all 40."""
    c = sheet(40, 37, seed=3, flips=0.1)
    v = random_velocity(c, 0.05, seed=2)
    ctx = B.Context.from_cloth(c)
    try:
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), dtype)
        _, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond="block", maxit=40, raise_on_error=False)
        assert info["status"] == B.PC_ERR_NOT_CONVERGED, info
        assert info["iters"] == 40 and info["sweeps"] >= 2, info
        # FP32 blocks run each sweep to the tolerance: no budget, one sweep
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), "f32")
        _, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond="block", maxit=40, raise_on_error=False)
        assert info["iters"] == 40 and info["sweeps"] == 1, info
    finally:
        ctx.close()


@pytest.mark.parametrize("precond", ["block", "jacobi"])
def test_f16_sweeps_keep_the_direction(torch, B, oracle_mod, precond):
    """FP16 refinement sweeps keep the search direction by default (the FP64
    residual replaces the recursive one and CG goes on, inner reduction 0.5).
    Against sweeps that restart CG (PC_OPT_KEEP_DIRECTION = 0, inner
    reduction 1e-2): both meet the tolerance through the oracle's matrix,
    and keeping the direction needs fewer iterations."""
    c = sheet(71, 53, seed=21, flips=0.1)
    v = random_velocity(c, 0.05, seed=2)
    P = oracle_mod.Problem.from_cloth(c)
    A = P.assemble(c.x0, v)
    out = {}
    for keep in (1, 0):
        ctx = B.Context.from_cloth(c)
        try:
            ctx.set_option(B.PC_OPT_KEEP_DIRECTION, keep)
            assert ctx.get_option(B.PC_OPT_KEEP_DIRECTION) == keep
            b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), "f16")
            dv, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond=precond)
            assert P.residual(A, dv.cpu().numpy()) <= 1e-6 * (1 + 1e-6)
            assert info["fallback"] == 0, info
            out[keep] = info
        finally:
            ctx.close()
    print(f"{precond}: keep {out[1]['iters']} iterations in {out[1]['sweeps']} sweeps, "
          f"restart {out[0]['iters']} in {out[0]['sweeps']}")
    assert out[1]["sweeps"] > out[0]["sweeps"]
    assert out[1]["iters"] < out[0]["iters"]
