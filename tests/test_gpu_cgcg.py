"""GPU parity of the single-reduction (Chronopoulos-Gear) CG against the FP64
oracle's form of the same method, through the C ABI:

* FP64 blocks: the iteration count agrees with the oracle's to rounding
  (the GPU keeps the preconditioned residual u as FP32 for the gather; 2%
  or 3 iterations), the solution is within the tolerance of the oracle's,
  and the true residual through the oracle's matrix meets the tolerance;
* every block storage and both preconditioners meet the tolerance through
  the oracle's matrix, with the refinement sweeps for BF16;
* HIP-graph replay of the iterations gives the same bits as plain launches;
* batched instances: each meets the tolerance through its own oracle system;
* an iteration budget ends the solve with exactly that many iterations."""
import numpy as np
import pytest

from gpu_helpers import random_velocity, require_gpu, sheet, to_dev
from paper_2008_00409_amd import meshgen as mg

pytestmark = pytest.mark.gpu
CG = "chronopoulos-gear"


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def B():
    from paper_2008_00409_amd import binding
    return binding


@pytest.mark.parametrize("precond", ["jacobi", "block"])
def test_fp64_matches_oracle(torch, B, oracle_mod, precond):
    c = sheet(43, 37, seed=31, flips=0.1)          # 1591 rows: 25 slices, ragged tail
    P = oracle_mod.Problem.from_cloth(c)
    v = random_velocity(c, seed=4)
    A = P.assemble(c.x0, v)
    xo, oinfo = P.pcg(A, tol=1e-9, precond=precond, method=CG)
    ctx = B.Context.from_cloth(c)
    try:
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), "f64")
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-9, precond=precond, method=CG)
        dv = dv.cpu().numpy()
    finally:
        ctx.close()
    assert abs(info["iters"] - oinfo["iters"]) <= max(3, 0.02 * oinfo["iters"]), (info["iters"], oinfo["iters"])
    assert P.residual(A, dv) <= 1e-9 * (1 + 1e-6)
    assert np.linalg.norm(dv - xo) <= 1e-6 * np.linalg.norm(xo)


@pytest.mark.parametrize("dtype,precond", [("f32", "jacobi"), ("f32", "block"), ("bf16", "block"),
                                           ("bf16", "jacobi")])
def test_low_precision_blocks_meet_tolerance(torch, B, oracle_mod, dtype, precond):
    c = sheet(71, 53, seed=21, flips=0.1)
    P = oracle_mod.Problem.from_cloth(c)
    v = random_velocity(c, 0.05, seed=2)
    A = P.assemble(c.x0, v)
    ctx = B.Context.from_cloth(c)
    try:
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), dtype)
        dv_t, it_t = ctx.cloth_pcg_solve(b, tol=1e-6, precond=precond)
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond=precond, method=CG)
        dv = dv.cpu().numpy()
    finally:
        ctx.close()
    assert info["rel_res_true"] <= 1e-6
    assert P.residual(A, dv) <= 1e-6 * (1 + 1e-6)
    # same method in exact arithmetic: iteration counts close to the textbook form's
    assert info["iters"] <= 1.25 * it_t["iters"] + 10, (info["iters"], it_t["iters"])
    print(f"{dtype}/{precond}: textbook {it_t['iters']} iterations ({it_t['sweeps']} sweeps), "
          f"single-reduction {info['iters']} ({info['sweeps']} sweeps)")


def test_graph_replay_bitwise(torch, B):
    c = sheet(64, 50, seed=33, flips=0.1)
    v = random_velocity(c, 0.05, seed=5)
    out = []
    for chunk in (0, 32):
        ctx = B.Context.from_cloth(c)
        try:
            ctx.set_option(B.PC_OPT_GRAPH_CHUNK, chunk)
            b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), "bf16")
            dv, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond="block", method=CG)
            out.append((dv.cpu().numpy(), info["iters"]))
        finally:
            ctx.close()
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0].view(np.uint64), out[1][0].view(np.uint64))


def test_batched_instances(torch, B, oracle_mod):
    c = mg.config_batch(seed=92, sizes=[11, 37, 8, 25])
    begins = [r[0] for r in c.sheet_ranges] + [c.nv]
    v = random_velocity(c, 0.05, seed=6)
    P = oracle_mod.Problem.from_cloth(c)
    A = P.assemble(c.x0, v)
    ctx = B.Context.from_cloth(c)
    try:
        ctx.set_instances(begins)
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), "f32")
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond="block", method=CG)
        per = ctx.instance_info()
        dv = dv.cpu().numpy()
    finally:
        ctx.close()
    r = A.b - P.spmv(A, dv)
    for k in range(len(begins) - 1):
        sl = slice(begins[k], begins[k + 1])
        assert np.linalg.norm(r[sl]) <= 1e-6 * (1 + 1e-6) * np.linalg.norm(A.b[sl])
        assert per[k]["rel_res_true"] <= 1e-6
    assert len({d["iters"] for d in per}) > 1      # the instances stop on their own


def test_iteration_budget(torch, B):
    c = sheet(40, 30, seed=34, flips=0.1)
    v = random_velocity(c, 0.05, seed=7)
    ctx = B.Context.from_cloth(c)
    try:
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), "f64")
        _dv, info = ctx.cloth_pcg_solve(b, tol=1e-12, maxit=7, precond="jacobi", method=CG, raise_on_error=False)
    finally:
        ctx.close()
    assert info["iters"] == 7
    assert info["status"] == B.PC_ERR_NOT_CONVERGED
