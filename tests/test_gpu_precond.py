"""GPU parity of the block-Jacobi preconditioner (P = the 3x3 diagonal blocks
of A, a solver variant of the PCG of paper Sec. 2.5) against the FP64 oracle,
through the C ABI:

* the inverse blocks stored at assembly against numpy inverses of the
  oracle's diagonal blocks (FP32 storage: 1e-5 of the block's largest entry);
* the solve with FP64 blocks against the oracle's block-Jacobi PCG: same
  iteration count up to rounding (2%), solution within the tolerance;
* every block storage type meets the tolerance through the oracle's matrix,
  with fewer iterations than Jacobi on the same system;
* instances batched in one launch give the same result as solo solves."""
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


def diag_blocks(A):
    nv = A.rowptr.size - 1
    rows = np.repeat(np.arange(nv), np.diff(A.rowptr))
    return A.vals[np.nonzero(A.colidx == rows)[0]]


def test_inverse_blocks_match_oracle(torch, B, oracle_mod):
    c = sheet(37, 29, seed=5, flips=0.1)     # 1073 rows: several slices, ragged tail
    P = oracle_mod.Problem.from_cloth(c)
    v = random_velocity(c)
    A = P.assemble(c.x0, v)
    ctx = B.Context.from_cloth(c)
    try:
        ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), "f32")
        dinv, binv = ctx.cloth_export_precond()
        dinv, binv = dinv.cpu().numpy().astype(np.float64), binv.cpu().numpy().astype(np.float64)
        want = np.linalg.inv(diag_blocks(A))
        scale = np.abs(want).reshape(-1, 9).max(axis=1)
        err = np.abs(binv - want).reshape(-1, 9).max(axis=1) / scale
        assert err.max() <= 1e-5, err.max()
        np.testing.assert_allclose(dinv, 1.0 / A.diag, rtol=1e-6)
        # pinned rows: A_ii = m_i I
        pin = c.pinned == 1
        np.testing.assert_allclose(binv[pin], np.eye(3)[None] / c.mass[pin, None, None], rtol=1e-6)
    finally:
        ctx.close()


def test_block_jacobi_fp64_matches_oracle_iterations(torch, B, oracle_mod):
    c = sheet(31, 23, seed=9, flips=0.1)
    P = oracle_mod.Problem.from_cloth(c)
    v = random_velocity(c)
    A = P.assemble(c.x0, v)
    xo, oinfo = P.pcg(A, tol=1e-8, precond="block")
    ctx = B.Context.from_cloth(c)
    try:
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), "f64")
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-8, precond="block")
        dv = dv.cpu().numpy()
        assert abs(info["iters"] - oinfo["iters"]) <= max(3, 0.02 * oinfo["iters"]), (info["iters"], oinfo["iters"])
        assert P.residual(A, dv) <= 1e-8 * (1 + 1e-6)
        assert np.linalg.norm(dv - xo) <= 1e-5 * np.linalg.norm(xo)
    finally:
        ctx.close()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_block_jacobi_residual_and_fewer_iterations(torch, B, oracle_mod, dtype):
    c = sheet(45, 41, seed=13, flips=0.1)
    P = oracle_mod.Problem.from_cloth(c)
    v = random_velocity(c)
    A = P.assemble(c.x0, v)
    ctx = B.Context.from_cloth(c)
    try:
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), dtype)
        dvj, ij = ctx.cloth_pcg_solve(b, tol=1e-6, precond="jacobi")
        dvb, ib = ctx.cloth_pcg_solve(b, tol=1e-6, precond="block")
        assert P.residual(A, dvb.cpu().numpy()) <= 1e-6 * (1 + 1e-6)
        assert ib["iters"] < ij["iters"], (ib["iters"], ij["iters"])
    finally:
        ctx.close()


def test_block_jacobi_batched_equals_solo(torch, B):
    c = mg.config_batch(seed=77, sizes=[11, 27, 16, 8, 21])   # grid sides: uneven, ragged slices
    begins = [r[0] for r in c.sheet_ranges] + [c.nv]
    v = random_velocity(c, 0.05, seed=4)
    x_d, v_d = to_dev(torch, c.x0), to_dev(torch, v)
    ctx = B.Context.from_cloth(c)
    try:
        ctx.set_instances(begins)
        b = ctx.cloth_assemble(x_d, v_d, "f32")
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond="block")
        dv = dv.cpu().numpy()
        per = ctx.instance_info()
    finally:
        ctx.close()
    for k, (v0, v1) in enumerate(c.sheet_ranges):
        t0, t1 = c.tri_ranges[k]
        sub = mg.Cloth("solo", c.rest[v0:v1], c.tris[t0:t1] - v0, c.mass[v0:v1], c.pinned[v0:v1], c.x0[v0:v1],
                       c.v0[v0:v1], c.h, c.tol, 1, [(0, v1 - v0)], [(0, t1 - t0)])
        solo = B.Context.from_cloth(sub)
        try:
            bs = solo.cloth_assemble(to_dev(torch, c.x0[v0:v1]), to_dev(torch, v[v0:v1]), "f32")
            ds, si = solo.cloth_pcg_solve(bs, tol=1e-6, precond="block")
            assert si["iters"] == per[k]["iters"]
            np.testing.assert_array_equal(ds.cpu().numpy(), dv[v0:v1])
        finally:
            solo.close()
