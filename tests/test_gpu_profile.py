"""Kernel timing with HIP events (pc_profile) observes a CG solve without
changing it: with sampling on, the solve returns the same iterate bit for bit
and the same iteration count as with sampling off, with plain launches and
with graph replay, and the three CG kernels are sampled."""
import numpy as np
import pytest

from gpu_helpers import random_velocity, require_gpu, sheet, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def B():
    from paper_2008_00409_amd import binding
    return binding


@pytest.mark.parametrize("chunk", [0, 16])
def test_profiling_changes_no_result(torch, B, chunk):
    c = sheet(48, 40, seed=11)
    v = random_velocity(c, 0.05, seed=12)
    ctx = B.Context.from_cloth(c)
    try:
        ctx.set_option(B.PC_OPT_GRAPH_CHUNK, chunk)
        x, vd = to_dev(torch, c.x0), to_dev(torch, v)
        b = ctx.cloth_assemble(x, vd, "bf16")
        ref, rinfo = ctx.cloth_pcg_solve(b, tol=1e-6, precond="block")
        ref = ref.cpu().numpy().copy()
        ctx.profile(2)
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond="block")
        prof = ctx.profile_read()
        ctx.profile(0)
        assert info["iters"] == rinfo["iters"]
        assert np.array_equal(dv.cpu().numpy().view(np.uint64), ref.view(np.uint64))
        for kind in ("spmv", "cg_update", "cg_dir"):
            p = prof[kind]
            assert p["samples"] >= 1
            assert 0.0 < p["min_ms"] <= p["median_ms"] <= p["max_ms"]
    finally:
        ctx.close()
