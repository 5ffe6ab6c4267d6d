"""GPU tests of many independent cloths in one context: each instance keeps
its own CG scalars, convergence and refinement, so the batched solve of an
instance equals (bit for bit) the solve of that instance alone, and every
instance meets the tolerance through the oracle's FP64 matrix."""
import numpy as np
import pytest

from gpu_helpers import require_gpu, to_dev
from paper_2008_00409_amd import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def B():
    from paper_2008_00409_amd import binding
    return binding


SIDES = [9, 23, 14, 31, 12]   # uneven instances, ragged slices at every boundary


def batch():
    return mg.config_batch(sizes=SIDES, seed=5100)


def sub_cloth(c, k):
    v0, v1 = c.sheet_ranges[k]
    t0, t1 = c.tri_ranges[k]
    return mg.Cloth(f"inst{k}", c.rest[v0:v1], c.tris[t0:t1] - v0, c.mass[v0:v1], c.pinned[v0:v1],
                    c.x0[v0:v1], c.v0[v0:v1], c.h, c.tol, 1, [(0, v1 - v0)], [(0, t1 - t0)])


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_batched_equals_solo_solves(torch, B, oracle_mod, dtype):
    c = batch()
    begins = [r[0] for r in c.sheet_ranges] + [c.nv]
    ctx = B.Context.from_cloth(c)
    try:
        ctx.set_instances(begins)
        x, v = to_dev(torch, c.x0), to_dev(torch, c.v0)
        b = ctx.cloth_assemble(x, v, dtype)
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-6)
        infos = ctx.instance_info()
        dv = dv.cpu().numpy()
    finally:
        ctx.close()
    assert len(infos) == len(SIDES)
    assert info["iters"] == max(i["iters"] for i in infos)
    for k in range(len(SIDES)):
        ck = sub_cloth(c, k)
        solo = B.Context.from_cloth(ck)
        try:
            xs, vs = to_dev(torch, ck.x0), to_dev(torch, ck.v0)
            bs = solo.cloth_assemble(xs, vs, dtype)
            dvs, sinfo = solo.cloth_pcg_solve(bs, tol=1e-6)
            dvs = dvs.cpu().numpy()
        finally:
            solo.close()
        v0, v1 = c.sheet_ranges[k]
        assert infos[k]["iters"] == sinfo["iters"]
        assert np.array_equal(dv[v0:v1].view(np.uint64), dvs.view(np.uint64))
        P = oracle_mod.Problem.from_cloth(ck)
        A = P.assemble(ck.x0, ck.v0)
        assert P.residual(A, dv[v0:v1]) <= 1e-6 * (1 + 1e-6)


def test_batched_graph_and_schedule_options(torch, B, oracle_mod):
    c = batch()
    begins = [r[0] for r in c.sheet_ranges] + [c.nv]
    ctx = B.Context.from_cloth(c)
    try:
        ctx.set_instances(begins)
        x, v = to_dev(torch, c.x0), to_dev(torch, c.v0)
        b = ctx.cloth_assemble(x, v, "f32")
        ref, rinfo = ctx.cloth_pcg_solve(b, tol=1e-6)
        ref = ref.cpu().numpy().copy()
        # a captured graph of 16 iterations replays the same kernels: same iterate
        ctx.set_option(B.PC_OPT_GRAPH_CHUNK, 16)
        for _ in range(2):
            dv, info = ctx.cloth_pcg_solve(b, tol=1e-6)
            assert np.array_equal(dv.cpu().numpy().view(np.uint64), ref.view(np.uint64))
        ctx.set_option(B.PC_OPT_GRAPH_CHUNK, 0)
        # other work-item sizes regroup the partial sums: same tolerance reached
        for spb, rpb in [(1, 64), (8, 1024), (2, 512)]:
            ctx.set_option(B.PC_OPT_SPMV_SLICES_PER_BLOCK, spb)
            ctx.set_option(B.PC_OPT_VECTOR_ROWS_PER_BLOCK, rpb)
            dv, info = ctx.cloth_pcg_solve(b, tol=1e-6)
            for k, inf in enumerate(ctx.instance_info()):
                assert inf["rel_res_true"] <= 1e-6
            assert abs(info["iters"] - rinfo["iters"]) <= 0.05 * rinfo["iters"] + 2
    finally:
        ctx.close()


def test_set_instances_rejects_bad_ranges(torch, B):
    c = batch()
    ctx = B.Context.from_cloth(c)
    try:
        with pytest.raises(B.PclothError, match="PC_ERR_ARG"):
            ctx.set_instances([0, 10, 5, c.nv])
        v0, v1 = c.sheet_ranges[1]
        with pytest.raises(B.PclothError, match="PC_ERR_MESH"):
            ctx.set_instances([0, v0 + 3, c.nv])   # cuts instance 1: a triangle joins two ranges
    finally:
        ctx.close()


def test_batched_steps(torch, B):
    c = batch()
    begins = [r[0] for r in c.sheet_ranges] + [c.nv]
    ctx = B.Context.from_cloth(c)
    try:
        ctx.set_instances(begins)
        x, v = to_dev(torch, c.x0), to_dev(torch, c.v0)
        infos = ctx.cloth_step(x, v, nsteps=3, dtype="f32", tol=1e-6)
        assert all(i["rel_res_true"] <= 1e-6 for i in infos)
        assert np.all(np.isfinite(x.cpu().numpy()))
        np.testing.assert_array_equal(x.cpu().numpy()[c.pinned == 1], c.x0[c.pinned == 1])
    finally:
        ctx.close()


def test_autotune_picks_a_valid_schedule(torch, B, tmp_path):
    """The autotuner times every candidate schedule on the assembled system,
    keeps the fastest, caches it by key, and the solve still meets the
    tolerance on every instance."""
    c = batch()
    begins = [r[0] for r in c.sheet_ranges] + [c.nv]
    ctx = B.Context.from_cloth(c)
    try:
        ctx.set_instances(begins)
        x, v = to_dev(torch, c.x0), to_dev(torch, c.v0)
        b = ctx.cloth_assemble(x, v, "f32")
        cache = str(tmp_path / "tune.json")
        res = ctx.autotune(b, iters=16, cache=cache, key="batch-test")
        spb, rpb, chunk = res["choice"]
        assert spb in (2, 4, 8, 16) and rpb % 64 == 0 and 64 <= rpb <= 4096 and chunk in (0, 32)
        assert res["ms_per_iter"] > 0 and not res["cached"]
        assert ctx.get_option(B.PC_OPT_SPMV_SLICES_PER_BLOCK) == spb
        again = ctx.autotune(b, iters=16, cache=cache, key="batch-test")
        assert again["cached"] and again["choice"] == [spb, rpb, chunk]
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-6)
        assert all(i["rel_res_true"] <= 1e-6 for i in ctx.instance_info())
    finally:
        ctx.close()
