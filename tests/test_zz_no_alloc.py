"""pc_ws_predict_noalloc, the prediction entry point for callers that cannot
allocate device memory: through the C ABI it must give pc_ws_predict's
result bit for bit (same kernels, features in the library's per-GPU
scratch), on two calls in a row, the second on a smaller mesh, and it must
allocate nothing (every device allocation of a context goes through the
context's allocator, here a counting one)."""
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


def _params(B, seed):
    p = B.Context.ws_init_params(seed).astype(np.float64)
    p[-(64 * 3 + 3):-3] *= 40.0        # a correction well away from zero
    p[-3:] = 0.01 * np.random.default_rng(seed).normal(size=3)
    return p


def _case(torch, B, c, seed, counting):
    ctx = B.Context.from_cloth(c, allocator=counting)
    ctx.ws_set_params(_params(B, seed))
    x = to_dev(torch, c.x0)
    v = to_dev(torch, random_velocity(c, 0.05, seed=seed))
    dvp = to_dev(torch, 0.01 * np.random.default_rng(seed + 1).normal(size=c.rest.shape))
    b = ctx.cloth_assemble(x, v, "f32")
    return ctx, x, v, b, dvp


def test_predict_noalloc_equals_predict_on_two_calls(torch, B):
    counting = B.TorchAllocator()
    for nx, ny, seed in ((61, 47, 3), (23, 19, 4)):     # 2,867 then 437 vertices (ragged last tile)
        c = sheet(nx, ny, seed=seed, flips=0.1)
        ctx, x, v, b, dvp = _case(torch, B, c, seed, counting)
        try:
            want = ctx.ws_predict(x, v, b, dvp)
            out = torch.full_like(want, float("nan"))
            torch.cuda.synchronize()
            n_alloc, n_free = counting.n_alloc, counting.n_free
            got = ctx.ws_predict_noalloc(x, v, b, dvp, out=out)
            torch.cuda.synchronize()
            assert counting.n_alloc == n_alloc and counting.n_free == n_free
            assert got.data_ptr() == out.data_ptr()
            assert torch.equal(got, want), float((got - want).abs().max())
            # a correction was predicted (the comparison is not of two copies of dv_prev)
            free = torch.from_numpy(c.pinned == 0).cuda()
            assert float((got - dvp)[free].abs().max()) > 1e-6
            assert torch.all(got[~free] == 0)
        finally:
            ctx.close()
    assert counting.n_free == counting.n_alloc


def test_predict_noalloc_rejects_meshes_beyond_its_scratch(torch, B):
    from paper_2008_00409_amd import meshgen as mg
    c = mg.config_grid(1025, seed=7)            # 1,050,625 vertices > 1,048,576 rows
    ctx = B.Context.from_cloth(c)
    try:
        x = to_dev(torch, c.x0)
        with pytest.raises(B.PclothError) as e:
            ctx.ws_predict_noalloc(x, x, x, x)
        assert e.value.status == B.PC_ERR_CAPACITY
    finally:
        ctx.close()


def test_predict_noalloc_needs_parameters(torch, B):
    c = sheet(23, 19, seed=5)
    ctx = B.Context.from_cloth(c)
    try:
        x = to_dev(torch, c.x0)
        v = torch.zeros_like(x)
        b = ctx.cloth_assemble(x, v, "f32")
        with pytest.raises(B.PclothError) as e:
            ctx.ws_predict_noalloc(x, v, b, v)
        assert e.value.status == B.PC_ERR_ARG
    finally:
        ctx.close()
