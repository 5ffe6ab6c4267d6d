"""Boundary conventions of the C ABI on the GPU: the device allocator hook
(pc_set_allocator) and the rule that cloth_step commits no failed step
(Sec. 2.5: a step of Eq. 3 is the solve followed by the update of v and x;
a step whose solve did not converge is not taken)."""
import numpy as np
import pytest

from gpu_helpers import require_gpu, sheet, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def B():
    from paper_2008_00409_amd import binding
    return binding


def _solve(torch, B, c, allocator):
    ctx = B.Context.from_cloth(c, allocator=allocator)
    try:
        x = to_dev(torch, c.x0)
        v = torch.zeros_like(x)
        b = ctx.cloth_assemble(x, v, "bf16")
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-7, precond="block")
        # a second step through cloth_step, which grows no buffer but runs the update
        infos = ctx.cloth_step(x, v, nsteps=2, dtype="f32", tol=1e-7, warm="prev", precond="block")
        torch.cuda.synchronize()
        return b.cpu().numpy(), dv.cpu().numpy(), x.cpu().numpy(), v.cpu().numpy(), info, infos
    finally:
        ctx.close()


def test_allocator_hook_routes_every_buffer_and_changes_no_result(torch, B):
    c = sheet(37, 29, seed=5, flips=0.1)
    counting = B.TorchAllocator()
    got = _solve(torch, B, c, counting)
    # every block the library took from the caller's allocator went back to it
    assert counting.n_alloc > 10, counting.n_alloc
    assert counting.n_free == counting.n_alloc and not counting.live, (counting.n_alloc, counting.n_free)
    assert counting.bytes > 9 * 8 * c.rest.shape[0]
    ref = _solve(torch, B, c, None)
    for a, r in zip(got[:4], ref[:4]):
        np.testing.assert_array_equal(a, r)
    assert got[4]["iters"] == ref[4]["iters"]
    assert [i["iters"] for i in got[5]] == [i["iters"] for i in ref[5]]


def test_allocator_hook_covers_grown_buffers(torch, B):
    """Buffers that grow after pc_create (a contact set, the warm-start
    network's state) come from the allocator installed on the context."""
    from paper_2008_00409_amd import meshgen as mg
    c, cs = mg.config_contact(21, 19)
    counting = B.TorchAllocator()
    ctx = B.Context.from_cloth(c, allocator=None)
    try:
        B.lib().pc_set_allocator(ctx.h, counting.alloc_fn, counting.free_fn, None)
        assert counting.n_alloc == 0
        ctx.cloth_set_contacts(cs.verts, cs.weights, cs.normals, cs.eta, cs.kc)
        ctx.ws_set_params(B.Context.ws_init_params(1))
        x = to_dev(torch, c.x0)
        v = torch.zeros_like(x)
        b = ctx.cloth_assemble(x, v, "bf16")
        ctx.ws_train_step(x, v, b, torch.zeros_like(x))
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond="block")
        torch.cuda.synchronize()
        assert info["rel_res_true"] <= 1e-6
        assert counting.n_alloc > 0 and counting.live
    finally:
        ctx.close()
    assert counting.n_free == counting.n_alloc and not counting.live, (counting.n_alloc, counting.n_free)


def test_set_allocator_rejects_half_a_pair(torch, B):
    a = B.TorchAllocator()
    st = B.lib().pc_set_allocator(None, a.alloc_fn, B._FREE_FN(), None)
    assert st == B.PC_ERR_ARG


def test_misaligned_allocator_is_refused(torch, B):
    """Blocks must be 256-byte aligned (the kernels' 16-byte vector loads rely
    on it): a block 16 bytes off is handed back and creation fails cleanly."""

    class Misaligned(B.TorchAllocator):
        def _alloc(self, nbytes, user):
            ptr = super()._alloc(int(nbytes) + 256, user)
            return None if ptr is None else ptr + 16

        def _free(self, ptr, user):
            super()._free(ptr - 16, user)

    bad = Misaligned()
    c = sheet(9, 8, seed=2)
    with pytest.raises(B.PclothError, match="PC_ERR_ARG"):
        B.Context.from_cloth(c, allocator=bad)
    assert bad.n_alloc >= 1 and bad.n_free == bad.n_alloc and not bad.live
    # a context created afterwards with torch's allocator works normally
    ctx = B.Context.from_cloth(c)
    try:
        x = to_dev(torch, c.x0)
        b = ctx.cloth_assemble(x, torch.zeros_like(x), "f32")
        _, info = ctx.cloth_pcg_solve(b, tol=1e-6)
        assert info["rel_res_true"] <= 1e-6
    finally:
        ctx.close()


def test_failed_step_is_not_committed(torch, B):
    c = sheet(29, 23, seed=4, flips=0.1)
    ctx = B.Context.from_cloth(c)
    try:
        x = to_dev(torch, c.x0)
        v = torch.zeros_like(x)
        ctx.cloth_step(x, v, nsteps=1, dtype="f64", tol=1e-8)
        x1, v1 = x.clone(), v.clone()
        with pytest.raises(B.PclothError) as e:
            ctx.cloth_step(x, v, nsteps=3, dtype="f64", tol=1e-8, maxit=5)
        assert e.value.status == B.PC_ERR_NOT_CONVERGED
        torch.cuda.synchronize()
        assert torch.equal(x, x1) and torch.equal(v, v1)
        # BF16 blocks with refinement: the budget ends inside a sweep
        with pytest.raises(B.PclothError) as e:
            ctx.cloth_step(x, v, nsteps=1, dtype="bf16", tol=1e-8, maxit=40, precond="block")
        assert e.value.status == B.PC_ERR_NOT_CONVERGED
        assert torch.equal(x, x1) and torch.equal(v, v1)
        # the context still steps normally afterwards
        infos = ctx.cloth_step(x, v, nsteps=1, dtype="f64", tol=1e-8)
        assert infos[0]["rel_res_true"] <= 1e-8 and not torch.equal(x, x1)
    finally:
        ctx.close()
