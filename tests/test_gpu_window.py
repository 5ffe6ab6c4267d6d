"""The SpMV's LDS window (the search direction's rows that a work item's
columns span, staged in LDS before the gathers) and its 16-bit column
offsets must not change any result:
solves with the window on and off are compared bit for bit, on a mesh in
grid order (every item's window fits), on the same mesh with randomly
renumbered vertices (windows span the whole mesh and fall back to global
gathers) and on a batch of instances."""
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


def renumbered(c, seed):
    perm = np.random.default_rng(seed).permutation(c.nv)      # old id -> new id
    inv = np.argsort(perm)                                     # new id -> old id
    return mg.Cloth(c.name + "-renumbered", c.rest[inv], perm[c.tris].astype(np.int32), c.mass[inv],
                    c.pinned[inv], c.x0[inv], c.v0[inv], c.h, c.tol, 1, [(0, c.nv)], [(0, c.nt)])


def solve(torch, B, c, v, window, dtype, precond, instances=None, narrow=1):
    ctx = B.Context.from_cloth(c)
    try:
        if instances is not None:
            ctx.set_instances(instances)
        ctx.set_option(B.PC_OPT_LDS_WINDOW, window)
        ctx.set_option(B.PC_OPT_NARROW_COLUMNS, narrow)
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), dtype)
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond=precond)
        return dv.cpu().numpy(), info
    finally:
        ctx.close()


@pytest.mark.parametrize("dtype,precond", [("f32", "jacobi"), ("bf16", "block"), ("f64", "block"),
                                           ("f16", "block")])
def test_window_on_off_identical_grid_order(torch, B, dtype, precond):
    c = sheet(71, 53, seed=21, flips=0.1)       # 3763 rows, 59 slices
    v = random_velocity(c, 0.05, seed=2)
    d1, i1 = solve(torch, B, c, v, 1, dtype, precond)
    d0, i0 = solve(torch, B, c, v, 0, dtype, precond)
    assert i1["iters"] == i0["iters"]
    assert np.array_equal(d1.view(np.uint64), d0.view(np.uint64))


def test_window_falls_back_on_scattered_columns(torch, B, oracle_mod):
    c = renumbered(sheet(90, 70, seed=22, flips=0.1), seed=5)   # 6300 rows, windows > 4096 rows
    v = random_velocity(c, 0.05, seed=3)
    d1, i1 = solve(torch, B, c, v, 1, "f32", "block")
    d0, i0 = solve(torch, B, c, v, 0, "f32", "block")
    assert i1["iters"] == i0["iters"]
    assert np.array_equal(d1.view(np.uint64), d0.view(np.uint64))
    P = oracle_mod.Problem.from_cloth(c)
    A = P.assemble(c.x0, v)
    assert P.residual(A, d1) <= 1e-6 * (1 + 1e-6)


def test_window_batched_instances(torch, B):
    c = mg.config_batch(seed=91, sizes=[13, 40, 9, 27])
    begins = [r[0] for r in c.sheet_ranges] + [c.nv]
    v = random_velocity(c, 0.05, seed=4)
    d1, i1 = solve(torch, B, c, v, 1, "bf16", "block", begins)
    d0, i0 = solve(torch, B, c, v, 0, "bf16", "block", begins)
    assert i1["iters"] == i0["iters"]
    assert np.array_equal(d1.view(np.uint64), d0.view(np.uint64))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_narrow_columns_identical(torch, B, dtype):
    c = sheet(71, 53, seed=21, flips=0.1)
    v = random_velocity(c, 0.05, seed=2)
    d1, i1 = solve(torch, B, c, v, 1, dtype, "block", narrow=1)
    d0, i0 = solve(torch, B, c, v, 1, dtype, "block", narrow=0)
    assert i1["iters"] == i0["iters"]
    assert np.array_equal(d1.view(np.uint64), d0.view(np.uint64))


def test_wide_columns_fall_back(torch, B, oracle_mod):
    """Randomly renumbered 42,000-vertex sheet: column offsets exceed 16 bits,
    the solver keeps 32-bit columns (and global gathers) and still solves."""
    c = renumbered(sheet(210, 200, seed=23, flips=0.0), seed=6)
    v = random_velocity(c, 0.05, seed=4)
    d1, i1 = solve(torch, B, c, v, 1, "f32", "block", narrow=1)
    d0, i0 = solve(torch, B, c, v, 0, "f32", "block", narrow=0)
    assert i1["iters"] == i0["iters"]
    assert np.array_equal(d1.view(np.uint64), d0.view(np.uint64))
