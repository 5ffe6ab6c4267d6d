"""The paper's own five-step matrix filling (index table, atomic index fill,
compacting, BELL value table, atomic value fill) and its BELL SpMV, built
beside the solver's assembly for comparison, against the FP64 oracle through
the C ABI: the compacted pattern is the oracle's block pattern (bit-exact),
the FP64 table's blocks match to 1e-12 of the row scale and b to 1e-10
(the atomics only reorder FP64 sums); the FP32 table's blocks to 4e-6 of
the row scale (each contribution and each atomic sum rounded to FP32, at
most ~60 terms per entry at 2^-24 each); padding slots repeat the row with
zero blocks; the SpMV matches the oracle's A times the FP32-rounded x.
The same system as cloth_assemble, so b agrees with it too."""
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


def bell_to_bsr(cols, vals, nv):
    """BELL table -> (rowptr, colidx, blocks); also the padding slots' values."""
    width = cols.shape[0]
    rowptr = [0]
    colidx, blocks, pad = [], [], []
    for i in range(nv):
        c = cols[:, i]
        uniq, first = np.unique(c, return_index=True)
        rest = np.setdiff1d(np.arange(width), first)
        assert np.all(c[rest] == i), "padding must repeat the row index"
        # the real slots come first, in ascending column order
        assert np.array_equal(np.sort(first), np.arange(uniq.size))
        colidx.append(uniq)
        blocks.append(vals[:, first, i].T.reshape(-1, 3, 3))
        pad.append(vals[:, rest, i].ravel())
        rowptr.append(rowptr[-1] + uniq.size)
    return (np.array(rowptr), np.concatenate(colidx), np.concatenate(blocks),
            np.concatenate(pad) if pad else np.zeros(0))


def row_scale(A, nv):
    return np.repeat(np.array([np.abs(A.vals[A.rowptr[i]:A.rowptr[i + 1]]).max() for i in range(nv)]),
                     np.diff(A.rowptr))


def run_bell(torch, B, c, v, dtype, contacts=None, rhs_mode=1):
    ctx = B.Context.from_cloth(c, rhs_mode=rhs_mode)
    try:
        if contacts is not None:
            ctx.cloth_set_contacts(*contacts)
        x_d, v_d = to_dev(torch, c.x0), to_dev(torch, v)
        b, width = ctx.cloth_assemble_bell(x_d, v_d, dtype)
        cols, vals = ctx.cloth_export_bell()
        xs = np.random.default_rng(11).normal(size=(c.nv, 3))
        y = ctx.cloth_spmv_bell(to_dev(torch, xs))
        b_ref = ctx.cloth_assemble(x_d, v_d, "f64")
        return dict(b=b.cpu().numpy(), width=width, cols=cols.cpu().numpy(), vals=vals.cpu().numpy(),
                    xs=xs, y=y.cpu().numpy(), b_solver=b_ref.cpu().numpy())
    finally:
        ctx.close()


@pytest.mark.parametrize("dtype,rhs_mode", [("f64", 1), ("f64", 0), ("f32", 1)])
def test_bell_matches_oracle(torch, B, oracle_mod, dtype, rhs_mode):
    c = sheet(71, 53, seed=21, flips=0.1)          # 3763 rows
    v = random_velocity(c, 0.05, seed=2)
    P = oracle_mod.Problem.from_cloth(c, oracle_mod.Material(rhs_mode=rhs_mode))
    A = P.assemble(c.x0, v)
    r = run_bell(torch, B, c, v, dtype, rhs_mode=rhs_mode)
    assert r["width"] == int(np.diff(A.rowptr).max())
    rowptr, colidx, blocks, pad = bell_to_bsr(r["cols"], r["vals"], c.nv)
    np.testing.assert_array_equal(rowptr, A.rowptr)
    np.testing.assert_array_equal(colidx, A.colidx)
    assert np.all(pad == 0.0)
    err = np.abs(blocks - A.vals).reshape(-1, 9).max(axis=1) / row_scale(A, c.nv)
    bar = 1e-12 if dtype == "f64" else 4e-6
    assert err.max() <= bar, err.max()
    if dtype == "f64":
        np.testing.assert_allclose(r["b"], A.b, rtol=1e-10, atol=1e-10 * np.abs(A.b).max())
    else:
        np.testing.assert_allclose(r["b"], A.b, rtol=0, atol=1e-5 * np.abs(A.b).max())
    np.testing.assert_allclose(r["b_solver"], A.b, rtol=1e-10, atol=1e-10 * np.abs(A.b).max())
    # SpMV: FP32-rounded x, FP64 accumulation
    x32 = r["xs"].astype(np.float32).astype(np.float64)
    yref = (A.dense() @ x32.ravel()).reshape(-1, 3)
    # |y - yref|_i <= (block bar) * rowscale_i * sum over the row's columns j of |x_j|_1
    rs = np.array([np.abs(A.vals[A.rowptr[i]:A.rowptr[i + 1]]).max() for i in range(c.nv)])
    ax = np.abs(x32).sum(axis=1)
    sx = np.array([ax[A.colidx[A.rowptr[i]:A.rowptr[i + 1]]].sum() for i in range(c.nv)])
    assert np.all(np.abs(r["y"] - yref) <= (bar * rs * sx)[:, None])


def test_bell_with_contacts_matches_oracle(torch, B, oracle_mod):
    c, cs = mg.config_contact(23, 19)
    v = random_velocity(c, 0.02, seed=5)
    P = oracle_mod.Problem.from_cloth(c)
    P.set_contacts(oracle_mod.Contacts(cs.verts, cs.weights, cs.normals, cs.eta, cs.kc))
    A = P.assemble(c.x0, v)
    r = run_bell(torch, B, c, v, "f64", contacts=(cs.verts, cs.weights, cs.normals, cs.eta, cs.kc))
    rowptr, colidx, blocks, pad = bell_to_bsr(r["cols"], r["vals"], c.nv)
    np.testing.assert_array_equal(rowptr, A.rowptr)
    np.testing.assert_array_equal(colidx, A.colidx)
    err = np.abs(blocks - A.vals).reshape(-1, 9).max(axis=1) / row_scale(A, c.nv)
    assert err.max() <= 1e-12, err.max()
    np.testing.assert_allclose(r["b"], A.b, rtol=1e-10, atol=1e-10 * np.abs(A.b).max())


def test_bell_rerun_within_rounding_solver_assembly_bitwise(torch, B):
    """Two FP32 fills of the same state agree to FP32 rounding of the atomic
    sums (the order varies); the solver's assembly is bit-identical."""
    c = sheet(120, 110, seed=24, flips=0.1)
    v = random_velocity(c, 0.05, seed=7)
    ctx = B.Context.from_cloth(c)
    try:
        x_d, v_d = to_dev(torch, c.x0), to_dev(torch, v)
        outs = []
        for _ in range(2):
            b, _w = ctx.cloth_assemble_bell(x_d, v_d, "f32")
            cols, vals = ctx.cloth_export_bell()
            outs.append((b.cpu().numpy(), cols.cpu().numpy(), vals.cpu().numpy()))
        mine = []
        for _ in range(2):
            bs = ctx.cloth_assemble(x_d, v_d, "f32")
            _rp, _ci, vs, _D = ctx.cloth_export_blocks(solver_blocks=True)
            mine.append((bs.cpu().numpy(), vs.cpu().numpy()))
    finally:
        ctx.close()
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    scale = np.abs(outs[0][2]).max(axis=(0, 1))
    assert np.all(np.abs(outs[0][2] - outs[1][2]).max(axis=(0, 1)) <= 4e-6 * scale)
    ndiff = int(np.count_nonzero(outs[0][2] != outs[1][2]))
    print(f"paper-layout FP32 fill: {ndiff} of {outs[0][2].size} values differ between two runs")
    assert np.array_equal(mine[0][0].view(np.uint64), mine[1][0].view(np.uint64))
    assert np.array_equal(mine[0][1].view(np.uint64), mine[1][1].view(np.uint64))


def test_bell_errors(torch, B):
    c = sheet(9, 8, seed=3)
    ctx = B.Context.from_cloth(c)
    try:
        x = to_dev(torch, c.x0)
        with pytest.raises(B.PclothError) as e:
            ctx.cloth_spmv_bell(x)
        assert e.value.status == B.PC_ERR_ARG
        with pytest.raises(B.PclothError) as e:
            ctx.cloth_assemble_bell(x, to_dev(torch, c.v0), "bf16")
        assert e.value.status == B.PC_ERR_ARG
        b, w = ctx.cloth_assemble_bell(x, to_dev(torch, c.v0), "f32")
        assert w > 0
        ctx.cloth_spmv_bell(x)
    finally:
        ctx.close()


def test_bell_long_rows_compact_without_lds(torch, B, oracle_mod):
    """One lower-sheet vertex in 70 contact pairs: its index-table row holds
    more than the 256 slots the LDS stage takes, so compaction runs from
    global memory; the table still matches the oracle."""
    c, cs = mg.config_contact(23, 19)
    nl = c.sheet_ranges[0][1]
    lo = c.tris[c.tris[:, 0] < nl]
    q = lo[len(lo) // 2]                                   # a lower triangle (q0, q1, q2)
    ups = np.arange(nl, c.nv)[:70]
    verts = np.column_stack([ups, np.repeat(q[None, :], 70, axis=0)]).astype(np.int32)
    weights = np.tile([1.0, -0.5, -0.3, -0.2], (70, 1))
    normals = np.tile([0.0, 0.0, 1.0], (70, 1))
    v = random_velocity(c, 0.02, seed=8)
    P = oracle_mod.Problem.from_cloth(c)
    P.set_contacts(oracle_mod.Contacts(verts, weights, normals, cs.eta, cs.kc))
    A = P.assemble(c.x0, v)
    ctx = B.Context.from_cloth(c)
    try:
        ctx.cloth_set_contacts(verts, weights, normals, cs.eta, cs.kc)
        b, width = ctx.cloth_assemble_bell(to_dev(torch, c.x0), to_dev(torch, v), "f64")
        cols, vals = ctx.cloth_export_bell()
        cols, vals, b = cols.cpu().numpy(), vals.cpu().numpy(), b.cpu().numpy()
    finally:
        ctx.close()
    assert width == int(np.diff(A.rowptr).max()) and width > 70
    rowptr, colidx, blocks, pad = bell_to_bsr(cols, vals, c.nv)
    np.testing.assert_array_equal(rowptr, A.rowptr)
    np.testing.assert_array_equal(colidx, A.colidx)
    assert np.all(pad == 0.0)
    err = np.abs(blocks - A.vals).reshape(-1, 9).max(axis=1) / row_scale(A, c.nv)
    assert err.max() <= 1e-12, err.max()
    np.testing.assert_allclose(b, A.b, rtol=1e-10, atol=1e-10 * np.abs(A.b).max())
