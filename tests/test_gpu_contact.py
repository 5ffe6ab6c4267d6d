"""GPU parity of the assembly with proximity (contact) elements against the
FP64 oracle, through the C ABI: the block pattern (bit-exact, with the
contact pairs), the FP64 blocks, b, diag(A) and the remainders; solves
through the oracle's matrix; a trajectory whose contact set changes every
step (so the pattern does); invalid contact sets rejected.

Bars as for the assembly without contacts: FP64 blocks to 1e-12 of the row
scale, b and diag(A) to 1e-10 relative."""
import numpy as np
import pytest

from gpu_helpers import random_velocity, require_gpu, to_dev
from paper_2008_00409_amd import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def B():
    from paper_2008_00409_amd import binding
    return binding


def two_sheets(n=23, m=19):
    return mg.config_contact(n, m)      # 2 x n x m vertices, every upper vertex paired


def oracle_contacts(oracle_mod, cs):
    return oracle_mod.Contacts(cs.verts, cs.weights, cs.normals, cs.eta, cs.kc)


def edge_edge_pairs(c, rng, count):
    """Synthetic edge-edge pairs between the two sheets (vertices of one lower
    and one upper triangle edge), weights (1-s, s, -(1-t), -t), unit normals."""
    nl = c.sheet_ranges[0][1]
    lo = c.tris[c.tris[:, 0] < nl]
    up = c.tris[c.tris[:, 0] >= nl]
    a = lo[rng.integers(0, len(lo), count)][:, :2]
    b = up[rng.integers(0, len(up), count)][:, :2]
    s, t = rng.uniform(0.1, 0.9, (2, count))
    n = rng.normal(size=(count, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    verts = np.column_stack([b, a]).astype(np.int32)
    w = np.column_stack([1 - t, t, -(1 - s), -s])
    return verts, w, n


@pytest.mark.parametrize("rhs_mode", [0, 1])
def test_assembly_with_contacts_matches_oracle(torch, B, oracle_mod, rhs_mode):
    c, cs = two_sheets()
    rng = np.random.default_rng(3)
    ev, ew, en = edge_edge_pairs(c, rng, 40)
    verts = np.concatenate([cs.verts, ev])
    weights = np.concatenate([cs.weights, ew])
    normals = np.concatenate([cs.normals, en])
    v = random_velocity(c, 0.02, seed=5)
    mat = oracle_mod.Material(rhs_mode=rhs_mode)
    P = oracle_mod.Problem.from_cloth(c, mat)
    P.set_contacts(oracle_mod.Contacts(verts, weights, normals, cs.eta, cs.kc))
    A = P.assemble(c.x0, v)
    ctx = B.Context.from_cloth(c, rhs_mode=rhs_mode)
    try:
        ctx.cloth_set_contacts(verts, weights, normals, cs.eta, cs.kc)
        x_d, v_d = to_dev(torch, c.x0), to_dev(torch, v)
        diag = torch.empty_like(x_d)
        b = ctx.cloth_assemble(x_d, v_d, "f32", diag=diag)
        rowptr, colidx, vals, D = ctx.cloth_export_blocks(solver_blocks=False)
        rowptr, colidx = rowptr.cpu().numpy(), colidx.cpu().numpy()
        vals, D = vals.cpu().numpy().reshape(-1, 3, 3), D.cpu().numpy().reshape(-1, 3, 3)
        b, diag = b.cpu().numpy(), diag.cpu().numpy()
    finally:
        ctx.close()
    np.testing.assert_array_equal(rowptr, A.rowptr)
    np.testing.assert_array_equal(colidx, A.colidx)
    scale = np.repeat(np.array([np.abs(A.vals[A.rowptr[i]:A.rowptr[i + 1]]).max() for i in range(P.nv)]),
                      np.diff(A.rowptr))
    err = np.abs(vals - A.vals).reshape(-1, 9).max(axis=1) / scale
    assert err.max() <= 1e-12, err.max()
    np.testing.assert_allclose(b, A.b, rtol=1e-10, atol=1e-10 * np.abs(A.b).max())
    np.testing.assert_allclose(diag, A.diag, rtol=1e-10)
    np.testing.assert_allclose(D, A.D, rtol=0, atol=1e-12 * np.abs(A.vals).max())


@pytest.mark.parametrize("dtype,precond", [("f32", "jacobi"), ("bf16", "block")])
def test_solve_with_contacts_through_oracle(torch, B, oracle_mod, dtype, precond):
    c, cs = two_sheets()
    v = random_velocity(c, 0.02, seed=6)
    P = oracle_mod.Problem.from_cloth(c)
    P.set_contacts(oracle_contacts(oracle_mod, cs))
    A = P.assemble(c.x0, v)
    ctx = B.Context.from_cloth(c)
    try:
        ctx.cloth_set_contacts(cs.verts, cs.weights, cs.normals, cs.eta, cs.kc)
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, v), dtype)
        dv, info = ctx.cloth_pcg_solve(b, tol=1e-6, precond=precond)
        dv = dv.cpu().numpy()
    finally:
        ctx.close()
    assert P.residual(A, dv) <= 1e-6 * (1 + 1e-6)


def test_changing_contacts_trajectory_matches_oracle(torch, B, oracle_mod):
    """Three steps: all pairs, then every other pair, then none; the GPU
    pattern follows and the states match the oracle's trajectory."""
    c, cs = two_sheets(17, 15)
    sets = [np.arange(cs.n), np.arange(0, cs.n, 2), np.arange(0)]
    P = oracle_mod.Problem.from_cloth(c)
    x, v = c.x0.copy(), c.v0.copy()
    ctx = B.Context.from_cloth(c)
    try:
        x_d, v_d = to_dev(torch, c.x0), to_dev(torch, c.v0)
        for sel in sets:
            if sel.size:
                P.set_contacts(oracle_mod.Contacts(cs.verts[sel], cs.weights[sel], cs.normals[sel], cs.eta, cs.kc))
                ctx.cloth_set_contacts(cs.verts[sel], cs.weights[sel], cs.normals[sel], cs.eta, cs.kc)
            else:
                P.set_contacts(None)
                ctx.cloth_set_contacts(None)
            x, v, dv, info = P.step(x, v, tol=1e-10)
            ctx.cloth_step(x_d, v_d, nsteps=1, dtype="f64", tol=1e-10)
            rowptr, colidx = ctx.pattern()
            np.testing.assert_array_equal(rowptr.cpu().numpy(), P.rowptr)
            np.testing.assert_array_equal(colidx.cpu().numpy(), P.colidx)
            vg = v_d.cpu().numpy()
            assert np.linalg.norm(vg - v) <= 1e-6 * np.linalg.norm(v)
            np.testing.assert_allclose(x_d.cpu().numpy(), x, rtol=0, atol=1e-9)
    finally:
        ctx.close()


def test_invalid_contacts_rejected(torch, B):
    c, cs = two_sheets(9, 8)
    ctx = B.Context.from_cloth(c)
    try:
        good = (cs.verts[:4].copy(), cs.weights[:4].copy(), cs.normals[:4].copy())
        bad_sets = []
        v = good[0].copy(); v[0, 1] = v[0, 0]                   # repeated vertex
        bad_sets.append((v, good[1], good[2]))
        v = good[0].copy(); v[1, 2] = c.nv                       # out of range
        bad_sets.append((v, good[1], good[2]))
        w = good[1].copy(); w[2, 0] += 0.1                        # weights do not sum to zero
        bad_sets.append((good[0], w, good[2]))
        n = good[2].copy(); n[3] *= 2.0                           # not unit length
        bad_sets.append((good[0], good[1], n))
        for verts, weights, normals in bad_sets:
            with pytest.raises(B.PclothError) as e:
                ctx.cloth_set_contacts(verts, weights, normals, cs.eta, cs.kc)
            assert e.value.status == B.PC_ERR_ARG
        # the context still assembles and solves (with no contacts)
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, c.v0), "f32")
        ctx.cloth_pcg_solve(b, tol=1e-6)
        # a valid set after the rejected ones
        ctx.cloth_set_contacts(*good, cs.eta, cs.kc)
        b = ctx.cloth_assemble(to_dev(torch, c.x0), to_dev(torch, c.v0), "f32")
        ctx.cloth_pcg_solve(b, tol=1e-6)
    finally:
        ctx.close()


def test_contacts_across_instances_rejected(torch, B):
    c, cs = two_sheets(9, 8)
    ctx = B.Context.from_cloth(c)
    try:
        ctx.set_instances([r[0] for r in c.sheet_ranges] + [c.nv])
        with pytest.raises(B.PclothError):
            ctx.cloth_set_contacts(cs.verts, cs.weights, cs.normals, cs.eta, cs.kc)
    finally:
        ctx.close()
