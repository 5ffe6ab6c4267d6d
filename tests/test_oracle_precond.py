"""Pins of the oracle's block-Jacobi preconditioned CG (P = the 3x3 diagonal
blocks of A) against special cases the mathematics fixes:

* block-diagonal A: the preconditioner is A^-1, so CG ends after one
  iteration at the exact solution (per-block solves by numpy);
* diagonal 3x3 blocks: block Jacobi and Jacobi are the same preconditioner,
  so the iterates coincide (same iteration count; solutions equal up to the
  combination order of the oracle's threaded dot products);
* on an assembled cloth system it reaches the tolerance in fewer iterations
  than Jacobi and meets the true residual bound."""
import numpy as np

from paper_2008_00409_amd import meshgen as mg


def block_system(rng, nv, offdiag):
    """Block-CSR SPD matrix with a ring of off-diagonal blocks (scaled by
    `offdiag`, 0 gives a block-diagonal matrix)."""
    rowptr, colidx, vals = [0], [], []
    for i in range(nv):
        cols = sorted({i, (i + 1) % nv, (i - 1) % nv})
        for j in cols:
            colidx.append(j)
            if i == j:
                G = rng.normal(size=(3, 3))
                vals.append(G @ G.T + 3.0 * np.eye(3))
            else:
                vals.append(np.zeros((3, 3)))
        rowptr.append(len(colidx))
    rowptr = np.array(rowptr, dtype=np.int32)
    colidx = np.array(colidx, dtype=np.int32)
    vals = np.array(vals)
    if offdiag:
        C = offdiag * rng.normal(size=(3, 3))
        for i in range(nv):
            j = (i + 1) % nv
            pij = rowptr[i] + list(colidx[rowptr[i]:rowptr[i + 1]]).index(j)
            pji = rowptr[j] + list(colidx[rowptr[j]:rowptr[j + 1]]).index(i)
            vals[pij] += C
            vals[pji] += C.T
    return rowptr, colidx, vals


def assembled(oracle_mod, rowptr, colidx, vals, b):
    nv = rowptr.size - 1
    dpos = [rowptr[i] + list(colidx[rowptr[i]:rowptr[i + 1]]).index(i) for i in range(nv)]
    diag = np.array([np.diag(vals[p]) for p in dpos])
    return oracle_mod.Assembled(rowptr, colidx, vals, b, diag, np.zeros((nv, 3, 3))), dpos


def run_pcg(oracle_mod, A, nv, **kw):
    P = oracle_mod.Problem.__new__(oracle_mod.Problem)
    P.nv = nv
    return oracle_mod.Problem.pcg(P, A, **kw)


def test_block_jacobi_solves_block_diagonal_system_in_one_iteration(oracle_mod):
    rng = np.random.default_rng(0)
    nv = 17
    rowptr, colidx, vals = block_system(rng, nv, 0.0)
    b = rng.normal(size=(nv, 3))
    A, dpos = assembled(oracle_mod, rowptr, colidx, vals, b)
    x, info = run_pcg(oracle_mod, A, nv, tol=1e-12, precond="block")
    want = np.array([np.linalg.solve(vals[dpos[i]], b[i]) for i in range(nv)])
    assert info["iters"] == 1
    np.testing.assert_allclose(x, want, rtol=1e-12, atol=1e-14)
    _, info_j = run_pcg(oracle_mod, A, nv, tol=1e-12, precond="jacobi")
    assert info_j["iters"] > 1


def test_block_jacobi_equals_jacobi_for_diagonal_blocks(oracle_mod):
    rng = np.random.default_rng(1)
    nv = 23
    rowptr, colidx, vals = block_system(rng, nv, 0.4)
    for i in range(nv):   # make every diagonal block diagonal (the system stays SPD)
        p = rowptr[i] + list(colidx[rowptr[i]:rowptr[i + 1]]).index(i)
        vals[p] = np.diag(np.diag(vals[p]) + 2.0)
    b = rng.normal(size=(nv, 3))
    A, _ = assembled(oracle_mod, rowptr, colidx, vals, b)
    xj, ij = run_pcg(oracle_mod, A, nv, tol=1e-10, precond="jacobi")
    xb, ib = run_pcg(oracle_mod, A, nv, tol=1e-10, precond="block")
    assert ij["iters"] == ib["iters"]
    np.testing.assert_allclose(xb, xj, rtol=1e-12, atol=1e-15)


def test_block_jacobi_on_cloth_system(oracle_mod):
    c = mg.config_grid(20, seed=2000, h=1.0 / 200)
    P = oracle_mod.Problem.from_cloth(c)
    v = 0.05 * np.random.default_rng(2).normal(size=c.x0.shape)
    v[c.pinned == 1] = 0
    A = P.assemble(c.x0, v)
    xj, ij = P.pcg(A, tol=1e-8, precond="jacobi")
    xb, ib = P.pcg(A, tol=1e-8, precond="block")
    assert ib["converged"] and ib["rel_res_true"] <= 1e-8 * (1 + 1e-6)
    assert ib["iters"] < ij["iters"]
    assert P.residual(A, xb) <= 1e-8 * (1 + 1e-6)
    # both solve the same system
    assert np.linalg.norm(xb - xj) <= 1e-5 * np.linalg.norm(xj)
