"""Pins of the oracle's single-reduction (Chronopoulos-Gear) preconditioned
CG against what the mathematics fixes:

* in exact arithmetic its iterates are those of the textbook recurrences, so
  after k iterations (k = 1..8, tolerance 0) the two oracles' solutions agree
  to rounding, with Jacobi and block-Jacobi preconditioning (a dropped or
  sign-flipped term of the alpha denominator, or an s recurrence on the wrong
  vector, breaks this from k = 2 on);
* a block-diagonal system with block Jacobi ends after one iteration at the
  exact per-block solutions (numpy);
* the solution of an assembled cloth system matches a dense solve
  (numpy.linalg.solve) and meets the true-residual bound, with the same
  iteration count as the textbook form to within one."""
import numpy as np
import pytest

from paper_2008_00409_amd import meshgen as mg
from test_oracle_precond import assembled, block_system, run_pcg


def cloth_system(oracle_mod, n=12, seed=3):
    c = mg.config_grid(n, seed=2000 + seed, h=1.0 / 200)
    P = oracle_mod.Problem.from_cloth(c)
    v = 0.05 * np.random.default_rng(seed).normal(size=c.x0.shape)
    v[c.pinned == 1] = 0
    return P, P.assemble(c.x0, v)


@pytest.mark.parametrize("precond", ["jacobi", "block"])
def test_iterates_match_textbook_cg(oracle_mod, precond):
    P, A = cloth_system(oracle_mod)
    for k in range(1, 9):
        xa, ia = P.pcg(A, tol=0.0, maxit=k, precond=precond)
        xb, ib = P.pcg(A, tol=0.0, maxit=k, precond=precond, method="chronopoulos-gear")
        assert ia["iters"] == ib["iters"] == k
        assert not ib["breakdown"]
        assert np.linalg.norm(xb - xa) <= 1e-9 * np.linalg.norm(xa), k


def test_block_diagonal_one_iteration(oracle_mod):
    rng = np.random.default_rng(4)
    nv = 19
    rowptr, colidx, vals = block_system(rng, nv, 0.0)
    b = rng.normal(size=(nv, 3))
    A, dpos = assembled(oracle_mod, rowptr, colidx, vals, b)
    x, info = run_pcg(oracle_mod, A, nv, tol=1e-12, precond="block", method="chronopoulos-gear")
    want = np.array([np.linalg.solve(vals[dpos[i]], b[i]) for i in range(nv)])
    assert info["iters"] == 1
    np.testing.assert_allclose(x, want, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("precond", ["jacobi", "block"])
def test_solution_matches_dense_solve(oracle_mod, precond):
    P, A = cloth_system(oracle_mod, n=14, seed=5)
    xd = np.linalg.solve(A.dense(), A.b.ravel()).reshape(-1, 3)
    xa, ia = P.pcg(A, tol=1e-10, precond=precond)
    xb, ib = P.pcg(A, tol=1e-10, precond=precond, method="chronopoulos-gear")
    assert ib["converged"] and ib["rel_res_true"] <= 1e-10 * (1 + 1e-3)
    assert abs(ib["iters"] - ia["iters"]) <= 1
    assert np.linalg.norm(xb - xd) <= 1e-7 * np.linalg.norm(xd)


def test_zero_rhs(oracle_mod):
    rng = np.random.default_rng(6)
    nv = 5
    rowptr, colidx, vals = block_system(rng, nv, 0.3)
    A, _ = assembled(oracle_mod, rowptr, colidx, vals, np.zeros((nv, 3)))
    x, info = run_pcg(oracle_mod, A, nv, x0=np.ones((nv, 3)), tol=1e-8, method="chronopoulos-gear")
    assert info["iters"] == 0 and np.all(x == 0.0)
