"""Pins of the learned-warm-start oracle (oracle/mlp.py): gradients against
central finite differences, the energy loss against its closed-form minimum,
Adam's first step against its closed form, bf16 rounding against hand-picked
values, and the features against invariances and direct definitions."""
import numpy as np
import pytest

from paper_2008_00409_amd import meshgen as mg


@pytest.fixture(scope="module")
def M():
    from oracle import mlp
    return mlp


def test_bf16_rounding_closed_form(M):
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.0e-3, 65504.0])
    # 3e-3 = 1.536 * 2^-9; 1.536 * 128 = 196.6 rounds to 197; 65504 rounds up to 2^16
    want = np.array([1.0, 1.0, 1 + 2 * 2 ** -7, -2.5, 197 / 128 * 2 ** -9, 65536.0])
    np.testing.assert_array_equal(M.bf16_round(vals), want)


def test_backward_matches_finite_differences(M):
    rng = np.random.default_rng(0)
    params = M.init_params(1)
    params[3][0] *= 100.0            # undo the small last-layer init for a well-scaled check
    for k in range(4):
        params[k][1] = 0.1 * rng.normal(size=params[k][1].shape)
    X = rng.normal(size=(7, M.IN))
    gy = rng.normal(size=(7, M.OUT))
    y, hs = M.forward(params, X)
    grads = M.backward(params, X, hs, gy)
    f = lambda p: float((M.forward(p, X)[0] * gy).sum())
    step = 1e-6
    for k in range(4):
        for q in range(2):
            arr = params[k][q]
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                old = arr[idx]
                arr[idx] = old + step
                fp = f(params)
                arr[idx] = old - step
                fm = f(params)
                arr[idx] = old
                fd = (fp - fm) / (2 * step)
                assert grads[k][q][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def small_system(oracle_mod, n=6):
    c = mg.config_grid(n, seed=31, h=0.01)
    P = oracle_mod.Problem.from_cloth(c)
    x = c.x0
    v = 0.05 * np.random.default_rng(2).normal(size=x.shape)
    v[c.pinned == 1] = 0
    A = P.assemble(x, v)
    return c, P, A, x, v


def test_energy_loss_gradient_and_minimum(M, oracle_mod):
    c, P, A, x, v = small_system(oracle_mod)
    apply_A = lambda z: P.spmv(A, z)
    sv = (1.0 / (6 - 1)) / c.h
    rng = np.random.default_rng(3)
    dv_prev = 0.01 * rng.normal(size=x.shape)
    y = 0.001 * rng.normal(size=x.shape)
    dv0 = M.start_from_output(y, dv_prev, c.pinned, sv)
    L, gy = M.energy_loss_grad(apply_A, A.b, A.diag, dv0, c.pinned, sv)
    step = 1e-7
    for idx in [(3, 0), (10, 2), (20, 1)]:
        yp, ym = y.copy(), y.copy()
        yp[idx] += step
        ym[idx] -= step
        Lp = M.energy_loss_grad(apply_A, A.b, A.diag, M.start_from_output(yp, dv_prev, c.pinned, sv),
                                c.pinned, sv)[0]
        Lm = M.energy_loss_grad(apply_A, A.b, A.diag, M.start_from_output(ym, dv_prev, c.pinned, sv),
                                c.pinned, sv)[0]
        assert gy[idx] == pytest.approx((Lp - Lm) / (2 * step), rel=1e-5)
    # at the exact solution the gradient vanishes and L = -0.5 b.A^-1 b / E0
    sol = np.linalg.solve(A.dense(), A.b.ravel()).reshape(-1, 3)
    Ls, gs = M.energy_loss_grad(apply_A, A.b, A.diag, sol, c.pinned, sv)
    E0 = float((A.b * A.b / A.diag).sum())
    assert Ls == pytest.approx(-0.5 * float((A.b * sol).sum()) / E0, rel=1e-10)
    assert np.abs(gs).max() < 1e-8 * sv / E0 * np.abs(A.b).max()


def test_adam_first_step_closed_form(M):
    params = M.init_params(2)
    grads = [[np.full_like(W, 0.5), np.full_like(c, -2.0)] for W, c in params]
    before = M.flatten(params)
    M.adam_step(params, grads, {}, lr=1e-3)
    delta = M.flatten(params) - before
    # first step: m_hat = g, v_hat = g^2  ->  update = -lr * g / (|g| + eps)
    gflat = M.flatten(grads)
    np.testing.assert_allclose(delta, -1e-3 * gflat / (np.abs(gflat) + 1e-8), rtol=1e-12)


def test_adam_constant_gradient_every_step(M):
    """With the same gradient g at every step, the bias-corrected moments are
    m_hat = g and v_hat = g^2 at every t (m_t = (1 - b1^t) g, v_t = (1 - b2^t)
    g^2), so every update is -lr g / (|g| + eps), not only the first."""
    params = M.init_params(4)
    rng = np.random.default_rng(8)
    grads = [[rng.normal(size=W.shape), rng.normal(size=c.shape)] for W, c in params]
    gflat = M.flatten(grads)
    state = {}
    for t in range(1, 6):
        before = M.flatten(params)
        M.adam_step(params, grads, state, lr=2e-3)
        delta = M.flatten(params) - before
        np.testing.assert_allclose(delta, -2e-3 * gflat / (np.abs(gflat) + 1e-8), rtol=1e-9,
                                   err_msg=f"step {t}")


def test_adam_alternating_gradient_closed_form(M):
    """Gradient +g, -g, +g: worked by hand from the moment recurrences
    (b1 = 0.9, b2 = 0.999).  v_hat = g^2 at every step since |g| is constant;
    m_1 = 0.1 g -> m_hat = g; m_2 = 0.09 g - 0.1 g = -0.01 g -> m_hat = -g/19
    (1 - 0.81 = 0.19); m_3 = -0.009 g + 0.1 g = 0.091 g -> m_hat = 91 g/271
    (1 - 0.729 = 0.271).  Updates: -lr g/(|g|+eps) times 1, -1/19, 91/271."""
    params = M.init_params(6)
    rng = np.random.default_rng(9)
    g = [[rng.normal(size=W.shape), rng.normal(size=c.shape)] for W, c in params]
    gflat = M.flatten(g)
    unit = gflat / (np.abs(gflat) + 1e-8)
    state = {}
    for sign, factor in ((1.0, 1.0), (-1.0, -1.0 / 19.0), (1.0, 91.0 / 271.0)):
        gs = [[sign * W, sign * c] for W, c in g]
        before = M.flatten(params)
        M.adam_step(params, gs, state, lr=1e-3)
        delta = M.flatten(params) - before
        np.testing.assert_allclose(delta, -1e-3 * factor * unit, rtol=1e-8, atol=1e-18)


def test_features_written_out_per_vertex(M, oracle_mod):
    """Every feature group of three vertices written out from its definition:
    neighbours from the oracle's dense matrix (nonzero off-diagonal blocks of
    row i), diag(A) from the dense diagonal, plain Python sums."""
    c, P, A, x, v = small_system(oracle_mod)
    rng = np.random.default_rng(12)
    dvp = rng.normal(size=x.shape)
    ell, h = 0.2, c.h
    sv = ell / h
    F = M.features(P.rowptr, P.colidx, x, v, A.b, A.diag, c.mass, c.pinned, dvp, ell, h)
    Ad = A.dense()
    nv = x.shape[0]
    pat = np.zeros((nv, nv), dtype=bool)
    for i in range(nv):
        for j in P.colidx[P.rowptr[i]:P.rowptr[i + 1]]:
            pat[i, j] = True
    for i in (0, 9, 17):
        nb = [j for j in range(nv) if j != i and pat[i, j]]
        d = np.array([Ad[3 * i + a, 3 * i + a] for a in range(3)])
        m = c.mass[i]
        mean = lambda arr: sum(arr[j] for j in nb) / len(nb)
        bm = A.b / c.mass[:, None]
        want = np.concatenate([
            v[i] / sv, (A.b[i] / m) / sv, dvp[i] / sv, mean(dvp) / sv, (A.b[i] / d) / sv,
            (mean(bm) - bm[i]) / sv, (mean(v) - v[i]) / sv, (mean(x) - x[i]) / ell,
            [float(c.pinned[i])], [np.log10(d.mean() / m)], [len(nb) / 12.0]])
        np.testing.assert_allclose(F[i], want, rtol=1e-12, atol=1e-14)


def test_features_invariances(M, oracle_mod):
    """Features 3-5 and 15-17 are linear in b; 6-8 and 9-11 linear in the
    previous increment; the Laplacian features (15-17, 18-20, 21-23) vanish
    for constant fields (b/m, v, a translation of x); feature 25 is unchanged
    when diag(A) and the masses are scaled together, and is 0 for a pinned
    vertex (diag(A)_i = m_i)."""
    c, P, A, x, v = small_system(oracle_mod)
    rng = np.random.default_rng(13)
    dvp = rng.normal(size=x.shape)
    ell, h = 0.2, c.h
    f = lambda x_, v_, b_, dg, m_, dv_: M.features(P.rowptr, P.colidx, x_, v_, b_, dg, m_, c.pinned, dv_, ell, h)
    F = f(x, v, A.b, A.diag, c.mass, dvp)
    F2 = f(x, v, 3 * A.b, A.diag, c.mass, -2 * dvp)
    np.testing.assert_allclose(F2[:, 3:6], 3 * F[:, 3:6], rtol=1e-13)
    np.testing.assert_allclose(F2[:, 15:18], 3 * F[:, 15:18], rtol=1e-12, atol=1e-14 * np.abs(F[:, 15:18]).max())
    np.testing.assert_allclose(F2[:, 6:12], -2 * F[:, 6:12], rtol=1e-13)
    const = np.tile([0.3, -1.2, 2.0], (x.shape[0], 1))
    Fc = f(const, const, const * c.mass[:, None], A.diag, c.mass, dvp)
    np.testing.assert_allclose(Fc[:, 15:24], 0.0, atol=1e-12 * np.abs(const).max() / min(ell, h))
    F4 = f(x, v, A.b, 5 * A.diag, 5 * c.mass, dvp)
    np.testing.assert_allclose(F4[:, 25], F[:, 25], rtol=1e-13, atol=1e-15)
    pinned = np.flatnonzero(c.pinned == 1)
    assert pinned.size > 0
    np.testing.assert_allclose(F[pinned, 25], 0.0, atol=1e-15)


def test_features_definitions_and_invariance(M, oracle_mod):
    c, P, A, x, v = small_system(oracle_mod)
    rng = np.random.default_rng(4)
    dvp = rng.normal(size=x.shape)
    ell, h = 0.2, c.h
    F = M.features(P.rowptr, P.colidx, x, v, A.b, A.diag, c.mass, c.pinned, dvp, ell, h)
    assert F.shape == (P.nv, 27)
    sv = ell / h
    np.testing.assert_allclose(F[:, 0:3], v / sv)
    np.testing.assert_allclose(F[:, 12:15], A.b / A.diag / sv)
    np.testing.assert_array_equal(F[:, 24], c.pinned)
    np.testing.assert_allclose(F[:, 26], (np.diff(P.rowptr) - 1) / 12.0)
    # vertex 7's neighbour mean of dv_prev, written out from its row
    i = 7
    nb = [j for j in P.colidx[P.rowptr[i]:P.rowptr[i + 1]] if j != i]
    np.testing.assert_allclose(F[i, 9:12], dvp[nb].mean(axis=0) / sv)
    # curvature feature is translation invariant; velocity features are linear
    F2 = M.features(P.rowptr, P.colidx, x + 3.0, v, A.b, A.diag, c.mass, c.pinned, dvp, ell, h)
    np.testing.assert_allclose(F2[:, 21:24], F[:, 21:24], atol=1e-12)
    F3 = M.features(P.rowptr, P.colidx, x, 2 * v, A.b, A.diag, c.mass, c.pinned, 2 * dvp, ell, h)
    np.testing.assert_allclose(F3[:, 0:3], 2 * F[:, 0:3])
    np.testing.assert_allclose(F3[:, 18:21], 2 * F[:, 18:21])


def test_energy_training_reduces_the_loss(M, oracle_mod):
    """Full-batch training on one small system lowers the energy loss of the
    start (the network can only improve on the previous-step start)."""
    c, P, A, x, v = small_system(oracle_mod, n=8)
    apply_A = lambda z: P.spmv(A, z)
    sv = (1.0 / 7) / c.h
    dvp = np.zeros_like(x)
    X = M.features(P.rowptr, P.colidx, x, v, A.b, A.diag, c.mass, c.pinned, dvp, 1.0 / 7, c.h)
    params = M.init_params(5)
    state = {}
    losses = []
    for it in range(200):
        y, hs = M.forward(params, X)
        dv0 = M.start_from_output(y, dvp, c.pinned, sv)
        L, gy = M.energy_loss_grad(apply_A, A.b, A.diag, dv0, c.pinned, sv)
        losses.append(L)
        M.adam_step(params, M.backward(params, X, hs, gy), state, lr=3e-3)
    assert losses[-1] < losses[0] - 0.1 * abs(losses[0])


def test_line_search_start_minimises_energy_along_the_correction(M, oracle_mod):
    """The start dv_prev + g u is the minimiser of the quadratic energy
    E(x) = x.A x / 2 - b.x on the line dv_prev + t u: E there is below E at
    dv_prev and at every other t, and dE/dt vanishes at g."""
    c, P, A, x, v = small_system(oracle_mod)
    apply_A = lambda z: P.spmv(A, z)
    rng = np.random.default_rng(9)
    dvp = 0.01 * rng.normal(size=x.shape)
    u = 0.01 * rng.normal(size=x.shape)
    u[c.pinned == 1] = 0
    E = lambda z: 0.5 * float((z * apply_A(z)).sum()) - float((A.b * z).sum())
    s0, g = M.line_search_start(apply_A, A.b, dvp, u)
    assert E(s0) <= E(dvp)
    for t in np.linspace(g - 1.0, g + 1.0, 11):
        assert E(s0) <= E(dvp + t * u) + 1e-15 * abs(E(s0))
    # stationarity: u.(A s0 - b) = 0
    assert abs(float((u * (apply_A(s0) - A.b)).sum())) <= 1e-9 * abs(float((u * A.b).sum()))
    # zero correction: g = 0 and the start is dv_prev
    s1, g1 = M.line_search_start(apply_A, A.b, dvp, np.zeros_like(u))
    assert g1 == 0.0 and np.array_equal(s1, dvp)
