"""Pins of the FP64 oracle's element physics against things other than itself:
central finite differences, closed forms, invariants and hand-derived special
cases.  The integrator needs per-element forces and their Jacobians (paper
Sec. 2.5, Eq. 2-3); the elements are the stretch and bending "assembly
elements" of Sec. 3.2."""
import math

import numpy as np
import pytest

MU, LAM, KB = 1000.0, 500.0, 1e-5


def rand_rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def random_triangle(rng, oracle_mod):
    X = rng.normal(size=(3, 3))
    B, A0 = oracle_mod.rest_triangles(X, np.array([[0, 1, 2]]))
    return X, B[0], A0[0]


def fd_grad(fun, x, step):
    g = np.zeros_like(x)
    for i in range(x.size):
        xp, xm = x.copy(), x.copy()
        xp.flat[i] += step
        xm.flat[i] -= step
        g.flat[i] = (fun(xp) - fun(xm)) / (2 * step)
    return g


def fd_jac(fun, x, step):
    cols = []
    for i in range(x.size):
        xp, xm = x.copy(), x.copy()
        xp.flat[i] += step
        xm.flat[i] -= step
        cols.append((fun(xp) - fun(xm)) / (2 * step))
    return np.stack(cols, axis=1)


# ---------------------------------------------------------------- stretch
def test_rest_frame_closed_form(oracle_mod):
    # right triangle with legs 2 and 3, rotated and translated: A0 = 3, and the
    # rest shape maps to an isometry (F^T F = I).
    rng = np.random.default_rng(1)
    R = rand_rot(rng)
    X = np.array([[0, 0, 0], [2.0, 0, 0], [0, 3.0, 0]]) @ R.T + rng.normal(size=3)
    B, A0 = oracle_mod.rest_triangles(X, np.array([[0, 1, 2]]))
    assert A0[0] == pytest.approx(3.0, rel=1e-14)
    Ds = np.stack([X[1] - X[0], X[2] - X[0]], axis=1)
    F = Ds @ B[0].reshape(2, 2)
    np.testing.assert_allclose(F.T @ F, np.eye(2), atol=1e-14)


def test_stretch_uniaxial_closed_form(oracle_mod):
    # legs 1, uniaxial stretch 1+eps along the first leg:
    # g = eps + eps^2/2, S = diag((2mu+lam) g, lam g), E = A0 (mu + lam/2) g^2,
    # f1 = -A0 ((1+eps)(2mu+lam) g, 0, 0), f2 = -A0 (0, lam g, 0), f0 = -f1-f2.
    X = np.array([[0, 0, 0], [1.0, 0, 0], [0, 1.0, 0]])
    B, A0 = oracle_mod.rest_triangles(X, np.array([[0, 1, 2]]))
    for eps in (1e-3, 0.05, -0.02):
        x = X.copy()
        x[1, 0] = 1 + eps
        g = eps + eps ** 2 / 2
        E = oracle_mod.stretch_energy(x.ravel(), B[0], A0[0], MU, LAM)
        assert E == pytest.approx(0.5 * (MU + LAM / 2) * g * g, rel=1e-12)
        f = oracle_mod.stretch_force(x.ravel(), B[0], A0[0], MU, LAM).reshape(3, 3)
        f1 = -0.5 * np.array([(1 + eps) * (2 * MU + LAM) * g, 0, 0])
        f2 = -0.5 * np.array([0, LAM * g, 0])
        np.testing.assert_allclose(f[1], f1, rtol=1e-12, atol=1e-14 * abs(f1[0]))
        np.testing.assert_allclose(f[2], f2, rtol=1e-12, atol=1e-14 * abs(f1[0]))
        np.testing.assert_allclose(f[0], -f1 - f2, rtol=1e-12, atol=1e-14 * abs(f1[0]))


@pytest.mark.parametrize("seed", range(6))
def test_stretch_force_is_minus_energy_gradient(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    X, B, A0 = random_triangle(rng, oracle_mod)
    x = X + 0.1 * rng.normal(size=(3, 3))
    f = oracle_mod.stretch_force(x.ravel(), B, A0, MU, LAM)
    g = fd_grad(lambda y: oracle_mod.stretch_energy(y, B, A0, MU, LAM), x.ravel(), 1e-6)
    np.testing.assert_allclose(f, -g, rtol=1e-6, atol=1e-6 * np.abs(f).max())


@pytest.mark.parametrize("seed", range(6))
def test_stretch_exact_K_is_force_jacobian(oracle_mod, seed):
    rng = np.random.default_rng(10 + seed)
    X, B, A0 = random_triangle(rng, oracle_mod)
    x = X + 0.2 * rng.normal(size=(3, 3))
    K = oracle_mod.stretch_K(x.ravel(), B, A0, MU, LAM, exact=True)
    J = fd_jac(lambda y: oracle_mod.stretch_force(y, B, A0, MU, LAM), x.ravel(), 1e-6)
    np.testing.assert_allclose(K, -J, rtol=1e-6, atol=1e-6 * np.abs(K).max())


def test_stretch_solver_K_psd_and_exact_in_tension(oracle_mod):
    rng = np.random.default_rng(3)
    X = np.array([[0, 0, 0], [1.0, 0, 0], [0.3, 0.9, 0]])
    B, A0 = oracle_mod.rest_triangles(X, np.array([[0, 1, 2]]))
    # tension: scale up by 1.1 and rotate -> S is positive definite
    x = (1.1 * X) @ rand_rot(rng).T
    Ke = oracle_mod.stretch_K(x.ravel(), B[0], A0[0], MU, LAM, exact=True)
    Ks = oracle_mod.stretch_K(x.ravel(), B[0], A0[0], MU, LAM, exact=False)
    np.testing.assert_allclose(Ks, Ke, rtol=1e-13, atol=1e-13 * np.abs(Ke).max())
    # compression: exact K is indefinite, solver K is PSD
    x = 0.8 * X
    Ke = oracle_mod.stretch_K(x.ravel(), B[0], A0[0], MU, LAM, exact=True)
    Ks = oracle_mod.stretch_K(x.ravel(), B[0], A0[0], MU, LAM, exact=False)
    assert np.linalg.eigvalsh(Ke).min() < -1e-6 * np.abs(Ke).max()
    assert np.linalg.eigvalsh(Ks).min() > -1e-10 * np.abs(Ks).max()


@pytest.mark.parametrize("exact", [False, True])
def test_stretch_invariants(oracle_mod, exact):
    rng = np.random.default_rng(4)
    for _ in range(5):
        X, B, A0 = random_triangle(rng, oracle_mod)
        x = X + 0.2 * rng.normal(size=(3, 3))
        f = oracle_mod.stretch_force(x.ravel(), B, A0, MU, LAM).reshape(3, 3)
        scale = np.abs(f).max()
        np.testing.assert_allclose(f.sum(0), 0, atol=1e-12 * scale)
        np.testing.assert_allclose(np.cross(x, f).sum(0), 0, atol=1e-11 * scale)
        K = oracle_mod.stretch_K(x.ravel(), B, A0, MU, LAM, exact=exact)
        np.testing.assert_allclose(K, K.T, atol=1e-12 * np.abs(K).max())
        Kb = K.reshape(3, 3, 3, 3)  # (k, a, l, b)
        np.testing.assert_allclose(Kb.sum(axis=2), 0, atol=1e-12 * np.abs(K).max())
        R = rand_rot(rng)
        E1 = oracle_mod.stretch_energy(x.ravel(), B, A0, MU, LAM)
        E2 = oracle_mod.stretch_energy((x @ R.T + 3.0).ravel(), B, A0, MU, LAM)
        assert E2 == pytest.approx(E1, rel=1e-10)


def test_stretch_zero_force_at_rest(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(5):
        X, B, A0 = random_triangle(rng, oracle_mod)
        f = oracle_mod.stretch_force(X.ravel(), B, A0, MU, LAM)
        assert np.abs(f).max() < 1e-10 * MU
        assert oracle_mod.stretch_energy(X.ravel(), B, A0, MU, LAM) < 1e-20 * MU


# ---------------------------------------------------------------- bending
def folded_hinge(phi, jitter=None):
    """a=(0,0,0), b=(1,0,0), c=(0.3,1,0); d starts at (0.6,-1,0) and is rotated
    by phi about the edge direction (+x, right-hand rule)."""
    x = np.array([[0, 0, 0], [1.0, 0, 0], [0.3, 1.0, 0], [0.6, -math.cos(phi), -math.sin(phi)]])
    return x


@pytest.mark.parametrize("phi", [0.0, 0.3, -0.7, 1.2, 2.5, -3.0])
def test_hinge_angle_closed_form(oracle_mod, phi):
    # By hand: n1 = (0,0,1), n2 = (0,-sin phi, cos phi), n1.n2 = cos phi,
    # (n1 x n2).e = sin phi, so theta = phi.  Any rigid motion keeps it.
    x = folded_hinge(phi)
    assert oracle_mod.hinge_angle(x.ravel()) == pytest.approx(phi, abs=1e-14)
    R = rand_rot(np.random.default_rng(6))
    assert oracle_mod.hinge_angle((x @ R.T - 2.0).ravel()) == pytest.approx(phi, abs=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_hinge_grad_fd(oracle_mod, seed):
    rng = np.random.default_rng(20 + seed)
    x = folded_hinge(rng.uniform(-2, 2)) + 0.1 * rng.normal(size=(4, 3))
    g = oracle_mod.hinge_grad(x.ravel())
    gfd = fd_grad(lambda y: oracle_mod.hinge_angle(y), x.ravel(), 1e-6)
    np.testing.assert_allclose(g, gfd, rtol=1e-7, atol=1e-7 * np.abs(g).max())
    np.testing.assert_allclose(g.reshape(4, 3).sum(0), 0, atol=1e-13 * np.abs(g).max())


@pytest.mark.parametrize("seed", range(4))
def test_bend_force_and_K(oracle_mod, seed):
    rng = np.random.default_rng(30 + seed)
    x = folded_hinge(rng.uniform(-1.5, 1.5)) + 0.05 * rng.normal(size=(4, 3))
    ch, tbar = 2.7, 0.2
    f = oracle_mod.bend_force(x.ravel(), ch, tbar, KB)
    gE = fd_grad(lambda y: oracle_mod.bend_energy(y, ch, tbar, KB), x.ravel(), 1e-6)
    np.testing.assert_allclose(f, -gE, rtol=1e-6, atol=1e-6 * np.abs(f).max())
    Ke = oracle_mod.bend_K(x.ravel(), ch, tbar, KB, exact=True)
    J = fd_jac(lambda y: oracle_mod.bend_force(y, ch, tbar, KB), x.ravel(), 1e-6)
    np.testing.assert_allclose(Ke, -J, rtol=1e-5, atol=1e-5 * np.abs(Ke).max())
    f4 = f.reshape(4, 3)
    np.testing.assert_allclose(f4.sum(0), 0, atol=1e-12 * np.abs(f).max())
    np.testing.assert_allclose(np.cross(x, f4).sum(0), 0, atol=1e-12 * np.abs(f).max())


def test_bend_gauss_newton_is_hessian_at_rest_angle(oracle_mod):
    x = folded_hinge(0.4)
    tbar = oracle_mod.hinge_angle(x.ravel())
    Kgn = oracle_mod.bend_K(x.ravel(), 1.5, tbar, KB, exact=False)
    J = fd_jac(lambda y: oracle_mod.bend_force(y, 1.5, tbar, KB), x.ravel(), 1e-6)
    np.testing.assert_allclose(Kgn, -J, rtol=1e-6, atol=1e-6 * np.abs(Kgn).max())
    assert np.linalg.eigvalsh(Kgn).min() > -1e-12 * np.abs(Kgn).max()
    Kb = Kgn.reshape(4, 3, 4, 3)
    np.testing.assert_allclose(Kb.sum(axis=2), 0, atol=1e-13 * np.abs(Kgn).max())


def test_bend_zero_force_at_rest(oracle_mod):
    x = folded_hinge(0.0)
    assert np.abs(oracle_mod.bend_force(x.ravel(), 3.0, 0.0, KB)).max() == 0.0
    assert oracle_mod.bend_energy(x.ravel(), 3.0, 0.0, KB) == 0.0


def test_bend_degenerate_hinge_contributes_nothing(oracle_mod):
    x = folded_hinge(0.3)
    x[2] = x[0] + 1e-14 * (x[1] - x[0])  # collapse the c wing onto the edge
    assert np.all(oracle_mod.bend_force(x.ravel(), 3.0, 0.0, KB) == 0.0)
    assert np.all(oracle_mod.bend_K(x.ravel(), 3.0, 0.0, KB) == 0.0)


def test_hinge_rest_coefficient_closed_form(oracle_mod):
    # unit right triangles sharing the edge (0,0)-(1,1)... use edge a-b of length
    # sqrt(2), wings at (1,0) and (0,1): areas 1/2 each -> c_h = 3*2/1 = 6.
    X = np.array([[0, 0, 0], [1.0, 1.0, 0], [0, 1.0, 0], [1.0, 0, 0]], dtype=float)
    ch, tb = oracle_mod.rest_hinges(X, np.array([[0, 1, 2, 3]]))
    assert ch[0] == pytest.approx(6.0, rel=1e-14)
    assert tb[0] == pytest.approx(0.0, abs=1e-15)


# ------------------------------------------------- PSD part of the stress
def _deformed_unit_triangle(S, R):
    """Corners of the unit right triangle (rest legs along x and y, so B = I
    and A0 = 1/2) deformed so that its StVK stress is the given symmetric S,
    then rotated by R.  The strain follows from inverting S = 2 mu G + lam
    tr(G) I; the in-plane deformation is the symmetric square root of
    C = I + 2 G (taken with eigh)."""
    trG = np.trace(S) / (2 * MU + 2 * LAM)
    G = (S - LAM * trG * np.eye(2)) / (2 * MU)
    w, V = np.linalg.eigh(np.eye(2) + 2 * G)
    assert w.min() > 0
    F2 = V @ np.diag(np.sqrt(w)) @ V.T
    rest2 = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    x = np.zeros((3, 3))
    x[:, :2] = rest2 @ F2.T
    return x @ R.T


def _psd_correction_from_K(oracle_mod, x):
    """S+ - S read off the oracle's stiffness: solver-mode K minus exact K is
    A0 (beta_k^T (S+ - S) beta_l) I_3 per block (k, l); with beta_1 = (1, 0)
    and beta_2 = (0, 1) the blocks (1,1), (1,2), (2,2) give the three entries.
    Also checks that every block of the difference is a multiple of I_3."""
    X = np.array([[0, 0, 0], [1.0, 0, 0], [0, 1.0, 0]])
    B, A0 = oracle_mod.rest_triangles(X, np.array([[0, 1, 2]]))
    np.testing.assert_allclose(B[0], [1, 0, 0, 1], atol=1e-15)
    Ks = oracle_mod.stretch_K(x.ravel(), B[0], A0[0], MU, LAM, exact=False)
    Ke = oracle_mod.stretch_K(x.ravel(), B[0], A0[0], MU, LAM, exact=True)
    D = (Ks - Ke).reshape(3, 3, 3, 3) / A0[0]          # (k, a, l, b)
    scale = np.abs(Ke).max()
    for k in range(3):
        for l in range(3):
            blk = D[k, :, l, :]
            np.testing.assert_allclose(blk, blk[0, 0] * np.eye(3), atol=1e-12 * scale)
    return np.array([[D[1, 0, 1, 0], D[1, 0, 2, 0]], [D[2, 0, 1, 0], D[2, 0, 2, 0]]])


def _psd_by_eigh(S):
    w, V = np.linalg.eigh(S)
    return V @ np.diag(np.maximum(w, 0.0)) @ V.T


@pytest.mark.parametrize("seed", range(8))
def test_stretch_psd_projection_matches_eigh_mixed_sign(oracle_mod, seed):
    """Solver Jacobian of Eq. 3 (Sec. 2.5): the geometric-stiffness term uses
    the positive part of the 2x2 stress.  For stresses with one positive and
    one negative eigenvalue (the indefinite case, in any orientation), the
    S+ that the oracle applies equals numpy's eigendecomposition with the
    negative eigenvalue set to zero."""
    rng = np.random.default_rng(700 + seed)
    ang = rng.uniform(0, np.pi)
    Q = np.array([[np.cos(ang), -np.sin(ang)], [np.sin(ang), np.cos(ang)]])
    s_pos, s_neg = rng.uniform(1.0, 40.0), -rng.uniform(1.0, 40.0)
    S = Q @ np.diag([s_pos, s_neg]) @ Q.T
    x = _deformed_unit_triangle(S, rand_rot(rng))
    got = _psd_correction_from_K(oracle_mod, x)
    want = _psd_by_eigh(S) - S
    np.testing.assert_allclose(got, want, atol=1e-9 * np.abs(S).max())


@pytest.mark.parametrize("ang_deg", [0.0, 30.0, 90.0, 135.0])
def test_stretch_psd_projection_stretched_x_compressed_y(oracle_mod, ang_deg):
    """A triangle stretched by 2% along one in-plane direction and compressed
    by 1% across it (direction at ang_deg to the first leg; 0 and 90 degrees
    take the diagonal-stress branch, the others the general one): the
    oracle's S+ - S equals the eigh projection of the stress computed from
    that deformation, and is nonzero."""
    a = np.deg2rad(ang_deg)
    d = np.array([np.cos(a), np.sin(a)])
    n = np.array([-d[1], d[0]])
    F2 = 1.02 * np.outer(d, d) + 0.99 * np.outer(n, n)
    G = 0.5 * (F2.T @ F2 - np.eye(2))
    S = 2 * MU * G + LAM * np.trace(G) * np.eye(2)
    w = np.linalg.eigvalsh(S)
    assert w[0] < 0 < w[1]
    rest2 = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    x = np.zeros((3, 3))
    x[:, :2] = rest2 @ F2.T
    got = _psd_correction_from_K(oracle_mod, x)
    want = _psd_by_eigh(S) - S
    assert np.abs(want).max() > 1.0
    np.testing.assert_allclose(got, want, atol=1e-9 * np.abs(S).max())


def test_stretch_psd_projection_definite_cases(oracle_mod):
    """Both eigenvalues positive: no change (S+ = S).  Both negative: the
    whole stress term is dropped (S+ = 0)."""
    rng = np.random.default_rng(77)
    for sgn in (1.0, -1.0):
        ang = rng.uniform(0, np.pi)
        Q = np.array([[np.cos(ang), -np.sin(ang)], [np.sin(ang), np.cos(ang)]])
        S = sgn * Q @ np.diag([rng.uniform(1, 30), rng.uniform(1, 30)]) @ Q.T
        got = _psd_correction_from_K(oracle_mod, _deformed_unit_triangle(S, rand_rot(rng)))
        want = np.zeros((2, 2)) if sgn > 0 else -S
        np.testing.assert_allclose(got, want, atol=1e-9 * np.abs(S).max())
