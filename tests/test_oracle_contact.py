"""Pins of the oracle's proximity (contact) elements and of the assembly with
contacts: forces against central differences of the energy, stiffness
against differences of the forces, a vertex-face pair written out by hand,
the inactive side of the thickness, translation invariance, and the
assembled system against a dense scatter of every element written out in
Python."""
import numpy as np
import pytest

from paper_2008_00409_amd import meshgen as mg


def random_contact(rng, active=True, eta=0.002):
    x12 = rng.normal(size=12) * 0.01
    s, t = rng.uniform(0.1, 0.9, 2)
    c = np.array([1 - s, s, -(1 - t), -t])            # edge-edge weights, sum zero
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    g = float(n @ (c @ x12.reshape(4, 3)))
    # move the first vertex along n so the gap is 0.4 eta (active) or 1.6 eta (inactive)
    want = 0.4 * eta if active else 1.6 * eta
    x12[:3] += (want - g) / c[0] * n
    return x12, c, n


def test_force_is_minus_energy_gradient(oracle_mod):
    rng = np.random.default_rng(0)
    x12, c, n = random_contact(rng)
    f = oracle_mod.contact_force(x12, c, n, 0.002, 800.0)
    step = 1e-9
    for j in range(12):
        xp, xm = x12.copy(), x12.copy()
        xp[j] += step
        xm[j] -= step
        fd = -(oracle_mod.contact_energy(xp, c, n, 0.002, 800.0) -
               oracle_mod.contact_energy(xm, c, n, 0.002, 800.0)) / (2 * step)
        assert f[j] == pytest.approx(fd, rel=1e-6, abs=1e-12)


def test_stiffness_is_minus_force_jacobian_and_psd(oracle_mod):
    rng = np.random.default_rng(1)
    x12, c, n = random_contact(rng)
    K = oracle_mod.contact_K(x12, c, n, 0.002, 800.0)
    step = 1e-8
    for j in range(12):
        xp, xm = x12.copy(), x12.copy()
        xp[j] += step
        xm[j] -= step
        col = -(oracle_mod.contact_force(xp, c, n, 0.002, 800.0) -
                oracle_mod.contact_force(xm, c, n, 0.002, 800.0)) / (2 * step)
        np.testing.assert_allclose(K[:, j], col, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(K, K.T, rtol=0, atol=1e-14 * np.abs(K).max())
    assert np.linalg.eigvalsh(K).min() > -1e-9 * np.abs(K).max()
    # block rows sum to zero (the weights do): translation invariance
    blocks = K.reshape(4, 3, 4, 3).sum(axis=2)
    assert np.abs(blocks).max() < 1e-12 * np.abs(K).max()


def test_vertex_face_closed_form(oracle_mod):
    # triangle a = 0, b = e_x, c = e_y in the plane z = 0; vertex p above the
    # point with barycentric weights (0.5, 0.2, 0.3), at height z
    eta, kc, z = 0.002, 1000.0, 0.0008
    xa, xb, xc = np.zeros(3), np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    xp = np.array([0.2, 0.3, z])
    x12 = np.concatenate([xp, xa, xb, xc])
    c = np.array([1.0, -0.5, -0.2, -0.3])
    n = np.array([0, 0, 1.0])
    assert oracle_mod.contact_energy(x12, c, n, eta, kc) == pytest.approx(0.5 * kc * (eta - z) ** 2, rel=1e-12)
    f = oracle_mod.contact_force(x12, c, n, eta, kc).reshape(4, 3)
    m = kc * (eta - z)
    np.testing.assert_allclose(f[0], [0, 0, m], rtol=1e-12)
    np.testing.assert_allclose(f[1:, 2], [-0.5 * m, -0.2 * m, -0.3 * m], rtol=1e-12)
    np.testing.assert_allclose(f[:, :2], 0.0, atol=0)
    K = oracle_mod.contact_K(x12, c, n, eta, kc)
    assert K[2, 2] == pytest.approx(kc)              # p, z-z
    assert K[2, 5] == pytest.approx(-0.5 * kc)       # p-a, z-z
    assert K[8, 11] == pytest.approx(0.2 * 0.3 * kc)  # b-c, z-z
    # beyond the thickness: nothing
    x12[2] = 1.5 * eta
    assert oracle_mod.contact_energy(x12, c, n, eta, kc) == 0.0
    assert np.all(oracle_mod.contact_force(x12, c, n, eta, kc) == 0.0)
    assert np.all(oracle_mod.contact_K(x12, c, n, eta, kc) == 0.0)


def two_sheets(oracle_mod, n=9):
    c, cs = mg.config_contact(n, n - 1)
    return c, cs


def dense_with_contacts(oracle_mod, P, C, x, mat):
    import test_oracle_system as TS
    TS.oracle_mod_ref = oracle_mod
    K = TS.dense_scatter(P, x, mat)
    for e in range(C.n):
        v = C.verts[e]
        Ke = oracle_mod.contact_K(x[v].ravel(), C.weights[e], C.normals[e], C.eta, C.kc)
        for k in range(4):
            for l in range(4):
                K[3 * v[k]:3 * v[k] + 3, 3 * v[l]:3 * v[l] + 3] += Ke[3 * k:3 * k + 3, 3 * l:3 * l + 3]
    return K


@pytest.mark.parametrize("rhs_mode", [0, 1])
def test_assembly_with_contacts_matches_dense_definition(oracle_mod, rhs_mode):
    import test_oracle_system as TS
    TS.oracle_mod_ref = oracle_mod
    c, cs = two_sheets(oracle_mod)
    assert cs.n > 20
    rng = np.random.default_rng(7)
    x = c.x0 + 0.0002 * rng.normal(size=c.x0.shape)
    v = 0.05 * rng.normal(size=c.x0.shape)
    v[c.pinned == 1] = 0
    mat = oracle_mod.Material(rhs_mode=rhs_mode)
    P = oracle_mod.Problem.from_cloth(c, mat)
    C = oracle_mod.Contacts(cs.verts, cs.weights, cs.normals, cs.eta, cs.kc)
    P.set_contacts(C)
    # the pattern holds every contact pair
    pairs = {(int(i), int(j)) for i in range(P.nv) for j in P.colidx[P.rowptr[i]:P.rowptr[i + 1]]}
    for e in range(cs.n):
        for k in range(4):
            for l in range(4):
                assert (int(cs.verts[e, k]), int(cs.verts[e, l])) in pairs
    A = P.assemble(x, v)
    K = dense_with_contacts(oracle_mod, P, C, x, mat)
    h = c.h
    Aref = np.diag(np.repeat(c.mass, 3)) + h * h * K
    f = TS.total_force_py(P, x + (h * v if rhs_mode == 0 else 0), mat)
    y = x + (h * v if rhs_mode == 0 else 0)
    for e in range(cs.n):
        vv = cs.verts[e]
        f[vv] += oracle_mod.contact_force(y[vv].ravel(), cs.weights[e], cs.normals[e], cs.eta,
                                          cs.kc).reshape(4, 3)
    bref = h * (f.ravel() - (0.0 if rhs_mode == 0 else h) * K @ v.ravel())
    pin3 = np.repeat(c.pinned, 3).astype(bool)
    Aref[pin3, :] = 0
    Aref[:, pin3] = 0
    Aref[pin3, pin3] = np.repeat(c.mass, 3)[pin3]
    bref[pin3] = 0
    np.testing.assert_allclose(A.dense(), Aref, rtol=0, atol=1e-12 * np.abs(Aref).max())
    np.testing.assert_allclose(A.b.ravel(), bref, rtol=0, atol=1e-12 * np.abs(bref).max())
    # still symmetric positive definite, and the contacts changed the system
    Ad = A.dense()
    np.testing.assert_allclose(Ad, Ad.T, rtol=0, atol=1e-14 * np.abs(Ad).max())
    np.linalg.cholesky(Ad)
    P.set_contacts(None)
    A0 = P.assemble(x, v)
    assert A0.colidx.size < A.colidx.size


def test_contacts_push_sheets_apart(oracle_mod):
    """One step with the upper sheet inside the thickness: the relative
    normal velocity of each contact pair becomes separating."""
    c, cs = two_sheets(oracle_mod, 11)
    P = oracle_mod.Problem.from_cloth(c, oracle_mod.Material())
    P.set_contacts(oracle_mod.Contacts(cs.verts, cs.weights, cs.normals, cs.eta, cs.kc))
    x1, v1, dv, info = P.step(c.x0, c.v0, tol=1e-10)
    assert info["converged"]
    vn = np.einsum("na,na->n", cs.normals, np.einsum("nk,nka->na", cs.weights, v1[cs.verts]))
    free = c.pinned[cs.verts].max(axis=1) == 0
    assert np.all(vn[free] > 0.0)
