"""GPU parity of the learned warm start (features, BF16-MFMA forward and
backward, Adam, learned CG start) against the FP64 oracle in oracle/mlp.py,
through the C ABI.

Bars: features and forward outputs within bf16 rounding of the oracle's
values computed with the same rounding points; per-tensor gradients to 3e-2
relative (bf16 operands, FP32 vs FP64 accumulation); the learned start
still solves Eq. 3 to the tolerance through the oracle's matrix."""
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


@pytest.fixture(scope="module")
def M():
    from oracle import mlp
    return mlp


def mean_edge(c):
    e = 0.0
    for k in range(3):
        a, b = c.tris[:, k], c.tris[:, (k + 1) % 3]
        e += np.linalg.norm(c.rest[a] - c.rest[b], axis=1).sum()
    return e / (3 * c.tris.shape[0])


def random_params(M, seed):
    p = M.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p[3][0] *= 30.0
    for k in range(4):
        p[k][1] = 0.05 * rng.normal(size=p[k][1].shape)
    return p


def setup_case(torch, B, oracle_mod, M, nx=29, ny=23, seed=3):
    c = sheet(nx, ny, seed=seed, flips=0.1)      # 667 vertices: 42 tiles, ragged last tile
    P = oracle_mod.Problem.from_cloth(c)
    v = random_velocity(c, 0.05, seed=seed)
    A = P.assemble(c.x0, v)
    dvp = 0.01 * np.random.default_rng(seed).normal(size=c.rest.shape)
    dvp[c.pinned == 1] = 0
    ctx = B.Context.from_cloth(c)
    x_d, v_d, dvp_d = to_dev(torch, c.x0), to_dev(torch, v), to_dev(torch, dvp)
    b_d = ctx.cloth_assemble(x_d, v_d, "f32")
    ell = mean_edge(c)
    X = M.features(P.rowptr, P.colidx, c.x0, v, A.b, A.diag, c.mass, c.pinned, dvp, ell, c.h)
    return c, P, A, v, dvp, ctx, (x_d, v_d, dvp_d, b_d), ell, X


def test_mfma_lane_layout(torch, B):
    from paper_2008_00409_amd import meshgen as mg
    c = mg.config_tiny()
    ctx = B.Context.from_cloth(c)
    try:
        out = ctx.mfma_probe()
        idx = np.arange(16)
        a = idx[:, None] * 16 + idx[None, :]
        np.testing.assert_array_equal(out[0], a)
        np.testing.assert_array_equal(out[1], a)
        # 16 x 16 x 32: the two K tiles of A come back apart
        np.testing.assert_array_equal(out[2], a)
        np.testing.assert_array_equal(out[3], 256 - a)
    finally:
        ctx.close()


def test_features_match_oracle(torch, B, oracle_mod, M):
    c, P, A, v, dvp, ctx, (x_d, v_d, dvp_d, b_d), ell, X = setup_case(torch, B, oracle_mod, M)
    try:
        F = ctx.ws_features(x_d, v_d, b_d, dvp_d).cpu().numpy().astype(np.uint16)
        got = (F.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        assert np.all(got[:, 27:] == 0)
        want = M.bf16_round(X)
        # within one bf16 ulp (values computed in FP64 on both sides, summation order differs)
        ulp = np.maximum(np.abs(want), 1e-30) * 2.0 ** -7
        assert np.all(np.abs(got[:, :27] - want) <= ulp + 1e-30)
    finally:
        ctx.close()


def test_forward_matches_oracle(torch, B, oracle_mod, M):
    c, P, A, v, dvp, ctx, (x_d, v_d, dvp_d, b_d), ell, X = setup_case(torch, B, oracle_mod, M)
    try:
        params = random_params(M, 7)
        ctx.ws_set_params(M.flatten(params))
        dv0 = ctx.ws_predict(x_d, v_d, b_d, dvp_d).cpu().numpy()
        y, hs = M.forward([[M.bf16_round(W), cb] for W, cb in params], X, bf16=True)
        want = M.start_from_output(y, dvp, c.pinned, ell / c.h)
        corr_g = (dv0 - dvp)[c.pinned == 0]
        corr_w = (want - dvp)[c.pinned == 0]
        err = np.linalg.norm(corr_g - corr_w) / np.linalg.norm(corr_w)
        assert err < 2e-2, err
        assert np.all(dv0[c.pinned == 1] == 0)
        # round trip of the parameters
        np.testing.assert_array_equal(ctx.ws_get_params(), M.flatten(params).astype(np.float32))
    finally:
        ctx.close()


def test_gradient_matches_oracle(torch, B, oracle_mod, M):
    c, P, A, v, dvp, ctx, (x_d, v_d, dvp_d, b_d), ell, X = setup_case(torch, B, oracle_mod, M)
    try:
        params = random_params(M, 11)
        ctx.ws_set_params(M.flatten(params))
        g_gpu, loss_gpu = ctx.ws_gradient(x_d, v_d, b_d, dvp_d)
        pb = [[M.bf16_round(W), cb] for W, cb in params]
        y, hs = M.forward(pb, X, bf16=True)
        sv = ell / c.h
        dv0 = M.start_from_output(y, dvp, c.pinned, sv)
        L, gy = M.energy_loss_grad(lambda z: P.spmv(A, z), A.b, A.diag, dv0, c.pinned, sv)
        grads = M.backward(pb, X, hs, gy, bf16=True)
        assert loss_gpu == pytest.approx(L, rel=2e-2, abs=1e-3 * abs(L))
        g_or = M.flatten(grads)
        o = 0
        for a, bdim in M.SHAPES:
            for n in (a * bdim, bdim):
                seg_g, seg_o = g_gpu[o:o + n], g_or[o:o + n]
                rel = np.linalg.norm(seg_g - seg_o) / max(np.linalg.norm(seg_o), 1e-30)
                assert rel < 3e-2, (o, n, rel)
                o += n
    finally:
        ctx.close()


def test_training_lowers_the_loss_and_learned_start_solves(torch, B, oracle_mod, M):
    c, P, A, v, dvp, ctx, (x_d, v_d, dvp_d, b_d), ell, X = setup_case(torch, B, oracle_mod, M)
    try:
        ctx.ws_set_params(M.flatten(M.init_params(3)))
        losses = [ctx.ws_train_step(x_d, v_d, b_d, dvp_d, lr=3e-3) for _ in range(60)]
        assert losses[-1] < losses[0] - 0.05 * abs(losses[0]), (losses[0], losses[-1])
        # learned start through cloth_pcg_solve: dv holds the previous increment on entry
        dv = dvp_d.clone()
        dv, info = ctx.cloth_pcg_solve(b_d, dv=dv, tol=1e-7, warm="learned")
        assert info["warm_used"] in (1, 2)
        assert P.residual(A, dv.cpu().numpy()) <= 1e-7 * (1 + 1e-6)
    finally:
        ctx.close()


def test_learned_start_matches_oracle_line_search(torch, B, oracle_mod, M):
    """pc_ws_start: previous increment plus the A-norm-optimal step along the
    network's correction, against the oracle's line search on the oracle's
    forward pass (bf16 rounding points) and FP64 matrix."""
    c, P, A, v, dvp, ctx, (x_d, v_d, dvp_d, b_d), ell, X = setup_case(torch, B, oracle_mod, M)
    try:
        params = random_params(M, 19)
        ctx.ws_set_params(M.flatten(params))
        start, g = ctx.ws_start(x_d, v_d, b_d, dvp_d)
        start = start.cpu().numpy()
        y, _ = M.forward([[M.bf16_round(W), cb] for W, cb in params], X, bf16=True)
        u = M.start_from_output(y, np.zeros_like(dvp), c.pinned, ell / c.h)
        want, g_want = M.line_search_start(lambda z: P.spmv(A, z), A.b, dvp, u)
        assert g == pytest.approx(g_want, rel=3e-2, abs=1e-3 * abs(g_want))
        corr_g, corr_w = (start - dvp)[c.pinned == 0], (want - dvp)[c.pinned == 0]
        assert np.linalg.norm(corr_g - corr_w) <= 3e-2 * np.linalg.norm(corr_w) + 1e-30
        # never worse than the previous increment in the A-norm (oracle matrix)
        E = lambda z: 0.5 * float((z * P.spmv(A, z)).sum()) - float((A.b * z).sum())
        assert E(start) <= E(dvp) + 1e-12 * abs(E(dvp))
    finally:
        ctx.close()


def test_trained_network_gain_on_held_out_step(torch, B, oracle_mod):
    """What the trained network adds over the method without it: the network
    is trained online on the first 20 steps of a 96 x 96 bumped sheet (3 Adam
    steps per step, the solver advancing with the learned start), then the
    next step's system is solved from the zero start, the previous increment
    and the learned start.  The learned start lowers the A-norm energy of the
    previous increment (through the oracle's matrix), and needs no more CG
    iterations than the zero start; the three counts are printed."""
    from paper_2008_00409_amd import meshgen as mg
    c = mg.config_grid(96, seed=2096, h=1.0 / 200)
    ctx = B.Context.from_cloth(c)
    try:
        ctx.ws_set_params(B.Context.ws_init_params(0))
        x = to_dev(torch, c.x0)
        v = torch.zeros_like(x)
        dvp = torch.zeros_like(x)
        pin = torch.from_numpy(c.pinned.astype(bool)).cuda()
        for _ in range(20):
            b = ctx.cloth_assemble(x, v, "f32")
            for _ in range(3):
                ctx.ws_train_step(x, v, b, dvp, lr=1e-3)
            dv, _ = ctx.cloth_pcg_solve(b, dv=dvp.clone(), tol=1e-6, warm="learned")
            v += dv
            v[pin] = 0
            x += c.h * v
            dvp = dv
        b = ctx.cloth_assemble(x, v, "f32")
        start, _g = ctx.ws_start(x, v, b, dvp)
        iters = {}
        for mode in ("zero", "prev", "learned"):
            dv0 = torch.zeros_like(x) if mode == "zero" else dvp.clone()
            _, info = ctx.cloth_pcg_solve(b, dv=dv0, tol=1e-6, warm=mode)
            assert info["rel_res_true"] <= 1e-6
            iters[mode] = info["iters"]
        P = oracle_mod.Problem.from_cloth(c)
        A = P.assemble(x.cpu().numpy(), v.cpu().numpy())
    finally:
        ctx.close()
    E = lambda z: 0.5 * float((z * P.spmv(A, z)).sum()) - float((A.b * z).sum())
    e_prev, e_learned = E(dvp.cpu().numpy()), E(start.cpu().numpy())
    print(f"held-out step: CG iterations zero {iters['zero']}, previous {iters['prev']}, "
          f"learned {iters['learned']}; energy previous {e_prev:.6e}, learned {e_learned:.6e}")
    assert e_learned < e_prev
    assert iters["learned"] <= iters["zero"]


def test_training_steps_match_oracle_adam(torch, B, oracle_mod, M):
    """k calls of pc_ws_train_step against k rounds of the oracle's forward
    pass, backward pass and Adam step (bias-corrected moments, Kingma and Ba
    2015), from the same parameters on the same assembled system of Eq. 3:

    1. before every step, the gradient the step applies (pc_ws_gradient at
       the GPU's current parameters) matches the oracle's gradient at those
       parameters per tensor, at the gradient bar above;
    2. after every step, the GPU's FP32 parameters equal the oracle's Adam
       driven by those same gradients, element by element to FP32 rounding
       of the update: this pins the first and second moments and the bias
       correction 1 - beta^t at every t (a correction frozen at t = 1, or
       one moment's factor swapped, moves some update by far more than the
       bar);
    3. after k steps, the GPU's parameter change matches the change of the
       oracle's own k-step trajectory (its gradients, its Adam) per tensor.
       Adam normalises each element's update to about lr, so an element whose
       gradient is near zero could take either sign on the two sides; with
       gradients within 2e-4 of the oracle's (measured) the change agrees to
       about 2e-3 per tensor, and the bar is 5e-2.  The figures are printed."""
    c, P, A, v, dvp, ctx, (x_d, v_d, dvp_d, b_d), ell, X = setup_case(torch, B, oracle_mod, M)
    k_steps, lr = 4, 2e-3
    sv = ell / c.h
    apply_A = lambda z: P.spmv(A, z)

    def oracle_grad(flat):
        pb = [[M.bf16_round(W), cb] for W, cb in M.unflatten(flat)]
        y, hs = M.forward(pb, X, bf16=True)
        dv0 = M.start_from_output(y, dvp, c.pinned, sv)
        L, gy = M.energy_loss_grad(apply_A, A.b, A.diag, dv0, c.pinned, sv)
        return M.flatten(M.backward(pb, X, hs, gy, bf16=True)), L

    def segments():
        o = 0
        for a, bdim in M.SHAPES:
            for n in (a * bdim, bdim):
                yield o, n
                o += n

    try:
        ctx.ws_set_params(M.flatten(random_params(M, 23)))
        p0 = ctx.ws_get_params().astype(np.float64)     # the FP32 values both sides start from
        p_fed = M.unflatten(p0)          # oracle Adam driven by the GPU's gradients
        st_fed, st_own = {}, {}
        p_own = M.unflatten(p0)          # oracle's own trajectory
        worst_grad, worst_step = 0.0, 0.0
        for t in range(1, k_steps + 1):
            p_gpu_before = ctx.ws_get_params().astype(np.float64)
            g_gpu, loss_gpu = ctx.ws_gradient(x_d, v_d, b_d, dvp_d)
            g_or, L_or = oracle_grad(p_gpu_before)
            assert loss_gpu == pytest.approx(L_or, rel=2e-2, abs=1e-3 * abs(L_or))
            for o, n in segments():
                rel = np.linalg.norm(g_gpu[o:o + n] - g_or[o:o + n]) / max(np.linalg.norm(g_or[o:o + n]), 1e-30)
                worst_grad = max(worst_grad, rel)
                assert rel < 3e-2, (t, o, n, rel)
            ctx.ws_train_step(x_d, v_d, b_d, dvp_d, lr=lr, want_loss=False)
            p_gpu = ctx.ws_get_params().astype(np.float64)
            M.adam_step(p_fed, M.unflatten(g_gpu.astype(np.float64)), st_fed, lr=lr)
            want = M.flatten(p_fed)
            # FP32 arithmetic of the update and FP32 storage of the weights, per step taken
            bar = t * (1e-5 * lr + 2.4e-7 * np.abs(want))
            err = np.abs(p_gpu - want)
            worst_step = max(worst_step, float(np.max(err / (1e-5 * lr + 2.4e-7 * np.abs(want)))) / t)
            assert np.all(err <= bar), (t, int(np.argmax(err - bar)), float(np.max(err)))
            # the step moved the weights: the comparison is not vacuous
            assert np.linalg.norm(p_gpu - p_gpu_before) > 0.3 * lr * np.sqrt(np.count_nonzero(g_gpu))
            g_own, _ = oracle_grad(M.flatten(p_own))
            M.adam_step(p_own, M.unflatten(g_own), st_own, lr=lr)
        d_gpu = ctx.ws_get_params().astype(np.float64) - p0
        d_own = M.flatten(p_own) - p0
        rels = []
        for o, n in segments():
            den = np.linalg.norm(d_own[o:o + n])
            if den == 0.0:
                assert np.linalg.norm(d_gpu[o:o + n]) == 0.0
                continue
            rels.append(np.linalg.norm(d_gpu[o:o + n] - d_own[o:o + n]) / den)
        print(f"adam parity: worst per-tensor gradient error {worst_grad:.2e}; worst element error "
              f"{worst_step:.3f} of the FP32 bar; k-step change against the oracle's own trajectory, per tensor: "
              + " ".join(f"{r:.3f}" for r in rels))
        assert max(rels) < 5e-2, rels
    finally:
        ctx.close()
