"""FP64 oracle of the learned CG warm start.  TEST INFRASTRUCTURE ONLY.

A per-vertex MLP over one-ring features predicts a correction to the
previous step's velocity increment; the prediction is the start of the CG
solve of Eq. 3 (paper Sec. 2.5).  Definitions (the HIP kernels implement the
same, independently):

* s_v = l / h with l the mean rest edge length and h the time step;
  N(i) = the block columns of row i other than i.
* 27 features per vertex, in this order:
   0-2  v_i / s_v
   3-5  (b_i / m_i) / s_v
   6-8  dv_prev_i / s_v
   9-11 mean_{j in N(i)} dv_prev_j / s_v
  12-14 (b_i / diag(A)_i) / s_v            (component-wise Jacobi estimate)
  15-17 (mean_j b_j/m_j - b_i/m_i) / s_v
  18-20 (mean_j v_j - v_i) / s_v
  21-23 (mean_j x_j - x_i) / l
  24    pinned flag
  25    log10(mean_a diag(A)_ia / m_i)
  26    |N(i)| / 12
* MLP 27 -> 64 -> 64 -> 64 -> 3, ReLU on the hidden layers:
  h_k = relu(h_{k-1} W_k + c_k), y = h_3 W_4 + c_4 (W_k stored in x out).
* Start: dv0_i = dv_prev_i + s_v y_i for free vertices, 0 for pinned ones
  (the training target); as the CG start the correction u = s_v y is added
  with the step g that minimises the A-norm error along u (line_search_start).
* Loss (energy norm of the start's error, scaled per system):
  L = (0.5 dv0^T A dv0 - b^T dv0) / E0,  E0 = b^T D^-1 b.
  dL/dy_i = s_v (A dv0 - b)_i / E0 for free vertices, 0 otherwise.
* Adam (beta1 0.9, beta2 0.999, eps 1e-8).
* Optional bf16 rounding at the kernels' rounding points: the features,
  the weights used in products, and each hidden activation after ReLU.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 27, 64, 3
SHAPES = [(IN, HID), (HID, HID), (HID, HID), (HID, OUT)]
N_PARAMS = sum(a * b + b for a, b in SHAPES)


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return out.reshape(np.shape(a))


def init_params(seed=0):
    """He-normal weights, zero biases, last layer scaled by 1e-2 so that the
    untrained start equals the previous step's increment."""
    rng = np.random.default_rng(seed)
    params = []
    for k, (a, b) in enumerate(SHAPES):
        W = rng.normal(size=(a, b)) * np.sqrt(2.0 / a)
        if k == 3:
            W *= 1e-2
        params.append([W, np.zeros(b)])
    return params


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), c]) for W, c in params])


def unflatten(vec):
    params, o = [], 0
    for a, b in SHAPES:
        W = vec[o:o + a * b].reshape(a, b)
        o += a * b
        c = vec[o:o + b]
        o += b
        params.append([W.copy(), c.copy()])
    return params


def neighbour_lists(rowptr, colidx):
    nv = rowptr.size - 1
    rows = np.repeat(np.arange(nv), np.diff(rowptr))
    keep = colidx != rows
    cnt = np.bincount(rows[keep], minlength=nv)
    return rows[keep], colidx[keep], cnt


def nb_mean(rows, cols, cnt, a):
    s = np.zeros_like(a)
    np.add.at(s, rows, a[cols])
    return s / np.maximum(cnt, 1)[:, None]


def features(rowptr, colidx, x, v, b, diag, mass, pinned, dv_prev, ell, h):
    """The 27 features above (float64, shape (nv, 27))."""
    sv = ell / h
    rows, cols, cnt = neighbour_lists(rowptr, colidx)
    m = mass[:, None]
    bm = b / m
    F = [v / sv, bm / sv, dv_prev / sv, nb_mean(rows, cols, cnt, dv_prev) / sv, (b / diag) / sv,
         (nb_mean(rows, cols, cnt, bm) - bm) / sv, (nb_mean(rows, cols, cnt, v) - v) / sv,
         (nb_mean(rows, cols, cnt, x) - x) / ell, pinned[:, None].astype(np.float64),
         np.log10(diag.mean(axis=1, keepdims=True) / m), (cnt / 12.0)[:, None]]
    return np.concatenate(F, axis=1)


def forward(params, X, bf16=False):
    """Returns (y, hidden activations [h1, h2, h3])."""
    r = bf16_round if bf16 else (lambda a: a)
    h = r(X)
    hs = []
    for k, (W, c) in enumerate(params):
        z = h @ r(W) + c
        if k < 3:
            h = r(np.maximum(z, 0.0))
            hs.append(h)
        else:
            h = z
    return h, hs


def backward(params, X, hs, gy, bf16=False):
    """Gradients of sum(gy * y) with respect to every weight and bias."""
    r = bf16_round if bf16 else (lambda a: a)
    inputs = [r(X)] + hs
    grads = [None] * 4
    g = r(gy)
    for k in range(3, -1, -1):
        W, c = params[k]
        grads[k] = [inputs[k].T @ g, g.sum(axis=0)]
        if k > 0:
            g = (g @ r(W).T) * (hs[k - 1] > 0)
            if bf16:
                g = r(g)
    return grads


def start_from_output(y, dv_prev, pinned, sv):
    dv0 = dv_prev + sv * y
    dv0[pinned == 1] = 0.0
    return dv0


def energy_loss_grad(apply_A, b, diag, dv0, pinned, sv):
    """(L, dL/dy) of the scaled energy loss for the start dv0."""
    E0 = float((b * b / diag).sum())
    Ad = apply_A(dv0)
    L = (0.5 * float((dv0 * Ad).sum()) - float((b * dv0).sum())) / E0
    gy = sv * (Ad - b) / E0
    gy[pinned == 1] = 0.0
    return L, gy


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    if "m" not in state:
        state["m"] = [[np.zeros_like(W), np.zeros_like(c)] for W, c in params]
        state["v"] = [[np.zeros_like(W), np.zeros_like(c)] for W, c in params]
    for k in range(4):
        for q in range(2):
            g = grads[k][q]
            state["m"][k][q] = b1 * state["m"][k][q] + (1 - b1) * g
            state["v"][k][q] = b2 * state["v"][k][q] + (1 - b2) * g * g
            mh = state["m"][k][q] / (1 - b1 ** t)
            vh = state["v"][k][q] / (1 - b2 ** t)
            params[k][q] = params[k][q] - lr * mh / (np.sqrt(vh) + eps)
    return params


def line_search_start(apply_A, b, dv_prev, u):
    """Start dv_prev + g u with g = u.(b - A dv_prev) / u.A u, the minimiser of
    the A-norm error along u (g = 0 when u.A u <= 0).  Returns (start, g)."""
    Au = apply_A(u)
    den = float((u * Au).sum())
    num = float((u * b).sum()) - float((u * apply_A(dv_prev)).sum())
    g = num / den if den > 0 and np.isfinite(num / den) else 0.0
    return dv_prev + g * u, g


def safeguard_scale(apply_A, b, dv0):
    """c = dv0.b / dv0.A dv0: the factor minimising the A-norm error of c dv0."""
    num = float((dv0 * b).sum())
    den = float((dv0 * apply_A(dv0)).sum())
    return num / den if den > 0 else 0.0
