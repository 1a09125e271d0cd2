"""Intersection network in the paper's own form (FP64): a ray as 16 points
along its line, gamma_10 of each, a residual MLP and a two-level classifier
of mu (Sec. "Neural Depth Fields", Sec. "Intersection network", Eq. 3-4 and
6, appendix "Architecture" and hyper-parameters).  Test infrastructure only.

Readings (the paper leaves these open; each is listed in the design notes):

* Points.  The 16 points regularise the ray to the segment of the line that
  can hold an intersection: mu in [-l, l] around the tangency point p_perp,
  the same range the classifier covers.  Point k sits at the centre of the
  k-th of 16 equal cells, x_k = p_perp + mu_k d with mu_k = l ((2k + 1)/16 - 1),
  and enters the encoding divided by l (so a line through the bounding sphere
  gives points within radius sqrt(2)).  Encoding per point as elsewhere:
  [x, sin(2^j pi x), cos(2^j pi x)] for j < 10, 63 values; the 16 blocks
  are concatenated in point order (1,008 values, D_i of the appendix).
* Layers.  head h_0 = ReLU(W_h gamma + b_h); block b:
  h_{b+1} = h_b + ReLU(W_{b,2} ReLU(W_{b,1} h_b + b_{b,1}) + b_{b,2});
  tail rows (hit logit alpha_hat, N_c coarse logits, N_f fine logits) =
  W_t h_16 + b_t, the first 1 + N_c rows being the paper's first branch and
  the N_f others its second.
* Segment operator S: u = (mu + l) / (2 l); coarse bin c = floor(N_c u),
  fine bin f = floor(N_f (N_c u - c)), each clamped to its range.  Its
  inverse (Eq. 4) is the lower edge of the fine bin:
  mu = 2 l c / N_c + (2 l / N_c) f / N_f - l.
* Decoding: first maximum on ties (argmax); p = sigmoid(alpha_hat).
* Loss (Eq. 6): binary cross-entropy with logits, averaged over the bins of
  each level, the two bin terms counted only for rays that hit (a miss has
  no mu to segment), everything averaged over the batch:
  L = (1/B) sum_i [ alpha_i (BCE_c,i + BCE_f,i) + 0.1 BCE(alpha_hat_i, alpha_i) ].

``gemm="bf16"`` emulates a bfloat16 matrix-core evaluation: the encoded
input, every weight matrix (head, blocks and tail), and every activation
that enters a matrix product (head output, block intermediate, the residual
stream after each addition) rounded to bfloat16, products accumulated in
float64; biases and the tail's logits stay unrounded.
"""
from __future__ import annotations

import numpy as np

from .geometry import encode
from .fields import sigmoid, softplus
from .rounding import round_bf16

F64 = np.float64


def _rnd(gemm):
    if gemm is None:
        return lambda a: a
    if gemm == "bf16":
        return round_bf16
    raise ValueError(gemm)


def line_points(o_l, d_l, l, n_points=16):
    """The ray's points, divided by l: [n, n_points, 3] (reading above;
    Fig. 2b, Sec. "Neural Depth Fields")."""
    o_l = np.asarray(o_l, F64)
    d_l = np.asarray(d_l, F64)
    t_perp = -np.sum(o_l * d_l, axis=-1)
    p_perp = o_l + t_perp[:, None] * d_l
    c = (2.0 * np.arange(n_points) + 1.0) / n_points - 1.0
    return p_perp[:, None, :] / l + c[None, :, None] * d_l[:, None, :]


def encode_points(x, L=10):
    """gamma_L of every point, blocks concatenated in point order:
    [n, n_points * 3 (1 + 2L)]."""
    n, k, _ = x.shape
    return np.concatenate([encode(x[:, j, :], L) for j in range(k)], axis=-1)


def segment(mu, l, nc=64, nf=128):
    """Segment operator S (Sec. "Intersection network"): mu in [-l, l] to
    (coarse bin, fine bin)."""
    u = (np.asarray(mu, F64) + l) / (2.0 * l)
    c = np.clip(np.floor(nc * u), 0, nc - 1)
    f = np.clip(np.floor(nf * (nc * u - c)), 0, nf - 1)
    return c.astype(np.int64), f.astype(np.int64)


def segment_inverse(c, f, l, nc=64, nf=128):
    """S^{-1} of Eq. 4: lambda_1 c / N_c + lambda_2 f / N_f - l with
    lambda_1 = 2 l, lambda_2 = 2 l / N_c."""
    lam1, lam2 = 2.0 * l, 2.0 * l / nc
    return lam1 * np.asarray(c, F64) / nc + lam2 * np.asarray(f, F64) / nf - l


def _layers(model):
    W = [np.asarray(w, F64) for w in model.trunk.W]
    b = [np.asarray(v, F64) for v in model.trunk.b]
    return W, b


def classifier_forward(model, feats, gemm=None, keep=False, acc=None):
    """Network on encoded inputs [n, D_i].  Returns (alpha_hat [n],
    coarse logits [n, N_c], fine logits [n, N_f]) and, with ``keep``, the
    activations needed by back-propagation.  ``acc="f32"`` sums every
    matrix product in float32 (in the BLAS routine's order) instead of
    float64: one of the orders a single-precision accumulator may take, used
    only to measure how much a result depends on that order, never as the
    expected value."""
    rnd = _rnd(gemm)
    W, b = _layers(model)
    nb = model.params["n_blocks"]
    nc = model.params["n_coarse"]

    def mm(h, w):
        if acc == "f32":
            return (h.astype(np.float32) @ w.T.astype(np.float32)).astype(F64)
        return h @ w.T

    x = rnd(np.asarray(feats, F64))
    acts = {"x": x, "h": [], "a": [], "r": []}
    h = rnd(np.maximum(mm(x, rnd(W[0])) + b[0], 0.0))
    acts["h"].append(h)
    for k in range(nb):
        a = rnd(np.maximum(mm(h, rnd(W[1 + 2 * k])) + b[1 + 2 * k], 0.0))
        r = np.maximum(mm(a, rnd(W[2 + 2 * k])) + b[2 + 2 * k], 0.0)
        h = rnd(h + r)
        acts["a"].append(a)
        acts["r"].append(r)
        acts["h"].append(h)
    out = mm(h, rnd(W[-1])) + b[-1]
    res = (out[:, 0], out[:, 1:1 + nc], out[:, 1 + nc:])
    return (res, acts) if keep else res


def argmax_first(v):
    """Index of the first maximum of each row."""
    return np.argmax(np.asarray(v, F64), axis=-1)


def classifier_decode(alpha_hat, vc, vf, l):
    """mu = S^{-1}(argmax vc, argmax vf) (Eq. 4) and p = sigmoid(alpha_hat)."""
    nc, nf = vc.shape[-1], vf.shape[-1]
    return segment_inverse(argmax_first(vc), argmax_first(vf), l, nc, nf), sigmoid(alpha_hat)


def classifier_eval(model, o_l, d_l, gemm=None, logits=False):
    """F_Phi of Eq. 3 on local rays, decoded.  Returns (mu / l, alpha_hat),
    the form the regression network's output takes (so that the routing and
    depth of Eq. 2 are shared), plus the logits with ``logits``."""
    l = model.bound
    feats = encode_points(line_points(o_l, d_l, l, model.params["n_points"]), model.params["enc_L"])
    a, vc, vf = classifier_forward(model, feats, gemm=gemm)
    mu, _ = classifier_decode(a, vc, vf, l)
    return (mu / l, a, vc, vf) if logits else (mu / l, a)


def bce_logits(z, y):
    """Binary cross-entropy of a logit z against a label y in {0, 1}."""
    z = np.asarray(z, F64)
    return softplus(z) - np.asarray(y, F64) * z


def classifier_loss_and_grads(model, o_l, d_l, mu_label, hit_label, w_hit=0.1, gemm=None):
    """Loss of Eq. 6 (reading above) and its gradients by back-propagation.
    ``mu_label`` in local units (mu of Eq. 2 before any division by l).
    Returns (loss, bin_term, hit_term, grads) with grads a list of
    (dW [out, in], db [out]) in layer order.  With ``gemm="bf16"`` the
    back-propagated gradients are rounded to bfloat16 where they enter a
    matrix product, as the activations are in the forward pass."""
    rnd = _rnd(gemm)
    l = model.bound
    nc, nf = model.params["n_coarse"], model.params["n_fine"]
    nb = model.params["n_blocks"]
    feats = encode_points(line_points(o_l, d_l, l, model.params["n_points"]), model.params["enc_L"])
    (ah, vc, vf), A = classifier_forward(model, feats, gemm=gemm, keep=True)
    B = ah.shape[0]
    alpha = np.asarray(hit_label, F64)
    c, f = segment(mu_label, l, nc, nf)
    yc = np.zeros((B, nc))
    yc[np.arange(B), c] = 1.0
    yf = np.zeros((B, nf))
    yf[np.arange(B), f] = 1.0
    bins = alpha * (bce_logits(vc, yc).mean(axis=1) + bce_logits(vf, yf).mean(axis=1))
    hitt = bce_logits(ah, alpha)
    loss = np.sum(bins + w_hit * hitt) / B
    # gradient of the loss at the tail's outputs
    g = np.zeros((B, 1 + nc + nf))
    g[:, 0] = w_hit * (sigmoid(ah) - alpha) / B
    g[:, 1:1 + nc] = alpha[:, None] * (sigmoid(vc) - yc) / (nc * B)
    g[:, 1 + nc:] = alpha[:, None] * (sigmoid(vf) - yf) / (nf * B)
    g = rnd(g)                              # enters the tail's two matrix products
    W, _ = _layers(model)
    Wm = [rnd(w) for w in W]
    n = len(W)
    grads = [None] * n
    h_last = A["h"][-1]
    grads[n - 1] = (g.T @ h_last, g.sum(axis=0))
    gh = g @ Wm[n - 1]                      # gradient at h_16
    for k in range(nb - 1, -1, -1):
        i1, i2 = 1 + 2 * k, 2 + 2 * k
        h_in, a, r = A["h"][k], A["a"][k], A["r"][k]
        g2 = rnd(gh * (r > 0))              # at the second layer's pre-activation
        grads[i2] = (g2.T @ a, g2.sum(axis=0))
        g1 = rnd((g2 @ Wm[i2]) * (a > 0))   # at the first layer's pre-activation
        grads[i1] = (g1.T @ h_in, g1.sum(axis=0))
        gh = gh + g1 @ Wm[i1]               # skip path plus the block's branch
    g0 = rnd(gh * (A["h"][0] > 0))
    grads[0] = (g0.T @ A["x"], g0.sum(axis=0))
    return loss, float(np.sum(bins) / B), float(np.sum(hitt) / B), grads
