"""NeDF training step: loss, gradients, Adam (FP64).  Test infrastructure only.

Reading of the loss (Eq. 6 in its regression form, keeping the 0.1 weight on
the mask term): for a batch of B local rays with labels mu* (in units of the
bounding radius, i.e. mu / l) and hit labels alpha in {0, 1},

    L = (1/B) sum_i [ alpha_i (mu_hat_i - mu*_i)^2 + 0.1 BCEwithLogits(z_i, alpha_i) ],
    BCEwithLogits(z, y) = softplus(z) - y z.

Gradients are the ordinary back-propagation of that loss through the ReLU
network.  Adam follows Kingma & Ba (2015) with bias correction, no weight
decay; the learning rate default 5e-4 is the paper's (training details).
"""
from __future__ import annotations

import numpy as np

from .geometry import encode, pluecker
from .fields import softplus, sigmoid
from .rounding import round_bf16

F64 = np.float64


def nedf_loss_and_grads(model, o_l, d_l, mu_label, hit_label, w_hit=0.1, gemm=None):
    """Returns (loss, mse_term, bce_term, grads) with grads a list of
    (dW [out,in], db [out]) per layer, all float64.

    ``gemm="bf16"`` emulates a bfloat16 matrix-core implementation: the
    encoded input, the hidden weights, every hidden activation and every
    back-propagated hidden-layer gradient are rounded to bfloat16 where they
    enter a matrix product (float64 accumulation); the head stays float64."""
    rnd = round_bf16 if gemm == "bf16" else (lambda a: a)
    pl, _ = pluecker(np.asarray(o_l, F64), np.asarray(d_l, F64))
    x = rnd(encode(pl, model.params["enc_L"]))
    Ws = [np.asarray(w, F64) for w in model.trunk.W]
    bs = [np.asarray(b, F64) for b in model.trunk.b]
    n = len(Ws)
    Wm = [rnd(w) if i < n - 1 else w for i, w in enumerate(Ws)]   # matrix-core copies
    B = x.shape[0]
    acts = [x]
    pre = []
    h = x
    for i in range(n):
        z = h @ Wm[i].T + bs[i]
        pre.append(z)
        h = rnd(np.maximum(z, 0.0)) if i < n - 1 else z
        acts.append(h)
    out = acts[-1]
    mu_hat, z = out[:, 0], out[:, 1]
    a = np.asarray(hit_label, F64)
    mu = np.asarray(mu_label, F64)
    mse = np.sum(a * (mu_hat - mu) ** 2) / B
    bce = np.sum(softplus(z) - a * z) / B
    loss = mse + w_hit * bce
    g = np.zeros_like(out)
    g[:, 0] = 2.0 * a * (mu_hat - mu) / B
    g[:, 1] = w_hit * (sigmoid(z) - a) / B
    grads = [None] * n
    for i in range(n - 1, -1, -1):
        if i < n - 1:
            g = rnd(g * (acts[i + 1] > 0))
        grads[i] = (g.T @ acts[i], g.sum(axis=0))
        g = g @ Wm[i]
    return loss, mse, bce, grads


def adam_step(params, grads, m, v, step, lr=5e-4, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of every array in ``params`` in
    place; ``step`` is the 1-based step number after this update."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= beta1
        mm += (1.0 - beta1) * g
        vv *= beta2
        vv += (1.0 - beta2) * g * g
        mhat = mm / (1.0 - beta1 ** step)
        vhat = vv / (1.0 - beta2 ** step)
        p -= lr * mhat / (np.sqrt(vhat) + eps)
