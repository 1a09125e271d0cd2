"""MX block-scaled E4M3 networks (FP64 emulation).  Test infrastructure only.

A finer alternative to per-layer FP8 scales: the OCP Microscaling (MX)
format gives every block of 32 values along the reduction dimension its own
power-of-two scale, kept as an E8M0 byte (exponent + 127, clamped to
0..254; an all-zero block takes the smallest scale), and each value is
stored as round_e4m3(v / X).  A product of an MX activation block and an MX
weight block is X_a X_w sum q_a q_w.

Reading of the scale choice: X is the smallest power of two with
amax / X <= 448 (E4M3's largest value), i.e. 2^(floor(log2 amax) - 8),
doubled when amax / that exceeds 448.  The format's suggested conversion
(2^(floor(log2 amax) - 8) alone) would clamp the largest values of about an
eighth of the blocks to 448 X, an error of up to 12.5 %; the doubled scale
costs only range at the bottom of E4M3's subnormals.

Reading (the method has no quantised form; this is the format's
definition applied to the regression-form intersection network): every
hidden layer's input and weight rows are quantised in blocks of 32
consecutive features; the encoded input groups the sine and cosine of 16
consecutive arguments (argument a = level * n + component, then the
identity components two per argument slot) into one block of 32; biases,
the float32 accumulation and the narrow head stay unquantised, the head
reading the last hidden layer's unrounded output.
"""
from __future__ import annotations

import numpy as np

from .geometry import encode, pluecker
from .rounding import round_e4m3

F64 = np.float64
E4M3_EMAX = 8
BLOCK = 32


def mx_exponent(amax):
    """Shared scale exponent of blocks with largest magnitude ``amax``: the
    smallest e with amax / 2^e <= 448 (floor(log2 amax) - 8, plus one when
    that leaves amax / 2^e above 448), clamped to the E8M0 range
    [-127, 127]; -127 for an all-zero block."""
    amax = np.asarray(amax, F64)
    pos = np.where(amax > 0, amax, 1.0)
    e = np.floor(np.log2(pos)) - E4M3_EMAX
    e = e + (pos / np.exp2(e) > 448.0)
    e = np.where(amax > 0, e, -127.0)
    return np.clip(e, -127.0, 127.0)


def mx_quantize(x, blocks):
    """Quantise the columns of x [n, K] block by block (``blocks``: list of
    column index arrays).  Returns (dequantised values q X [n, K],
    exponents [n, n_blocks]); columns in no block become zero."""
    x = np.asarray(x, F64)
    out = np.zeros_like(x)
    exps = np.zeros((x.shape[0], len(blocks)))
    for j, idx in enumerate(blocks):
        idx = np.asarray(idx, np.int64)
        if idx.size == 0:
            continue
        v = x[:, idx]
        e = mx_exponent(np.max(np.abs(v), axis=1))
        X = np.exp2(e)[:, None]
        out[:, idx] = round_e4m3(v / X) * X
        exps[:, j] = e
    return out, exps


def hidden_blocks(K):
    """Blocks of 32 consecutive features of a hidden layer's input."""
    return [np.arange(s, min(s + BLOCK, K)) for s in range(0, K, BLOCK)]


def encoded_blocks(n, L):
    """Blocks of the encoded input gamma_L of n components (natural feature
    order [p, sin 2^0 pi p, cos 2^0 pi p, ...]): argument slot a < n L is
    (level a // n, component a % n) and holds its sine and cosine; the
    identity components follow two per slot; a block takes the two features
    of each of 16 consecutive slots."""
    feats = []
    for a in range(n * L):
        level, comp = divmod(a, n)
        feats.append([n + 2 * n * level + comp, n + 2 * n * level + n + comp])
    for i in range((n + 1) // 2):
        feats.append([f for f in (2 * i, 2 * i + 1) if f < n])
    blocks = []
    for s in range(0, len(feats), BLOCK // 2):
        blocks.append(np.array([f for slot in feats[s:s + BLOCK // 2] for f in slot], np.int64))
    return blocks


def mlp_forward_mx(x, weights, in_blocks, acc=None):
    """Hidden layers h' = ReLU(MX(h) . MX(W)^T + b) with the weights' rows
    quantised over the same blocks as the input, then the linear head on the
    last unrounded hidden output.  ``acc="f32"`` sums in float32 (an
    alternative summation order, for measuring sensitivity only)."""
    h = np.asarray(x, F64)
    n = len(weights.W)
    blocks = in_blocks
    for i in range(n - 1):
        W = np.asarray(weights.W[i], F64)
        b = np.asarray(weights.b[i], F64)
        hq, _ = mx_quantize(h, blocks)
        Wq, _ = mx_quantize(W, blocks)
        if acc == "f32":
            z = (hq.astype(np.float32) @ Wq.T.astype(np.float32)).astype(F64) + b
        else:
            z = hq @ Wq.T + b
        h = np.maximum(z, 0.0)
        blocks = hidden_blocks(h.shape[1])
    return h @ np.asarray(weights.W[-1], F64).T + np.asarray(weights.b[-1], F64)


def nedf_eval_mx(model, o_l, d_l, acc=None):
    """The regression-form intersection network (Eq. 1) with MX E4M3
    inputs: (mu_hat, hit logit)."""
    pl, _ = pluecker(np.asarray(o_l, F64), np.asarray(d_l, F64))
    L = model.params["enc_L"]
    out = mlp_forward_mx(encode(pl, L), model.trunk, encoded_blocks(6, L), acc=acc)
    return out[..., 0], out[..., 1]
