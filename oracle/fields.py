"""Networks and density fields (FP64).  Test infrastructure only.

Network reading (stated in the design notes): fully connected ReLU layers of
the given widths followed by a linear head, no skip connections, weights
stored [out, in] as in PyTorch.  ``gemm`` selects how the GPU's matrix-core
layers are emulated: ``None`` is plain float64; ``"bf16"`` / ``"e4m3"`` round
every input of a hidden (matrix-core) layer, activations and weights, to that
format and accumulate in float64.  Narrow output heads always take unrounded
activations and weights.
"""
from __future__ import annotations

import numpy as np

from .geometry import encode, pluecker
from .rounding import round_bf16, round_e4m3

F64 = np.float64


def sigmoid(x):
    x = np.asarray(x, F64)
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-x))


def softplus(u):
    u = np.asarray(u, F64)
    return np.maximum(u, 0.0) + np.log1p(np.exp(-np.abs(u)))


def _rounder(gemm):
    if gemm is None:
        return lambda a: a
    if gemm == "bf16":
        return round_bf16
    if gemm == "e4m3":
        raise ValueError("e4m3 emulation needs per-layer scales: use mlp_forward(scales=...)")
    raise ValueError(gemm)


def mlp_forward(x, weights, gemm=None, scales=None, return_hidden=False, acc=None):
    """Hidden layers h_{i+1} = ReLU(W_i h_i + b_i), then a linear head.

    ``scales`` (E4M3 emulation): list of (w_scale, a_scale) per hidden layer;
    the layer computes (q(h/a) . q(W/w)^T) * a * w + b with q = round_e4m3.
    ``acc="f32"`` sums each hidden layer's products in float32 (in the BLAS
    routine's order) instead of float64: one of the summation orders a
    single-precision accumulator may take, used only to measure how much a
    result depends on that order, never as the expected value.
    Returns the head output, and optionally the last hidden activation."""
    h = np.asarray(x, F64)
    n = len(weights.W)
    rnd = _rounder(gemm) if scales is None else None
    for i in range(n):
        W = np.asarray(weights.W[i], F64)
        b = np.asarray(weights.b[i], F64)
        if i < n - 1:
            if scales is not None:
                ws, as_ = scales[i]
                qa, qw = round_e4m3(h / as_), round_e4m3(W / ws)
                if acc == "f32":
                    z = (qa.astype(np.float32) @ qw.T.astype(np.float32)).astype(F64) * (as_ * ws) + b
                else:
                    z = (qa @ qw.T) * (as_ * ws) + b
            elif acc == "f32":
                z = (rnd(h).astype(np.float32) @ rnd(W).T.astype(np.float32)).astype(F64) + b
            else:
                z = rnd(h) @ rnd(W).T + b
            h = np.maximum(z, 0.0)
        else:
            out = h @ W.T + b
    if return_hidden:
        return out, h
    return out


def sdf(shape, x):
    """Analytic signed distances for the SDF-biased synthetic objects:
    0 sphere r=0.6; 1 rounded box half-size 0.45 (rounding 0.05);
    2 torus (R=0.5, r=0.2) around y; 3 ellipsoid radii (0.7, 0.45, 0.35)
    (first-order distance approximation k0 (k0 - 1) / k1)."""
    x = np.asarray(x, F64)
    if shape == 0:
        return np.linalg.norm(x, axis=-1) - 0.6
    if shape == 1:
        q = np.abs(x) - (0.45 - 0.05)
        outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
        inside = np.minimum(np.max(q, axis=-1), 0.0)
        return outside + inside - 0.05
    if shape == 2:
        qx = np.sqrt(x[..., 0] ** 2 + x[..., 2] ** 2) - 0.5
        return np.sqrt(qx ** 2 + x[..., 1] ** 2) - 0.2
    if shape == 3:
        r = np.array([0.7, 0.45, 0.35])
        k0 = np.linalg.norm(x / r, axis=-1)
        k1 = np.linalg.norm(x / (r * r), axis=-1)
        return np.where(k1 > 0, k0 * (k0 - 1.0) / np.where(k1 > 0, k1, 1.0), -r.min())
    raise ValueError(shape)


def density(model, x, gemm=None, scales=None):
    """Volume density sigma(x) of a model at local points x [n,3].

    * sphere: sigma_max * sigmoid((radius - |x|) / width)   (density A)
    * slab:   sigma0 where z0 <= z <= z1, else 0
    * hard_sphere: sigma0 where |x| < radius, else 0
    * linear: c0 + c . x (a test field: affine along every ray)
    * mlp / nerf trunk: u = MLP(gamma_L(x)); ``softplus`` gives
      softplus(u), optionally zero outside |x| <= bound; ``sdf`` gives
      sigma_max * sigmoid(u - sdf(x) / width).
    """
    x = np.asarray(x, F64)
    p = model.params
    k = model.kind
    if k == "sphere":
        return p["sigma_max"] * sigmoid((p["radius"] - np.linalg.norm(x, axis=-1)) / p["width"])
    if k == "slab":
        z = x[..., 2]
        return np.where((z >= p["z0"]) & (z <= p["z1"]), p["sigma0"], 0.0)
    if k == "hard_sphere":
        return np.where(np.linalg.norm(x, axis=-1) < p["radius"], p["sigma0"], 0.0)
    if k == "linear":
        return p["c0"] + x @ np.asarray(p["c"], F64)
    if k in ("mlp", "nerf"):
        u = mlp_forward(encode(x, p["enc_L"]), model.trunk, gemm=gemm, scales=scales)[..., 0]
        return _sigma_from_raw(model, x, u)
    raise ValueError(k)


def _sigma_from_raw(model, x, u):
    p = model.params
    if p["sigma_mode"] == "softplus":
        s = softplus(u)
        if p.get("masked", False):
            s = np.where(np.linalg.norm(x, axis=-1) <= model.bound, s, 0.0)
        return s
    if p["sigma_mode"] == "sdf":
        return p["sigma_max"] * sigmoid(u - sdf(p["sdf_shape"], x) / p["width"])
    raise ValueError(p["sigma_mode"])


def surface_value(model, x, gemm=None):
    """Signed surface function used by the secant refinement: the logit of
    sigma / sigma_max for fields of the form sigma_max * sigmoid(q(x)), i.e.
    q(x), whose zero set is the iso-surface sigma = sigma_max / 2; positive
    inside.  ``linear`` (test field) gives c0 + c . x - iso."""
    x = np.asarray(x, F64)
    p = model.params
    if model.kind == "sphere":
        return (p["radius"] - np.linalg.norm(x, axis=-1)) / p["width"]
    if model.kind == "linear":
        return p["c0"] + x @ np.asarray(p["c"], F64) - p["iso"]
    if model.kind in ("mlp", "nerf") and p.get("sigma_mode") == "sdf":
        u = mlp_forward(encode(x, p["enc_L"]), model.trunk, gemm=gemm)[..., 0]
        return u - sdf(p["sdf_shape"], x) / p["width"]
    raise ValueError("no surface for this field")


def nerf_eval(model, x, d, gemm=None):
    """NeRF F_Theta(x, d) -> (sigma, rgb) in local space (Eq. 8).  Reading of
    the colour branch: concat(h_last, gamma_dirL(d)) -> ReLU layer -> 3 ->
    sigmoid; sigma as in ``density``."""
    x = np.asarray(x, F64)
    d = np.asarray(d, F64)
    p = model.params
    u, h = mlp_forward(encode(x, p["enc_L"]), model.trunk, gemm=gemm, return_hidden=True)
    sigma = _sigma_from_raw(model, x, u[..., 0])
    feat = np.concatenate([h, encode(d, p["dir_L"])], axis=-1)
    rgb = sigmoid(mlp_forward(feat, model.rgb, gemm=gemm))
    return sigma, rgb


def nedf_eval(model, o_l, d_l, gemm=None, scales=None):
    """Intersection network F_Phi (Eq. 1) in its regression form: input
    gamma_L of the line coordinates (d, o x d), output (mu_hat, hit logit z).
    A ``nedf16`` model is the multi-level classifier (Eq. 3-4), decoded to
    the same (mu / l, z) form."""
    if model.kind == "nedf16":
        from .classifier import classifier_eval
        if scales is not None:
            raise ValueError("the classifier network has no E4M3 form")
        return classifier_eval(model, o_l, d_l, gemm=gemm)
    pl, _ = pluecker(np.asarray(o_l, F64), np.asarray(d_l, F64))
    out = mlp_forward(encode(pl, model.params["enc_L"]), model.trunk, gemm=gemm, scales=scales)
    return out[..., 0], out[..., 1]


def fp8_calibrate(model, o_l, d_l):
    """Per-hidden-layer E4M3 scales of an intersection network from a
    calibration batch: w_scale = max|W| / 448 and a_scale = max|layer input|
    / 448 over the batch (float64 forward; 448 is the largest finite E4M3
    value).  Returns an array [n_hidden, 2] of (w_scale, a_scale)."""
    pl, _ = pluecker(np.asarray(o_l, F64), np.asarray(d_l, F64))
    h = encode(pl, model.params["enc_L"])
    n = len(model.trunk.W)
    out = []
    for i in range(n - 1):
        W = np.asarray(model.trunk.W[i], F64)
        out.append((np.abs(W).max() / 448.0, np.abs(h).max() / 448.0))
        h = np.maximum(h @ W.T + np.asarray(model.trunk.b[i], F64), 0.0)
    return np.array(out)
