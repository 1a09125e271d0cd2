"""Pins for the oracle's network evaluation: hand-computed outputs and the
paper's own architecture constants (CPU only)."""
import json
import os

import numpy as np

import synthetic as syn
from oracle import mlp_forward, encode, round_bf16

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_hand_computed_two_layer_net():
    w = syn.MLPWeights([np.array([[1.0, -1.0], [2.0, 0.5]], np.float32), np.array([[1.0, 2.0]], np.float32)],
                       [np.array([0.5, -3.0], np.float32), np.array([0.1], np.float32)])
    # x=(1,2): z1 = (-0.5, 0) -> relu 0 -> 0.1 ; x=(3,1): z1=(2.5, 3.5) -> 2.5 + 7 + 0.1
    out = mlp_forward(np.array([[1.0, 2.0], [3.0, 1.0]]), w)
    assert np.allclose(out[:, 0], [0.1, 9.6], atol=1e-6)
    out_h, h = mlp_forward(np.array([[3.0, 1.0]]), w, return_hidden=True)
    assert np.allclose(h, [[2.5, 3.5]])


def test_bf16_emulation_is_exact_on_representable_inputs():
    g = np.random.default_rng(3)
    w = syn.MLPWeights([round_bf16(g.integers(-8, 8, (4, 3)) / 8.0).astype(np.float32),
                        np.array([[0.5, -0.25, 1.0, 2.0]], np.float32)],
                       [np.zeros(4, np.float32), np.zeros(1, np.float32)])
    x = g.integers(-16, 16, (5, 3)) / 16.0
    assert np.array_equal(mlp_forward(x, w, gemm="bf16"), mlp_forward(x, w))
    # a non-representable activation is rounded before the hidden layer
    x2 = np.array([[1.0 + 2.0 ** -10, 0.0, 0.0]])
    w2 = syn.MLPWeights([np.array([[1.0, 0, 0]], np.float32), np.array([[1.0]], np.float32)],
                        [np.zeros(1, np.float32), np.zeros(1, np.float32)])
    assert mlp_forward(x2, w2, gemm="bf16")[0, 0] == 1.0
    assert mlp_forward(x2, w2)[0, 0] == 1.0 + 2.0 ** -10


def test_paper_architecture_reading_matches_storage():
    c = json.load(open(GOLDEN))
    Di = c["intersection_network_input_dim"]["value"]
    assert Di == c["points_per_ray"]["value"] * encode(np.zeros((1, 3)), c["encoding_levels"]["value"]).shape[1]
    Df = c["feature_dim"]["value"]
    nb = c["residual_blocks"]["value"]
    Nc, Nf = c["coarse_bins"]["value"], c["fine_bins"]["value"]
    head = Di * Df + Df
    body = nb * 2 * (Df * Df + Df)
    tail = Df * (1 + Nc) + (1 + Nc) + Df * Nf + Nf       # (alpha, v_c) branch and v_f branch
    params = head + body + tail
    assert params == 2413249
    mb = params * 4 / 1e6
    nedf_mb = c["storage_nedf_plus_nerf_MB"]["value"] - c["storage_nerf_MB"]["value"]
    assert abs(mb - nedf_mb) < 0.5                         # 9.65 MB vs "13 MB - 3 MB"
    # the NeRF-shaped objects used here have the stated parameter count
    m = syn.nerf_model(2, 0)
    n = sum(w.size + b.size for w, b in zip(m.trunk.W + m.rgb.W, m.trunk.b + m.rgb.b))
    assert n == 513924


def test_fp8_calibration_amax_definition():
    """The calibration scales are the largest magnitudes / 448: scaling a
    batch so that its amax is known fixes them exactly."""
    from oracle import fp8_calibrate, round_e4m3
    g = np.random.default_rng(5)
    t = syn.normal_mlp(syn.rng(0, 63), [6 * 3, 8, 8, 2], hidden_gain=2.0)
    m = syn.Model(kind="nedf", bound=1.0, trunk=t, params=dict(enc_L=1))
    o = g.standard_normal((50, 3)) * 3
    d = g.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    sc = fp8_calibrate(m, o, d)
    assert sc.shape == (2, 2)
    assert np.isclose(sc[0, 0], np.abs(t.W[0]).max() / 448) and np.isclose(sc[1, 0], np.abs(t.W[1]).max() / 448)
    # the first layer's input amax is the largest |encoded feature|: sin/cos <= 1, |d| = 1, |o x d| <= |o|
    pl = np.concatenate([d, np.cross(o, d)], axis=1)
    assert np.abs(d).max() <= sc[0, 1] * 448 <= max(1.0, np.abs(pl).max()) + 1e-12
    # the scaled maxima quantise to the top code
    assert round_e4m3(np.abs(t.W[0]).max() / sc[0, 0]) == 448.0
