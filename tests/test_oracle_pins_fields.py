"""Pins for parts of the oracle that the first pin set left open (CPU only):

* the four analytic signed distances of the SDF-biased objects, against
  points known to lie on each surface, the sign inside and outside, and
  brute-force distances (box by clamping, torus by a sampled circle);
* the E4M3 emulation of ``mlp_forward(scales=...)`` on hand-set operands
  whose quantisation and products are known exactly, plus a tie and a
  saturating case;
* the bfloat16 emulation of the training gradients: exact agreement with
  float64 on bfloat16-representable operands, and one hand-rounded case.
"""
import math

import numpy as np
import pytest

import synthetic as syn
from oracle import sdf, mlp_forward, nedf_loss_and_grads, round_bf16


# ---------------------------------------------------------------- sdf shapes
SURFACE = {
    0: [(0.6, 0, 0), (0, -0.6, 0), (0, 0, 0.6), (0.6 / math.sqrt(3),) * 3],
    # rounded box: half-size 0.45 on the faces, 0.4 + 0.05 n on the rounded corner
    1: [(0.45, 0, 0), (0, 0.45, 0.1), (-0.2, 0.3, -0.45), tuple(0.4 + 0.05 / math.sqrt(3) for _ in range(3))],
    # torus around y, tube centre radius 0.5, tube radius 0.2
    2: [(0.7, 0, 0), (0.3, 0, 0), (0.5, 0.2, 0), (0, -0.2, 0.5), (0, 0, -0.7),
        (0.5 * math.cos(1.0) + 0.2 * math.cos(1.0) * math.cos(0.4), 0.2 * math.sin(0.4),
         0.5 * math.sin(1.0) + 0.2 * math.sin(1.0) * math.cos(0.4))],
    # ellipsoid radii (0.7, 0.45, 0.35)
    3: [(0.7, 0, 0), (0, 0.45, 0), (0, 0, 0.35), (-0.7 * 0.6, 0.45 * 0.8, 0)],
}
INSIDE = {0: [(0, 0, 0), (0.3, 0.2, 0.1)], 1: [(0, 0, 0), (0.42, 0.1, -0.2)],
          2: [(0.5, 0, 0), (0, 0.1, 0.55)], 3: [(0, 0, 0), (0.5, 0.2, 0.1)]}
OUTSIDE = {0: [(0.7, 0, 0), (0.4, 0.4, 0.4)], 1: [(0.5, 0, 0), (0.44, 0.44, 0.44)],
           2: [(0, 0, 0), (0, 0.7, 0), (0.5, 0.25, 0)], 3: [(0, 0.5, 0), (0.5, 0.3, 0.2)]}


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_sdf_zero_on_known_surface_points(shape):
    x = np.array(SURFACE[shape], np.float64)
    assert np.allclose(sdf(shape, x), 0.0, atol=1e-12), sdf(shape, x)


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_sdf_sign_inside_and_outside(shape):
    assert np.all(sdf(shape, np.array(INSIDE[shape], np.float64)) < 0)
    assert np.all(sdf(shape, np.array(OUTSIDE[shape], np.float64)) > 0)


def test_sdf_exact_distances_at_hand_points():
    # sphere: |x| - 0.6
    assert abs(sdf(0, np.array([[0.0, 0.0, 0.0]]))[0] + 0.6) < 1e-15
    # rounded box: the centre is 0.45 from every face
    assert abs(sdf(1, np.array([[0.0, 0.0, 0.0]]))[0] + 0.45) < 1e-15
    # torus: tube centre is 0.2 inside; the origin is 0.3 outside; the y axis point (0, 0.7, 0)
    # is sqrt(0.5^2 + 0.7^2) - 0.2 from the tube (distinguishes the y axis from x or z)
    assert abs(sdf(2, np.array([[0.5, 0.0, 0.0]]))[0] + 0.2) < 1e-15
    assert abs(sdf(2, np.array([[0.0, 0.0, 0.0]]))[0] - 0.3) < 1e-15
    assert abs(sdf(2, np.array([[0.0, 0.7, 0.0]]))[0] - (math.hypot(0.5, 0.7) - 0.2)) < 1e-15
    # ellipsoid: along a principal axis the first-order form is the exact distance
    for axis, r in enumerate((0.7, 0.45, 0.35)):
        p = np.zeros((1, 3))
        p[0, axis] = 2 * r
        assert abs(sdf(3, p)[0] - r) < 1e-12
    assert abs(sdf(3, np.zeros((1, 3)))[0] + 0.35) < 1e-15


def test_sdf_box_and_torus_match_brute_force():
    g = np.random.default_rng(11)
    x = g.uniform(-1.0, 1.0, (400, 3))
    # rounded box = box of half-size 0.4 grown by 0.05: distance by clamping outside,
    # by the nearest face inside
    c = np.clip(x, -0.4, 0.4)
    out = np.linalg.norm(x - c, axis=1)
    inside = np.all(np.abs(x) <= 0.4, axis=1)
    face = np.min(0.4 - np.abs(x), axis=1)
    ref = np.where(inside, -face, out) - 0.05
    assert np.allclose(sdf(1, x), ref, atol=1e-12)
    # torus = points within 0.2 of the circle of radius 0.5 in the xz-plane
    phi = np.linspace(0, 2 * np.pi, 200001)
    circ = np.stack([0.5 * np.cos(phi), np.zeros_like(phi), 0.5 * np.sin(phi)], axis=1)
    for p in x[:40]:
        dmin = np.min(np.linalg.norm(circ - p, axis=1))
        assert abs(sdf(2, p[None])[0] - (dmin - 0.2)) < 1e-9


def test_sdf_ellipsoid_zero_set_is_the_ellipsoid():
    g = np.random.default_rng(12)
    v = g.standard_normal((500, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = np.array([0.7, 0.45, 0.35])
    on = v * r                                      # x^2/a^2 + y^2/b^2 + z^2/c^2 = 1
    assert np.allclose(sdf(3, on), 0.0, atol=1e-12)
    assert np.all(sdf(3, 1.05 * on) > 0) and np.all(sdf(3, 0.95 * on) < 0)


# ---------------------------------------------------------------- E4M3 emulation
def _net(Ws, bs):
    return syn.MLPWeights([np.asarray(w, np.float64) for w in Ws], [np.asarray(b, np.float64) for b in bs])


def test_fp8_scaled_layer_on_exact_operands():
    """h/a and W/w are E4M3 values, so the layer is (h/a).(W/w)^T a w + b
    with no rounding: computed by hand."""
    a_s, w_s = 0.25, 0.5
    h = np.array([[0.375, -0.5]])                  # h/a = (1.5, -2)
    W1 = np.array([[0.5, 0.25], [-1.5, 1.0]])      # W/w = ((1, 0.5), (-3, 2))
    b1 = np.array([0.1, 0.2])
    W2 = np.array([[2.0, 3.0]])
    b2 = np.array([0.5])
    # (h/a).(W/w)^T = (1.5 - 1, -4.5 - 4) = (0.5, -8.5); x a w = (0.0625, -1.0625); + b -> (0.1625, -0.8625)
    # ReLU -> (0.1625, 0); head 2 * 0.1625 + 0.5 = 0.825
    out, hid = mlp_forward(h, _net([W1, W2], [b1, b2]), scales=[(w_s, a_s)], return_hidden=True)
    assert np.allclose(hid, [[0.1625, 0.0]], atol=1e-15)
    assert abs(out[0, 0] - 0.825) < 1e-15


def test_fp8_scaled_layer_rounds_ties_to_even_and_saturates():
    W1 = np.array([[1.0, 0.0], [0.0, 1.0]])
    W2 = np.array([[1.0, 1.0]])
    z = [np.zeros(2), np.zeros(1)]
    # 1.0625 lies halfway between the E4M3 values 1 and 1.125: ties to even -> 1;
    # 1.1875 halfway between 1.125 and 1.25 -> 1.25 (even mantissa); 500 saturates to 448
    h = np.array([[1.0625, 1.1875], [500.0, 0.0]])
    out, hid = mlp_forward(h, _net([W1, W2], z), scales=[(1.0, 1.0)], return_hidden=True)
    assert np.array_equal(hid, [[1.0, 1.25], [448.0, 0.0]])
    # the weights are quantised with their own scale: W / 0.25 = 4.25 lies halfway between the
    # E4M3 values 4 and 4.5 (spacing 0.5 at 4) -> ties to even -> 4
    out2, hid2 = mlp_forward(np.array([[1.0, 0.0]]), _net([np.array([[1.0625, 0.0]]), np.array([[1.0]])],
                                                        [np.zeros(1), np.zeros(1)]),
                             scales=[(0.25, 1.0)], return_hidden=True)
    assert hid2[0, 0] == 1.0                       # 4 * 0.25
    # the head stays unquantised
    assert out2[0, 0] == 1.0


# ---------------------------------------------------------------- bf16 training emulation
def _dyadic_nedf():
    """A two-hidden-layer intersection network with enc_L = 0 (input = the
    line coordinates) whose weights are small dyadic numbers, chosen so that
    on the rays below every activation and every back-propagated hidden
    gradient is a bfloat16 value (8 significant bits)."""
    W = [np.array([[1.0, -0.5, 0.5, 0.25, 0.25, 0.0], [0.0, 0.0, 0.0, 1.0, -0.5, -1.0],
                   [0.5, 0.5, -1.0, -0.5, -0.5, 0.5], [0.5, -1.0, 0.25, 1.0, -0.5, 0.0]], np.float32),
         np.array([[-0.25, 1.0, 0.5, 0.0], [1.0, -0.5, 1.0, 0.0], [0.0, 1.0, 0.0, 0.5]], np.float32),
         np.array([[0.0, 0.25, -0.25], [-0.25, -0.25, 0.0]], np.float32)]
    b = [np.array([0.0, 0.0, 0.0, 0.25], np.float32), np.array([0.125, 0.125, 0.0], np.float32),
         np.zeros(2, np.float32)]
    return syn.Model(kind="nedf", bound=1.0, trunk=syn.MLPWeights(W, b), params=dict(enc_L=0))


def test_bf16_training_emulation_exact_on_representable_operands():
    m = _dyadic_nedf()
    # d = +z; o = (0.5, 0.25, -3) -> o x d = (0.25, -0.5, 0): every input a short dyadic number
    o = np.array([[0.5, 0.25, -3.0], [-1.0, 0.5, 2.0]])
    d = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    mu = np.array([0.25, -0.5])
    a = np.array([1.0, 1.0])
    # w_hit = 0 keeps the output gradient dyadic (the BCE derivative is not)
    r64 = nedf_loss_and_grads(m, o, d, mu, a, w_hit=0.0)
    r16 = nedf_loss_and_grads(m, o, d, mu, a, w_hit=0.0, gemm="bf16")
    assert r64[0] == r16[0]
    for (dw64, db64), (dw16, db16) in zip(r64[3], r16[3]):
        assert np.array_equal(dw64, dw16) and np.array_equal(db64, db16)
    # and the gradients are not trivially zero
    assert any(np.abs(g[0]).sum() > 0 for g in r64[3])
    # the weight gradients themselves are not all bfloat16 values: they are
    # float32-accumulated outputs, never rounded by the emulation
    assert any(not np.array_equal(round_bf16(g[0]), g[0]) for g in r64[3])


def test_bf16_training_emulation_hand_rounded_one_layer():
    """One hidden unit, enc_L = 0, input m_x = 1 + 2^-9 (rounds to 1 in
    bfloat16, which keeps 8 significant bits), all other inputs zero.
    Hidden h = ReLU(w m_x) with w = 1 + 2^-7 (a bfloat16 value); head
    mu_hat = 2 h, z = 0; label mu* = 0, alpha = 1, B = 1, w_hit = 0.

    bfloat16 emulation: x = 1, h = w = 1 + 2^-7 (representable, kept),
    mu_hat = 2 + 2^-6, dL/dmu_hat = 2 mu_hat = 4 + 2^-5;
    head gradient dW = g h = (4 + 2^-5)(1 + 2^-7);
    back-propagated g_h = 2 (4 + 2^-5) = 8 + 2^-4, which is a bfloat16 value
    (the spacing at 8 is 2^-4) and is kept; first-layer dW = g_h x = 8 + 2^-4.
    float64: x = 1 + 2^-9, h = (1 + 2^-7)(1 + 2^-9), and the gradients follow."""
    W = [np.zeros((1, 6), np.float32), np.array([[2.0], [0.0]], np.float32)]
    W[0][0, 3] = 1.0 + 2.0 ** -7
    b = [np.zeros(1, np.float32), np.zeros(2, np.float32)]
    m = syn.Model(kind="nedf", bound=1.0, trunk=syn.MLPWeights(W, b), params=dict(enc_L=0))
    # line coordinates (d, o x d) with d = +z and o = (0, 1 + 2^-9, 0): o x d = (1 + 2^-9, 0, 0)
    o = np.array([[0.0, 1.0 + 2.0 ** -9, 0.0]])
    d = np.array([[0.0, 0.0, 1.0]])
    mu, a = np.array([0.0]), np.array([1.0])
    loss, mse, bce, gr = nedf_loss_and_grads(m, o, d, mu, a, w_hit=0.0, gemm="bf16")
    w = 1.0 + 2.0 ** -7
    muh = 2.0 * w
    assert mse == muh ** 2
    g_out = 2.0 * muh
    assert gr[1][0][0, 0] == g_out * w and gr[1][0][1, 0] == 0.0
    g_h = 2.0 * g_out
    assert round_bf16(g_h) == g_h                  # 8 + 2^-4 is representable
    assert gr[0][0][0, 3] == g_h * 1.0             # the rounded input, not 1 + 2^-9
    assert gr[0][1][0] == g_h
    # float64 reference keeps the unrounded input
    loss64, mse64, _, gr64 = nedf_loss_and_grads(m, o, d, mu, a, w_hit=0.0)
    x = 1.0 + 2.0 ** -9
    assert mse64 == (2.0 * w * x) ** 2
    assert gr64[0][0][0, 3] == 2.0 * 2.0 * (2.0 * w * x) * x
    # a back-propagated gradient that is not a bfloat16 value is rounded:
    # with head weight 2 + 2^-6 the hidden gradient 2 mu_hat (2 + 2^-6) needs more than 8 significant bits
    W2 = [W[0].copy(), np.array([[2.0 + 2.0 ** -6], [0.0]], np.float32)]
    m2 = syn.Model(kind="nedf", bound=1.0, trunk=syn.MLPWeights(W2, b), params=dict(enc_L=0))
    _, _, _, g2 = nedf_loss_and_grads(m2, o, d, mu, a, w_hit=0.0, gemm="bf16")
    muh2 = (2.0 + 2.0 ** -6) * w
    gh2 = 2.0 * muh2 * (2.0 + 2.0 ** -6)
    assert round_bf16(gh2) != gh2
    assert g2[0][1][0] == round_bf16(gh2)
