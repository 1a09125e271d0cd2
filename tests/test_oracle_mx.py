"""Pins of the oracle's MX block-scaled E4M3 emulation (OCP Microscaling:
one power-of-two scale per block of 32 values) against hand-computed
blocks, its scale covariance, saturation and the block partitions."""
import numpy as np

import synthetic as syn
from oracle.mx import mx_exponent, mx_quantize, hidden_blocks, encoded_blocks, mlp_forward_mx
from oracle import mlp_forward


def test_exponent_hand_values():
    # floor(log2 amax) - 8, one more when amax / 2^e would exceed 448
    assert list(mx_exponent(np.array([448.0, 256.0, 255.9, 1.0, 0.3, 0.0, 2.0 ** 200, 448.5, 500.0, 1.76]))) == \
        [0.0, 0.0, 0.0, -8.0, -10.0, -127.0, 127.0, 1.0, 1.0, -7.0]


def test_quantize_hand_block():
    blk = [np.arange(32)]
    x = np.zeros((3, 32))
    x[0, :4] = [448.0, 1.0, -3.0, 0.5]          # scale 1: all representable
    x[1, :3] = [500.0, 300.0, 17.0]             # scale 2: 250 -> 256, 150 -> 144, 8.5 -> 8 (tie to even)
    x[2, :2] = [0.3, 0.01]                      # scale 2^-10: 307.2 -> 320, 10.24 -> 10
    q, e = mx_quantize(x, blk)
    assert np.array_equal(q[0, :4], x[0, :4]) and e[0, 0] == 0.0
    assert q[1, 0] == 512.0 and q[1, 1] == 288.0 and q[1, 2] == 16.0 and e[1, 0] == 1.0
    assert e[2, 0] == -10.0
    assert np.isclose(q[2, 0], 320.0 / 1024) and np.isclose(q[2, 1], 10.0 / 1024)


def test_quantize_scale_covariance_and_independent_blocks():
    g = np.random.default_rng(1)
    x = g.standard_normal((5, 64)) * 3
    q, e = mx_quantize(x, hidden_blocks(64))
    x2 = x.copy()
    x2[:, 32:] *= 2.0 ** 7                      # one block scaled by a power of two
    q2, e2 = mx_quantize(x2, hidden_blocks(64))
    assert np.array_equal(q2[:, :32], q[:, :32]) and np.array_equal(e2[:, 0], e[:, 0])
    assert np.array_equal(q2[:, 32:], q[:, 32:] * 2.0 ** 7) and np.array_equal(e2[:, 1], e[:, 1] + 7)
    # per block, v / X stays within 448 (nothing saturates) and above 224
    # for the largest value; in E4M3's normal range a value is off by at
    # most half a step (2^-4 relative)
    X = np.repeat(np.exp2(e), 32, axis=1)
    r = np.abs(x) / X
    assert np.all(r <= 448.0) and np.all(r.reshape(5, 2, 32).max(axis=2) > 224.0)
    normal = r >= 2.0 ** -6
    assert np.all(np.abs(q - x)[normal] <= np.abs(x)[normal] * 2.0 ** -4)


def test_block_partitions_cover_every_feature_once():
    for n, L in ((6, 8), (3, 10), (6, 0)):
        blocks = encoded_blocks(n, L)
        allf = np.concatenate(blocks)
        assert sorted(allf.tolist()) == list(range(n * (1 + 2 * L)))
        assert all(len(b) <= 32 for b in blocks)
    b = encoded_blocks(6, 8)
    # first block: sine and cosine of levels 0, 1 (all 6 components) and level 2 components 0..3
    assert sorted(b[0].tolist()) == sorted([6 + c for c in range(6)] + [12 + c for c in range(6)] +
                                           [18 + c for c in range(6)] + [24 + c for c in range(6)] +
                                           [30 + c for c in range(4)] + [36 + c for c in range(4)])
    assert [len(x) for x in hidden_blocks(256)] == [32] * 8


def test_forward_equals_plain_mlp_on_representable_operands():
    # weights and inputs already E4M3 values of one scale per block, and the
    # ReLU outputs representable too: MX quantisation changes nothing
    W = [np.array([[1.0, -2.0, 0.5, 0.0] * 8] * 32), np.eye(32)[:2] * 0.25]
    b = [np.zeros(32), np.zeros(2)]
    net = syn.MLPWeights(W, b)
    x = np.array([[1.0, 0.5, 2.0, 4.0] * 8, [0.25, 0.0, 1.0, 2.0] * 8])
    want = mlp_forward(x, net)
    got = mlp_forward_mx(x, net, hidden_blocks(32))
    assert np.allclose(got, want, rtol=0, atol=0)
