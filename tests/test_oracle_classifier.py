"""Pins of the oracle's multi-level classifier network (16 points, gamma_10,
residual MLP, S and S^-1 of Eq. 4, loss of Eq. 6) against closed forms,
special cases, brute force and finite differences."""
import numpy as np
import pytest

import synthetic as syn
from oracle import (line_points, encode_points, segment, segment_inverse, classifier_forward, classifier_decode,
                    classifier_eval, classifier_loss_and_grads, mlp_forward, nedf_pair, to_local)
from oracle.classifier import argmax_first


def _tiny(n_points=2, L=1, width=4, n_blocks=2, nc=4, nf=8, seed=0, bias_std=0.3):
    m = syn.classifier_model(1, 500 + seed, enc_L=L, n_points=n_points, width=width, n_blocks=n_blocks,
                             n_coarse=nc, n_fine=nf, bias_std=bias_std, block_scale=1.0)
    return m


def test_line_points_hand_example():
    # origin 3 units before the tangency point (0, 0.5, 0), bound 2
    o = np.array([[0.0, 0.5, -3.0]])
    d = np.array([[0.0, 0.0, 1.0]])
    x = line_points(o, d, 2.0)
    assert x.shape == (1, 16, 3)
    assert np.allclose(x[0, 0], [0.0, 0.25, -15.0 / 16.0], atol=0, rtol=0)
    assert np.allclose(x[0, 15], [0.0, 0.25, 15.0 / 16.0], atol=0, rtol=0)
    assert np.allclose(np.diff(x[0, :, 2]), 0.125, atol=0, rtol=0)


def test_line_points_depend_on_the_line_only():
    g = np.random.default_rng(1)
    o = g.standard_normal((50, 3)) * 3
    d = g.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x1 = line_points(o, d, 1.5)
    x2 = line_points(o + g.standard_normal((50, 1)) * 4 * d, d, 1.5)
    assert np.allclose(x1, x2, atol=1e-12)
    # symmetric about p_perp / l, which is orthogonal to d; spacing 2 / 16
    mid = x1.mean(axis=1)
    assert np.allclose(np.sum(mid * d, axis=1), 0.0, atol=1e-12)
    assert np.allclose(np.linalg.norm(np.diff(x1, axis=1), axis=2), 0.125, atol=1e-12)


def test_encode_points_layout():
    g = np.random.default_rng(2)
    x = g.uniform(-1.4, 1.4, (3, 16, 3))
    f = encode_points(x, 10)
    assert f.shape == (3, 1008)   # D_i of the appendix
    for j in (0, 7, 15):
        blk = f[:, 63 * j:63 * (j + 1)]
        assert np.array_equal(blk[:, :3], x[:, j])
        for lev in (0, 4, 9):
            for c in range(3):
                assert np.allclose(blk[:, 3 + 6 * lev + c], np.sin(2.0 ** lev * np.pi * x[:, j, c]), atol=1e-12)
                assert np.allclose(blk[:, 6 + 6 * lev + c], np.cos(2.0 ** lev * np.pi * x[:, j, c]), atol=1e-12)


def test_segment_edges_and_known_bins():
    l = 2.0
    c, f = segment(np.array([-l, l, 0.0, -l + 2 * l * 5 / 64 + (2 * l / 64) * 7 / 128]), l)
    assert list(c) == [0, 63, 32, 5] and list(f) == [0, 127, 0, 7]
    assert segment_inverse(5, 7, l) == -l + 2 * l * 5 / 64 + (2 * l / 64) * 7 / 128
    assert segment_inverse(0, 0, l) == -l


def test_segment_is_one_uniform_partition():
    # brute force: the (coarse, fine) pair is the cell of mu in a uniform
    # partition of [-l, l] into N_c N_f cells, and S^-1 gives its lower edge
    l, nc, nf = 1.25, 64, 128
    g = np.random.default_rng(3)
    mu = np.concatenate([g.uniform(-l, l, 20000), np.linspace(-l, l, 8193)[:-1] + 1e-9])
    c, f = segment(mu, l, nc, nf)
    cell = np.floor((mu + l) / (2 * l) * nc * nf)
    assert np.array_equal(c * nf + f, cell.astype(np.int64))
    lo = segment_inverse(c, f, l, nc, nf)
    assert np.all(lo <= mu + 1e-12) and np.all(mu < lo + 2 * l / (nc * nf) + 1e-12)


def test_argmax_first_maximum():
    v = np.array([[0.0, 3.0, 1.0, 3.0], [2.0, 2.0, 2.0, 2.0]])
    assert list(argmax_first(v)) == [1, 0]
    mu, p = classifier_decode(np.array([0.0, 2.0]), v, np.array([[0, 1, 5, 5, 0, 0, 0, 0.0]] * 2), 1.0)
    assert np.allclose(mu, [segment_inverse(1, 2, 1.0, 4, 8), segment_inverse(0, 2, 1.0, 4, 8)])
    assert np.allclose(p, [0.5, 1.0 / (1.0 + np.exp(-2.0))])


def test_forward_without_blocks_is_the_plain_mlp():
    m = _tiny(n_blocks=2)
    for k in range(1, 5):   # zero every block layer: h_16 = h_0
        m.trunk.W[k][:] = 0
        m.trunk.b[k][:] = 0
    g = np.random.default_rng(4)
    feats = g.standard_normal((7, m.trunk.W[0].shape[1]))
    a, vc, vf = classifier_forward(m, feats)
    plain = syn.MLPWeights([m.trunk.W[0], m.trunk.W[-1]], [m.trunk.b[0], m.trunk.b[-1]])
    out = mlp_forward(feats, plain)
    assert np.allclose(np.concatenate([a[:, None], vc, vf], axis=1), out, atol=1e-12)


def test_identity_blocks_double_the_stream():
    # W_1 = W_2 = I, zero biases: h + ReLU(ReLU(h)) = 2 h for h >= 0, so n
    # blocks scale the head output by 2^n (pins the skip path and the order)
    m = _tiny(width=4, n_blocks=3)
    for k in range(1, 7):
        m.trunk.W[k][:] = np.eye(4, dtype=np.float32)
        m.trunk.b[k][:] = 0
    g = np.random.default_rng(5)
    feats = g.standard_normal((5, m.trunk.W[0].shape[1]))
    a, vc, vf = classifier_forward(m, feats)
    h0 = np.maximum(feats @ m.trunk.W[0].T.astype(np.float64) + m.trunk.b[0], 0.0)
    want = (8.0 * h0) @ m.trunk.W[-1].T.astype(np.float64) + m.trunk.b[-1]
    assert np.allclose(np.concatenate([a[:, None], vc, vf], axis=1), want, atol=1e-12)


def test_constant_tail_gives_known_depth_and_routing():
    # zero tail weights, one-hot biases: every ray decodes to mu = S^-1(10, 20)
    m = syn.classifier_model(1, 7, n_blocks=2)
    m.trunk.W[-1][:] = 0
    b = np.zeros(193, np.float32)
    b[0] = 5.0
    b[1 + 10] = 1.0
    b[1 + 64 + 20] = 1.0
    m.trunk.b[-1][:] = b
    inst = syn.Instance(model=0, R=np.eye(3), T=np.array([0.0, 0.0, -5.0]), s=1.5)
    o = np.zeros((3, 3))
    d = np.array([[0.0, 0.0, -1.0], [0.05, 0.0, -1.0], [0.0, 0.3, -1.0]])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    hit, D, p, path = nedf_pair(m, None, inst, o, d, fallback=False)
    o_l, d_l = to_local(inst, o, d)
    t_perp = -np.sum(o_l * d_l, axis=1)
    mu = segment_inverse(10, 20, 1.0)
    assert np.all(hit) and np.all(path == 0)
    assert np.allclose(D, 1.5 * (t_perp - mu), atol=1e-12)
    assert np.allclose(p, 1.0 / (1.0 + np.exp(-5.0)))
    mu_l, z = classifier_eval(m, o_l, d_l)
    assert np.allclose(mu_l, mu) and np.allclose(z, 5.0)


def test_loss_at_zero_logits():
    # every logit 0: each BCE term is ln 2
    m = syn.classifier_model(1, 8, n_blocks=1)
    m.trunk.W[-1][:] = 0
    m.trunk.b[-1][:] = 0
    o, d = syn.training_rays(1, 9, 40)
    alpha = (np.arange(40) % 3 == 0).astype(np.float64)
    mu = np.linspace(-0.9, 0.9, 40)
    loss, bins, hitt, _ = classifier_loss_and_grads(m, o, d, mu, alpha)
    n_hit = alpha.sum()
    assert np.isclose(bins, 2 * np.log(2) * n_hit / 40)
    assert np.isclose(hitt, np.log(2))
    assert np.isclose(loss, bins + 0.1 * hitt)


def test_gradients_match_finite_differences():
    m = _tiny(n_points=2, L=1, width=5, n_blocks=2, nc=4, nf=8, seed=3)
    g = np.random.default_rng(6)
    o = g.standard_normal((12, 3)) * 2
    d = -o + g.standard_normal((12, 3)) * 0.3
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    alpha = (g.random(12) < 0.6).astype(np.float64)
    mu = g.uniform(-0.95, 0.95, 12)
    for k in range(len(m.trunk.W)):
        m.trunk.W[k] = m.trunk.W[k].astype(np.float64)
        m.trunk.b[k] = m.trunk.b[k].astype(np.float64)
    _, _, _, grads = classifier_loss_and_grads(m, o, d, mu, alpha)
    eps = 1e-6
    for k in range(len(m.trunk.W)):
        W = m.trunk.W[k]
        for (i, j) in [(0, 0), (W.shape[0] - 1, W.shape[1] - 1), (W.shape[0] // 2, W.shape[1] // 3)]:
            old = W[i, j]
            W[i, j] = old + eps
            lp = classifier_loss_and_grads(m, o, d, mu, alpha)[0]
            W[i, j] = old - eps
            lm = classifier_loss_and_grads(m, o, d, mu, alpha)[0]
            W[i, j] = old
            assert np.isclose(grads[k][0][i, j], (lp - lm) / (2 * eps), rtol=1e-5, atol=1e-9), (k, i, j)
        bb = m.trunk.b[k]
        old = bb[0]
        bb[0] = old + eps
        lp = classifier_loss_and_grads(m, o, d, mu, alpha)[0]
        bb[0] = old - eps
        lm = classifier_loss_and_grads(m, o, d, mu, alpha)[0]
        bb[0] = old
        assert np.isclose(grads[k][1][0], (lp - lm) / (2 * eps), rtol=1e-5, atol=1e-9), k
