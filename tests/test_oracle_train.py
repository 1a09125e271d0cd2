"""Pins for the oracle's NeDF loss, gradients and Adam (CPU only)."""
import math

import numpy as np

import synthetic as syn
from oracle import nedf_loss_and_grads, adam_step
from oracle.fields import nedf_eval, softplus


def _tiny_nedf(stream=0):
    g = syn.rng(0, 40 + stream)
    trunk = syn.normal_mlp(g, [18, 8, 8, 2], hidden_gain=2.0)
    for b in trunk.b:
        b[:] = (g.standard_normal(b.shape) * 0.1).astype(np.float32)
    return syn.Model(kind="nedf", bound=1.0, trunk=trunk, params=dict(enc_L=1))


def _batch(n=32):
    o, d = syn.training_rays(0, 50, n)
    g = syn.rng(0, 51)
    mu = g.uniform(-1, 1, n)
    a = (g.random(n) < 0.6).astype(np.float64)
    return o.astype(np.float64), d.astype(np.float64), mu, a


def test_gradients_match_central_differences():
    m = _tiny_nedf()
    o, d, mu, a = _batch()
    loss, mse, bce, grads = nedf_loss_and_grads(m, o, d, mu, a)
    # the loss is the stated sum, evaluated independently through the forward pass
    mh, z = nedf_eval(m, o, d)
    ref = np.mean(a * (mh - mu) ** 2) + 0.1 * np.mean(softplus(z) - a * z)
    assert abs(loss - ref) < 1e-13
    h = 1e-6
    for li in range(3):
        for arr, gi in ((m.trunk.W[li], grads[li][0]), (m.trunk.b[li], grads[li][1])):
            base = arr.astype(np.float64).copy()
            flat = base.reshape(-1)
            for k in range(0, flat.size, max(1, flat.size // 7)):
                orig = flat[k]
                vals = []
                for sgn in (+1, -1):
                    flat[k] = orig + sgn * h
                    tm = syn.Model(kind="nedf", bound=1.0, params=m.params,
                                   trunk=syn.MLPWeights([w.astype(np.float64) for w in m.trunk.W],
                                                        [b.astype(np.float64) for b in m.trunk.b]))
                    if arr is m.trunk.W[li]:
                        tm.trunk.W[li] = base.reshape(arr.shape).copy()
                    else:
                        tm.trunk.b[li] = base.reshape(arr.shape).copy()
                    vals.append(nedf_loss_and_grads(tm, o, d, mu, a)[0])
                flat[k] = orig
                fd = (vals[0] - vals[1]) / (2 * h)
                an = gi.reshape(-1)[k]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-8, (li, k, fd, an)


def test_bce_derivative_is_sigmoid_minus_label():
    for z in (-3.0, -0.2, 0.0, 1.7):
        for y in (0.0, 1.0):
            h = 1e-6
            fd = ((softplus(z + h) - y * (z + h)) - (softplus(z - h) - y * (z - h))) / (2 * h)
            assert abs(fd - (1 / (1 + math.exp(-z)) - y)) < 1e-9


def test_adam_first_and_second_step_closed_form():
    p = np.array([1.0, -2.0, 0.5, 3.0])
    g1 = np.array([0.3, -1e-3, 2.0, 0.0])
    m = np.zeros(4)
    v = np.zeros(4)
    p0 = p.copy()
    adam_step([p], [g1], [m], [v], step=1, lr=5e-4)
    # first step: m_hat = g, v_hat = g^2  =>  dp = -lr g / (|g| + eps)
    assert np.allclose(p - p0, -5e-4 * g1 / (np.abs(g1) + 1e-8), atol=1e-15)
    g2 = np.array([-0.1, 2e-3, 2.0, 1.0])
    p1 = p.copy()
    adam_step([p], [g2], [m], [v], step=2, lr=5e-4)
    m2 = 0.9 * 0.1 * g1 + 0.1 * g2
    v2 = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    mh = m2 / (1 - 0.81)
    vh = v2 / (1 - 0.999 ** 2)
    assert np.allclose(p - p1, -5e-4 * mh / (np.sqrt(vh) + 1e-8), atol=1e-15)
