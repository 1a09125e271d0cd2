"""Pins for the oracle's rays, transforms and encodings (CPU only)."""
import math

import numpy as np
import pytest

import synthetic as syn
from oracle import camera_rays, to_local, pluecker, encode, sphere_chord, inverse_transform


def test_camera_ray_passes_through_projected_point():
    # Pin by the inverse map: perspective projection with focal length
    # f = H / (2 tan(fov/2)) sends a camera-frame point (X, Y, Z) (Z < 0 in
    # front) to pixel centre coordinates (W/2 + f X/-Z, H/2 - f Y/-Z).
    cam = syn.Camera(eye=(0.3, -0.2, 5.0), at=(0.3, -0.2, 0.0), up=(0, 1, 0),
                     fov_y_deg=40.0, width=64, height=48)
    f = cam.height / (2 * math.tan(math.radians(20.0)))
    for (i, j) in [(0, 0), (63, 47), (10, 30), (32, 24)]:
        depth = 3.7
        X = (i + 0.5 - cam.width / 2) * depth / f
        Y = -(j + 0.5 - cam.height / 2) * depth / f
        P = np.array(cam.eye) + np.array([X, Y, -depth])
        o, d = camera_rays(cam, [j * cam.width + i])
        v = P - o[0]
        assert np.linalg.norm(np.cross(v / np.linalg.norm(v), d[0])) < 1e-12
        assert np.dot(v, d[0]) > 0
        assert abs(np.linalg.norm(d[0]) - 1) < 1e-14


def test_camera_basis_and_symmetry():
    cam = syn.config1_camera()
    o, d = camera_rays(cam)
    assert np.allclose(o, [0, 0, 4])
    d = d.reshape(32, 32, 3)
    # mirror symmetry about the optical axis
    assert np.allclose(d[:, ::-1, 0], -d[:, :, 0], atol=1e-15)
    assert np.allclose(d[::-1, :, 1], -d[:, :, 1], atol=1e-15)
    assert np.all(d[..., 2] < 0)
    # rows run top to bottom (+y first)
    assert d[0, 0, 1] > 0 and d[-1, 0, 1] < 0


def test_rigid_inverse_roundtrip_and_scale():
    g = syn.rng(0, 3)
    for _ in range(5):
        R = syn.shoemake_rotation(g)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14) and abs(np.linalg.det(R) - 1) < 1e-13
        T = g.uniform(-3, 3, 3)
        s = float(g.uniform(0.5, 1.5))
        inst = syn.Instance(0, R, T, s)
        q = g.standard_normal((7, 3))
        v = s * q @ R.T + T                      # G(q) = s R q + T
        o_l, _ = to_local(inst, v, np.tile([1.0, 0, 0], (7, 1)))
        assert np.allclose(o_l, q, atol=1e-13)
        M, c = inverse_transform(R, T, s)
        assert np.allclose(v @ M.T + c, q, atol=1e-13)
        # a world point o + t d maps to o_l + (t/s) d_l
        o = g.standard_normal(3) * 4
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        t = 2.5
        ol, dl = to_local(inst, o[None], d[None])
        pl, _ = to_local(inst, (o + t * d)[None], d[None])
        assert np.allclose(pl[0], ol[0] + (t / s) * dl[0], atol=1e-13)
        assert abs(np.linalg.norm(dl) - 1) < 1e-14


def test_encoding_special_values_and_layout():
    # sin/cos of pi/6, pi/4, pi/3, pi/2 have closed forms
    p = np.array([[1 / 6, 1 / 4, 1 / 2]])
    e = encode(p, 2)
    assert e.shape == (1, 3 * 5)
    assert np.allclose(e[0, 0:3], [1 / 6, 1 / 4, 1 / 2])
    assert np.allclose(e[0, 3:6], [0.5, math.sqrt(2) / 2, 1.0], atol=1e-15)           # sin(pi p)
    assert np.allclose(e[0, 6:9], [math.sqrt(3) / 2, math.sqrt(2) / 2, 0.0], atol=1e-15)  # cos(pi p)
    assert np.allclose(e[0, 9:12], [math.sqrt(3) / 2, 1.0, 0.0], atol=1e-15)           # sin(2 pi p)
    assert np.allclose(e[0, 12:15], [0.5, 0.0, -1.0], atol=1e-15)                      # cos(2 pi p)
    # paper appendix: 16 points x 10 levels gives D_i = 1008
    assert encode(np.zeros((1, 16 * 3)), 10).shape[1] == 1008
    # config widths: xyz L=10 -> 63, dir L=4 -> 27, Pluecker L=8 -> 102, L=6 -> 39
    assert encode(np.zeros((1, 3)), 10).shape[1] == 63
    assert encode(np.zeros((1, 3)), 4).shape[1] == 27
    assert encode(np.zeros((1, 6)), 8).shape[1] == 102
    assert encode(np.zeros((1, 3)), 6).shape[1] == 39


def test_pluecker_origin_shift():
    g = syn.rng(0, 4)
    o = g.standard_normal((10, 3)) * 3
    d = g.standard_normal((10, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    lam = g.standard_normal(10)
    pl0, tp0 = pluecker(o, d)
    pl1, tp1 = pluecker(o + lam[:, None] * d, d)
    assert np.allclose(pl0, pl1, atol=1e-13)
    assert np.allclose(tp1, tp0 - lam, atol=1e-13)
    # tangency point is the closest point of the line to the local origin
    p = o + tp0[:, None] * d
    assert np.allclose(np.sum(p * d, axis=1), 0, atol=1e-13)
    assert np.allclose(np.linalg.norm(p, axis=1), np.linalg.norm(pl0[:, 3:], axis=1), atol=1e-13)


def test_sphere_chord_brute_force():
    g = syn.rng(0, 5)
    o = g.standard_normal((200, 3)) * 2.5
    d = g.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    a, b, valid = sphere_chord(o, d, 1.0)
    ts = np.linspace(0, 8, 80001)
    for k in range(200):
        inside = np.linalg.norm(o[k][None] + ts[:, None] * d[k][None], axis=1) <= 1.0
        if not inside.any():
            assert not valid[k] or (b[k] - a[k]) < 2e-4
            continue
        assert valid[k]
        assert abs(ts[inside].min() - a[k]) <= 1e-4 + 1e-12
        assert abs(ts[inside].max() - b[k]) <= 1e-4 + 1e-12
