"""Pins for the oracle's marcher and composition against closed forms and
brute force (CPU only)."""
import math

import numpy as np

import synthetic as syn
from oracle import march, march_compose, camera_rays, density, to_local, sphere_chord
from oracle.render import march_instance

IDENT = syn.Instance(0, np.eye(3), np.zeros(3), 1.0)


def _axis_ray():
    return np.array([[0.0, 0.0, 4.0]]), np.array([[0.0, 0.0, -1.0]])


def _geo_depth(q, n, t0, delta):
    """sum_{k<n} q^k (1-q) (t0 + (k + 1/2) delta), by the geometric series."""
    S0 = (1 - q ** n)
    Sk = q * (1 - n * q ** (n - 1) + (n - 1) * q ** n) / (1 - q) ** 2
    return S0 * (t0 + delta / 2) + delta * (1 - q) * Sk


def test_slab_sample_aligned_exact_and_continuous():
    # slab |z| <= 1/2 crossed along -z from z = 4: path length 1 = 32 samples
    sigma0 = 3.0
    slab = syn.Model(kind="slab", params=dict(sigma0=sigma0, z0=-0.5, z1=0.5))
    o, d = _axis_ray()
    A, D, raw = march(lambda x: density(slab, x), o, d, np.array([2.0]), np.array([6.0]), 128)
    delta = 4.0 / 128
    q = math.exp(-sigma0 * delta)
    assert abs(A[0] - (1 - math.exp(-sigma0))) < 1e-12           # discrete A exact
    assert abs(raw[0] - _geo_depth(q, 32, 3.5, delta)) < 1e-12    # geometric series
    cont = 3.5 + 1 / sigma0 - math.exp(-sigma0) / (1 - math.exp(-sigma0))
    assert abs(D[0] - cont) < 2 * delta                            # O(delta)
    # convergence: finer sampling approaches the continuous depth
    A2, D2, _ = march(lambda x: density(slab, x), o, d, np.array([2.0]), np.array([6.0]), 4096)
    assert abs(D2[0] - cont) < abs(D[0] - cont) + 1e-15 and abs(D2[0] - cont) < 1e-3


def test_hard_sphere_discrete_and_analytic():
    sigma0, r = 7.0, 0.5
    hs = syn.Model(kind="hard_sphere", params=dict(sigma0=sigma0, radius=r))
    g = syn.rng(0, 11)
    N, tn, tf = 256, 2.0, 6.0
    delta = (tf - tn) / N
    for _ in range(20):
        o = np.array([[0.0, 0.0, 4.0]])
        ang, rad = g.uniform(0, 2 * math.pi), 0.45 * math.sqrt(g.uniform())
        tgt = np.array([rad * math.cos(ang), rad * math.sin(ang), 0.0])
        d = (tgt - o[0])
        d = (d / np.linalg.norm(d))[None]
        A, D, raw = march(lambda x: density(hs, x), o, d, np.array([tn]), np.array([tf]), N)
        tp = -float(o[0] @ d[0])
        b2 = float(o[0] @ o[0]) - tp * tp
        h = math.sqrt(r * r - b2)
        t_in, t_out = tp - h, tp + h
        tk = tn + (np.arange(N) + 0.5) * delta
        inside = (tk > t_in) & (tk < t_out)
        n_in = int(inside.sum())
        k0 = int(np.argmax(inside))
        q = math.exp(-sigma0 * delta)
        assert abs(A[0] - (1 - q ** n_in)) < 1e-12
        assert abs(raw[0] - _geo_depth(q, n_in, tk[k0] - delta / 2, delta)) < 1e-11
        c = t_out - t_in
        Ac = 1 - math.exp(-sigma0 * c)
        Dc = t_in + 1 / sigma0 - c * math.exp(-sigma0 * c) / Ac
        assert abs(A[0] - Ac) < 2 * sigma0 * delta
        assert abs(D[0] - Dc) < 2 * delta


def test_opacity_telescopes_for_any_field():
    _, b = syn.config1_models()
    cam = syn.config1_camera(8, 8)
    o, d = camera_rays(cam)
    N = 64
    a = np.full(len(o), 2.0)
    bb = np.full(len(o), 6.0)
    A, D, raw = march(lambda x: density(b, x), o, d, a, bb, N)
    delta = 4.0 / N
    t = 2.0 + (np.arange(N) + 0.5) * delta
    x = o[:, None, :] + t[None, :, None] * d[:, None, :]
    tauN = density(b, x.reshape(-1, 3)).reshape(len(o), N).sum(axis=1) * delta
    assert np.allclose(A, 1 - np.exp(-tauN), atol=1e-13, rtol=0)
    assert np.all((D >= 2.0) & (D <= 6.0))


def test_density_A_matches_analytic_sphere():
    a, _ = syn.config1_models()
    cam = syn.config1_camera()
    o, d = camera_rays(cam)
    depth, ident, opac = march_compose([a], [IDENT], o, d, 128, interval=(2.0, 6.0))
    tp = -np.sum(o * d, axis=1)
    b2 = np.sum(o * o, axis=1) - tp ** 2
    geo_hit = b2 < 0.25
    t_in = tp - np.sqrt(np.maximum(0.25 - b2, 0))
    hit = ident == 0
    assert np.all(hit[np.sqrt(b2) < 0.49])
    assert not np.any(hit[np.sqrt(b2) > 0.56])
    assert np.all(np.abs(depth[hit & geo_hit] - t_in[hit & geo_hit]) <= 4.0 / 128 + 0.03)
    assert 60 < hit.sum() < 140


def test_rigid_and_scale_invariance():
    _, b = syn.config1_models()
    model = syn.Model(kind="mlp", bound=1.0, trunk=b.trunk,
                      params=dict(enc_L=6, sigma_mode="softplus", masked=True))
    g = syn.rng(0, 12)
    R = syn.shoemake_rotation(g)
    T = np.array([0.3, -0.4, 0.2])
    s = 1.3
    inst = syn.Instance(0, R, T, s)
    cam = syn.Camera(eye=(0.2, 0.1, 5.0), at=(0.3, -0.4, 0.2), up=(0, 1, 0), fov_y_deg=30.0,
                     width=6, height=6)
    o, d = camera_rays(cam)
    v1, A1, D1 = march_instance(model, inst, o, d, 48)
    ol, dl = to_local(inst, o, d)
    v0, A0, D0 = march_instance(model, IDENT, ol, dl, 48)
    assert np.array_equal(v0, v1)
    assert np.allclose(A1[v1], A0[v0], atol=1e-12)
    assert np.allclose(D1[v1], s * D0[v0], atol=1e-11)


def test_compose_brute_force_and_permutation():
    g = syn.rng(0, 13)
    models = [syn.Model(kind="sphere", bound=1.0, params=dict(syn.SPHERE_A))]
    insts = []
    for k in range(6):
        insts.append(syn.Instance(0, syn.shoemake_rotation(g), g.uniform(-1.0, 1.0, 3),
                                  float(g.uniform(0.6, 1.4))))
    cam = syn.Camera(eye=(0.0, 0.0, 6.0), at=(0, 0, 0), up=(0, 1, 0), fov_y_deg=35.0,
                     width=8, height=8)
    o, d = camera_rays(cam)
    depth, ident, opac = march_compose(models, insts, o, d, 64)
    for p in range(64):
        best, bid, bA = np.inf, -1, 0.0
        for k, inst in enumerate(insts):
            v, A, D = march_instance(models[0], inst, o[p:p + 1], d[p:p + 1], 64)
            bA = max(bA, A[0])
            if v[0] and A[0] >= 0.5 and D[0] < best:
                best, bid = D[0], k
        assert bid == ident[p]
        assert (best == depth[p]) or (abs(best - depth[p]) < 1e-12)
        assert abs(bA - opac[p]) < 1e-15
    perm = [3, 0, 5, 1, 4, 2]
    depth2, ident2, _ = march_compose(models, [insts[i] for i in perm], o, d, 64)
    mapped = np.where(ident2 >= 0, np.array(perm)[ident2], -1)
    assert np.array_equal(mapped, ident)
    assert np.allclose(depth2, depth, atol=1e-12) or np.array_equal(depth2, depth)
